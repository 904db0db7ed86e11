"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the header declares, and plan creation validates descriptors."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2505_03352_amd import _abi
from paper_2505_03352_amd.plan import Plan, freqs_of, grid_design_of
from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "yeeopt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(yo_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.yo_version()


def _create(dev, **over):
    grid, design = grid_design_of(dev)
    grid.update(over.pop("grid", {}))
    design.update(over.pop("design", {}))
    freqs = over.pop("freqs", freqs_of(dev))
    srcs = over.pop("srcs", [m.plane for m in dev.sources])
    ports = over.pop("ports", [m.plane for m in dev.ports])
    return Plan(grid, design, over.pop("n_steps", dev.n_steps), freqs, srcs, ports, device="cpu")


def test_plan_create_and_workspace_size():
    dev = configs.realistic()
    p = _create(dev)
    # fields alone: 6 rhs x 2 buffers x 6 components x padded cells x 4 B
    cells = dev.nz * dev.ny * ((dev.nx + 31) // 32 * 32)
    assert p.workspace_bytes > 6 * 12 * cells * 4
    assert p.workspace_bytes < 6 * 12 * cells * 4 * 1.5
    assert p.n_rhs == 6
    p.close()


def test_multiport_fits_one_gpu():
    dev = configs.multiport()
    p = _create(dev)
    assert p.n_rhs == 25
    assert p.workspace_bytes < 60e9
    p.close()


def test_unstable_courant_rejected():
    dev = configs.tiny()
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, grid={"courant": 0.6})
    assert e.value.status == _abi.YO_EUNSTABLE


def test_design_touching_pml_rejected():
    dev = configs.tiny()
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, design={"i0": 8})
    assert e.value.status == _abi.YO_EINVAL


def test_plane_inside_pml_rejected():
    dev = configs.tiny()
    from workloads import Plane
    bad = Plane(0, 3, 20, 10, 5, 5)
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, srcs=[bad])
    assert e.value.status == _abi.YO_EINVAL


def test_odd_supersample_rejected():
    dev = configs.tiny()
    with pytest.raises(_abi.YeeOptError):
        _create(dev, design={"supersample": 3})


def test_window_outside_run_rejected():
    dev = configs.tiny()
    f = freqs_of(dev)
    f[0].win_start = dev.n_steps - 10
    f[0].win_len = 20
    with pytest.raises(_abi.YeeOptError):
        _create(dev, freqs=f)


def test_too_many_ports_unsupported():
    dev = configs.tiny()
    ports = [dev.ports[0].plane] * 9
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, ports=ports)
    assert e.value.status == _abi.YO_EUNSUPPORTED


def test_calls_before_bind_fail_cleanly():
    dev = configs.tiny()
    p = _create(dev)
    L = _abi.lib()
    assert L.yo_reset(p.handle, _abi.YO_BOTH, None) == _abi.YO_EWORKSPACE
    assert L.yo_finalize(p.handle, _abi.YO_BOTH, None) == _abi.YO_EWORKSPACE
    assert L.yo_set_tiling(p.handle, 8, 16, 0) == _abi.YO_EINVAL
    assert L.yo_set_tiling(p.handle, 4, 3, 0) == _abi.YO_EINVAL
    assert L.yo_set_tiling(p.handle, 4, 64, 0) == _abi.YO_EINVAL
    assert L.yo_set_tiling(p.handle, 4, 16, 512) == _abi.YO_EINVAL
    assert L.yo_set_tiling(p.handle, 4, 8, 3) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 511) == _abi.YO_OK
    p.close()


def test_model_bytes_matches_traffic_model():
    dev = configs.realistic()
    p = _create(dev)
    b, c = p.model_bytes(_abi.YO_BOTH)
    assert c == 6 * dev.cells
    per = b / c
    assert 48 + 2 <= per <= 70
    p.close()


def test_size_limits_rejected():
    dev = configs.tiny()
    # a state array of one right-hand side beyond 2 GiB
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, grid={"nx": 700, "ny": 700, "nz": 300})
    assert e.value.status == _abi.YO_EUNSUPPORTED
    # a grid too small for its CPML and tiles
    with pytest.raises(_abi.YeeOptError) as e:
        _create(dev, grid={"nx": 3})
    assert e.value.status == _abi.YO_EINVAL


def test_morphology_arguments_and_workspace():
    dev = configs.tiny()
    p = _create(dev)
    base = p.workspace_bytes
    L = _abi.lib()
    h = p.handle
    assert L.yo_set_morphology(h, b"edx", 3.0, 20.0) == _abi.YO_EINVAL
    assert L.yo_set_morphology(h, b"ededededd", 3.0, 20.0) == _abi.YO_EINVAL
    assert L.yo_set_morphology(h, b"ed", 0.0, 20.0) == _abi.YO_EINVAL
    assert L.yo_set_morphology(h, b"ed", 3.0, 0.0) == _abi.YO_EINVAL
    assert L.yo_set_morphology(h, b"ed", 3.0, 81.0) == _abi.YO_EINVAL
    assert L.yo_set_morphology(h, b"ed", 16.5, 20.0) == _abi.YO_EUNSUPPORTED   # radius 33
    assert L.yo_set_morphology(h, b"edde", 3.0, 20.0) == _abi.YO_OK
    nb = ct.c_size_t()
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK
    S, U, V = dev.supersample, dev.supersample * (dev.md + 4), dev.supersample * (dev.nd + 4)
    DD = S * dev.md * S * dev.nd
    assert nb.value >= base + 4 * (5 * U * V + 4 * DD + 4 * DD + 2 * 113)
    assert nb.value < base + 4 * (5 * U * V + 8 * DD + 2 * 113) + 4096
    assert L.yo_set_morphology(h, None, 0.0, 0.0) == _abi.YO_OK          # off again
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK and nb.value == base
    p.close()
    # through the binding: the device description carries the filters
    dev.morph_ops, dev.morph_d, dev.morph_alpha = "edde", 3.0, 20.0
    q = _create(dev)
    assert q.morph_ops == "edde" and q.workspace_bytes > base
    q.close()


def test_pulse_arguments_and_workspace():
    dev = configs.realistic()
    p = _create(dev)
    base = p.workspace_bytes
    L = _abi.lib()
    h = p.handle
    w0, sig, t0 = dev.pulse()
    om = w0 / dev.dt()
    assert L.yo_set_pulse(h, -om, sig, t0) == _abi.YO_EINVAL
    assert L.yo_set_pulse(h, om, sig, -1.0) == _abi.YO_EINVAL
    assert L.yo_set_pulse(h, 1.2 * np.pi / dev.dt(), sig, t0) == _abi.YO_EINVAL   # above pi / dt
    assert L.yo_set_pulse(h, om, sig, t0) == _abi.YO_OK
    nb = ct.c_size_t()
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK
    # 2 stepped right-hand sides instead of 6: fields and CPML memories shrink 3x
    assert nb.value < 0.45 * base
    n = ct.c_int()
    assert L.yo_rhs_count(h, ct.byref(n)) == _abi.YO_OK and n.value == 6   # output numbering kept
    b, c = ct.c_double(), ct.c_double()
    assert L.yo_model_bytes(h, _abi.YO_BOTH, ct.byref(b), ct.byref(c)) == _abi.YO_OK
    assert c.value == 2 * dev.cells
    assert L.yo_set_pulse(h, 0.0, 0.0, 0.0) == _abi.YO_OK                 # off again
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK and nb.value == base
    p.close()


def test_two_term_coefficient_arguments_and_workspace():
    dev = configs.micro_demux()
    p = _create(dev)
    base = p.workspace_bytes
    L = _abi.lib()
    h = p.handle
    assert L.yo_set_alpha_terms(h, 3) == _abi.YO_EINVAL
    assert L.yo_set_alpha_terms(h, 2) == _abi.YO_OK
    nb = ct.c_size_t()
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK and nb.value > base
    w0, sig, t0 = dev.pulse()
    assert L.yo_set_pulse(h, w0 / dev.dt(), sig, t0) == _abi.YO_EUNSUPPORTED
    assert L.yo_set_alpha_terms(h, 1) == _abi.YO_OK
    assert L.yo_workspace_bytes(h, ct.byref(nb)) == _abi.YO_OK and nb.value == base
    assert L.yo_set_pulse(h, w0 / dev.dt(), sig, t0) == _abi.YO_OK
    assert L.yo_set_alpha_terms(h, 2) == _abi.YO_EUNSUPPORTED
    p.close()
    # a port whose next plane would enter the CPML
    m = dev.ports[0].plane
    edge = type(m)(m.axis, dev.nx - dev.npml[1] - 1, m.lo0, m.lo1, m.n0, m.n1)
    q = _create(dev, ports=[edge, dev.ports[1].plane])
    assert _abi.lib().yo_set_alpha_terms(q.handle, 2) == _abi.YO_EINVAL
    q.close()


def test_static_workspace_rejects_a_plan_beyond_its_size():
    """The allocation-free binding refuses, before touching any device, a plan
    whose workspace exceeds the static array (32 MiB)."""
    dev = configs.realistic()
    p = _create(dev)
    assert p.workspace_bytes > 32 << 20
    with pytest.raises(_abi.YeeOptError) as e:
        _abi.call("yo_bind_static_workspace", p.handle, None)
    assert e.value.status == _abi.YO_EWORKSPACE
    assert "static workspace" in str(e.value)
    p.close()


def test_dft_stride_arguments():
    """yo_set_dft_stride needs a pulse, a stride in [1, 64], a pulse whose
    spectrum vanishes at the aliases, and no workspace yet."""
    dev = configs.tiny()
    p = _create(dev)
    L = _abi.lib()
    assert L.yo_set_dft_stride(p.handle, 4) == _abi.YO_EINVAL          # no pulse
    w0 = 2 * np.pi * 299792458.0 / 1.55e-6
    assert L.yo_set_pulse(p.handle, w0, 80.0, 400.0) == _abi.YO_OK
    assert L.yo_set_dft_stride(p.handle, 0) == _abi.YO_EINVAL
    assert L.yo_set_dft_stride(p.handle, 65) == _abi.YO_EINVAL
    assert L.yo_set_dft_stride(p.handle, 4) == _abi.YO_OK
    # a pulse a few steps long has a spectrum wide enough to alias
    assert L.yo_set_pulse(p.handle, w0, 1.5, 10.0) == _abi.YO_OK
    assert L.yo_set_dft_stride(p.handle, 8) == _abi.YO_EINVAL
    assert b"alias" in L.yo_last_error()
    p.close()


def test_time_blocking_arguments_and_workspace():
    """yo_set_time_blocking adds one state buffer per right-hand side; tiling
    flag 512 needs it and does not combine with flag 16; flag 1024 needs 512."""
    dev = configs.tiny()
    p = _create(dev)
    L = _abi.lib()
    b1 = p.workspace_bytes
    assert L.yo_set_tiling(p.handle, 4, 16, 512) == _abi.YO_EINVAL
    assert L.yo_set_time_blocking(p.handle, 3) == _abi.YO_EINVAL
    assert L.yo_set_time_blocking(p.handle, 2) == _abi.YO_OK
    nb = ct.c_size_t()
    assert L.yo_workspace_bytes(p.handle, ct.byref(nb)) == _abi.YO_OK
    nxp = (dev.nx + 2 + 31) // 32 * 32
    one_buffer = 6 * 4 * (dev.nz + 2) * (dev.ny + 2) * nxp
    assert nb.value - b1 >= 2 * one_buffer          # forward + adjoint right-hand side
    assert L.yo_set_tiling(p.handle, 4, 16, 512) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 16) == _abi.YO_EINVAL
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 256) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 1024) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 1024) == _abi.YO_EINVAL         # needs 512
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 2048 | 128) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 2048) == _abi.YO_EINVAL         # needs 512
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 4096) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 4096) == _abi.YO_EINVAL         # needs 512
    assert L.yo_set_tiling(p.handle, 4, 16, 512 | 8192) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 8192) == _abi.YO_EINVAL         # needs 512
    assert L.yo_set_tiling(p.handle, 4, 16, 16384) == _abi.YO_OK
    assert L.yo_set_tiling(p.handle, 4, 16, 16384 | 4) == _abi.YO_EINVAL     # not cooperative
    assert L.yo_set_tiling(p.handle, 4, 16, 32768) == _abi.YO_EINVAL
    assert L.yo_set_time_blocking(p.handle, 1) == _abi.YO_OK
    assert L.yo_workspace_bytes(p.handle, ct.byref(nb)) == _abi.YO_OK and nb.value == b1
    p.close()
