"""Python handle of one yeeopt plan.  Torch supplies device memory and the
stream; every computation runs in the HIP library through the C ABI."""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import YO_ADJOINT, YO_BOTH, YO_FORWARD, call

C0 = 299792458.0


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ct.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if t.is_conj() or t.is_neg():
        # a lazy conjugate/negative view: data_ptr() holds the unconjugated values
        raise ValueError("resolve conjugate/negative views before passing them to the library")
    return ct.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, device, dtype) -> torch.Tensor:
    """Materialised, contiguous device copy (resolves lazy conj/neg views)."""
    return t.to(device, dtype).resolve_conj().resolve_neg().contiguous()


def _host_c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, np.complex128))


@dataclass
class FreqSpec:
    omega: float            # rad/s
    ramp_steps: float
    win_start: int
    win_len: int


class Plan:
    """One geometry with its forward sources, output ports and wavelengths.

    Right-hand sides: forward (src s, freq f) -> f*n_src + s; adjoint (port p,
    freq f) -> n_src*n_freq + f*n_ports + p.
    """

    def __init__(self, grid: dict, design: dict, n_steps: int, freqs: Sequence[FreqSpec],
                 src_planes: Sequence, port_planes: Sequence, device="cuda", pulse=None,
                 two_term: bool = False, time_blocking: int = 1):
        """pulse: None, or (omega0 rad/s, sigma steps, t0 steps[, DFT stride])
        for pulse excitation (one run per source and per port for all
        wavelengths; the DFT samples every stride-th step, default 1).
        two_term: the modal coefficient with both of its terms (App. A).
        time_blocking: 2 gives the plan a third state buffer so that tiling
        flag 512 can advance its interior two steps per launch."""
        self.device = torch.device(device)
        self.grid = dict(grid)
        self.design = dict(design)
        self.n_steps = int(n_steps)
        self.freqs = list(freqs)
        self.n_freq = len(self.freqs)
        self.n_src = len(src_planes)
        self.n_ports = len(port_planes)
        self.src_planes = list(src_planes)
        self.port_planes = list(port_planes)
        g = _abi.yo_grid(grid["nx"], grid["ny"], grid["nz"], grid["dx"], grid["dy"], grid["dz"],
                         grid["courant"], (ct.c_int * 6)(*grid["npml"]), grid.get("pml_m", 3.0),
                         grid.get("pml_sigma_scale", 1.0), grid.get("pml_kappa_max", 1.0),
                         grid.get("pml_a_max", 0.0))
        d = _abi.yo_design(design["i0"], design["j0"], design["md"], design["nd"], design["k_lo"],
                           design["k_hi"], design["mc"], design["nc"], design["filter_r"],
                           design["supersample"], design["eps_core"], design["eps_clad"],
                           design["sobel_delta"])
        fr = (_abi.yo_freq * self.n_freq)(*[_abi.yo_freq(f.omega, f.ramp_steps, f.win_start,
                                                          f.win_len) for f in self.freqs])
        sp = (_abi.yo_plane * max(1, self.n_src))(*[_abi.yo_plane(p.axis, p.index, p.lo0, p.lo1,
                                                                  p.n0, p.n1) for p in src_planes])
        pp = (_abi.yo_plane * max(1, self.n_ports))(*[_abi.yo_plane(p.axis, p.index, p.lo0, p.lo1,
                                                                    p.n0, p.n1) for p in port_planes])
        h = ct.c_void_p()
        call("yo_plan_create", ct.byref(g), ct.byref(d), self.n_steps, self.n_freq, fr,
             self.n_src, sp, self.n_ports, pp, ct.byref(h))
        self._h = h
        self.morph_ops = design.get("morph_ops", "") or ""
        if self.morph_ops:
            # Eqs. (4)-(6): before the workspace is sized and bound
            call("yo_set_morphology", self._h, self.morph_ops.encode(),
                 float(design["morph_d"]), float(design.get("morph_alpha", 20.0)))
        self.mon_nc = 5 if two_term else 2
        if two_term:
            call("yo_set_alpha_terms", self._h, 2)
        self.pulse = tuple(pulse) if pulse is not None else None
        if self.pulse is not None:
            call("yo_set_pulse", self._h, float(pulse[0]), float(pulse[1]), float(pulse[2]))
            if len(self.pulse) > 3 and int(self.pulse[3]) != 1:
                call("yo_set_dft_stride", self._h, int(self.pulse[3]))
        self.time_blocking = int(time_blocking)
        if self.time_blocking != 1:
            call("yo_set_time_blocking", self._h, self.time_blocking)
        nb = ct.c_size_t()
        call("yo_workspace_bytes", self._h, ct.byref(nb))
        self.workspace_bytes = int(nb.value)
        self.workspace = None
        n = ct.c_int()
        call("yo_rhs_count", self._h, ct.byref(n))
        self.n_rhs = int(n.value)
        self.n_fwd = self.n_src * self.n_freq
        # stepped right-hand sides (get_fields / set_fields numbering)
        self.n_stepped = (self.n_src + self.n_ports) if self.pulse is not None else self.n_rhs
        self.n_stepped_fwd = self.n_src if self.pulse is not None else self.n_fwd
        nz, ny, nx = grid["nz"], grid["ny"], grid["nx"]
        self.shape = (3, nz, ny, nx)
        self.box = (design["i0"] - 1, design["j0"] - 1, design["k_lo"] - 1, design["md"] + 2,
                    design["nd"] + 2, design["k_hi"] - design["k_lo"] + 3)
        S = design["supersample"]
        self.canvas_shape = (S * (design["nd"] + 4), S * (design["md"] + 4))
        self.control_shape = (design["nc"], design["mc"])
        self.beta = None
        self._keep = []

    # ----------------------------------------------------------- lifecycle
    def bind(self, workspace: Optional[torch.Tensor] = None, stream=None):
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-workspace.data_ptr()) % 256
        view = workspace[off:]
        if view.numel() < self.workspace_bytes:
            raise ValueError("workspace too small")
        self.workspace = workspace
        call("yo_bind_workspace", self._h, ct.c_void_p(view.data_ptr()),
             ct.c_size_t(view.numel()), _stream(stream))
        return self

    def bind_static(self, stream=None):
        """Bind the library's static per-device workspace (no allocation;
        at most 32 MiB, shared by every plan bound this way on the device:
        the last one bound owns it)."""
        call("yo_bind_static_workspace", self._h, _stream(stream))
        self.workspace = None
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _abi.lib().yo_plan_destroy(self._h)
            self._h = ct.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ----------------------------------------------------------- setup
    def set_background(self, kappa: torch.Tensor, mask: torch.Tensor, stream=None):
        kappa = _dev(kappa, self.device, torch.float32)
        mask = _dev(mask, self.device, torch.float32)
        assert tuple(kappa.shape) == self.shape and tuple(mask.shape) == self.canvas_shape
        call("yo_set_background", self._h, _ptr(kappa), _ptr(mask), _stream(stream))
        self._keep = [kappa, mask]

    def set_source_mode(self, s: int, h, stream=None):
        h = _host_c128(h)
        pl = self.src_planes[s]
        assert h.shape == (2, pl.n1, pl.n0)
        call("yo_set_source_mode", self._h, s, h.ctypes.data_as(ct.c_void_p), _stream(stream))

    def set_port_mode(self, p: int, e, h, stream=None):
        e, h = _host_c128(e), _host_c128(h)
        pl = self.port_planes[p]
        assert e.shape == h.shape == (2, pl.n1, pl.n0)
        call("yo_set_port_mode", self._h, p, e.ctypes.data_as(ct.c_void_p),
             h.ctypes.data_as(ct.c_void_p), _stream(stream))

    def set_design(self, C: torch.Tensor, beta: float, stream=None):
        C = _dev(C, self.device, torch.float32)
        assert tuple(C.shape) == self.control_shape
        call("yo_set_design", self._h, _ptr(C), float(beta), _stream(stream))
        self.beta = float(beta)
        self._C = C

    def set_tiling(self, rows: int, zchunk: int, flags: int = 0):
        """Work split of the time-stepping kernel (see yo_set_tiling)."""
        call("yo_set_tiling", self._h, int(rows), int(zchunk), int(flags))
        self.tiling = (int(rows), int(zchunk), int(flags))

    # ----------------------------------------------------------- stepping
    def run(self, which=YO_BOTH, chunk=64, use_graph=True, stream=None):
        call("yo_run", self._h, which, chunk, int(bool(use_graph)), _stream(stream))

    def reset(self, which=YO_BOTH, stream=None):
        call("yo_reset", self._h, which, _stream(stream))

    def advance(self, which, n_steps, stream=None):
        call("yo_advance", self._h, which, int(n_steps), _stream(stream))

    def finalize(self, which=YO_BOTH, stream=None):
        call("yo_finalize", self._h, which, _stream(stream))

    def steps_done(self) -> int:
        n = ct.c_int()
        call("yo_steps_done", self._h, ct.byref(n))
        return int(n.value)

    # ----------------------------------------------------------- outputs
    def alpha(self, stream=None) -> torch.Tensor:
        out = torch.zeros((self.n_src, self.n_ports, self.n_freq), dtype=torch.complex64,
                          device=self.device)
        call("yo_alpha", self._h, _ptr(out), _stream(stream))
        return out

    def gradient(self, coef: torch.Tensor, stream=None) -> torch.Tensor:
        coef = _dev(coef, self.device, torch.complex64)
        assert tuple(coef.shape) == (self.n_src, self.n_ports, self.n_freq)
        out = torch.empty(self.control_shape, dtype=torch.float32, device=self.device)
        call("yo_gradient", self._h, _ptr(coef), _ptr(out), _stream(stream))
        return out

    def gradient_kappa(self, coef: torch.Tensor, stream=None) -> torch.Tensor:
        coef = _dev(coef, self.device, torch.complex64)
        x0, y0, z0, bx, by, bz = self.box
        out = torch.empty((3, bz, by, bx), dtype=torch.float32, device=self.device)
        call("yo_gradient_kappa", self._h, _ptr(coef), _ptr(out), _stream(stream))
        return out

    def chain_vjp(self, gkappa: torch.Tensor, stream=None) -> torch.Tensor:
        gkappa = _dev(gkappa, self.device, torch.float32)
        x0, y0, z0, bx, by, bz = self.box
        assert tuple(gkappa.shape) == (3, bz, by, bx)
        out = torch.empty(self.control_shape, dtype=torch.float32, device=self.device)
        call("yo_chain_vjp", self._h, _ptr(gkappa), _ptr(out), _stream(stream))
        return out

    def get_dft(self, rhs: int, region: int = 0, stream=None) -> torch.Tensor:
        if region == 0:
            x0, y0, z0, bx, by, bz = self.box
            shape = (3, bz, by, bx)
        else:
            pl = self.port_planes[region - 1]
            shape = (self.mon_nc, pl.n1, pl.n0)
        out = torch.empty(shape, dtype=torch.complex64, device=self.device)
        call("yo_get_dft", self._h, rhs, region, _ptr(out), _stream(stream))
        return out

    def set_fields(self, rhs: int, E: torch.Tensor, H: torch.Tensor, stream=None):
        E = _dev(E, self.device, torch.float32)
        H = _dev(H, self.device, torch.float32)
        call("yo_set_fields", self._h, rhs, _ptr(E), _ptr(H), _stream(stream))
        torch.cuda.current_stream().synchronize()

    def get_fields(self, rhs: int, stream=None):
        E = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        H = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        call("yo_get_fields", self._h, rhs, _ptr(E), _ptr(H), _stream(stream))
        return E, H

    def get_kappa(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        call("yo_get_kappa", self._h, _ptr(out), _stream(stream))
        return out

    def time_kernel(self, cls: int = 0, n_launch: int = 20, stream=None):
        """(avg ms per launch, algorithmic bytes per launch, cell-updates per
        launch) of one part of the time-stepping kernel (0: interior tiles,
        1: CPML shell, 2: the two-step region, 3: the interior around it, 4:
        the z-slabs under it, 5: the shell of paired steps), by HIP events on
        the stream.  An empty part gives zeros."""
        ms, b, c = ct.c_float(), ct.c_double(), ct.c_double()
        call("yo_time_kernel", self._h, int(cls), int(n_launch), ct.byref(ms), ct.byref(b),
             ct.byref(c), _stream(stream))
        return float(ms.value), float(b.value), float(c.value)

    def tile_table(self, part: int):
        """The tiles of launch part `part` (see time_kernel) under the current
        tiling: an int array [n][7] of x0, x1, y0, y1, z0, z1, CPML class
        (host only)."""
        n = ct.c_int()
        call("yo_tile_table", self._h, int(part), None, 0, ct.byref(n))
        out = (ct.c_int * (7 * max(n.value, 1)))()
        call("yo_tile_table", self._h, int(part), out, n.value, ct.byref(n))
        import numpy as np
        return np.ctypeslib.as_array(out)[: 7 * n.value].reshape(n.value, 7).copy()

    def unbinarity(self, lo: float = 0.01, hi: float = 0.99, stream=None) -> torch.Tensor:
        """Fraction of grey design sub-pixels (lo < rho < hi) of the design
        last set, as a one-element device tensor."""
        out = torch.empty(1, dtype=torch.float32, device=self.device)
        call("yo_unbinarity", self._h, float(lo), float(hi), _ptr(out), _stream(stream))
        return out

    def set_timing(self, part: int = 0, n_last: int = 100):
        """Time the launches of one part (0 interior, 1 CPML shell, 2 both)
        over the last `n_last` steps of every later advance (0: off); clears
        what was recorded."""
        call("yo_set_timing", self._h, int(part), int(n_last))

    def timing(self, part: int = 0):
        """(mean ms per timed launch, launches timed) of launch part `part`
        (0 to 5, see time_kernel) since the last set_timing."""
        ms, n = ct.c_float(), ct.c_int()
        call("yo_get_timing", self._h, int(part), ct.byref(ms), ct.byref(n))
        return float(ms.value), int(n.value)

    def model_bytes(self, which=YO_BOTH):
        b, c = ct.c_double(), ct.c_double()
        call("yo_model_bytes", self._h, which, ct.byref(b), ct.byref(c))
        return float(b.value), float(c.value)


def adam_step(C: torch.Tensor, G: torch.Tensor, M: torch.Tensor, V: torch.Tensor, step: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, stream=None):
    """One Adam step on device FP32 tensors of equal size, in place (C, M, V)."""
    for t in (C, G, M, V):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("contiguous float32 device tensors expected")
    n = C.numel()
    if not (G.numel() == M.numel() == V.numel() == n):
        raise ValueError("size mismatch")
    call("yo_adam_step", _ptr(C), _ptr(G), _ptr(M), _ptr(V), n, int(step), float(lr), float(b1),
         float(b2), float(eps), _stream(stream))


def advance_many(plans: Sequence[Plan], which: Sequence[int], n_steps: int, chunk: int = 64,
                 use_graph: bool = True, stream=None):
    """Step several plans in the same launches (each keeps its own counter)."""
    n = len(plans)
    arr = (ct.c_void_p * n)(*[p.handle.value for p in plans])
    wh = (ct.c_int * n)(*which)
    call("yo_advance_many", arr, wh, n, int(n_steps), int(chunk), int(bool(use_graph)),
         _stream(stream))


# ------------------------------------------------------------------ marshalling
def grid_design_of(dev):
    """Grid/design dictionaries from a device description (duck-typed: any
    object with the attributes of ``workloads.Device``)."""
    grid = dict(nx=dev.nx, ny=dev.ny, nz=dev.nz, dx=dev.dx, dy=dev.dx, dz=dev.dx,
                courant=dev.courant, npml=tuple(dev.npml), pml_m=dev.pml_m,
                pml_sigma_scale=dev.pml_sigma_scale, pml_kappa_max=dev.pml_kappa_max,
                pml_a_max=dev.pml_a_max)
    design = dict(i0=dev.i0, j0=dev.j0, md=dev.md, nd=dev.nd, k_lo=dev.k_lo, k_hi=dev.k_hi,
                  mc=dev.mc, nc=dev.nc, filter_r=dev.filter_r, supersample=dev.supersample,
                  eps_core=dev.eps_core, eps_clad=dev.eps_clad, sobel_delta=dev.sobel_delta)
    if getattr(dev, "morph_ops", ""):
        design.update(morph_ops=dev.morph_ops, morph_d=dev.morph_d, morph_alpha=dev.morph_alpha)
    return grid, design


def freqs_of(dev) -> List[FreqSpec]:
    out = []
    for lam in dev.wavelengths:
        ws, wl = dev.window(lam)
        out.append(FreqSpec(2 * np.pi * C0 / lam, dev.ramp_steps(lam), ws, wl))
    return out


def plan_for(dev, device="cuda", stream=None, C=None, beta=None, set_design=True,
             workspace: Optional[torch.Tensor] = None, pulse=None, two_term: bool = False,
             static_workspace: bool = False, time_blocking: int = 1) -> Plan:
    """Create, bind and fill a plan for a device description.  pulse:
    (omega0 rad/s, sigma steps, t0 steps[, DFT stride]) for pulse excitation;
    two_term: the two-term modal coefficient; static_workspace: bind the
    library's static workspace instead of allocating one; time_blocking: 2
    for a plan that may take two steps per launch (tiling flag 512)."""
    grid, design = grid_design_of(dev)
    p = Plan(grid, design, dev.n_steps, freqs_of(dev), [m.plane for m in dev.sources],
             [m.plane for m in dev.ports], device=device, pulse=pulse, two_term=two_term,
             time_blocking=time_blocking)
    if static_workspace:
        p.bind_static(stream)
    else:
        p.bind(workspace, stream)
    p.set_background(torch.as_tensor(dev.kappa_bg, dtype=torch.float32),
                     torch.as_tensor(dev.mask_hr, dtype=torch.float32), stream)
    for s, m in enumerate(dev.sources):
        p.set_source_mode(s, m.h, stream)
    for q, m in enumerate(dev.ports):
        p.set_port_mode(q, m.e, m.h, stream)
    if set_design:
        Cv = dev.C if C is None else C
        p.set_design(torch.as_tensor(np.asarray(Cv), dtype=torch.float32),
                     dev.beta if beta is None else beta, stream)
    return p
