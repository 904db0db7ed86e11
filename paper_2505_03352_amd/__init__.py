"""MI355X-native adjoint FDTD hot path for inverse design of passive Si
photonics (arXiv 2505.03352): a C-ABI library of HIP kernels for gfx950
(``libyeeopt.so``, interface in ``include/yeeopt.h``) and a thin Python
binding that uses PyTorch only for device memory and streams.

Modules:
  _abi     ctypes declarations of the C ABI
  plan     Plan (one geometry, its right-hand sides and workspace)
  fn       torch.autograd.Function over C -> alpha
  batch    batched stepping of many plans in shared launches, autotuner
  serve    continuous-batching request loop
"""
from ._abi import YO_ADJOINT, YO_BOTH, YO_FORWARD, YeeOptError  # noqa: F401

__all__ = ["YO_FORWARD", "YO_ADJOINT", "YO_BOTH", "YeeOptError"]
