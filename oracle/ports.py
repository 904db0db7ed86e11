"""Mode sources and modal coefficients (paper Appendix A).  TEST INFRASTRUCTURE ONLY.

On a plane with unit normal n and tangential components (t1, t2) ordered so
that (t1, t2, n) is right-handed:
  * the forward mode source is the electric current J = n x h, i.e.
    J_t1 = -h_t2, J_t2 = h_t1;
  * the modal coefficient keeps only the term that depends on E:
    alpha = (1/(2N)) sum (E_t1 h_t2^* - E_t2 h_t1^*) dA, with the mode
    normalisation N = (1/2) sum (e_t1 h_t2^* - e_t2 h_t1^*) dA taken over the
    mode's own fields, so alpha = 1 when E is the mode;
  * hence alpha = w . E with w_t1 = h_t2^*/(2N), w_t2 = -h_t1^*/(2N), and the
    adjoint source w is -(J^F)^*/(2N).
Arrays follow the plane convention of ``workloads``: index 0 = t1, 1 = t2;
``h[1]`` (h_t2) is stored at the E_t1 sites and ``h[0]`` at the E_t2 sites.
The cell area is the unit of dA and cancels.
"""
import numpy as np


def norm_N(e, h):
    return 0.5 * np.sum(e[0] * np.conj(h[1]) - e[1] * np.conj(h[0]))


def monitor_weights(e, h):
    N = norm_N(e, h)
    w = np.empty_like(np.asarray(e, np.complex128))
    w[0] = np.conj(h[1]) / (2.0 * N)
    w[1] = -np.conj(h[0]) / (2.0 * N)
    return w


def source_current(h):
    j = np.empty(np.shape(h), np.complex128)
    j[0] = -h[1]
    j[1] = h[0]
    return j


def alpha(w, Ehat_plane):
    return np.sum(w * Ehat_plane)
