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

The two-term coefficient of Appendix A,
    alpha = (1/4) ( (1/N) sum (E x h^*) . n + (1/N^*) sum (e^* x H) . n ),
reads the tangential H on the H sites half a cell past the plane along n
(H_t1 shares the E_t2 sites' transverse position, H_t2 the E_t1 sites'):
alpha = wE . E + u . H with wE the E-only weights halved and
u_t1 = -e_t2^*/(4 N^*), u_t2 = e_t1^*/(4 N^*).
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


def two_term_weights(e, h, axis: int):
    """(wE, u) of the two-term coefficient; u[0] weighs H_t1, u[1] H_t2.
    u[0] is zeroed on the plane's last row along t2 and u[1] on its last
    column along t1 (H sites whose curl would reach past the plane; the
    mode is negligible there)."""
    N = norm_N(e, h)
    wE = 0.5 * monitor_weights(e, h)
    u = np.empty_like(np.asarray(e, np.complex128))
    u[0] = -np.conj(e[1]) / (4.0 * np.conj(N))
    u[1] = np.conj(e[0]) / (4.0 * np.conj(N))
    t1 = (axis + 1) % 3
    if t1 == min(t1, (axis + 2) % 3):     # t1 along the columns of [n1][n0]
        u[0][-1, :] = 0.0
        u[1][:, -1] = 0.0
    else:
        u[0][:, -1] = 0.0
        u[1][-1, :] = 0.0
    return wE, u


def alpha_two_term(wE, u, Ehat_plane, Hhat_plane):
    return np.sum(wE * Ehat_plane) + np.sum(u * Hhat_plane)


def h_term_on_e_sites(u, axis: int, s_axis: float, s_t1: float, s_t2: float, theta: float):
    """The H term u . Hhat rewritten on E sites through the discrete Faraday
    law of the Yee update (Ht^{n+1/2} = Ht^{n-1/2} - curl_e E^n gives
    Hhat = curl_e Ehat / (2 i sin theta)): returns (q_i [2], q_n, q_i1 [2]),
    the weights of the tangential E on the plane, the normal E half a cell
    past it, and the tangential E one cell past it.  Arrays are [n1][n0] in
    the plane's storage order (c0 = the lower-numbered of the two in-plane
    axes); u must vanish on the last row along t2 (u[0]) and the last column
    along t1 (u[1]) so every weight stays on the plane."""
    u = np.asarray(u, np.complex128)
    t1 = (axis + 1) % 3
    c0 = min(t1, (axis + 2) % 3)
    # storage shift of one cell along t1 / t2: (d1 along rows, d0 along columns)
    along_t1 = (0, 1) if t1 == c0 else (1, 0)
    along_t2 = (1, 0) if t1 == c0 else (0, 1)
    f = 1.0 / (2j * np.sin(theta))
    q_i = np.zeros_like(u)
    q_i1 = np.zeros_like(u)
    q_i[1] = s_axis * u[0] * f
    q_i1[1] = -s_axis * u[0] * f
    q_i[0] = -s_axis * u[1] * f
    q_i1[0] = s_axis * u[1] * f
    q_n = (-s_t2 * u[0] + s_t1 * u[1]) * f

    def shifted(a, d):          # a moved one cell forward along storage direction d
        out = np.zeros_like(a)
        if d == (1, 0):
            out[1:, :] = a[:-1, :]
        else:
            out[:, 1:] = a[:, :-1]
        return out

    q_n = q_n + s_t2 * shifted(u[0], along_t2) * f - s_t1 * shifted(u[1], along_t1) * f
    return q_i, q_n, q_i1
