// Parametrization chain (paper Sec. 3) and its vector-Jacobian product, plus
// the small kernels around the time stepping: fills, pitched copies, the
// steady-state fit, the modal overlap and the Eq. (1) gradient assembly.
// All of this is 2-D or plane-sized work next to the 3-D time stepping; the
// kernels are plain one-thread-per-output gathers (no atomics, fixed
// summation order, so results do not depend on scheduling).
#include "yo_internal.h"

namespace {

constexpr int BS = 256;

inline int nblk(size_t n) { return (int)((n + BS - 1) / BS); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ------------------------------------------------------------- utilities
__global__ void k_fill(float *p, size_t n, float v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// dense [ncomp][nz][ny][nx] -> components c0.. of a ghost-layout array of nc
// components (interior only; ghosts untouched)
__global__ void k_to_ghost(const float *src, float *dst, int ncomp, int c0, int nc, int nz, int ny,
                           int nx, int nxp)
{
    const size_t n = (size_t)ncomp * nz * ny * nx;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        size_t q = i;
        const int x = (int)(q % nx); q /= nx;
        const int y = (int)(q % ny); q /= ny;
        const int z = (int)(q % nz); q /= nz;
        dst[yo_off(c0 + (int)q, x, y, z, ny, nxp, nc)] = src[i];
    }
}

__global__ void k_from_ghost(const float *src, float *dst, int ncomp, int c0, int nc, int nz, int ny,
                             int nx, int nxp)
{
    const size_t n = (size_t)ncomp * nz * ny * nx;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        size_t q = i;
        const int x = (int)(q % nx); q /= nx;
        const int y = (int)(q % ny); q /= ny;
        const int z = (int)(q % nz); q /= nz;
        dst[i] = src[yo_off(c0 + (int)q, x, y, z, ny, nxp, nc)];
    }
}

// Ehat = (g00 Re S + g01 Im S) + i (g10 Re S + g11 Im S): least-squares
// amplitude/phase from the DFT sums S = sum E^n exp(+i w n dt).  Any
// non-finite phasor (all-ones exponent bits) sets *bad to 1: one atomic per
// wave that holds one.
__global__ void k_finalize(float2 *a, size_t n, float g00, float g01, float g10, float g11, int *bad)
{
    unsigned int nonfinite = 0u;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float2 s = a[i];
        const float2 e = make_float2(fmaf(g00, s.x, g01 * s.y), fmaf(g10, s.x, g11 * s.y));
        a[i] = e;
        nonfinite |= (__float_as_uint(e.x) & 0x7f800000u) == 0x7f800000u;
        nonfinite |= (__float_as_uint(e.y) & 0x7f800000u) == 0x7f800000u;
    }
    const unsigned long long m = __ballot(nonfinite != 0u);
    if ((threadIdx.x & 63) == 0 && m) atomicOr(bad, 1);
}

// alpha = sum w * Ehat over one port plane; one block, fixed-order tree
__global__ void k_alpha(const float2 *e, const float2 *w, int n, float2 *out)
{
    __shared__ float sr[BS], si[BS];
    float ar = 0.0f, ai = 0.0f;
    for (int i = threadIdx.x; i < n; i += BS) {
        const float2 a = w[i], b = e[i];
        ar = fmaf(a.x, b.x, fmaf(-a.y, b.y, ar));
        ai = fmaf(a.x, b.y, fmaf(a.y, b.x, ai));
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sr[threadIdx.x] += sr[threadIdx.x + s];
            si[threadIdx.x] += si[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = make_float2(sr[0], si[0]);
}

// ------------------------------------------------------------- forward chain
// Eq. (2) with the truncated Gaussian basis (separable taps with clamped
// control indices), then the tanh projection Eq. (3)/(6) into the canvas
// `out`, whose margin takes the background fill.
__global__ void k_project(YoChainBufs c, const float *C, float beta, float *out)
{
    const int n = c.U * c.V;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const int v = i / c.U, u = i - v * c.U;
    const int ud = u - 2 * c.S, vd = v - 2 * c.S;
    if (ud < 0 || ud >= c.S * c.md || vd < 0 || vd >= c.S * c.nd) {
        out[i] = c.mask[i];
        return;
    }
    const int xlo = c.tap_lo_x[ud], xn = c.tap_n_x[ud];
    const int ylo = c.tap_lo_y[vd], yn = c.tap_n_y[vd];
    float phi = 0.0f;
    for (int ty = 0; ty < yn; ++ty) {
        const int b = clampi(ylo + ty, 0, c.nc - 1);
        float row = 0.0f;
        for (int tx = 0; tx < xn; ++tx) {
            const int a = clampi(xlo + tx, 0, c.mc - 1);
            row = fmaf(c.tap_w_x[ud * c.tmax + tx], C[b * c.mc + a], row);
        }
        phi = fmaf(c.tap_w_y[vd * c.tmax + ty], row, phi);
    }
    phi -= 0.5f;
    const float t = tanhf(beta * phi);
    c.tanh_[vd * (c.S * c.md) + ud] = t;
    out[i] = 0.5f * (1.0f + t);
}

// Eqs. (4)-(5): one soft dilation or erosion of the canvas `in` with the
// normalised disc (mean over the taps), on the design area; taps are
// clamped into the canvas, so near the design edge they read the fixed
// margin.  Exponents are shifted so every term is at most one:
// dilation 1 + log(mean e^{a(rho-1)}) / a, erosion -log(mean e^{-a rho}) / a
// (the same values as Eqs. (4)-(5)).  The mean is kept for the transpose.
__global__ void k_morph(YoChainBufs c, const float *in, float *out, float *sum, int dilate)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= c.U * c.V) return;
    const int v = i / c.U, u = i - v * c.U;
    const int ud = u - 2 * c.S, vd = v - 2 * c.S;
    if (ud < 0 || ud >= c.S * c.md || vd < 0 || vd >= c.S * c.nd) {
        out[i] = c.mask[i];
        return;
    }
    const float a = c.malpha;
    float acc = 0.0f;
    for (int t = 0; t < c.n_mtaps; ++t) {
        const int vv = clampi(v + c.mtap[2 * t], 0, c.V - 1);
        const int uu = clampi(u + c.mtap[2 * t + 1], 0, c.U - 1);
        const float r = in[vv * c.U + uu];
        acc += dilate ? expf(a * (r - 1.0f)) : expf(-a * r);
    }
    const float m = acc * c.minv;
    sum[vd * (c.S * c.md) + ud] = m;
    const float l = logf(m) / a;
    out[i] = dilate ? 1.0f + l : -l;
}

// The projection after the morphological stages, Eq. (6):
// rho = (1 + tanh(beta (rho~ - 1/2))) / 2 on the design area.
__global__ void k_morph_project(YoChainBufs c, const float *in, float beta)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= c.U * c.V) return;
    const int v = i / c.U, u = i - v * c.U;
    const int ud = u - 2 * c.S, vd = v - 2 * c.S;
    if (ud < 0 || ud >= c.S * c.md || vd < 0 || vd >= c.S * c.nd) {
        c.rho[i] = c.mask[i];
        return;
    }
    const float t = tanhf(beta * (in[i] - 0.5f));
    c.tanh2[vd * (c.S * c.md) + ud] = t;
    c.rho[i] = 0.5f * (1.0f + t);
}

// Eq. (8): S x S box means centred on each E component (E_x window shifted
// half a cell in x, E_y in y), of 1/eps, eps and rho.
__global__ void k_box(YoChainBufs c)
{
    const int gsz = c.G0 * c.G1;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= 3 * gsz) return;
    const int comp = i / gsz, pix = i - comp * gsz;
    const int n = pix / c.G0, m = pix - n * c.G0;
    const int half = c.S / 2;
    const int shx = comp == 0 ? half : 0, shy = comp == 1 ? half : 0;
    const float de = c.eps_core - c.eps_clad;
    float p = 0.0f, q = 0.0f, r = 0.0f;
    for (int b = 0; b < c.S; ++b) {
        const int v = clampi(c.S * n + shy + b, 0, c.V - 1);
        for (int a = 0; a < c.S; ++a) {
            const int u = clampi(c.S * m + shx + a, 0, c.U - 1);
            const float rho = c.rho[v * c.U + u];
            const float eps = fmaf(de, rho, c.eps_clad);
            p += 1.0f / eps;
            q += eps;
            r += rho;
        }
    }
    const float inv = 1.0f / (float)(c.S * c.S);
    c.P[i] = p * inv;
    c.Q[i] = q * inv;
    c.R[i] = r * inv;
}

__device__ __forceinline__ void sobel(const float *R, int G0, int G1, int n, int m, float &gx,
                                      float &gy)
{
    const float w[3] = {1.0f, 2.0f, 1.0f};
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int dn = -1; dn <= 1; ++dn) {
#pragma unroll
        for (int dm = -1; dm <= 1; ++dm) {
            const float v = R[clampi(n + dn, 0, G1 - 1) * G0 + clampi(m + dm, 0, G0 - 1)];
            sx = fmaf(w[dn + 1] * (float)dm, v, sx);
            sy = fmaf(w[dm + 1] * (float)dn, v, sy);
        }
    }
    gx = sx * 0.125f;
    gy = sy * 0.125f;
}

// Sobel normals, Eq. (7), extrusion through the slab into the 3-D kappa.
__global__ void k_smooth(YoChainBufs c, float *kappa, int nx, int ny, int nz, int nxp, int i0,
                         int j0, int k_lo, int k_hi)
{
    const int wm = c.md + 2, wn = c.nd + 2;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= wm * wn) return;
    const int n = 1 + i / wm, m = 1 + i % wm;
    const int gsz = c.G0 * c.G1;
    const int pix = n * c.G0 + m;
    float gxx, gyx, gxy, gyy;
    sobel(c.R, c.G0, c.G1, n, m, gxx, gyx);             // on the E_x grid
    sobel(c.R + gsz, c.G0, c.G1, n, m, gxy, gyy);       // on the E_y grid
    const float n2x = gxx * gxx / (gxx * gxx + gyx * gyx + c.delta);
    const float n2y = gyy * gyy / (gxy * gxy + gyy * gyy + c.delta);
    const float kx = fmaf(n2x, c.P[pix], (1.0f - n2x) / c.Q[pix]);
    const float ky = fmaf(n2y, c.P[gsz + pix], (1.0f - n2y) / c.Q[gsz + pix]);
    const float kzi = 1.0f / c.Q[2 * gsz + pix];
    const float kzf = 0.5f * (c.P[2 * gsz + pix] + 1.0f / c.eps_clad);
    c.aux[0 * gsz + pix] = n2x;
    c.aux[1 * gsz + pix] = n2y;
    c.aux[2 * gsz + pix] = gxx;
    c.aux[3 * gsz + pix] = gyx;
    c.aux[4 * gsz + pix] = gxy;
    c.aux[5 * gsz + pix] = gyy;
    const int x = i0 - 2 + m, y = j0 - 2 + n;
    for (int k = k_lo; k <= k_hi; ++k) {
        kappa[yo_off(0, x, y, k, ny, nxp, 3)] = kx;
        kappa[yo_off(1, x, y, k, ny, nxp, 3)] = ky;
    }
    for (int k = k_lo; k < k_hi; ++k) kappa[yo_off(2, x, y, k, ny, nxp, 3)] = kzi;
    kappa[yo_off(2, x, y, k_lo - 1, ny, nxp, 3)] = kzf;
    kappa[yo_off(2, x, y, k_hi, ny, nxp, 3)] = kzf;
    (void)nx;
    (void)nz;
}

// ------------------------------------------------------------- Eq. (1)
// dF/deps_c(r) = sum_{f,s,p} 2 Re[coef_{s,p,f} (-2 i sin theta_f) E_F E_A]
//             = sum 4 sin theta_f Im[coef E_F E_A];  dF/dkappa = -dF/deps / kappa^2
// One thread per in-plane box cell, looping over the box planes; also forms
// the z sums of the extrusion's transpose.
__global__ void k_grad(const YoGradArgs a)
{
    const int bx = a.box[3], by = a.box[4], bz = a.box[5];
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= bx * by) return;
    const int bj = i / bx, bi = i - bj * bx;
    const size_t bsz = (size_t)bx * by * bz;
    float sx = 0.0f, sy = 0.0f, szi = 0.0f, szf = 0.0f;
    for (int c = 0; c < 3; ++c) {
        for (int bk = 0; bk < bz; ++bk) {
            const size_t o = ((size_t)c * bz + bk) * (size_t)bx * by + i;
            float ge = 0.0f;
            for (int f = 0; f < a.n_freq; ++f) {
                const float s4 = 4.0f * a.sinth[f];
                for (int s = 0; s < a.n_src; ++s) {
                    const float2 ef = a.EF[f * a.n_src + s][o];
                    for (int p = 0; p < a.n_ports; ++p) {
                        const float2 ea = a.EA[f * a.n_ports + p][o];
                        const float2 cf = a.coef[(s * a.n_ports + p) * a.n_freq + f];
                        // prod = ef * ea
                        const float pr = fmaf(ef.x, ea.x, -ef.y * ea.y);
                        const float pi = fmaf(ef.x, ea.y, ef.y * ea.x);
                        // Im(cf * prod)
                        const float im = fmaf(cf.x, pi, cf.y * pr);
                        ge = fmaf(s4, im, ge);
                    }
                }
            }
            const int x = a.box[0] + bi, y = a.box[1] + bj, z = a.box[2] + bk;
            const float kap = a.kappa[yo_off(c, x, y, z, a.ny, a.nxp, 3)];
            const float gk = -ge / (kap * kap);
            if (a.gbox) a.gbox[o] = gk;
            if (c < 2) {
                if (z >= a.k_lo && z <= a.k_hi) {
                    if (c == 0) sx += gk; else sy += gk;
                }
            } else {
                if (z >= a.k_lo && z < a.k_hi) szi += gk;
                if (z == a.k_lo - 1 || z == a.k_hi) szf += gk;
            }
        }
    }
    (void)bsz;
    if (a.gmap) {
        // box cell (bi, bj) is component-grid pixel (bi + 1, bj + 1)
        const int gsz = a.G0 * a.G1;
        const int pix = (bj + 1) * a.G0 + (bi + 1);
        a.gmap[pix] = sx;
        a.gmap[gsz + pix] = sy;
        a.gmap[2 * gsz + pix] = szi;
        a.gmap[3 * gsz + pix] = szf;
    }
}

// Transpose of the extrusion through the slab: dF/dkappa on the box -> the
// four z-summed maps (E_x planes, E_y planes, interior E_z, face E_z).
__global__ void k_zsum(const float *gbox, int x0, int y0, int z0, int bx, int by, int bz,
                       int k_lo, int k_hi, float *gmap, int G0, int G1)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= bx * by) return;
    const int bj = i / bx, bi = i - bj * bx;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    for (int bk = 0; bk < bz; ++bk) {
        const int z = z0 + bk;
        const size_t o = (size_t)bk * bx * by + i;
        const size_t cs = (size_t)bx * by * bz;
        if (z >= k_lo && z <= k_hi) {
            s0 += gbox[o];
            s1 += gbox[cs + o];
        }
        if (z >= k_lo && z < k_hi) s2 += gbox[2 * cs + o];
        if (z == k_lo - 1 || z == k_hi) s3 += gbox[2 * cs + o];
    }
    const int gsz = G0 * G1, pix = (bj + 1) * G0 + (bi + 1);
    gmap[pix] = s0;
    gmap[gsz + pix] = s1;
    gmap[2 * gsz + pix] = s2;
    gmap[3 * gsz + pix] = s3;
    (void)x0; (void)y0;
}

// ------------------------------------------------------------- chain VJP
// Eq. (7) partials and the normal-vector partials (written region only).
__global__ void k_vjp_pointwise(YoChainBufs c)
{
    const int gsz = c.G0 * c.G1;
    const int pix = blockIdx.x * BS + threadIdx.x;
    if (pix >= gsz) return;
    const int n = pix / c.G0, m = pix - n * c.G0;
    const bool w = (n >= 1 && n <= c.nd + 2 && m >= 1 && m <= c.md + 2);
    float gP[3] = {0, 0, 0}, gQ[3] = {0, 0, 0}, gG[4] = {0, 0, 0, 0};
    if (w) {
        for (int comp = 0; comp < 2; ++comp) {
            const float g = c.gmap[comp * gsz + pix];
            const float n2 = c.aux[comp * gsz + pix];
            const float Gx = c.aux[(2 + 2 * comp) * gsz + pix];
            const float Gy = c.aux[(3 + 2 * comp) * gsz + pix];
            const float P = c.P[comp * gsz + pix], Q = c.Q[comp * gsz + pix];
            gP[comp] = g * n2;
            gQ[comp] = -g * (1.0f - n2) / (Q * Q);
            const float gn = g * (P - 1.0f / Q);
            const float D = Gx * Gx + Gy * Gy + c.delta;
            const float D2 = D * D;
            if (comp == 0) {
                gG[0] = gn * 2.0f * Gx * (Gy * Gy + c.delta) / D2;
                gG[1] = -gn * 2.0f * Gy * Gx * Gx / D2;
            } else {
                gG[3] = gn * 2.0f * Gy * (Gx * Gx + c.delta) / D2;
                gG[2] = -gn * 2.0f * Gx * Gy * Gy / D2;
            }
        }
        const float Qz = c.Q[2 * gsz + pix];
        gP[2] = 0.5f * c.gmap[3 * gsz + pix];
        gQ[2] = -c.gmap[2 * gsz + pix] / (Qz * Qz);
    }
    for (int k = 0; k < 3; ++k) {
        c.gPQ[k * gsz + pix] = gP[k];
        c.gPQ[(3 + k) * gsz + pix] = gQ[k];
    }
    for (int k = 0; k < 4; ++k) c.gG[k * gsz + pix] = gG[k];
}

// Transpose of the clamped Sobel stencils: gather every (pixel, tap) whose
// clamped source is this pixel.
__global__ void k_vjp_sobel(YoChainBufs c)
{
    const int gsz = c.G0 * c.G1;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= 2 * gsz) return;
    const int comp = i / gsz, pix = i - comp * gsz;
    const int nq = pix / c.G0, mq = pix - nq * c.G0;
    const float *gx = c.gG + (2 * comp) * gsz;
    const float *gy = c.gG + (2 * comp + 1) * gsz;
    const float w[3] = {1.0f, 2.0f, 1.0f};
    float acc = 0.0f;
    for (int n = nq - 1; n <= nq + 1; ++n) {
        if (n < 0 || n >= c.G1) continue;
        for (int m = mq - 1; m <= mq + 1; ++m) {
            if (m < 0 || m >= c.G0) continue;
            const float ax = gx[n * c.G0 + m], ay = gy[n * c.G0 + m];
            for (int dn = -1; dn <= 1; ++dn) {
                if (clampi(n + dn, 0, c.G1 - 1) != nq) continue;
                for (int dm = -1; dm <= 1; ++dm) {
                    if (clampi(m + dm, 0, c.G0 - 1) != mq) continue;
                    acc = fmaf(w[dn + 1] * (float)dm * 0.125f, ax, acc);
                    acc = fmaf(w[dm + 1] * (float)dn * 0.125f, ay, acc);
                }
            }
        }
    }
    c.gR[i] = acc;
}

// number of window sub-pixels of pixel m (shift sh) that clamp onto u
__device__ __forceinline__ int win_count(int m, int sh, int S, int u, int n_hr)
{
    int cnt = 0;
    for (int a = 0; a < S; ++a) cnt += (clampi(S * m + sh + a, 0, n_hr - 1) == u);
    return cnt;
}

// Transpose of the box means to the canvas, the density mix and the
// derivative (beta/2)(1 - t^2) of the last projection (t = its tanh values)
// on the design area, into gout [S nd][S md].
__global__ void k_vjp_canvas(YoChainBufs c, float beta, const float *tproj, float *gout)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= c.U * c.V) return;
    const int v = i / c.U, u = i - v * c.U;
    const int ud = u - 2 * c.S, vd = v - 2 * c.S;
    if (ud < 0 || ud >= c.S * c.md || vd < 0 || vd >= c.S * c.nd) return;
    const int gsz = c.G0 * c.G1;
    const int half = c.S / 2;
    const float invS2 = 1.0f / (float)(c.S * c.S);
    float gi = 0.0f, ge = 0.0f, gr = 0.0f;
    for (int comp = 0; comp < 3; ++comp) {
        const int shx = comp == 0 ? half : 0, shy = comp == 1 ? half : 0;
        const int mc0 = (u - shx) / c.S, nc0 = (v - shy) / c.S;
        for (int n = nc0 - 1; n <= nc0 + 1; ++n) {
            if (n < 0 || n >= c.G1) continue;
            const int cy = win_count(n, shy, c.S, v, c.V);
            if (!cy) continue;
            for (int m = mc0 - 1; m <= mc0 + 1; ++m) {
                if (m < 0 || m >= c.G0) continue;
                const int cx = win_count(m, shx, c.S, u, c.U);
                if (!cx) continue;
                const float wgt = (float)(cx * cy) * invS2;
                const int pix = n * c.G0 + m;
                gi = fmaf(wgt, c.gPQ[comp * gsz + pix], gi);
                ge = fmaf(wgt, c.gPQ[(3 + comp) * gsz + pix], ge);
                if (comp < 2) gr = fmaf(wgt, c.gR[comp * gsz + pix], gr);
            }
        }
    }
    const float de = c.eps_core - c.eps_clad;
    const float eps = fmaf(de, c.rho[i], c.eps_clad);
    const float grho = fmaf(gi, -de / (eps * eps), fmaf(ge, de, gr));
    const float t = tproj[vd * (c.S * c.md) + ud];
    gout[vd * (c.S * c.md) + ud] = grho * 0.5f * beta * (1.0f - t * t);
}

// Transpose of a morphological stage, first half: q = g / mean.
__global__ void k_morph_q(YoChainBufs c, const float *g, const float *sum)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= c.S * c.md * c.S * c.nd) return;
    c.mq[i] = g[i] / sum[i];
}

// Second half: d rho~(x) / d rho(x') = e(x') / (n mean(x)) for every tap
// with x + delta = x', e the stage's shifted exponential, so the gradient at
// x' gathers q over x = x' - delta (the disc is symmetric) within the
// design area (taps that were clamped land in the margin, which has no
// gradient).  With tproj, the Eq. (3) projection's derivative follows.
__global__ void k_morph_vjp(YoChainBufs c, const float *in, int dilate, const float *tproj, float beta,
                            float *gout)
{
    const int nud = c.S * c.md, nvd = c.S * c.nd;
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= nud * nvd) return;
    const int vd = i / nud, ud = i - vd * nud;
    float acc = 0.0f;
    for (int t = 0; t < c.n_mtaps; ++t) {
        const int vq = vd - c.mtap[2 * t], uq = ud - c.mtap[2 * t + 1];
        if (vq < 0 || vq >= nvd || uq < 0 || uq >= nud) continue;
        acc += c.mq[vq * nud + uq];
    }
    const float r = in[(vd + 2 * c.S) * c.U + ud + 2 * c.S];
    const float e = dilate ? expf(c.malpha * (r - 1.0f)) : expf(-c.malpha * r);
    float g = e * acc * c.minv;
    if (tproj) {
        const float t = tproj[i];
        g *= 0.5f * beta * (1.0f - t * t);
    }
    gout[i] = g;
}

// Transpose of the separable filter, x then y.  tmp[vd][a] = sum_ud gphi W_x(ud, a)
__global__ void k_vjp_filter_x(YoChainBufs c)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    const int nvd = c.S * c.nd, nud = c.S * c.md;
    if (i >= nvd * c.mc) return;
    const int vd = i / c.mc, a = i - vd * c.mc;
    float acc = 0.0f;
    for (int ud = c.urange_x[2 * a]; ud <= c.urange_x[2 * a + 1]; ++ud) {
        const int lo = c.tap_lo_x[ud], nt = c.tap_n_x[ud];
        float w = 0.0f;
        for (int t = 0; t < nt; ++t)
            if (clampi(lo + t, 0, c.mc - 1) == a) w += c.tap_w_x[ud * c.tmax + t];
        acc = fmaf(w, c.gphi[vd * nud + ud], acc);
    }
    c.tmp[i] = acc;
}

__global__ void k_vjp_filter_y(YoChainBufs c, float *dFdC)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= c.nc * c.mc) return;
    const int b = i / c.mc, a = i - b * c.mc;
    float acc = 0.0f;
    for (int vd = c.urange_y[2 * b]; vd <= c.urange_y[2 * b + 1]; ++vd) {
        const int lo = c.tap_lo_y[vd], nt = c.tap_n_y[vd];
        float w = 0.0f;
        for (int t = 0; t < nt; ++t)
            if (clampi(lo + t, 0, c.nc - 1) == b) w += c.tap_w_y[vd * c.tmax + t];
        acc = fmaf(w, c.tmp[vd * c.mc + a], acc);
    }
    dFdC[i] = acc;
}


// Unbinarity (Sec. 4): grey sub-pixels of the design area, those whose
// final density lies strictly between the two thresholds, given as tanh
// values of the last projection (rho = (1 + t) / 2).  One atomic add per wave (vector atomic
// on an integer, so the count does not depend on the order).
__global__ void k_gray_count(YoChainBufs c, const float *tproj, float tlo, float thi, int *count)
{
    const int n = c.S * c.md * c.S * c.nd;
    const int i = blockIdx.x * BS + threadIdx.x;
    const float t = i < n ? tproj[i] : -2.0f;
    const bool grey = t > tlo && t < thi;
    const unsigned long long m = __ballot(grey);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, __popcll(m));
}

__global__ void k_gray_finish(const int *count, float inv_total, float *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = (float)count[0] * inv_total;
}

__global__ void k_set_int(int *p, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

// Adam (Sec. 4, Eqs. (10)-(11)) on the controls: M, V moving averages of the
// gradient and its square; the update divides the bias-corrected first
// moment by the square root of the bias-corrected second plus eps.
// inv1 = 1 / (1 - b1^i), inv2 = 1 / (1 - b2^i) for step i (from the host).
__global__ void k_adam(float *C, const float *G, float *M, float *V, int n, float lr, float b1,
                       float b2, float eps, float inv1, float inv2)
{
    const int i = blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = fmaf(b1, M[i], (1.0f - b1) * g);
    const float v = fmaf(b2, V[i], (1.0f - b2) * (g * g));
    M[i] = m;
    V[i] = v;
    C[i] = C[i] - lr * ((m * inv1) / (sqrtf(v * inv2) + eps));
}

}  // namespace

hipError_t yo_launch_fill(float *p, size_t n, float v, hipStream_t s)
{
    if (!n) return hipSuccess;
    int blocks = nblk(n);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(BS), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t yo_launch_to_ghost(const float *dense, float *ghost, int ncomp, int c0, int nc, int nz,
                              int ny, int nx, int nxp, hipStream_t s)
{
    const size_t n = (size_t)ncomp * nz * ny * nx;
    if (!n) return hipSuccess;
    int blocks = nblk(n);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_to_ghost, dim3(blocks), dim3(BS), 0, s, dense, ghost, ncomp, c0, nc, nz, ny,
                       nx, nxp);
    return hipGetLastError();
}

hipError_t yo_launch_from_ghost(const float *ghost, float *dense, int ncomp, int c0, int nc, int nz,
                                int ny, int nx, int nxp, hipStream_t s)
{
    const size_t n = (size_t)ncomp * nz * ny * nx;
    if (!n) return hipSuccess;
    int blocks = nblk(n);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_from_ghost, dim3(blocks), dim3(BS), 0, s, ghost, dense, ncomp, c0, nc, nz,
                       ny, nx, nxp);
    return hipGetLastError();
}

hipError_t yo_launch_finalize(float2 *a, size_t n, float g00, float g01, float g10, float g11,
                              int *bad, hipStream_t s)
{
    if (!n) return hipSuccess;
    int blocks = nblk(n);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_finalize, dim3(blocks), dim3(BS), 0, s, a, n, g00, g01, g10, g11, bad);
    return hipGetLastError();
}

hipError_t yo_launch_alpha(const float2 *mon, const float2 *w, int n, float2 *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(BS), 0, s, mon, w, n, out);
    return hipGetLastError();
}

hipError_t yo_launch_chain_forward(const YoChainBufs &c, const float *C, float beta, float *kappa,
                                   int nx, int ny, int nz, int nxp, int i0, int j0, int k_lo,
                                   int k_hi, hipStream_t s)
{
    const size_t UV = (size_t)c.U * c.V;
    const size_t DD = (size_t)c.S * c.md * c.S * c.nd;
    hipLaunchKernelGGL(k_project, dim3(nblk(UV)), dim3(BS), 0, s, c, C, beta, c.n_morph ? c.mcan : c.rho);
    for (int k = 0; k < c.n_morph; ++k)
        hipLaunchKernelGGL(k_morph, dim3(nblk(UV)), dim3(BS), 0, s, c, c.mcan + k * UV, c.mcan + (k + 1) * UV,
                           c.msum + k * DD, (int)((c.mdil >> k) & 1u));
    if (c.n_morph)
        hipLaunchKernelGGL(k_morph_project, dim3(nblk(UV)), dim3(BS), 0, s, c, c.mcan + c.n_morph * UV, beta);
    hipLaunchKernelGGL(k_box, dim3(nblk((size_t)3 * c.G0 * c.G1)), dim3(BS), 0, s, c);
    hipLaunchKernelGGL(k_smooth, dim3(nblk((size_t)(c.md + 2) * (c.nd + 2))), dim3(BS), 0, s, c,
                       kappa, nx, ny, nz, nxp, i0, j0, k_lo, k_hi);
    return hipGetLastError();
}

hipError_t yo_launch_grad_assemble(const YoGradArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad, dim3(nblk((size_t)a.box[3] * a.box[4])), dim3(BS), 0, s, a);
    return hipGetLastError();
}

hipError_t yo_launch_chain_vjp(const YoChainBufs &c, float beta, float *dFdC, hipStream_t s)
{
    const size_t gsz = (size_t)c.G0 * c.G1;
    hipLaunchKernelGGL(k_vjp_pointwise, dim3(nblk(gsz)), dim3(BS), 0, s, c);
    hipLaunchKernelGGL(k_vjp_sobel, dim3(nblk(2 * gsz)), dim3(BS), 0, s, c);
    const size_t UV = (size_t)c.U * c.V;
    const size_t DD = (size_t)c.S * c.md * c.S * c.nd;
    float *g = c.n_morph ? c.mg : c.gphi;
    hipLaunchKernelGGL(k_vjp_canvas, dim3(nblk(UV)), dim3(BS), 0, s, c, beta, c.n_morph ? c.tanh2 : c.tanh_, g);
    for (int k = c.n_morph - 1; k >= 0; --k) {
        hipLaunchKernelGGL(k_morph_q, dim3(nblk(DD)), dim3(BS), 0, s, c, (const float *)g, c.msum + k * DD);
        float *next = k == 0 ? c.gphi : (g == c.mg ? c.mg + DD : c.mg);
        hipLaunchKernelGGL(k_morph_vjp, dim3(nblk(DD)), dim3(BS), 0, s, c, (const float *)(c.mcan + k * UV),
                           (int)((c.mdil >> k) & 1u), k == 0 ? (const float *)c.tanh_ : (const float *)nullptr,
                           beta, next);
        g = next;
    }
    hipLaunchKernelGGL(k_vjp_filter_x, dim3(nblk((size_t)c.S * c.nd * c.mc)), dim3(BS), 0, s, c);
    hipLaunchKernelGGL(k_vjp_filter_y, dim3(nblk((size_t)c.nc * c.mc)), dim3(BS), 0, s, c, dFdC);
    return hipGetLastError();
}

hipError_t yo_launch_zsum(const float *gbox, const int *box, int k_lo, int k_hi, float *gmap, int G0,
                          int G1, hipStream_t s)
{
    hipLaunchKernelGGL(k_zsum, dim3(nblk((size_t)box[3] * box[4])), dim3(BS), 0, s, gbox, box[0],
                       box[1], box[2], box[3], box[4], box[5], k_lo, k_hi, gmap, G0, G1);
    return hipGetLastError();
}

hipError_t yo_launch_unbinarity(const YoChainBufs &c, float tlo, float thi, int *count, float *out,
                                hipStream_t s)
{
    const size_t n = (size_t)c.S * c.md * c.S * c.nd;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, count, 0);
    hipLaunchKernelGGL(k_gray_count, dim3(nblk(n)), dim3(BS), 0, s, c,
                       (const float *)(c.n_morph ? c.tanh2 : c.tanh_), tlo, thi, count);
    hipLaunchKernelGGL(k_gray_finish, dim3(1), dim3(64), 0, s, count, (float)(1.0 / (double)n), out);
    return hipGetLastError();
}

hipError_t yo_launch_adam(float *C, const float *G, float *M, float *V, int n, float lr, float b1, float b2,
                          float eps, float inv1, float inv2, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(nblk((size_t)n)), dim3(BS), 0, s, C, G, M, V, n, lr, b1, b2, eps, inv1,
                       inv2);
    return hipGetLastError();
}
