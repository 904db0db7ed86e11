// Fused Yee time step for gfx950: one launch advances every tile of every
// selected right-hand side by one full step (Ht half step, then E step),
// with the CPML memories, the soft current source and the running DFT of the
// design region and port planes folded into the same sweep.
//
// Update (paper Sec. 2: time-harmonic sources, steady-state phasors):
//   Ht^{n+1/2} = Ht^{n-1/2} - curl_e E^n          (forward differences)
//   E^{n+1}    = E^n + kappa (curl_h Ht^{n+1/2} - j^{n+1/2})  (backward)
// every difference along axis a scaled by S_a = c dt / d_a; in a CPML slab
// the difference d becomes d/k + psi with psi <- b psi + c d.
//
// Work decomposition (one wave = 64 lanes is the unit of work; waves of a
// block are independent, there is no LDS and no barrier):
//   * lane l handles x = 62*tx - 1 + l.  Lanes 1..62 own their cells; lane 0
//     (x-1) and lane 63 (x+62) are halo lanes whose values reach the owners
//     through cross-lane shuffles.
//   * a wave owns TY rows j0..j0+TY-1 and additionally recomputes the Ht of
//     row j0-1, which the E update of row j0 needs.
//   * a wave marches z-planes k0..k1-1, carrying E of the next plane and the
//     Ht of the previous plane in registers; it starts one plane early to
//     recompute Ht(k0-1).
// E and Ht (and the Ht CPML memories) are double-buffered by step parity, so
// a halo recompute always reads old values that no other wave overwrites in
// this launch, and every recomputed halo value is bitwise equal to the one
// its owner stores (same expression, same inputs, no contraction).
//
// Launch: blocks of 4 waves.  Blocks are dispatched round-robin over the 8
// XCDs; the block index is remapped so each XCD receives one contiguous run
// of tiles and neighbouring tiles (sharing halo rows) meet in the same L2.
#include "yo_internal.h"

namespace {

__device__ __forceinline__ float shfl_next(float v)   // value of lane+1
{
    return __shfl_down(v, 1, 64);
}
__device__ __forceinline__ float shfl_prev(float v)   // value of lane-1
{
    return __shfl_up(v, 1, 64);
}

__device__ __forceinline__ int slab_index(int u, int n, int lo, int hi)
{
    if (u < lo) return u;
    if (u >= n - hi) return u - (n - hi) + lo;
    return -1;
}

// one CPML-modified difference: psi_new = b psi_old + c d, returns d/k + psi_new
struct Cpml {
    float b, c, ki;
};
__device__ __forceinline__ Cpml cpml_at(const float *prof, int n, int which, int u)
{
    // prof layout [6][n]: bE cE kiE bH cH kiH ; which = 0 (E sites) or 3 (H sites)
    Cpml p;
    p.b = prof[(which + 0) * n + u];
    p.c = prof[(which + 1) * n + u];
    p.ki = prof[(which + 2) * n + u];
    return p;
}
__device__ __forceinline__ float pml_diff(float d, const Cpml &p, float psi_old, float &psi_new)
{
    psi_new = fmaf(p.b, psi_old, p.c * d);
    return fmaf(d, p.ki, psi_new);
}

__device__ __forceinline__ int sel3(int a, int v0, int v1, int v2)
{
    return a == 0 ? v0 : (a == 1 ? v1 : v2);
}
__device__ __forceinline__ float self3(int a, float v0, float v1, float v2)
{
    return a == 0 ? v0 : (a == 1 ? v1 : v2);
}

// does a plane cross the box [xlo,xhi] x [jlo,jhi] x [klo,khi] (inclusive)?
__device__ __forceinline__ bool plane_hits(const YoPlaneD &pl, int xlo, int xhi, int jlo, int jhi,
                                           int klo, int khi)
{
    const int nlo = sel3(pl.axis, xlo, jlo, klo), nhi = sel3(pl.axis, xhi, jhi, khi);
    const int alo = pl.axis == 0 ? jlo : xlo, ahi = pl.axis == 0 ? jhi : xhi;
    const int blo = pl.axis == 2 ? jlo : klo, bhi = pl.axis == 2 ? jhi : khi;
    return pl.index >= nlo && pl.index <= nhi && pl.lo0 <= ahi && pl.lo0 + pl.n0 > alo &&
           pl.lo1 <= bhi && pl.lo1 + pl.n1 > blo;
}

struct Geo {
    int nx, ny, nz, nxp;
    size_t plane, comp;
};

template <int TY, bool PML>
__device__ __forceinline__ void wave_step(const YoPlanD &P, const YoRhsD &R, const int step,
                                          const int tx, const int ty, const int tz, const int kc,
                                          const int lane)
{
    Geo g;
    g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.nxp = P.nxp;
    g.plane = (size_t)g.ny * g.nxp;
    g.comp = g.plane * g.nz;
    const int par = step & 1;
    const float *__restrict__ Eo = R.E[par];
    float *__restrict__ En = R.E[par ^ 1];
    const float *__restrict__ Ho = R.H[par];
    float *__restrict__ Hn = R.H[par ^ 1];
    const float *__restrict__ K = P.kappa;
    const float sx = P.sx, sy = P.sy, sz = P.sz;

    const int x = tx * YO_TX - 1 + lane;
    const bool xin = (x >= 0) && (x < g.nx);
    const bool own_x = (lane >= 1) && (lane <= YO_TX) && xin;
    const int j0 = ty * TY;
    const int k0 = tz * kc;
    const int k1 = min(k0 + kc, g.nz);

    // ---- DFT and source participation of this wave (uniform) ----
    const int wstep = step - R.win_start;
    const bool in_window = (wstep >= 0) && (wstep < R.win_len);
    float4 st = R.steptab[step];
    const int xlo = tx * YO_TX, xhi = tx * YO_TX + YO_TX - 1;   // owned x range
    const int jlo = j0, jhi = j0 + TY - 1;
    bool box_hit = false;
    if (in_window) {
        box_hit = !(xhi < P.box[0] || xlo >= P.box[0] + P.box[3] || jhi < P.box[1] ||
                    jlo >= P.box[1] + P.box[4] || k1 <= P.box[2] || k0 >= P.box[2] + P.box[5]);
    }
    unsigned port_mask = 0;
    if (in_window) {
        for (int p = 0; p < P.n_ports; ++p)
            if (plane_hits(P.ports[p], xlo, xhi, jlo, jhi, k0, k1 - 1)) port_mask |= 1u << p;
    }
    const bool has_src = (R.src_j != nullptr) && plane_hits(R.src, xlo, xhi, jlo, jhi, k0, k1 - 1);

    // ---- PML per-lane x data ----
    int pxE = -1;   // slab index along x of this lane (same for E and H sites)
    const float *profx = P.prof[0], *profy = P.prof[1], *profz = P.prof[2];
    const int Wx = P.plo[0] + P.phi[0], Wy = P.plo[1] + P.phi[1], Wz = P.plo[2] + P.phi[2];
    Cpml cxE = {1.0f, 0.0f, 1.0f}, cxH = {1.0f, 0.0f, 1.0f};
    if (PML && xin) {
        pxE = slab_index(x, g.nx, P.plo[0], P.phi[0]);
        if (pxE >= 0) {
            cxE = cpml_at(profx, g.nx, 0, x);
            cxH = cpml_at(profx, g.nx, 3, x);
        }
    }

    float Ec[3][TY + 2], Enx[3][TY + 2];
    float Hp[2][TY];          // Ht_x, Ht_y of the previous plane, rows j0..j0+TY-1
    float Hc[3][TY + 1];      // Ht of the current plane, rows j0-1..j0+TY-1

    // row pointers are wave-uniform; only the 32-bit lane offset x varies
    auto row = [&](const float *base, int c, int k, int j) -> const float * {
        return base + (size_t)c * g.comp + (size_t)k * g.plane + (size_t)j * g.nxp;
    };
    auto ld = [&](const float *base, int c, int k, int j) -> float {
        const bool ok = xin && (unsigned)j < (unsigned)g.ny && (unsigned)k < (unsigned)g.nz;
        return ok ? row(base, c, k, j)[x] : 0.0f;
    };

#pragma unroll
    for (int r = 0; r < TY + 2; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Ec[c][r] = ld(Eo, c, k0 - 1, j0 - 1 + r);
    }
#pragma unroll
    for (int r = 0; r < TY; ++r) { Hp[0][r] = 0.0f; Hp[1][r] = 0.0f; }

    for (int k = k0 - 1; k < k1; ++k) {
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Enx[c][r] = ld(Eo, c, k + 1, j0 - 1 + r);
        }
        if (k >= 0) {
            const bool own_k = (k >= k0);
            int pz = -1;
            if (PML) pz = slab_index(k, g.nz, P.plo[2], P.phi[2]);
            // ---------------- Ht at plane k, rows j0-1 .. j0+TY-1 ----------------
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                const int j = j0 - 1 + r;
                const float ez_i1 = shfl_next(Ec[2][r]);
                const float ey_i1 = shfl_next(Ec[1][r]);
                float dyEz = Ec[2][r + 1] - Ec[2][r];
                float dzEy = Enx[1][r] - Ec[1][r];
                float dzEx = Enx[0][r] - Ec[0][r];
                float dxEz = ez_i1 - Ec[2][r];
                float dxEy = ey_i1 - Ec[1][r];
                float dyEx = Ec[0][r + 1] - Ec[0][r];
                const bool jin = (unsigned)j < (unsigned)g.ny;
                const bool own = own_x && own_k && (r >= 1) && jin;
                if (PML && jin && xin) {
                    const int py = slab_index(j, g.ny, P.plo[1], P.phi[1]);
                    float *const *psiO = R.psiH[par];
                    float *const *psiN = R.psiH[par ^ 1];
                    if (pxE >= 0) {
                        const size_t r0 = ((size_t)0 * g.nz + k) * g.ny * Wx + (size_t)j * Wx;
                        const size_t r1 = ((size_t)1 * g.nz + k) * g.ny * Wx + (size_t)j * Wx;
                        float n0, n1;
                        dxEz = pml_diff(dxEz, cxH, (psiO[0] + r0)[pxE], n0);   // Hy
                        dxEy = pml_diff(dxEy, cxH, (psiO[0] + r1)[pxE], n1);   // Hz
                        if (own) { (psiN[0] + r0)[pxE] = n0; (psiN[0] + r1)[pxE] = n1; }
                    }
                    if (py >= 0) {
                        const Cpml cy = cpml_at(profy, g.ny, 3, j);
                        const size_t r0 = (((size_t)0 * g.nz + k) * Wy + py) * g.nxp;
                        const size_t r1 = (((size_t)1 * g.nz + k) * Wy + py) * g.nxp;
                        float n0, n1;
                        dyEz = pml_diff(dyEz, cy, (psiO[1] + r0)[x], n0);   // Hx
                        dyEx = pml_diff(dyEx, cy, (psiO[1] + r1)[x], n1);   // Hz
                        if (own) { (psiN[1] + r0)[x] = n0; (psiN[1] + r1)[x] = n1; }
                    }
                    if (pz >= 0) {
                        const Cpml cz = cpml_at(profz, g.nz, 3, k);
                        const size_t r0 = (((size_t)0 * Wz + pz) * g.ny + j) * g.nxp;
                        const size_t r1 = (((size_t)1 * Wz + pz) * g.ny + j) * g.nxp;
                        float n0, n1;
                        dzEy = pml_diff(dzEy, cz, (psiO[2] + r0)[x], n0);   // Hx
                        dzEx = pml_diff(dzEx, cz, (psiO[2] + r1)[x], n1);   // Hy
                        if (own) { (psiN[2] + r0)[x] = n0; (psiN[2] + r1)[x] = n1; }
                    }
                }
                const float hx0 = ld(Ho, 0, k, j), hy0 = ld(Ho, 1, k, j), hz0 = ld(Ho, 2, k, j);
                const float hx = hx0 - fmaf(sy, dyEz, -(sz * dzEy));
                const float hy = hy0 - fmaf(sz, dzEx, -(sx * dxEz));
                const float hz = hz0 - fmaf(sx, dxEy, -(sy * dyEx));
                const bool valid = jin && xin;
                Hc[0][r] = valid ? hx : 0.0f;
                Hc[1][r] = valid ? hy : 0.0f;
                Hc[2][r] = valid ? hz : 0.0f;
                if (own) {
                    float *hrow = Hn + (size_t)k * g.plane + (size_t)j * g.nxp;
                    hrow[x] = hx;
                    hrow[g.comp + x] = hy;
                    hrow[2 * g.comp + x] = hz;
                }
            }
            // ---------------- E at plane k, rows j0 .. j0+TY-1 ----------------
            if (own_k) {
#pragma unroll
                for (int r = 1; r <= TY; ++r) {
                    const int j = j0 - 1 + r;
                    const float hz_im = shfl_prev(Hc[2][r]);
                    const float hy_im = shfl_prev(Hc[1][r]);
                    if (j >= g.ny) continue;
                    float dyHz = Hc[2][r] - Hc[2][r - 1];
                    float dzHy = Hc[1][r] - Hp[1][r - 1];
                    float dzHx = Hc[0][r] - Hp[0][r - 1];
                    float dxHz = Hc[2][r] - hz_im;
                    float dxHy = Hc[1][r] - hy_im;
                    float dyHx = Hc[0][r] - Hc[0][r - 1];
                    if (PML && own_x) {
                        const int py = slab_index(j, g.ny, P.plo[1], P.phi[1]);
                        if (pxE >= 0) {
                            float *ps = R.psiE[0];
                            const size_t r0 = ((size_t)0 * g.nz + k) * g.ny * Wx + (size_t)j * Wx;
                            const size_t r1 = ((size_t)1 * g.nz + k) * g.ny * Wx + (size_t)j * Wx;
                            float n0, n1;
                            dxHz = pml_diff(dxHz, cxE, (ps + r0)[pxE], n0);   // Ey
                            dxHy = pml_diff(dxHy, cxE, (ps + r1)[pxE], n1);   // Ez
                            (ps + r0)[pxE] = n0; (ps + r1)[pxE] = n1;
                        }
                        if (py >= 0) {
                            float *ps = R.psiE[1];
                            const Cpml cy = cpml_at(profy, g.ny, 0, j);
                            const size_t r0 = (((size_t)0 * g.nz + k) * Wy + py) * g.nxp;
                            const size_t r1 = (((size_t)1 * g.nz + k) * Wy + py) * g.nxp;
                            float n0, n1;
                            dyHz = pml_diff(dyHz, cy, (ps + r0)[x], n0);   // Ex
                            dyHx = pml_diff(dyHx, cy, (ps + r1)[x], n1);   // Ez
                            (ps + r0)[x] = n0; (ps + r1)[x] = n1;
                        }
                        if (pz >= 0) {
                            float *ps = R.psiE[2];
                            const Cpml cz = cpml_at(profz, g.nz, 0, k);
                            const size_t r0 = (((size_t)0 * Wz + pz) * g.ny + j) * g.nxp;
                            const size_t r1 = (((size_t)1 * Wz + pz) * g.ny + j) * g.nxp;
                            float n0, n1;
                            dzHy = pml_diff(dzHy, cz, (ps + r0)[x], n0);   // Ex
                            dzHx = pml_diff(dzHx, cz, (ps + r1)[x], n1);   // Ey
                            (ps + r0)[x] = n0; (ps + r1)[x] = n1;
                        }
                    }
                    if (!own_x) continue;
                    const size_t ro = (size_t)k * g.plane + (size_t)j * g.nxp;
                    const float *krow = K + ro;
                    const float kx = krow[x], ky = krow[g.comp + x], kz = krow[2 * g.comp + x];
                    const float ex0 = Ec[0][r], ey0 = Ec[1][r], ez0 = Ec[2][r];
                    float ex = fmaf(kx, fmaf(sy, dyHz, -(sz * dzHy)), ex0);
                    float ey = fmaf(ky, fmaf(sz, dzHx, -(sx * dxHz)), ey0);
                    float ez = fmaf(kz, fmaf(sx, dxHy, -(sy * dyHx)), ez0);

                    // running DFT of E^n (the old field) over the window
                    if (box_hit) {
                        const int bi = x - P.box[0], bj = j - P.box[1], bk = k - P.box[2];
                        if ((unsigned)bi < (unsigned)P.box[3] && (unsigned)bj < (unsigned)P.box[4] &&
                            (unsigned)bk < (unsigned)P.box[5]) {
                            const size_t bs = (size_t)P.box[3] * P.box[4] * P.box[5];
                            const size_t bo = ((size_t)bk * P.box[4] + bj) * P.box[3] + bi;
                            float2 *d = R.dft_box;
                            float2 a0 = d[bo], a1 = d[bs + bo], a2 = d[2 * bs + bo];
                            a0.x = fmaf(ex0, st.z, a0.x); a0.y = fmaf(ex0, st.w, a0.y);
                            a1.x = fmaf(ey0, st.z, a1.x); a1.y = fmaf(ey0, st.w, a1.y);
                            a2.x = fmaf(ez0, st.z, a2.x); a2.y = fmaf(ez0, st.w, a2.y);
                            d[bo] = a0; d[bs + bo] = a1; d[2 * bs + bo] = a2;
                        }
                    }
                    for (int p = 0; port_mask >> p; ++p) {
                        if (!((port_mask >> p) & 1u)) continue;
                        const YoPlaneD pl = P.ports[p];
                        if (sel3(pl.axis, x, j, k) != pl.index) continue;
                        const int a0i = (pl.axis == 0 ? j : x) - pl.lo0;
                        const int a1i = (pl.axis == 2 ? j : k) - pl.lo1;
                        if ((unsigned)a0i >= (unsigned)pl.n0 || (unsigned)a1i >= (unsigned)pl.n1) continue;
                        const int t1 = (pl.axis + 1) % 3, t2 = (pl.axis + 2) % 3;
                        const float e1 = self3(t1, ex0, ey0, ez0), e2 = self3(t2, ex0, ey0, ez0);
                        float2 *d = R.dft_mon + P.mon_off[p];
                        const size_t o1 = (size_t)a1i * pl.n0 + a0i;
                        const size_t o2 = (size_t)pl.n1 * pl.n0 + o1;
                        float2 v1 = d[o1], v2 = d[o2];
                        v1.x = fmaf(e1, st.z, v1.x); v1.y = fmaf(e1, st.w, v1.y);
                        v2.x = fmaf(e2, st.z, v2.x); v2.y = fmaf(e2, st.w, v2.y);
                        d[o1] = v1; d[o2] = v2;
                    }
                    // soft current source at (n+1/2) dt
                    if (has_src) {
                        const YoPlaneD pl = R.src;
                        if (sel3(pl.axis, x, j, k) == pl.index) {
                            const int a0i = (pl.axis == 0 ? j : x) - pl.lo0;
                            const int a1i = (pl.axis == 2 ? j : k) - pl.lo1;
                            if ((unsigned)a0i < (unsigned)pl.n0 && (unsigned)a1i < (unsigned)pl.n1) {
                                const size_t o1 = (size_t)a1i * pl.n0 + a0i;
                                const size_t o2 = (size_t)pl.n1 * pl.n0 + o1;
                                const float2 j1 = R.src_j[o1], j2 = R.src_j[o2];
                                const float jv1 = fmaf(j1.x, st.x, j1.y * st.y);
                                const float jv2 = fmaf(j2.x, st.x, j2.y * st.y);
                                const int t1 = (pl.axis + 1) % 3;
                                if (pl.axis != 0) ex = fmaf(-kx, t1 == 0 ? jv1 : jv2, ex);
                                if (pl.axis != 1) ey = fmaf(-ky, t1 == 1 ? jv1 : jv2, ey);
                                if (pl.axis != 2) ez = fmaf(-kz, t1 == 2 ? jv1 : jv2, ez);
                            }
                        }
                    }
                    // perfect conductor: tangential E on the planes i=0, j=0, k=0
                    if (j == 0 || k == 0) ex = 0.0f;
                    if (x == 0 || k == 0) ey = 0.0f;
                    if (x == 0 || j == 0) ez = 0.0f;
                    float *erow = En + ro;
                    erow[x] = ex;
                    erow[g.comp + x] = ey;
                    erow[2 * g.comp + x] = ez;
                }
            }
        }
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            Hp[0][r - 1] = (k >= 0) ? Hc[0][r] : 0.0f;
            Hp[1][r - 1] = (k >= 0) ? Hc[1][r] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Ec[c][r] = Enx[c][r];
        }
    }
}

template <int TY, bool PML>
__global__ __launch_bounds__(256) void k_yee_step(const YoStepArgs a)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, rem = nb & 7, xcd = b & 7, pos = b >> 3;
    const int lb = (xcd < rem) ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
    const int wave = lb * YO_WAVES_PER_BLOCK + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= a.total_waves) return;
    int s = 0;
    while (s + 1 < a.n_slots && wave >= a.prefix[s + 1]) ++s;
    const YoSlot sl = a.slot[s];
    const YoPlanD &P = *sl.plan;
    const int step = *P.step_ctr + a.k_offset;
    if (step >= P.n_steps) return;
    // right-hand sides of one tile are adjacent waves (they share kappa)
    const int local = wave - a.prefix[s];
    const int r = sl.rhs0 + local % sl.nrhs;
    const int t = sl.tiles[local / sl.nrhs];
    const int ty = t & 2047, tx = (t >> 11) & 2047, tz = t >> 22;
    wave_step<TY, PML>(P, P.rhs[r], step, tx, ty, tz, sl.kc, lane);
}

__global__ void k_ctr(const YoCtrArgs a, int set_value)
{
    const int i = threadIdx.x;
    if (i < a.n) {
        if (set_value)
            *a.ctr[i] = a.add;
        else
            *a.ctr[i] += a.add;
    }
}

}  // namespace

hipError_t yo_launch_step(int ty, int pml, const YoStepArgs &args, int blocks, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    if (ty == 4 && !pml)
        hipLaunchKernelGGL((k_yee_step<4, false>), dim3(blocks), dim3(256), 0, s, args);
    else if (ty == 4 && pml)
        hipLaunchKernelGGL((k_yee_step<4, true>), dim3(blocks), dim3(256), 0, s, args);
    else if (ty == 8 && !pml)
        hipLaunchKernelGGL((k_yee_step<8, false>), dim3(blocks), dim3(256), 0, s, args);
    else if (ty == 8 && pml)
        hipLaunchKernelGGL((k_yee_step<8, true>), dim3(blocks), dim3(256), 0, s, args);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t yo_launch_ctr(const YoCtrArgs &args, int set_value, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctr, dim3(1), dim3(64), 0, s, args, set_value);
    return hipGetLastError();
}
