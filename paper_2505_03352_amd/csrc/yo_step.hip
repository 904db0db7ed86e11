// Fused Yee time step for gfx950.  Each step is two launches over every
// selected right-hand side of every plan in the call: the interior tiles
// (clear of every absorbing slab, no CPML code) and the CPML shell; each
// advances its tiles by one full step (Ht half step, then E step).  Two
// small kernels bracket them: the running DFT of E^n (design box and port
// planes) before the step, and the soft current source after it.
//
// Update (paper Sec. 2: time-harmonic sources, steady-state phasors):
//   Ht^{n+1/2} = Ht^{n-1/2} - curl_e E^n                        (forward differences)
//   E^{n+1}    = E^n + kappa curl_h Ht^{n+1/2} - kappa j^{n+1/2} (backward differences)
// every difference along axis a scaled by S_a = c dt / d_a; in a CPML slab
// the difference d becomes d/k + psi with psi <- b psi + c d.
//
// Work decomposition (one wave = 64 lanes):
//   * lane l handles x = x0 - 1 + l.  Lanes 1..xn own their cells; lane 0
//     (x0-1) and the lane after the last owned one are halo lanes whose
//     values reach the owners through DPP whole-wave shifts.
//   * a wave owns rows j0..j0+jn-1 (jn <= 4) and recomputes the Ht of row
//     j0-1, which the E update of row j0 needs (or, in cooperative blocks,
//     takes it and the E row above from its neighbours through LDS).
//   * a wave marches z-planes k0..k1-1, carrying E of the next plane and the
//     Ht of the previous plane in registers; it starts one plane early to
//     recompute Ht(k0-1).
// A step reads the state buffer of step n and writes that of step n+1 (two
// buffers, or three in rotation when the plan's interior may take two steps
// per sweep); the Ht CPML memories are double-buffered by step parity, so a
// halo recompute reads old values no other wave overwrites in this launch,
// and every recomputed halo value is bitwise equal to the one its owner
// stores (same expression, same inputs, no contraction).  Field arrays carry
// a zero ghost layer, so every load is unconditional: indices outside the
// grid are clamped onto the ghost layer and read zero.
//
// A CPML tile's class (bit a: it meets the absorbing slab of axis a) picks
// an instantiation with the CPML code of exactly those axes, or the shell
// runs the code of all three.
//
// Launch: blocks of 4 (or 8) waves, dispatched round-robin over the 8 XCDs;
// the block index is remapped so each XCD receives one contiguous run of
// tiles and neighbouring tiles (sharing halo rows) meet in the same L2.
#include "yo_internal.h"

namespace {

// Neighbour exchange along x with DPP whole-wave shifts (one VALU move, no
// LDS round trip).  The lane with no neighbour gets 0; those are halo lanes,
// whose results are never used.
__device__ __forceinline__ float shfl_next(float v)   // value of lane+1 (wave_shl:1)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float shfl_prev(float v)   // value of lane-1 (wave_shr:1)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Raw buffer access: the resource (base, size) and the row offset are
// wave-uniform scalars, the only per-lane operand is the column offset, so a
// load costs no vector address arithmetic.  Reads past the buffer return 0.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc rsrc_of(const float *p, size_t n_floats)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0,
                                             (int)(n_floats * sizeof(float)), 0x00020000);
}
__device__ __forceinline__ float bload(Rsrc r, int voff, int soff)
{
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float v, Rsrc r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, voff, soff, 0);
}

// Store of a new field value: no wave of this launch reads it again, so it
// is marked non-temporal (cache-policy bit 1) to leave the caches to the
// halo rows and planes that neighbouring tiles do re-read.  (The CPML
// memories keep the default policy: marked the same way, measured slower.)
__device__ __forceinline__ void bstore_nt(float v, Rsrc r, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, voff, soff, 2);
}

__device__ __forceinline__ int slab_index(int u, int n, int lo, int hi)
{
    if (u < 0 || u >= n) return -1;
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

// What the CPML code needs of the plan and the right-hand side, read once
// per tile before any store (a store to global memory would otherwise make
// the compiler reload the descriptors with vector loads and wait for them),
// plus the y and z profile coefficients of the tile's rows and planes, one
// row (plane) per lane, taken out with readlane when used.
struct CpmlCtx {
    int nx, ny, nz, nxp;
    int plo[3], phi[3], W[3];
    int off[3], n[3];        // CPML memory layout (floats), see YoRhsD
    int qEo, qEn, qHo, qHn;  // memories (first component) read and written this step, E and Ht
    Rsrc ps;                 // this right-hand side's CPML memories
    Cpml cyE, cyH;           // lane l: row j0 - 1 + l
    Cpml czE, czH;           // lane l: plane k0 - 1 + l
    int j0m, k0m;            // j0 - 1, k0 - 1
};

__device__ __forceinline__ float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ Cpml lane_cpml(const Cpml &c, int l)
{
    Cpml o;
    o.b = lane_value(c.b, l);
    o.c = lane_value(c.c, l);
    o.ki = lane_value(c.ki, l);
    return o;
}

// CPML memory slots of each axis, as first components (two components per
// slot): with two state buffers, E one slot (0) read and written in place
// and Ht two (2, 4) by step parity, since halo rows recompute Ht from the
// old step's memory while its owner writes the new one; with three state
// buffers (two steps per launch) three slots each, E at 0, 2, 4 and Ht at
// 6, 8, 10, the step's memories in slot step % 3: a two-step launch reads
// slot n % 3 around its cells and writes slot (n + 2) % 3 of its own while
// single steps write (n + 1) % 3.
__device__ __forceinline__ void cpml_slots(int nbuf, int step, int &qEo, int &qEn, int &qHo, int &qHn)
{
    if (nbuf == 3) {
        const int s0 = step % 3, s1 = (step + 1) % 3;
        qEo = 2 * s0;
        qEn = 2 * s1;
        qHo = 6 + 2 * s0;
        qHn = 6 + 2 * s1;
    } else {
        const int par = step & 1;
        qEo = qEn = 0;
        qHo = 2 + 2 * par;
        qHn = 2 + 2 * (par ^ 1);
    }
}

// Byte offsets of CPML memory q (a slot's first component + c, see
// cpml_slots) of axis A at site (x, j, k): the lane part (voff) and the wave-uniform part
// (soff); false when the site is outside the axis' slabs.
template <int A>
__device__ __forceinline__ bool psi_at(const CpmlCtx &C, int q, int x, int j, int k, int pxs,
                                       int &voff, int &soff)
{
    if (A == 0) {
        voff = pxs * (int)sizeof(float);
        soff = (C.off[0] + q * C.n[0] + (k * C.ny + j) * C.W[0]) * (int)sizeof(float);
        return pxs >= 0;
    }
    if (A == 1) {
        const int py = slab_index(j, C.ny, C.plo[1], C.phi[1]);
        voff = x * (int)sizeof(float);
        soff = (C.off[1] + q * C.n[1] + (k * C.W[1] + py) * C.nxp) * (int)sizeof(float);
        return py >= 0;
    }
    const int pz = slab_index(k, C.nz, C.plo[2], C.phi[2]);
    voff = x * (int)sizeof(float);
    soff = (C.off[2] + q * C.n[2] + (pz * C.ny + j) * C.nxp) * (int)sizeof(float);
    return pz >= 0;
}

// CPML corrections of the six differences of one Ht site row (x = this
// lane, row j, plane k): each difference inside an absorbing slab of its
// axis becomes d/kp + psi with psi <- b psi + c d.  Ht's memories are read
// from one slot and written to another (halo rows recompute Ht, reading psi
// of the old step); only the owner writes the new value.  PRE: the old
// values were loaded with the plane's fields (q[axis][component]); else they
// are loaded here.
template <int PM, bool PRE>
__device__ __forceinline__ void h_cpml(const CpmlCtx &C, int x, int j, int k, int pxs,
                                       const Cpml &cxH, bool own, const float (&q)[3][2],
                                       float &dxEz, float &dxEy, float &dyEz, float &dyEx,
                                       float &dzEy, float &dzEx)
{
    const bool xin = (x >= 0) && (x < C.nx);
    const bool jin = (j >= 0) && (j < C.ny);
    if (!(jin && xin && k >= 0)) return;
    const int qo = C.qHo, qn = C.qHn;
    int v, s0, s1, t0, t1;
    if ((PM & 1) && psi_at<0>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<0>(C, qo + 1, x, j, k, pxs, v, s1);
        float n0, n1;
        dxEz = pml_diff(dxEz, cxH, PRE ? q[0][0] : bload(C.ps, v, s0), n0);   // Hy
        dxEy = pml_diff(dxEy, cxH, PRE ? q[0][1] : bload(C.ps, v, s1), n1);   // Hz
        if (own) {
            psi_at<0>(C, qn, x, j, k, pxs, v, t0);
            psi_at<0>(C, qn + 1, x, j, k, pxs, v, t1);
            bstore(n0, C.ps, v, t0);
            bstore(n1, C.ps, v, t1);
        }
    }
    if ((PM & 2) && psi_at<1>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<1>(C, qo + 1, x, j, k, pxs, v, s1);
        const Cpml cy = lane_cpml(C.cyH, j - C.j0m);
        float n0, n1;
        dyEz = pml_diff(dyEz, cy, PRE ? q[1][0] : bload(C.ps, v, s0), n0);   // Hx
        dyEx = pml_diff(dyEx, cy, PRE ? q[1][1] : bload(C.ps, v, s1), n1);   // Hz
        if (own) {
            psi_at<1>(C, qn, x, j, k, pxs, v, t0);
            psi_at<1>(C, qn + 1, x, j, k, pxs, v, t1);
            bstore(n0, C.ps, v, t0);
            bstore(n1, C.ps, v, t1);
        }
    }
    if ((PM & 4) && psi_at<2>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<2>(C, qo + 1, x, j, k, pxs, v, s1);
        const Cpml cz = lane_cpml(C.czH, k - C.k0m);
        float n0, n1;
        dzEy = pml_diff(dzEy, cz, PRE ? q[2][0] : bload(C.ps, v, s0), n0);   // Hx
        dzEx = pml_diff(dzEx, cz, PRE ? q[2][1] : bload(C.ps, v, s1), n1);   // Hy
        if (own) {
            psi_at<2>(C, qn, x, j, k, pxs, v, t0);
            psi_at<2>(C, qn + 1, x, j, k, pxs, v, t1);
            bstore(n0, C.ps, v, t0);
            bstore(n1, C.ps, v, t1);
        }
    }
}

// CPML corrections of the six differences of one owned E site (each E
// memory is read and written by its owner only: one slot, read and written
// in place, or with three state buffers the slot of the step read and the
// next one written).  PRE as for h_cpml.
template <int PM, bool PRE>
__device__ __forceinline__ void e_cpml(const CpmlCtx &C, int x, int j, int k, int pxs, const Cpml &cxE,
                                       const float (&q)[3][2], float &dxHz, float &dxHy, float &dyHz,
                                       float &dyHx, float &dzHy, float &dzHx)
{
    const int qo = C.qEo, qn = C.qEn;
    int v, s0, s1, t0, t1;
    if ((PM & 1) && psi_at<0>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<0>(C, qo + 1, x, j, k, pxs, v, s1);
        float n0, n1;
        dxHz = pml_diff(dxHz, cxE, PRE ? q[0][0] : bload(C.ps, v, s0), n0);   // Ey
        dxHy = pml_diff(dxHy, cxE, PRE ? q[0][1] : bload(C.ps, v, s1), n1);   // Ez
        psi_at<0>(C, qn, x, j, k, pxs, v, t0);
        psi_at<0>(C, qn + 1, x, j, k, pxs, v, t1);
        bstore(n0, C.ps, v, t0);
        bstore(n1, C.ps, v, t1);
    }
    if ((PM & 2) && psi_at<1>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<1>(C, qo + 1, x, j, k, pxs, v, s1);
        const Cpml cy = lane_cpml(C.cyE, j - C.j0m);
        float n0, n1;
        dyHz = pml_diff(dyHz, cy, PRE ? q[1][0] : bload(C.ps, v, s0), n0);   // Ex
        dyHx = pml_diff(dyHx, cy, PRE ? q[1][1] : bload(C.ps, v, s1), n1);   // Ez
        psi_at<1>(C, qn, x, j, k, pxs, v, t0);
        psi_at<1>(C, qn + 1, x, j, k, pxs, v, t1);
        bstore(n0, C.ps, v, t0);
        bstore(n1, C.ps, v, t1);
    }
    if ((PM & 4) && psi_at<2>(C, qo, x, j, k, pxs, v, s0)) {
        psi_at<2>(C, qo + 1, x, j, k, pxs, v, s1);
        const Cpml cz = lane_cpml(C.czE, k - C.k0m);
        float n0, n1;
        dzHy = pml_diff(dzHy, cz, PRE ? q[2][0] : bload(C.ps, v, s0), n0);   // Ex
        dzHx = pml_diff(dzHx, cz, PRE ? q[2][1] : bload(C.ps, v, s1), n1);   // Ey
        psi_at<2>(C, qn, x, j, k, pxs, v, t0);
        psi_at<2>(C, qn + 1, x, j, k, pxs, v, t1);
        bstore(n0, C.ps, v, t0);
        bstore(n1, C.ps, v, t1);
    }
}

// Old CPML memories q (a slot's first component, see cpml_slots) of every axis in PM at one
// site, or 0 where `use` is false or the site is outside the slab (such a
// lane's offset is past the buffer, so the load moves no data and the
// loads need no branch).
template <int PM>
__device__ __forceinline__ void psi_preload(const CpmlCtx &C, int q, int x, int j, int k, int pxs,
                                            bool use, float (&out)[3][2])
{
    const int far = (int)0x80000000;
    int v, s0, s1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!(PM & (1 << a))) continue;
        bool in = false;
        if (a == 0) {
            in = psi_at<0>(C, q, x, j, k, pxs, v, s0);
            psi_at<0>(C, q + 1, x, j, k, pxs, v, s1);
        } else if (a == 1) {
            in = psi_at<1>(C, q, x, j, k, pxs, v, s0);
            psi_at<1>(C, q + 1, x, j, k, pxs, v, s1);
        } else {
            in = psi_at<2>(C, q, x, j, k, pxs, v, s0);
            psi_at<2>(C, q + 1, x, j, k, pxs, v, s1);
        }
        in = in && use;
        out[a][0] = bload(C.ps, in ? v : far, in ? s0 : 0);
        out[a][1] = bload(C.ps, in ? v : far, in ? s1 : 0);
    }
}

// Exchange slots of a cooperative block, per plane parity and wave: Ex and
// Ez of the wave's first row (next plane), Ht_x and Ht_z of its last row.
#define YO_XS_FLOATS (2 * YO_MAX_WPB * 4 * 64)

__device__ __forceinline__ void block_sync_lds()
{
    // LDS-only ordering: outstanding global loads and stores stay in flight
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One wave's share of a tile.  COOP = false: the tile is the wave's own
// (rows j0 .. j0+jn-1); the wave loads the E rows above and below and
// recomputes the Ht row below.  COOP = true: the tile is the block's, its
// waves are stacked in y (wave w owns rows J0 + w TY ...), and neighbouring
// waves hand each other the one row they share through LDS: Ex, Ez of the
// row above and Ht_x, Ht_z of the row below.  Only the block's bottom wave
// recomputes the Ht row below the block and only its top wave loads the E
// row above it; one barrier per plane.
template <int TY, int PM, bool COOP, bool PF>
__device__ __forceinline__ void wave_step(const YoPlanD &P, const YoRhsD &R, const int step,
                                          const int4 t, const int w, const int lane, float *xs)
{
    const int nx = P.nx, ny = P.ny, nz = P.nz, nxp = P.nxp;
    const int rows = ny + 2;
    const size_t groups = (size_t)(nz + 2) * rows;           // row groups (j, k)
    const int rowb = nxp * (int)sizeof(float);                // one component row, bytes
    // state: 6 component rows per group (E then Ht); kappa: 3
    const Rsrc Fo = rsrc_of(R.F[step % P.nbuf], 6 * groups * nxp);
    const Rsrc Fn = rsrc_of(R.F[(step + 1) % P.nbuf], 6 * groups * nxp);
    const Rsrc K = rsrc_of(P.kappa, 3 * groups * nxp);
    const int eb = 0, hb = 3 * rowb;                          // E and Ht within a state group
    const float sx = P.sx, sy = P.sy, sz = P.sz;

    const int x0 = t.x & 0xffff, xn = t.x >> 16;
    const int J0 = t.y & 0xffff, JN = t.y >> 16;
    const int k0 = t.z & 0xffff, k1 = t.z >> 16;
    const int j0 = COOP ? J0 + w * TY : J0;
    const int jn = COOP ? clampi(JN - w * TY, 0, TY) : JN;
    const bool bottom = !COOP || w == 0;
    const bool top = !COOP || JN - w * TY <= TY;        // no rows of the tile above this wave
    if (COOP && jn == 0) {
        // past the tile's last row: nothing to compute, but keep the barriers
        for (int k = k0 - 1; k < k1; ++k) block_sync_lds();
        return;
    }
    // this wave's slots; a neighbour's are 4 * 64 floats below or above
    float *const xme = COOP ? xs + w * 4 * 64 + lane : nullptr;
    auto xslot = [&](int pp, int dw, int c) -> float & {
        return xme[(pp * YO_MAX_WPB + dw) * 4 * 64 + c * 64];
    };
    const int x = x0 - 1 + lane;
    // lanes past the halo lane after the last owned one take no part: their
    // column offset lies past every buffer, so their loads move no data (a
    // narrow strip costs only its own columns)
    const bool lane_used = lane <= xn + 1;
    const int xo = lane_used ? (clampi(x, -1, nx) + 1) * (int)sizeof(float) : 0x40000000;
    const bool own_x = (lane >= 1) && (lane <= xn);
    // wave-uniform byte offsets of row group (j, k) in the state and kappa arrays
    auto ro = [&](int j, int k) -> int {
        return ((k + 1) * rows + (clampi(j, -1, ny) + 1)) * 6 * rowb;
    };
    auto rk = [&](int j, int k) -> int {
        return ((k + 1) * rows + (clampi(j, -1, ny) + 1)) * 3 * rowb;
    };

    // ---- CPML data (CPML classes only), read before any store ----
    const bool xin = (x >= 0) && (x < nx);
    int pxs = -1;
    Cpml cxE = {1.0f, 0.0f, 1.0f}, cxH = {1.0f, 0.0f, 1.0f};
    CpmlCtx C;
    if (PM) {
        C.nx = nx; C.ny = ny; C.nz = nz; C.nxp = nxp;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C.plo[a] = P.plo[a];
            C.phi[a] = P.phi[a];
            C.W[a] = P.plo[a] + P.phi[a];
            C.off[a] = P.psi_off[a];
            C.n[a] = P.psi_n[a];
        }
        C.ps = rsrc_of(R.psi, (size_t)P.psi_total);
        cpml_slots(P.nbuf, step, C.qEo, C.qEn, C.qHo, C.qHn);
        C.j0m = j0 - 1;
        C.k0m = k0 - 1;
        const Cpml one = {1.0f, 0.0f, 1.0f};
        C.cyE = C.cyH = C.czE = C.czH = one;
        if ((PM & 2) && lane <= TY) {
            const int jj = j0 - 1 + lane;
            if (jj >= 0 && jj < ny && slab_index(jj, ny, P.plo[1], P.phi[1]) >= 0) {
                C.cyE = cpml_at(P.prof[1], ny, 0, jj);
                C.cyH = cpml_at(P.prof[1], ny, 3, jj);
            }
        }
        if (PM & 4) {
            const int kk = k0 - 1 + lane;
            if (kk >= 0 && kk < k1 && slab_index(kk, nz, P.plo[2], P.phi[2]) >= 0) {
                C.czE = cpml_at(P.prof[2], nz, 0, kk);
                C.czH = cpml_at(P.prof[2], nz, 3, kk);
            }
        }
        if ((PM & 1) && xin && lane_used) {
            pxs = slab_index(x, nx, P.plo[0], P.phi[0]);
            if (pxs >= 0) {
                cxE = cpml_at(P.prof[0], nx, 0, x);
                cxH = cpml_at(P.prof[0], nx, 3, x);
            }
        }
    }

    float Ec[3][TY + 2], Enx[3][TY + 2];
    float Hp[2][TY];          // Ht_x, Ht_y of the previous plane, rows j0..j0+TY-1
    float Hc[3][TY + 1];      // Ht of the current plane, rows j0-1..j0+TY-1
    float Ho_[3][TY + 1], Kv[3][TY];

    // Plane k works on E(k) in Ec, E(k+1) in Enx, old Ht(k) in Ho_ and
    // kappa(k) in Kv.  PF (prefetch): those are in registers when plane k
    // starts, and the loads for plane k+1 are issued before plane k's stores,
    // because the vector-memory counter also counts stores and a wait placed
    // after them would wait for the stores too.  Without PF a plane loads its
    // own operands (fewer registers, more waves to hide the latency).
    // rows a wave never loads (the row below unless bottom, the row above
    // unless top) are filled from neighbours or never read
    auto load_plane = [&](int k, float (&en)[3][TY + 2], float (&ho)[3][TY + 1],
                          float (&kv)[3][TY]) {
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            const int o = ro(j0 - 1 + r, k + 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) en[c][r] = bload(Fo, xo, eb + c * rowb + o);
        }
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            const int o = ro(j0 - 1 + r, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) ho[c][r] = bload(Fo, xo, hb + c * rowb + o);
        }
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            const int o = rk(j0 - 1 + r, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) kv[c][r - 1] = bload(K, xo, c * rowb + o);
        }
        // last, so that the branches do not blur the wait counts of the rest
        if (bottom) {
            const int oe = ro(j0 - 1, k + 1), oh = ro(j0 - 1, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                en[c][0] = bload(Fo, xo, eb + c * rowb + oe);
                ho[c][0] = bload(Fo, xo, hb + c * rowb + oh);
            }
        }
        if (top) {
            // only Ex and Ez of the row above enter (as y-differences)
            const int o = ro(j0 + TY, k + 1);
            en[0][TY + 1] = bload(Fo, xo, eb + o);
            en[2][TY + 1] = bload(Fo, xo, eb + 2 * rowb + o);
        }
    };

#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Ec[c][0] = Enx[c][0] = Ho_[c][0] = Hc[c][0] = 0.0f;
        Ec[c][TY + 1] = Enx[c][TY + 1] = 0.0f;
    }
#pragma unroll
    for (int r = 0; r < TY + 2; ++r) {
        if (r == 0 && !bottom) continue;
        const int o = ro(j0 - 1 + r, k0 - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) Ec[c][r] = bload(Fo, xo, eb + c * rowb + o);
    }
#pragma unroll
    for (int r = 0; r < TY; ++r) { Hp[0][r] = 0.0f; Hp[1][r] = 0.0f; }
    if (PF) load_plane(k0 - 1, Enx, Ho_, Kv);

    for (int k = k0 - 1; k < k1; ++k) {
        const bool own_k = (k >= k0);
        float Enx2[3][TY + 2], Ho2[3][TY + 1], Kv2[3][TY];
        if (PF) {
            // unconditional (the last plane re-reads itself) so the wait counts stay exact
            load_plane(k + 1 < k1 ? k + 1 : k, Enx2, Ho2, Kv2);
        } else {
            load_plane(k, Enx, Ho_, Kv);
        }
        // CPML tiles without prefetch: the plane's old CPML memories are
        // loaded here with its fields, so one wait covers both
        constexpr bool PRE = PM != 0 && !PF;
        float qH[TY + 1][3][2], qE[TY][3][2];
        if constexpr (PRE) {
            const bool kin = k >= 0 && k < nz;
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
                const int j = j0 - 1 + r;
                const bool use = (r > 0 || bottom) && xin && lane_used && kin && j >= 0 && j < ny;
                psi_preload<PM>(C, C.qHo, x, j, k, pxs, use, qH[r]);
            }
#pragma unroll
            for (int r = 1; r <= TY; ++r) {
                const bool use = own_x && k >= k0 && r <= jn;
                psi_preload<PM>(C, C.qEo, x, j0 - 1 + r, k, pxs, use, qE[r - 1]);
            }
        }
        const int pp = k & 1;
        if (COOP) {
            // E of plane k+1, first row: the wave below's row above
            xslot(pp, 0, 0) = Enx[0][1];
            xslot(pp, 0, 1) = Enx[2][1];
        }

        // ---------------- Ht at plane k, rows j0-1 .. j0+TY-1 ----------------
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            if (r == 0 && !bottom) continue;
            const int j = j0 - 1 + r;
            const float ez_i1 = shfl_next(Ec[2][r]);
            const float ey_i1 = shfl_next(Ec[1][r]);
            float dyEz = Ec[2][r + 1] - Ec[2][r];
            float dzEy = Enx[1][r] - Ec[1][r];
            float dzEx = Enx[0][r] - Ec[0][r];
            float dxEz = ez_i1 - Ec[2][r];
            float dxEy = ey_i1 - Ec[1][r];
            float dyEx = Ec[0][r + 1] - Ec[0][r];
            const bool own = own_x && own_k && (r >= 1) && (r <= jn);
            if (PM)
                h_cpml<PM, PRE>(C, lane_used ? x : -1, j, k, pxs, cxH, own, qH[r], dxEz, dxEy,
                                dyEz, dyEx, dzEy, dzEx);
            const float hx = Ho_[0][r] - fmaf(sy, dyEz, -(sz * dzEy));
            const float hy = Ho_[1][r] - fmaf(sz, dzEx, -(sx * dxEz));
            const float hz = Ho_[2][r] - fmaf(sx, dxEy, -(sy * dyEx));
            Hc[0][r] = hx;
            Hc[1][r] = hy;
            Hc[2][r] = hz;
            if (own) {
                const int o = ro(j, k) + hb;
                bstore_nt(hx, Fn, xo, o);
                bstore_nt(hy, Fn, xo, rowb + o);
                bstore_nt(hz, Fn, xo, 2 * rowb + o);
            }
        }
        if (COOP) {
            xslot(pp, 0, 2) = Hc[0][TY];
            xslot(pp, 0, 3) = Hc[2][TY];
            block_sync_lds();
            if (!bottom) {
                Hc[0][0] = xslot(pp, -1, 2);
                Hc[2][0] = xslot(pp, -1, 3);
            }
            if (!top) {
                Enx[0][TY + 1] = xslot(pp, 1, 0);
                Enx[2][TY + 1] = xslot(pp, 1, 1);
            }
        }
        // ---------------- E at plane k, rows j0 .. j0+jn-1 ----------------
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            const int j = j0 - 1 + r;
            const float hz_im = shfl_prev(Hc[2][r]);
            const float hy_im = shfl_prev(Hc[1][r]);
            if (!own_k || r > jn) continue;
            float dyHz = Hc[2][r] - Hc[2][r - 1];
            float dzHy = Hc[1][r] - Hp[1][r - 1];
            float dzHx = Hc[0][r] - Hp[0][r - 1];
            float dxHz = Hc[2][r] - hz_im;
            float dxHy = Hc[1][r] - hy_im;
            float dyHx = Hc[0][r] - Hc[0][r - 1];
            if (PM && own_x)
                e_cpml<PM, PRE>(C, x, j, k, pxs, cxE, qE[r - 1], dxHz, dxHy, dyHz, dyHx, dzHy, dzHx);
            float ex = fmaf(Kv[0][r - 1], fmaf(sy, dyHz, -(sz * dzHy)), Ec[0][r]);
            float ey = fmaf(Kv[1][r - 1], fmaf(sz, dzHx, -(sx * dxHz)), Ec[1][r]);
            float ez = fmaf(Kv[2][r - 1], fmaf(sx, dxHy, -(sy * dyHx)), Ec[2][r]);
            // perfect conductor: tangential E on the planes i=0, j=0, k=0
            ex = (j == 0 || k == 0) ? 0.0f : ex;
            ey = (x == 0 || k == 0) ? 0.0f : ey;
            ez = (x == 0 || j == 0) ? 0.0f : ez;
            if (own_x) {
                const int o = ro(j, k) + eb;
                bstore_nt(ex, Fn, xo, o);
                bstore_nt(ey, Fn, xo, rowb + o);
                bstore_nt(ez, Fn, xo, 2 * rowb + o);
            }
        }
#pragma unroll
        for (int r = 1; r <= TY; ++r) {
            Hp[0][r - 1] = Hc[0][r];
            Hp[1][r - 1] = Hc[1][r];
        }
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Ec[c][r] = Enx[c][r];
                if (PF) Enx[c][r] = Enx2[c][r];
            }
        }
        if (PF) {
#pragma unroll
            for (int r = 0; r <= TY; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Ho_[c][r] = Ho2[c][r];
            }
#pragma unroll
            for (int r = 0; r < TY; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Kv[c][r] = Kv2[c][r];
            }
        }
    }
}

// PM = YO_PM_ANY: tiles of every CPML class in one launch, each tile's class
// (int4 .w) selecting its code.
#define YO_PM_ANY 8
template <int PM, bool COOP, bool PF, int TY>
__device__ __forceinline__ void tile_step(const YoPlanD &P, const YoRhsD &R, int step, const int4 t,
                                          int w, int lane, float *xs)
{
    if constexpr (PM == YO_PM_ANY) {
        switch (t.w) {
        case 1: wave_step<TY, 1, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 2: wave_step<TY, 2, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 3: wave_step<TY, 3, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 4: wave_step<TY, 4, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 5: wave_step<TY, 5, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 6: wave_step<TY, 6, COOP, PF>(P, R, step, t, w, lane, xs); break;
        case 7: wave_step<TY, 7, COOP, PF>(P, R, step, t, w, lane, xs); break;
        default: wave_step<TY, 0, COOP, PF>(P, R, step, t, w, lane, xs); break;
        }
    } else {
        wave_step<TY, PM, COOP, PF>(P, R, step, t, w, lane, xs);
    }
}

// TY: rows per wave (YO_TY; YO_TY2 for the taller shell tiles)
template <int PM, bool COOP, bool PF, int TY = YO_TY>
__global__ __launch_bounds__(64 * YO_MAX_WPB) void k_yee_step(const YoStepArgs a)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, rem = nb & 7, xcd = b & 7, pos = b >> 3;
    const int lb = (xcd < rem) ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
    const int wpb = a.wpb;
    // the wave index is the same in every lane: say so, so that everything
    // derived from it (slot, tile, row offsets) lives in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(lb * wpb + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // every early exit below is uniform over the block (slot prefixes are
    // whole blocks), as the cooperative variant's barriers require
    if (wave >= a.total_waves) return;
    int s = 0;
    while (s + 1 < a.n_slots && wave >= a.prefix[s + 1]) ++s;
    const YoSlot sl = a.slot[s];
    const YoPlanD &P = *sl.plan;
    const int step = *P.step_ctr + a.k_offset;
    if (step >= P.n_steps) return;
    const int local = wave - a.prefix[s];
    if (COOP) {
        // one tile per block; consecutive blocks take the same tile for the
        // next right-hand sides, which share kappa
        __shared__ float xs[YO_XS_FLOATS];
        const int blk = local / wpb;
        const int w = local - blk * wpb;
        const int r = sl.rhs0 + blk % sl.nrhs;
        const int ti = blk / sl.nrhs;
        if (ti >= sl.ntile) return;
        tile_step<PM, true, PF, TY>(P, P.rhs[r], step, sl.tiles[ti], w, lane, xs);
    } else {
        // A block's waves take consecutive tiles (neighbouring x-strips of
        // the same rows) of one right-hand side, so together they stream
        // contiguous row segments and share the cache lines at the strips'
        // edges; consecutive blocks take the same tiles for the next
        // right-hand sides, which share kappa.
        const int grp = local / (wpb * sl.nrhs);
        const int in_grp = local - grp * (wpb * sl.nrhs);
        const int r = sl.rhs0 + in_grp / wpb;
        const int ti = grp * wpb + in_grp % wpb;
        if (ti >= sl.ntile) return;
        tile_step<PM, false, PF, TY>(P, P.rhs[r], step, sl.tiles[ti], 0, lane, nullptr);
    }
}

// ---------------------------------------------------------------------------
// Two steps per sweep (temporal blocking) for the tiles of the two-step region
// R2 (YoPlanD::r2), which lies two cells clear of every absorbing slab and of
// every source plane, so neither step needs CPML code or a source term there.
// A wave owns x in [x0, x0+xn) (xn <= 60; lane l holds x = x0 - 2 + l), rows
// j0..j0+jn-1 (jn <= TY) and planes k0..k1-1, reads the state after step n
// (buffer n % 3) and writes the state after step n+2 (buffer (n+2) % 3),
// recomputing from step n's values everything the second step needs around
// its cells: step n+1 on lanes 1..62, rows j0-1..j0+TY and planes k0-1..k1,
// step n+1's Ht on one more lane, row and plane below.  Marching up z, it
// takes step n+1 at plane k and step n+2 at plane k-1 in the same pass (a
// wavefront in z-t), so each plane's state is read once for both steps.
// The cells of R2's outermost layer also get their step-n+1 state written
// (buffer (n+1) % 3): the single steps of the tiles around R2 read it.
// Every value is computed with the expression and the operand order of the
// single-step kernel, so the two paths give bitwise the same fields.
// ZP: the tiles of the z-slabs under R2's x-y footprint (planes down to 0 and
// up to nz - 1), with the z-axis CPML code of the single-step kernel: a wave
// reads the memories of slot n % 3 around its cells, keeps step n+1's new
// ones in registers for the second step, and writes slot (n+2) % 3 of its own
// cells and, for R2's outermost layer, the Ht memories of step n+1 (slot
// (n+1) % 3), which the single steps around read.  Planes past the grid are
// the perfect conductor's zeros.
// COOP: the tile is the block's, its waves stacked in y (wave w owns rows
// J0 + w TY ...); each wave loads its own rows of step n and the rows it
// shares with the waves below and above come through LDS (E^n of the two
// rows below and above, Ht^{n-1/2} of the two below and one above; one
// barrier per plane, two parities), so only the block's bottom and top
// waves load the block's halo rows.
template <int TY, bool ZP, bool COOP = false>
__device__ __forceinline__ void wave_step2(const YoPlanD &P, const YoRhsD &R, const int step,
                                           const int4 t, const int w, const int wpb, const int lane,
                                           float *xs)
{
    const int nx = P.nx, ny = P.ny, nxp = P.nxp;
    const int rows = ny + 2;
    const size_t groups = (size_t)(P.nz + 2) * rows;
    const int rowb = nxp * (int)sizeof(float);
    const int nb = P.nbuf;
    const Rsrc FA = rsrc_of(R.F[step % nb], 6 * groups * nxp);          // after step n
    const Rsrc FB = rsrc_of(R.F[(step + 1) % nb], 6 * groups * nxp);    // after n+1 (rim)
    const Rsrc FC = rsrc_of(R.F[(step + 2) % nb], 6 * groups * nxp);    // after n+2
    const Rsrc K = rsrc_of(P.kappa, 3 * groups * nxp);
    const int eb = 0, hb = 3 * rowb;
    const float sx = P.sx, sy = P.sy, sz = P.sz;

    const int x0 = t.x & 0xffff, xn = t.x >> 16;
    const int J0 = t.y & 0xffff, JN = t.y >> 16;
    const int k0 = t.z & 0xffff, k1 = t.z >> 16;
    const int j0 = COOP ? J0 + w * TY : J0;
    const int jn = COOP ? clampi(JN - w * TY, 0, TY) : JN;
    const bool bottom = !COOP || w == 0;
    const bool top = !COOP || JN - w * TY <= TY;        // no rows of the tile above this wave
    if (COOP && jn == 0) {
        // past the tile's last row: nothing to compute, but keep the barriers
        for (int k = k0 - 2; k <= k1; ++k) block_sync_lds();
        return;
    }
    // exchange slots of this wave (20 per parity: E^n rows TY, TY+1 and Ht
    // rows TY, TY+1 for the wave above; E^n row 2, row 3's Ex and Ez, and Ht
    // row 2 for the wave below); a neighbour's are 20 * 64 floats away
    float *const xme = COOP ? xs + w * 20 * 64 + lane : nullptr;
    auto xslot = [&](int pp, int dw, int q) -> float & {
        return xme[(pp * wpb + dw) * 20 * 64 + q * 64];
    };
    const int x = x0 - 2 + lane;
    const int xo = (clampi(x, -1, nx) + 1) * (int)sizeof(float);
    const bool own_x = (lane >= 2) && (lane < 2 + xn);
    // R2's outermost layer, whose step-n+1 state the tiles around R2 read
    const int ra0 = P.r2[0], ra1 = P.r2[1], rb0 = P.r2[2], rb1 = P.r2[3], rc0 = P.r2[4], rc1 = P.r2[5];
    const bool rim_x = own_x && (x == ra0 || x == ra1 - 1);
    // z-axis CPML memories (ZP): slots as in cpml_slots, byte offsets of
    // component c of slot q at row j of slab plane pz
    const int nz = P.nz, zlo = P.plo[2], zhi = P.phi[2];
    const Rsrc PS = rsrc_of(R.psi, (size_t)P.psi_total);
    const int s0 = step % 3, s1 = (step + 1) % 3, s2 = (step + 2) % 3;
    const int xv = clampi(x, 0, nx - 1) * (int)sizeof(float);
    auto zo = [&](int q, int pz, int j) -> int {
        return (P.psi_off[2] + q * P.psi_n[2] + (pz * ny + j) * nxp) * (int)sizeof(float);
    };
    auto ro = [&](int j, int k) -> int {
        return ((k + 1) * rows + (clampi(j, -1, ny) + 1)) * 6 * rowb;
    };
    auto rk = [&](int j, int k) -> int {
        return ((k + 1) * rows + (clampi(j, -1, ny) + 1)) * 3 * rowb;
    };
    // row index r: j = j0 - 2 + r
    constexpr int NE = TY + 4;     // E^n rows 0..TY+3 (the last: Ex and Ez only)
    constexpr int NH = TY + 3;     // Ht^{n-1/2} and Ht^{n+1/2} rows 0..TY+2
    float Ec[3][NE], Enx[3][NE];   // E^n at planes k and k+1
    float Ho[3][NH];               // Ht^{n-1/2} at plane k
    float Hh[3][NH], Hhp[3][NH];   // Ht^{n+1/2} at planes k and k-1
    float Kc[3][NH], Kp[3][NH];    // kappa at planes k and k-1 (rows 1..TY+2)
    float E1c[3][NH], E1p[3][NH];  // E^{n+1} at planes k and k-1 (rows 1..TY+2)
    float H2[3][NH], H2p[2][NH];   // Ht^{n+3/2} at planes k-1 and k-2 (rows 1..TY+1)
    // ZP: z memories of step n+1 (Ht rows 0..TY+2, E rows 1..TY+2) at
    // planes k and k-1, with the planes' coefficients
    float qH1[2][NH], qH1p[2][NH], qE1[2][NH], qE1p[2][NH];
    Cpml czH = {1.0f, 0.0f, 1.0f}, czE = czH, czHp = czH, czEp = czH;
    int pzp = -1;

    // all: every row from memory; else (COOP) the rows a neighbour passes on
    // are left for the exchange
    auto load_e = [&](int k, float (&e)[3][NE], bool all) {
        if (ZP && (k < -1 || k > nz)) {   // past the ghost planes
#pragma unroll
            for (int r = 0; r < NE; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) e[c][r] = 0.0f;
            return;
        }
#pragma unroll
        for (int r = 0; r < NE; ++r) {
            if (COOP && !all && ((r < 2 && !bottom) || (r >= TY + 2 && !top))) continue;
            const int o = ro(j0 - 2 + r, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (r == NE - 1 && c == 1) { e[c][r] = 0.0f; continue; }
                e[c][r] = bload(FA, xo, eb + c * rowb + o);
            }
        }
    };
    load_e(k0 - 2, Ec, true);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < NH; ++r) Hhp[c][r] = E1p[c][r] = Kp[c][r] = H2[c][r] = 0.0f;
#pragma unroll
    for (int r = 0; r < NH; ++r) {
        H2p[0][r] = H2p[1][r] = 0.0f;
        qH1[0][r] = qH1[1][r] = qE1[0][r] = qE1[1][r] = 0.0f;
    }

    for (int k = k0 - 2; k <= k1; ++k) {
        load_e(k + 1, Enx, false);
        if (ZP && k < -1) {
#pragma unroll
            for (int r = 0; r < NH; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) Ho[c][r] = 0.0f;
        } else {
#pragma unroll
            for (int r = 0; r < NH; ++r) {
                if (COOP && ((r < 2 && !bottom) || (r >= TY + 2 && !top))) continue;
                const int o = ro(j0 - 2 + r, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) Ho[c][r] = bload(FA, xo, hb + c * rowb + o);
            }
        }
        if (COOP) {
            // the rows the neighbours share, then theirs
            const int pp = k & 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xslot(pp, 0, c) = Enx[c][TY];
                xslot(pp, 0, 3 + c) = Enx[c][TY + 1];
                xslot(pp, 0, 6 + c) = Ho[c][TY];
                xslot(pp, 0, 9 + c) = Ho[c][TY + 1];
                xslot(pp, 0, 12 + c) = Enx[c][2];
                xslot(pp, 0, 17 + c) = Ho[c][2];
            }
            xslot(pp, 0, 15) = Enx[0][3];
            xslot(pp, 0, 16) = Enx[2][3];
            block_sync_lds();
            if (!bottom) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Enx[c][0] = xslot(pp, -1, c);
                    Enx[c][1] = xslot(pp, -1, 3 + c);
                    Ho[c][0] = xslot(pp, -1, 6 + c);
                    Ho[c][1] = xslot(pp, -1, 9 + c);
                }
            }
            if (!top) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Enx[c][TY + 2] = xslot(pp, 1, 12 + c);
                    Ho[c][TY + 2] = xslot(pp, 1, 17 + c);
                }
                Enx[0][TY + 3] = xslot(pp, 1, 15);
                Enx[1][TY + 3] = 0.0f;
                Enx[2][TY + 3] = xslot(pp, 1, 16);
            }
        }
        // ZP: plane k's z coefficients (its memories of step n, slot n % 3,
        // are loaded where used)
        const int pz = ZP ? slab_index(k, nz, zlo, zhi) : -1;
        if (ZP && pz >= 0) {
            czH = cpml_at(P.prof[2], nz, 3, k);
            czE = cpml_at(P.prof[2], nz, 0, k);
        }
        const bool do_e1 = k >= k0 - 1;
        if (do_e1) {
#pragma unroll
            for (int r = 1; r < NH; ++r) {
                const int o = rk(j0 - 2 + r, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) Kc[c][r] = bload(K, xo, c * rowb + o);
            }
        }
        // ---- step n+1's Ht at plane k, rows 0..TY+2 ----
#pragma unroll
        for (int r = 0; r < NH; ++r) {
            const float ez_i1 = shfl_next(Ec[2][r]);
            const float ey_i1 = shfl_next(Ec[1][r]);
            const float dyEz = Ec[2][r + 1] - Ec[2][r];
            const float dzEy = Enx[1][r] - Ec[1][r];
            const float dzEx = Enx[0][r] - Ec[0][r];
            const float dxEz = ez_i1 - Ec[2][r];
            const float dxEy = ey_i1 - Ec[1][r];
            const float dyEx = Ec[0][r + 1] - Ec[0][r];
            float dzEy_ = dzEy, dzEx_ = dzEx;
            if (ZP && pz >= 0) {
                const int o = zo(6 + 2 * s0, pz, j0 - 2 + r);
                dzEy_ = pml_diff(dzEy, czH, bload(PS, xv, o), qH1[0][r]);                       // Hx
                dzEx_ = pml_diff(dzEx, czH, bload(PS, xv, o + P.psi_n[2] * 4), qH1[1][r]);   // Hy
            }
            Hh[0][r] = Ho[0][r] - fmaf(sy, dyEz, -(sz * dzEy_));
            Hh[1][r] = Ho[1][r] - fmaf(sz, dzEx_, -(sx * dxEz));
            Hh[2][r] = Ho[2][r] - fmaf(sx, dxEy, -(sy * dyEx));
            if (ZP && k < 0) Hh[0][r] = Hh[1][r] = Hh[2][r] = 0.0f;   // ghost plane
        }
        if (do_e1) {
            // ---- step n+1's E at plane k, rows 1..TY+2 ----
            const bool own_k = k >= k0 && k < k1;
            const bool rim_k = k == rc0 || k == rc1 - 1;
#pragma unroll
            for (int r = 1; r < NH; ++r) {
                const int j = j0 - 2 + r;
                const float hz_im = shfl_prev(Hh[2][r]);
                const float hy_im = shfl_prev(Hh[1][r]);
                const float dyHz = Hh[2][r] - Hh[2][r - 1];
                const float dzHy = Hh[1][r] - Hhp[1][r];
                const float dzHx = Hh[0][r] - Hhp[0][r];
                const float dxHz = Hh[2][r] - hz_im;
                const float dxHy = Hh[1][r] - hy_im;
                const float dyHx = Hh[0][r] - Hh[0][r - 1];
                float dzHy_ = dzHy, dzHx_ = dzHx;
                if (ZP && pz >= 0) {
                    const int o = zo(2 * s0, pz, j);
                    dzHy_ = pml_diff(dzHy, czE, bload(PS, xv, o), qE1[0][r]);                       // Ex
                    dzHx_ = pml_diff(dzHx, czE, bload(PS, xv, o + P.psi_n[2] * 4), qE1[1][r]);   // Ey
                }
                float ex = fmaf(Kc[0][r], fmaf(sy, dyHz, -(sz * dzHy_)), Ec[0][r]);
                float ey = fmaf(Kc[1][r], fmaf(sz, dzHx_, -(sx * dxHz)), Ec[1][r]);
                float ez = fmaf(Kc[2][r], fmaf(sx, dxHy, -(sy * dyHx)), Ec[2][r]);
                ex = (j == 0 || k == 0) ? 0.0f : ex;
                ey = (x == 0 || k == 0) ? 0.0f : ey;
                ez = (x == 0 || j == 0) ? 0.0f : ez;
                if (ZP && (k < 0 || k >= nz)) ex = ey = ez = 0.0f;   // ghost planes stay zero
                E1c[0][r] = ex;
                E1c[1][r] = ey;
                E1c[2][r] = ez;
                // the step-n+1 state of R2's outermost layer
                const bool own_r = r >= 2 && r - 2 < jn;
                if (own_k && own_r && own_x && (rim_k || rim_x || j == rb0 || j == rb1 - 1)) {
                    const int o = ro(j, k);
                    bstore_nt(ex, FB, xo, eb + o);
                    bstore_nt(ey, FB, xo, eb + rowb + o);
                    bstore_nt(ez, FB, xo, eb + 2 * rowb + o);
                    bstore_nt(Hh[0][r], FB, xo, hb + o);
                    bstore_nt(Hh[1][r], FB, xo, hb + rowb + o);
                    bstore_nt(Hh[2][r], FB, xo, hb + 2 * rowb + o);
                    if (ZP && pz >= 0) {
                        bstore(qH1[0][r], PS, xv, zo(6 + 2 * s1, pz, j));
                        bstore(qH1[1][r], PS, xv, zo(6 + 2 * s1 + 1, pz, j));
                    }
                }
            }
        }
        if (k >= k0) {
            // ---- step n+2 at plane km = k-1: Ht rows 1..TY+1, E rows 2..TY+1 ----
            const int km = k - 1;
#pragma unroll
            for (int r = 1; r <= TY + 1; ++r) {
                const float ez_i1 = shfl_next(E1p[2][r]);
                const float ey_i1 = shfl_next(E1p[1][r]);
                const float dyEz = E1p[2][r + 1] - E1p[2][r];
                const float dzEy = E1c[1][r] - E1p[1][r];
                const float dzEx = E1c[0][r] - E1p[0][r];
                const float dxEz = ez_i1 - E1p[2][r];
                const float dxEy = ey_i1 - E1p[1][r];
                const float dyEx = E1p[0][r + 1] - E1p[0][r];
                float dzEy_ = dzEy, dzEx_ = dzEx;
                if (ZP && pzp >= 0) {
                    float n0, n1;
                    dzEy_ = pml_diff(dzEy, czHp, qH1p[0][r], n0);   // Hx
                    dzEx_ = pml_diff(dzEx, czHp, qH1p[1][r], n1);   // Hy
                    if (own_x && r >= 2 && r - 2 < jn && km >= k0 && km < k1) {
                        const int j = j0 - 2 + r;
                        bstore(n0, PS, xv, zo(6 + 2 * s2, pzp, j));
                        bstore(n1, PS, xv, zo(6 + 2 * s2 + 1, pzp, j));
                    }
                }
                H2[0][r] = Hhp[0][r] - fmaf(sy, dyEz, -(sz * dzEy_));
                H2[1][r] = Hhp[1][r] - fmaf(sz, dzEx_, -(sx * dxEz));
                H2[2][r] = Hhp[2][r] - fmaf(sx, dxEy, -(sy * dyEx));
                if (ZP && km < 0) H2[0][r] = H2[1][r] = H2[2][r] = 0.0f;   // ghost plane
            }
            if (km >= k0) {
#pragma unroll
                for (int r = 2; r <= TY + 1; ++r) {
                    const int j = j0 - 2 + r;
                    const float hz_im = shfl_prev(H2[2][r]);
                    const float hy_im = shfl_prev(H2[1][r]);
                    if (r - 2 >= jn) continue;
                    const float dyHz = H2[2][r] - H2[2][r - 1];
                    const float dzHy = H2[1][r] - H2p[1][r];
                    const float dzHx = H2[0][r] - H2p[0][r];
                    const float dxHz = H2[2][r] - hz_im;
                    const float dxHy = H2[1][r] - hy_im;
                    const float dyHx = H2[0][r] - H2[0][r - 1];
                    float dzHy_ = dzHy, dzHx_ = dzHx;
                    if (ZP && pzp >= 0) {
                        float n0, n1;
                        dzHy_ = pml_diff(dzHy, czEp, qE1p[0][r], n0);   // Ex
                        dzHx_ = pml_diff(dzHx, czEp, qE1p[1][r], n1);   // Ey
                        if (own_x) {
                            bstore(n0, PS, xv, zo(2 * s2, pzp, j));
                            bstore(n1, PS, xv, zo(2 * s2 + 1, pzp, j));
                        }
                    }
                    float ex = fmaf(Kp[0][r], fmaf(sy, dyHz, -(sz * dzHy_)), E1p[0][r]);
                    float ey = fmaf(Kp[1][r], fmaf(sz, dzHx_, -(sx * dxHz)), E1p[1][r]);
                    float ez = fmaf(Kp[2][r], fmaf(sx, dxHy, -(sy * dyHx)), E1p[2][r]);
                    ex = (j == 0 || km == 0) ? 0.0f : ex;
                    ey = (x == 0 || km == 0) ? 0.0f : ey;
                    ez = (x == 0 || j == 0) ? 0.0f : ez;
                    if (own_x) {
                        const int o = ro(j, km);
                        bstore_nt(ex, FC, xo, eb + o);
                        bstore_nt(ey, FC, xo, eb + rowb + o);
                        bstore_nt(ez, FC, xo, eb + 2 * rowb + o);
                        bstore_nt(H2[0][r], FC, xo, hb + o);
                        bstore_nt(H2[1][r], FC, xo, hb + rowb + o);
                        bstore_nt(H2[2][r], FC, xo, hb + 2 * rowb + o);
                    }
                }
            }
#pragma unroll
            for (int r = 1; r <= TY + 1; ++r) {
                H2p[0][r] = H2[0][r];
                H2p[1][r] = H2[1][r];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int r = 0; r < NE; ++r) Ec[c][r] = Enx[c][r];
#pragma unroll
            for (int r = 0; r < NH; ++r) {
                Hhp[c][r] = Hh[c][r];
                E1p[c][r] = E1c[c][r];
                Kp[c][r] = Kc[c][r];
            }
        }
        if (ZP) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < NH; ++r) {
                    qH1p[c][r] = qH1[c][r];
                    qE1p[c][r] = qE1[c][r];
                }
            czHp = czH;
            czEp = czE;
            pzp = pz;
        }
    }
}

template <bool ZP, int TY, bool COOP>
__global__ __launch_bounds__(64 * YO_MAX_WPB) void k_yee_step2(const YoStepArgs a)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb >> 3, rem = nb & 7, xcd = b & 7, pos = b >> 3;
    const int lb = (xcd < rem) ? xcd * (q + 1) + pos : rem * (q + 1) + (xcd - rem) * q + pos;
    const int wpb = a.wpb;
    const int wave = __builtin_amdgcn_readfirstlane(lb * wpb + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (wave >= a.total_waves) return;
    int s = 0;
    while (s + 1 < a.n_slots && wave >= a.prefix[s + 1]) ++s;
    const YoSlot sl = a.slot[s];
    const YoPlanD &P = *sl.plan;
    const int step = *P.step_ctr + a.k_offset;
    // the host schedules a pair only where both steps remain
    if (step + 1 >= P.n_steps) return;
    const int local = wave - a.prefix[s];
    if (COOP) {
        // one tile per block; consecutive blocks take the same tile for the
        // next right-hand sides (every early exit above is uniform over the
        // block, as the barriers require)
        extern __shared__ float xs2[];
        const int blk = local / wpb;
        const int w = local - blk * wpb;
        const int r = sl.rhs0 + blk % sl.nrhs;
        const int ti = blk / sl.nrhs;
        if (ti >= sl.ntile) return;
        wave_step2<TY, ZP, true>(P, P.rhs[r], step, sl.tiles[ti], w, wpb, lane, xs2);
        return;
    }
    const int grp = local / (wpb * sl.nrhs);
    const int in_grp = local - grp * (wpb * sl.nrhs);
    const int r = sl.rhs0 + in_grp / wpb;
    const int ti = grp * wpb + in_grp % wpb;
    if (ti >= sl.ntile) return;
    wave_step2<TY, ZP, false>(P, P.rhs[r], step, sl.tiles[ti], 0, wpb, lane, nullptr);
}

// locate point q of slot s in the aux work list
__device__ __forceinline__ bool aux_point(const YoAuxArgs &a, int &s, int &r, int &q)
{
    const int blk = blockIdx.x;
    s = 0;
    while (s + 1 < a.n_slots && blk >= a.prefix[s + 1]) ++s;
    const long g = (long)(blk - a.prefix[s]) * blockDim.x + threadIdx.x;
    const long per = a.npts[s];
    if (per <= 0 || g >= per * a.nrhs[s]) return false;
    r = a.rhs0[s] + (int)(g / per);
    q = (int)(g % per);
    return true;
}

// Component plane tt of a port or source plane (normal `axis`, cell index
// `index`): 0, 1 the tangential E (t1, t2) on the plane; 2 the normal E
// (its sites lie half a cell past the plane, stored at the same index);
// 3, 4 the tangential E on the next plane.
__device__ __forceinline__ void plane_component(int axis, int index, int tt, int &c, int &idx)
{
    c = tt == 2 ? axis : (axis + 1 + (tt < 2 ? tt : tt - 3)) % 3;
    idx = index + (tt >= 3 ? 1 : 0);
}

// Running DFT of E^n (called before step n): S += E^n exp(+i w n dt) on the
// design box (3 components) and the port planes (2 tangential components),
// for each frequency the right-hand side accumulates; under a pulse with a
// DFT stride m > 1 only the steps divisible by m add.
__global__ __launch_bounds__(256) void k_dft(const YoAuxArgs a)
{
    int s, r, q;
    if (!aux_point(a, s, r, q)) return;
    const YoPlanD &P = *a.plan[s];
    const int step = *P.step_ctr + a.k_offset;
    if (step >= P.n_steps) return;
    const YoRhsD &R = P.rhs[r];
    const int w = step - R.win_start;
    if (w < 0 || w >= R.win_len) return;
    if (P.dft_stride > 1 && step % P.dft_stride) return;
    const float *F = R.F[step % P.nbuf];
    const int bx = P.box[3], by = P.box[4], bz = P.box[5];
    const int bsz = bx * by * bz;
    float e;
    float2 *acc;
    int fstride;
    if (q < 3 * bsz) {
        const int c = q / bsz, rem = q - c * bsz;
        const int bk = rem / (bx * by), rem2 = rem - bk * bx * by;
        const int bj = rem2 / bx, bi = rem2 - bj * bx;
        e = F[yo_off(c, P.box[0] + bi, P.box[1] + bj, P.box[2] + bk, P.ny, P.nxp, 6)];
        acc = R.dft_box + q;
        fstride = R.box_fstride;
    } else {
        const int qm = q - 3 * bsz;
        int p = 0;
        while (p + 1 < P.n_ports && qm >= P.mon_off[p + 1]) ++p;
        const YoPlaneD pl = P.ports[p];
        const int loc = qm - P.mon_off[p];
        const int plane = pl.n0 * pl.n1;
        const int tt = loc / plane, rem = loc - tt * plane;
        const int b = rem / pl.n0, ai = rem - b * pl.n0;
        int c, idx;
        plane_component(pl.axis, pl.index, tt, c, idx);
        const int cx = sel3(pl.axis, idx, pl.lo0 + ai, pl.lo0 + ai);
        const int cy = sel3(pl.axis, pl.lo0 + ai, idx, pl.lo1 + b);
        const int cz = sel3(pl.axis, pl.lo1 + b, pl.lo1 + b, idx);
        e = F[yo_off(c, cx, cy, cz, P.ny, P.nxp, 6)];
        acc = R.dft_mon + qm;
        fstride = R.mon_fstride;
    }
    for (int f = 0; f < R.n_dft; ++f) {
        const float4 st = R.dfttab[(size_t)f * P.n_steps + step];
        float2 v = acc[(size_t)f * fstride];
        v.x = fmaf(e, st.z, v.x);
        v.y = fmaf(e, st.w, v.y);
        acc[(size_t)f * fstride] = v;
    }
}

// Soft current source of step n (called after step n): E^{n+1} -= kappa j^{n+1/2}
// on the right-hand side's source plane.
__global__ __launch_bounds__(256) void k_source(const YoAuxArgs a)
{
    int s, r, q;
    if (!aux_point(a, s, r, q)) return;
    const YoPlanD &P = *a.plan[s];
    const int step = *P.step_ctr + a.k_offset;
    if (step >= P.n_steps) return;
    const YoRhsD &R = P.rhs[r];
    if (!R.src_j) return;
    const YoPlaneD pl = R.src;
    const int plane = pl.n0 * pl.n1;
    if (q >= R.src_nc * plane) return;
    const float4 st = R.steptab[step];
    const int tt = q / plane, rem = q - tt * plane;
    const int b = rem / pl.n0, ai = rem - b * pl.n0;
    int c, idx;
    plane_component(pl.axis, pl.index, tt, c, idx);
    const int cx = sel3(pl.axis, idx, pl.lo0 + ai, pl.lo0 + ai);
    const int cy = sel3(pl.axis, pl.lo0 + ai, idx, pl.lo1 + b);
    const int cz = sel3(pl.axis, pl.lo1 + b, pl.lo1 + b, idx);
    const size_t o = yo_off(c, cx, cy, cz, P.ny, P.nxp, 6);
    const float2 jv = R.src_j[q];
    const float j = fmaf(jv.x, st.x, jv.y * st.y);
    float *F = R.F[(step + 1) % P.nbuf];
    F[o] = fmaf(-P.kappa[yo_off(c, cx, cy, cz, P.ny, P.nxp, 3)], j, F[o]);
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

template <int PM, bool COOP, bool PF, int TY = YO_TY>
static void launch_one(const YoStepArgs &args, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_yee_step<PM, COOP, PF, TY>), dim3(blocks), dim3(64 * args.wpb), 0, s, args);
}

template <int PM>
static void launch_pm(bool coop, bool pf, const YoStepArgs &args, int blocks, hipStream_t s)
{
    if (coop) {
        if (pf) launch_one<PM, true, true>(args, blocks, s);
        else launch_one<PM, true, false>(args, blocks, s);
    } else {
        if (pf) launch_one<PM, false, true>(args, blocks, s);
        else launch_one<PM, false, false>(args, blocks, s);
    }
}

hipError_t yo_launch_step(int pm, bool coop, bool prefetch, const YoStepArgs &args, int blocks,
                          hipStream_t s, int rows)
{
    if (blocks <= 0) return hipSuccess;
    if (args.wpb != 4 && args.wpb != 8) return hipErrorInvalidValue;
    if (rows == YO_TY2) {
        // taller tiles: the CPML shell's independent waves only
        if (coop) return hipErrorInvalidValue;
        if (pm == YO_PM_ANY && prefetch) launch_one<YO_PM_ANY, false, true, YO_TY2>(args, blocks, s);
        else if (pm == YO_PM_ANY) launch_one<YO_PM_ANY, false, false, YO_TY2>(args, blocks, s);
        else if (pm == 7 && prefetch) launch_one<7, false, true, YO_TY2>(args, blocks, s);
        else if (pm == 7) launch_one<7, false, false, YO_TY2>(args, blocks, s);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (rows != YO_TY) return hipErrorInvalidValue;
    switch (pm) {
    case 0: launch_pm<0>(coop, prefetch, args, blocks, s); break;
    case 1: launch_pm<1>(coop, prefetch, args, blocks, s); break;
    case 7: launch_pm<7>(coop, prefetch, args, blocks, s); break;
    case YO_PM_ANY: launch_pm<YO_PM_ANY>(coop, prefetch, args, blocks, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t yo_launch_step2(bool zslab, int rows, bool coop, const YoStepArgs &args, int blocks,
                           hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    if (args.wpb != 4 && args.wpb != 8) return hipErrorInvalidValue;
    const dim3 g(blocks), b(64 * args.wpb);
    // cooperative: 20 exchange slots of 64 floats per wave and parity
    const size_t lds = (size_t)2 * args.wpb * 20 * 64 * sizeof(float);
    if (zslab && rows == YO_TY && !coop)
        hipLaunchKernelGGL((k_yee_step2<true, YO_TY, false>), g, b, 0, s, args);
    else if (!zslab && rows == YO_TY && !coop)
        hipLaunchKernelGGL((k_yee_step2<false, YO_TY, false>), g, b, 0, s, args);
    else if (!zslab && rows == YO_TY2 && !coop)
        hipLaunchKernelGGL((k_yee_step2<false, YO_TY2, false>), g, b, 0, s, args);
    else if (!zslab && rows == YO_TY && coop)
        hipLaunchKernelGGL((k_yee_step2<false, YO_TY, true>), g, b, lds, s, args);
    else if (!zslab && rows == YO_TY2 && coop)
        hipLaunchKernelGGL((k_yee_step2<false, YO_TY2, true>), g, b, lds, s, args);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t yo_launch_dft(const YoAuxArgs &args, hipStream_t s)
{
    if (args.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dft, dim3(args.total_blocks), dim3(256), 0, s, args);
    return hipGetLastError();
}

hipError_t yo_launch_source(const YoAuxArgs &args, hipStream_t s)
{
    if (args.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_source, dim3(args.total_blocks), dim3(256), 0, s, args);
    return hipGetLastError();
}

hipError_t yo_launch_ctr(const YoCtrArgs &args, int set_value, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctr, dim3(1), dim3(64), 0, s, args, set_value);
    return hipGetLastError();
}
