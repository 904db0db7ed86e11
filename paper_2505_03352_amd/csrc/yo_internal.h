// Internal device descriptors and kernel entry points of libyeeopt (not part
// of the public ABI).  Host runtime and kernels share these layouts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define YO_MAX_PORTS 8
#define YO_MAX_SLOTS 32
#define YO_TX 62          // owned x-cells per wave (lanes 1..62; lanes 0 and 63 are halo)
#define YO_TY 4           // rows per wave
#define YO_TY2 6          // rows per wave of the two-step region's taller tiles
#define YO_MAX_WPB 8      // waves per block of the step kernel: 4 or 8

// Field arrays carry one ghost layer on every face and keep the components
// of one (j, k) row together: component c of cell (x, j, k), x in [-1, nx],
// j in [-1, ny], k in [-1, nz], of an array with nc components sits at
//   (((k + 1) * (ny + 2) + (j + 1)) * nc + c) * nxp + (x + 1).
// The state of one right-hand side and step parity is one such array with
// nc = 6 (Ex Ey Ez Ht_x Ht_y Ht_z), kappa one with nc = 3, so a row group
// of all components is one contiguous block of memory.  Ghosts are zero and
// never written, which realises the perfect-conductor box (values outside
// the grid read as zero) without branches.

struct YoPlaneD {
    int axis, index, lo0, lo1, n0, n1;
};

// One right-hand side: its own field state, absorbing-layer memories, DFT
// sums, source plane and per-step phase table.
struct YoRhsD {
    // state buffers, ghost layout, nc = 6 (E then Ht): the state after step
    // s is in F[s % nbuf]; nbuf = 3 (a third buffer) when the plan may
    // advance its interior two steps per sweep, else 2 (F[2] null)
    float *F[3];
    // CPML memories: per axis a, at float offset psi_off[a] of the plan,
    // arrays of psi_n[a] floats, two components per slot: with nbuf = 2 six
    // (E one slot, Ht two by step parity), with nbuf = 3 twelve (E three
    // slots, Ht three, the step's in slot step % 3); each [2 comps] of the
    // axis' slab layout
    // (x [nz][ny][Wx], y [nz][Wy][nxp], z [Wz][ny][nxp])
    float *psi;
    float2 *dft_box;         // [3][bz][by][bx]
    float2 *dft_mon;         // concatenated port planes [2][n1][n0]
    const float4 *steptab;   // [n_steps]: source signal (x, y) at (n+1/2)dt, (cos, sin) at n dt
    const float2 *src_j;     // [2][n1][n0], nullptr if no source
    YoPlaneD src;
    int win_start, win_len;
    float ginv[4];           // inverse Gram matrix of the steady-state fit
    int freq;
    int n_dft;               // frequencies this right-hand side's DFT accumulates (1, or all under a pulse)
    const float4 *dfttab;    // DFT phases (.z, .w) of frequency f at step n: dfttab[f * n_steps + n]
    int box_fstride;         // float2 entries from one frequency's DFT box to the next
    int mon_fstride;         // the same for the port planes
    int src_nc;              // component planes of the source (see YoPlanD::mon_nc)
    int pad2;
};

// One plan (one geometry): shared material and geometry description.
struct YoPlanD {
    int nx, ny, nz, nxp;     // nxp: padded row pitch of the ghost layout
    float sx, sy, sz, pad0;
    int plo[3], phi[3];      // PML cells low/high per axis
    const float *kappa;      // ghost layout (ghost values unused)
    const float *prof[3];    // per axis [6][n_a]: bE cE kiE bH cH kiH
    int psi_off[3], psi_n[3];
    int psi_total;           // floats of CPML memory per right-hand side
    int box[6];              // x0 y0 z0 bx by bz
    int n_ports;
    int n_steps;
    int dft_stride;          // the DFT adds E^n of the steps n divisible by it (1: every step)
    int nbuf;                // state buffers per right-hand side (2 or 3)
    int r2[6];               // two-step region [x0, x1) x [y0, y1) x [z0, z1) (empty: x1 <= x0)
    YoPlaneD ports[YO_MAX_PORTS];
    int mon_off[YO_MAX_PORTS];
    int mon_total;
    int *step_ctr;           // device step counter of this plan
    int n_rhs;
    // component planes of a port's monitor (and of its adjoint source): 2 =
    // the tangential E on the plane; 5 = those, the normal E half a cell past
    // the plane, and the tangential E one cell past it
    int mon_nc;
    const YoRhsD *rhs;       // [n_rhs]
};

// A tile is one wave's work (or, in the cooperative layout, one block's):
// owned x in [x0, x0+xn) (xn <= 62), rows [j0, j0+jn) (jn <= YO_TY, or
// YO_TY * waves per block), planes [k0, k1).  Packed as int4
// (x0 | xn << 16, j0 | jn << 16, k0 | k1 << 16, tile class).
struct YoSlot {
    const YoPlanD *plan;
    const int4 *tiles;       // tile list of this launch's class
    int rhs0, nrhs;
    int ntile, pad_;
};

struct YoStepArgs {
    int n_slots;
    int k_offset;            // launch index inside the chunk; step = counter + k_offset
    int total_waves;
    int wpb;                 // waves per block (4 or 8)
    int prefix[YO_MAX_SLOTS + 1];
    YoSlot slot[YO_MAX_SLOTS];
};

// Work list of the small per-step kernels (DFT accumulation and source
// injection): per slot, the plan, its right-hand side range and the number
// of points per right-hand side.
struct YoAuxArgs {
    int n_slots;
    int k_offset;
    int total_blocks;
    int pad_;
    int prefix[YO_MAX_SLOTS + 1];   // blocks
    const YoPlanD *plan[YO_MAX_SLOTS];
    int rhs0[YO_MAX_SLOTS], nrhs[YO_MAX_SLOTS];
    int npts[YO_MAX_SLOTS];         // points per right-hand side
};

struct YoCtrArgs {
    int n;
    int add;
    int *ctr[YO_MAX_SLOTS];
};

// Parametrization buffers of one plan.
struct YoChainBufs {
    int md, nd, mc, nc, S, U, V, G0, G1;   // G0 = md+4 (x), G1 = nd+4 (y)
    int tmax;                               // filter taps per sub-pixel (max)
    float eps_core, eps_clad, delta;
    // filter tables
    int *tap_lo_x, *tap_n_x, *tap_lo_y, *tap_n_y;   // [S md], [S nd]
    float *tap_w_x, *tap_w_y;                        // [S md][tmax], [S nd][tmax]
    int *urange_x, *urange_y;                        // per control: [2] first/last sub-pixel
    // forward state
    float *mask;      // [V][U]
    float *rho;       // [V][U]
    float *tanh_;     // [S nd][S md]
    float *P, *Q, *R; // [3][G1][G0]
    float *aux;       // [6][G1][G0]: n2x n2y Gx_x Gy_x Gx_y Gy_y
    // backward
    float *gmap;      // [4][G1][G0]: gx gy gz_in gz_face
    float *gPQ;       // [6][G1][G0]: gP(x,y,z) gQ(x,y,z)
    float *gG;        // [4][G1][G0]: gGx_x gGy_x gGx_y gGy_y
    float *gR;        // [2][G1][G0]
    float *gphi;      // [S nd][S md]
    float *tmp;       // [S nd][mc]
    // morphological filters (n_morph = 0: none; rho = the Eq. (3) projection)
    int n_morph;      // stages
    unsigned mdil;    // bit k set: stage k dilates, else erodes
    int n_mtaps;      // disc taps
    float malpha;     // sharpness
    float minv;       // 1 / n_mtaps
    int *mtap;        // [n_mtaps][2]: dy, dx (sub-pixels)
    float *mcan;      // [n_morph + 1][V][U]: stage inputs, then the last output
    float *msum;      // [n_morph][S nd][S md]: each stage's kernel sums
    float *tanh2;     // [S nd][S md]: tanh of the projection after the stages
    float *mg;        // [2][S nd][S md]: gradients between stages
    float *mq;        // [S nd][S md]: gradient / kernel sum of the stage being transposed
};

// ---- kernel launchers ----
// pm: 0 = interior tiles (no CPML code), 1 = interior tiles plus tiles inside
// the x-slabs only (the x-axis CPML code), 7 = CPML tiles with the code of all
// three axes, 8 = CPML tiles each running its own class's code (int4 .w);
// coop: one tile per block, its waves stacked in y (tiles of YO_TY * wpb
// rows); prefetch: operands of the next plane loaded during this one
// rows: rows per wave, YO_TY, or YO_TY2 for the shell (pm 7 or 8, not coop)
hipError_t yo_launch_step(int pm, bool coop, bool prefetch, const YoStepArgs &args, int blocks,
                          hipStream_t s, int rows = YO_TY);
// two steps per sweep over the tiles of the two-step region (independent
// waves); zslab: the tiles of the z-slabs under it, with z-axis CPML code;
// rows: rows per wave, YO_TY, or YO_TY2 for the region itself; coop: one
// tile per block, its waves stacked in y and sharing rows through LDS
hipError_t yo_launch_step2(bool zslab, int rows, bool coop, const YoStepArgs &args, int blocks,
                           hipStream_t s);
hipError_t yo_launch_dft(const YoAuxArgs &args, hipStream_t s);
hipError_t yo_launch_source(const YoAuxArgs &args, hipStream_t s);
hipError_t yo_launch_ctr(const YoCtrArgs &args, int set_value, hipStream_t s);
hipError_t yo_launch_fill(float *p, size_t n, float v, hipStream_t s);
// dense [ncomp][nz][ny][nx] <-> components c0 .. c0+ncomp-1 of a ghost-layout
// array with nc components
hipError_t yo_launch_to_ghost(const float *dense, float *ghost, int ncomp, int c0, int nc, int nz,
                              int ny, int nx, int nxp, hipStream_t s);
hipError_t yo_launch_from_ghost(const float *ghost, float *dense, int ncomp, int c0, int nc, int nz,
                                int ny, int nx, int nxp, hipStream_t s);
// in-place phasor fit of n complex sums; sets *bad to 1 if a result is not
// finite (*bad is left alone otherwise)
hipError_t yo_launch_finalize(float2 *a, size_t n, float g00, float g01, float g10, float g11,
                              int *bad, hipStream_t s);
hipError_t yo_launch_alpha(const float2 *mon_dft, const float2 *weights, int n, float2 *out,
                           hipStream_t s);
hipError_t yo_launch_chain_forward(const YoChainBufs &c, const float *C, float beta,
                                   float *kappa, int nx, int ny, int nz, int nxp, int i0, int j0,
                                   int k_lo, int k_hi, hipStream_t s);
#define YO_MAX_GF 32
#define YO_MAX_GA 64
#define YO_MAX_FREQ 16
struct YoGradArgs {
    const float2 *EF[YO_MAX_GF];   // forward box phasors, index f*n_src + s
    const float2 *EA[YO_MAX_GA];   // adjoint box phasors, index f*n_ports + p
    float sinth[YO_MAX_FREQ];      // sin(w dt / 2) per frequency
    const float2 *coef;            // [n_src][n_ports][n_freq]
    const float *kappa;            // ghost layout
    float *gbox;                   // optional [3][bz][by][bx] dF/dkappa
    float *gmap;                   // optional [4][G1][G0] z-summed maps
    int n_src, n_ports, n_freq;
    int nxp, ny, nz;
    int box[6];
    int k_lo, k_hi, G0, G1;
};
hipError_t yo_launch_grad_assemble(const YoGradArgs &a, hipStream_t s);
hipError_t yo_launch_chain_vjp(const YoChainBufs &c, float beta, float *dFdC, hipStream_t s);
// grey fraction of the design area: rho in (lo, hi) as tanh in (tlo, thi)
hipError_t yo_launch_unbinarity(const YoChainBufs &c, float tlo, float thi, int *count, float *out,
                                hipStream_t s);
hipError_t yo_launch_adam(float *C, const float *G, float *M, float *V, int n, float lr, float b1, float b2,
                          float eps, float inv1, float inv2, hipStream_t s);
hipError_t yo_launch_zsum(const float *gbox, const int *box, int k_lo, int k_hi, float *gmap, int G0,
                          int G1, hipStream_t s);

// ghost-layout offset of component c of (x, j, k) in an array of nc components
__host__ __device__ inline size_t yo_off(int c, int x, int j, int k, int ny, int nxp, int nc)
{
    return (((size_t)(k + 1) * (ny + 2) + (size_t)(j + 1)) * nc + c) * nxp + (size_t)(x + 1);
}
