/*
 * yeeopt: adjoint FDTD hot path for inverse design of passive Si photonics
 * on MI355X (gfx950).  C ABI.
 *
 * The library computes, for control variables C and projection strength
 * beta (paper Sec. 3, Eqs. (2), (3)/(6), (7), (8)), the per-component
 * anisotropic permittivity on the Yee grid; advances the Yee scheme with
 * time-harmonic electric-current mode sources (Sec. 2 and Appendix A) once
 * for every forward right-hand side (input source x wavelength) and once for
 * every adjoint right-hand side (output port x wavelength, unit amplitude);
 * reads amplitude and phase of the steady state in the design region and on
 * the port planes; forms the modal coefficients alpha (Appendix A); and pulls
 * dF/dalpha back to dF/dC through Eq. (1) and the parametrization's
 * vector-Jacobian product, without forming the Jacobian.
 *
 * Conventions
 *   - Grid: nx x ny x nz cells, the CPML included.  Yee sites in cell units:
 *     E_x(i+1/2,j,k), E_y(i,j+1/2,k), E_z(i,j,k+1/2), Ht_x(i,j+1/2,k+1/2),
 *     Ht_y(i+1/2,j,k+1/2), Ht_z(i+1/2,j+1/2,k); Ht = eta0 H.  The outer box is
 *     a perfect electric conductor.  Dense 3-D arrays exchanged with the
 *     caller are FP32 [3][nz][ny][nx], x fastest.
 *   - Time: dt = courant * min(dx,dy,dz) / c.  E^n lives at n dt, Ht at
 *     (n+1/2) dt.  Phasors follow E(t) = Re(Ehat exp(-i w t)).
 *   - Planes: normal `axis` (0,1,2) at cell `index`; (c0,c1) are the other
 *     two axes in increasing order with extents [lo0,lo0+n0) x [lo1,lo1+n1);
 *     plane arrays are [2][n1][n0], components ordered cyclically
 *     (axis x: (y,z); axis y: (z,x); axis z: (x,y)).
 *   - Complex arrays are interleaved (re, im): complex64 on the device,
 *     complex128 (double pairs) on the host.
 *   - Design canvas: the design area (md x nd pixels at (i0, j0)) plus a
 *     2-pixel margin, `supersample` sub-pixels per pixel, FP32
 *     [S(nd+4)][S(md+4)]; sub-pixel (v,u) covers x in
 *     [i0-2.5+u/S, i0-2.5+(u+1)/S) and the same in y.  Controls are FP32
 *     [nc][mc] (x fastest) spread over the design area.
 *
 * Memory and streams
 *   - The library never allocates device memory.  Every device pointer is
 *     owned by the caller; a plan keeps non-owning pointers to its bound
 *     workspace and the caller keeps it alive until yo_plan_destroy.
 *   - Calls taking a hipStream_t are asynchronous on that stream, except
 *     where noted; host arrays passed to them are copied before return.
 *   - Errors: a negative yo_status and a thread-local message from
 *     yo_last_error().  Device faults surface as YO_EHIP; a run that
 *     diverged surfaces as YO_EUNSTABLE from yo_finalize (watchdog below).
 */
#ifndef YEEOPT_H
#define YEEOPT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *yo_stream;   /* same type as hipStream_t */
typedef struct yo_plan yo_plan;
typedef int yo_status;

enum {
    YO_OK = 0,
    YO_EINVAL = -1,        /* bad argument or descriptor                        */
    YO_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. too many ports)   */
    YO_EHIP = -3,          /* HIP runtime error                                 */
    YO_EWORKSPACE = -4,    /* no workspace bound or too small                   */
    YO_EUNSTABLE = -5,     /* Courant number above the stability limit, or a run
                              whose phasors came out non-finite (watchdog)      */
    YO_ESTATE = -6         /* call out of order (e.g. gradient before a run)    */
};

enum { YO_FORWARD = 1, YO_ADJOINT = 2, YO_BOTH = 3 };

/* Grid and absorbing boundary (CPML on every face with npml > 0; the PML is
 * graded as sigma = scale * 0.8 (m+1) (c dt / d_a) * xi^m with depth xi in
 * [0,1], stretch 1 + (kappa_max - 1) xi^m and CFS shift a_max (1 - xi)). */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;          /* metres */
    double courant;             /* c dt / min(dx, dy, dz) */
    int npml[6];                /* cells on faces -x,+x,-y,+y,-z,+z */
    double pml_m, pml_sigma_scale, pml_kappa_max, pml_a_max;
} yo_grid;

/* Design region and parametrization (paper Sec. 3).  The Si slab holds the
 * E_x/E_y planes k_lo..k_hi; E_z planes k_lo..k_hi-1 are inside and the E_z
 * planes k_lo-1 and k_hi lie on the slab faces. */
typedef struct {
    int i0, j0, md, nd;         /* design area pixels [i0,i0+md) x [j0,j0+nd) */
    int k_lo, k_hi;
    int mc, nc;                 /* control grid, x count and y count */
    double filter_r;            /* Gaussian basis support radius, control pixels (sigma = r/2) */
    int supersample;            /* S, even */
    double eps_core, eps_clad;
    double sobel_delta;         /* regulariser in n^2 = G^2 / (|G|^2 + delta) */
} yo_design;

typedef struct { int axis, index, lo0, lo1, n0, n1; } yo_plane;

/* Per-wavelength time-stepping description. */
typedef struct {
    double omega;               /* angular frequency, rad/s */
    double ramp_steps;          /* raised-cosine source ramp length in steps (0: none) */
    int win_start, win_len;     /* E^n for n in [win_start, win_start+win_len) is fitted */
} yo_freq;

/* Create a plan (host only, no device work).  Validates the descriptors:
 * YO_EUNSTABLE if c dt sqrt(sum 1/d_a^2) >= 1; YO_EINVAL for an odd
 * supersample, a design canvas that leaves the grid or touches the CPML,
 * a source or port plane outside the grid or inside the CPML, an empty or
 * out-of-range window, or non-positive sizes.  The plan has n_src forward
 * sources and n_ports output ports (their planes fixed here, their mode
 * profiles set later); it owns (n_src + n_ports) * n_freq right-hand sides.
 * Limits: n_ports <= 8, n_freq <= 16, n_src*n_freq <= 32,
 * n_ports*n_freq <= 64 (YO_EUNSUPPORTED beyond). */
yo_status yo_plan_create(const yo_grid *grid, const yo_design *design, int n_steps,
                         int n_freq, const yo_freq *freqs, int n_src, const yo_plane *src_planes,
                         int n_ports, const yo_plane *port_planes, yo_plan **out);
void yo_plan_destroy(yo_plan *plan);

/* Morphological filters (Sec. 3, Eqs. (4)-(6)), host only, before
 * yo_bind_workspace (YO_ESTATE after).  `ops` names the stages applied to
 * the Eq. (3) density in order, 'd' for the soft dilation of Eq. (4) and
 * 'e' for the soft erosion of Eq. (5), at most 8 (e.g. "edde": opening then
 * closing); the stages are followed by the projection of Eq. (6) with the
 * same beta.  The kernel K_m is the disc of `diameter` design pixels (every
 * sub-pixel offset of length at most diameter * S / 2), normalised to unit
 * sum; `alpha` is the sharpness.  Stages act on the design area; taps
 * outside it read the canvas margin (the background fill), taps beyond the
 * canvas its nearest edge sub-pixel.  NULL or "" turns the filters off.
 * YO_EINVAL for other characters, more than 8 stages, diameter <= 0 or
 * alpha outside (0, 80]; YO_EUNSUPPORTED for a disc radius above 32
 * sub-pixels.  Changes yo_workspace_bytes. */
yo_status yo_set_morphology(yo_plan *plan, const char *ops, double diameter, double alpha);

/* Modal coefficient (App. A), host only, before yo_bind_workspace
 * (YO_ESTATE after).  terms = 1 (default): the E-dependent term alone,
 * alpha = (1/(2N)) sum (E_t1 h_t2* - E_t2 h_t1*) dA.  terms = 2: both terms,
 * alpha = (1/4) ((1/N) sum (E x h*) . n + (1/N*) sum (e* x H) . n) dA, with
 * H the tangential H on the sites half a cell past the plane along its
 * normal.  The library evaluates the H term on E sites through the Yee
 * update's H step (Hhat = curl_e Ehat / (2 i sin(w dt / 2))): each port then
 * records five component planes (E_t1, E_t2 on the plane, the normal E half
 * a cell past it, E_t1, E_t2 on the next plane; yo_get_dft region 1+p is
 * complex64 [5][n1][n0]), and its adjoint source carries the same weights,
 * which depend on the wavelength.  Weights of H sites whose curl would reach
 * past the plane (its last row along t2 for H_t1, last column along t1 for
 * H_t2) are dropped.  Call yo_set_port_mode after this.  YO_EINVAL for
 * other values or a port whose next plane leaves the grid interior;
 * YO_EUNSUPPORTED under a pulse.  Changes yo_workspace_bytes. */
yo_status yo_set_alpha_terms(yo_plan *plan, int terms);

/* Pulse excitation (Sec. 2's other route to frequency-domain fields:
 * Fourier transforms of field transients), host only, before
 * yo_bind_workspace (YO_ESTATE after).  With sigma_steps > 0 every source
 * and every port is stepped once instead of once per wavelength: its
 * current is g(t) Re(jhat e^{-i omega0 t}), g(t) = exp(-(t - t0)^2 /
 * (2 sigma^2)), t = (n + 1/2) dt in steps, and the DFT of every step is
 * accumulated at each wavelength of the plan.  yo_finalize turns the sums
 * into the phasors 2 DFT(w) / S(w), S(w) = sum_n s_n e^{+i w (n + 1/2) dt}
 * of the injected samples s_n = g e^{-i omega0 t}, so yo_get_dft, yo_alpha
 * and the gradients keep their meaning and numbering (one output
 * right-hand side per source or port and wavelength).  The phasors are
 * exact when the field has died away by the end of the run and the pulse
 * spectrum at -w is negligible; the caller picks n_steps, sigma and t0 for
 * that.  The yo_freq windows and ramps are not used.  YO_EUNSUPPORTED with
 * the two-term coefficient.  The stepped
 * right-hand sides (yo_set_fields / yo_get_fields) are the sources, then
 * the ports.  sigma_steps <= 0 turns the pulse off.  YO_EINVAL for a
 * carrier outside (0, pi/dt) or t0 < 0.  Changes yo_workspace_bytes. */
yo_status yo_set_pulse(yo_plan *plan, double omega0, double sigma_steps, double t0_steps);

/* Under a pulse (yo_set_pulse first), host only, before yo_bind_workspace
 * (YO_ESTATE after): the DFT adds E^n only on the steps n divisible by
 * `stride` (1..64; 1, the default, is every step), and the phasors become
 * 2 stride DFT(w) / S(w).  The sampled sum is (1/stride) times the sum of
 * the full DFT at w + 2 pi q / stride, q = 0..stride-1, so the phasors stay
 * those of the full DFT when the pulse's spectrum vanishes at every alias
 * q != 0: YO_EINVAL unless it is below 1e-6 of its value at w there (and for
 * the pulse's conjugate part) at every wavelength; the FP32 rounding of the
 * stored samples alone leaves about 1e-8.  The DFT's memory traffic
 * drops by the stride.  YO_EINVAL without a pulse or for a stride outside
 * [1, 64]; turning the pulse off resets it to 1. */
yo_status yo_set_dft_stride(yo_plan *plan, int stride);

/* Temporal blocking (Sec. 2: the diamond / wavefront tilings of x-y-z-t that
 * fdtd-z shares with DiamondTorre, advancing several steps per pass over
 * memory), host only, before yo_bind_workspace (YO_ESTATE after).  steps = 2
 * gives every right-hand side a third state buffer (the state after step s
 * lives in buffer s % 3), so that the interior cells two clear of every
 * absorbing slab and of every source and port plane (the two-step region)
 * can be advanced two steps in one launch that reads each of their planes
 * once; tiling flag 512 (yo_set_tiling) then turns the pairs on.  Steps
 * whose DFT the plan needs (the time-harmonic window) and a run's odd last
 * step go one at a time.  Results are bitwise those of single steps.
 * steps = 1 (the default) removes the buffer.  Changes yo_workspace_bytes.
 * YO_EINVAL for other values. */
yo_status yo_set_time_blocking(yo_plan *plan, int steps);

/* Device bytes the plan needs (host only). */
yo_status yo_workspace_bytes(const yo_plan *plan, size_t *bytes);

/* Bind a caller-owned device buffer of at least yo_workspace_bytes bytes
 * (256-byte aligned) and upload the plan's tables (PML profiles, step
 * phases, filter taps) on `stream`.  YO_EWORKSPACE if too small. */
yo_status yo_bind_workspace(yo_plan *plan, void *dev, size_t bytes, yo_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bind the
 * library's own static workspace of the current device instead of a
 * caller-owned buffer; everything else works as after yo_bind_workspace.
 * Allocates nothing (no hipMalloc, no allocating library call).  The static
 * workspace holds at most 32 MiB (the tiny 56x56x36 device with one forward
 * and one adjoint right-hand side needs about 21 MiB): a plan whose
 * yo_workspace_bytes exceeds that gets YO_EWORKSPACE and stays unbound.  The
 * device's array is shared by every plan bound to it and keeps the last
 * binding's contents; this call clears the plan's part of it to zero and
 * uploads the plan's tables (synchronising `stream`).  Binding another plan
 * to the same device's static workspace takes the memory over: every later
 * call on the earlier plan returns YO_EWORKSPACE until it is bound again.
 * Calls on plans sharing it that overlap in time (other host threads or
 * streams) race and give undefined results.  Each device holds its own
 * copy until the process ends. */
yo_status yo_bind_static_workspace(yo_plan *plan, yo_stream stream);

/* Background: dev_kappa = 1/eps_r per E component, FP32 [3][nz][ny][nx];
 * dev_mask = background fill of the design canvas, FP32 [S(nd+4)][S(md+4)]
 * (only its margin is used).  Both are copied into the workspace. */
yo_status yo_set_background(yo_plan *plan, const float *dev_kappa, const float *dev_mask,
                            yo_stream stream);

/* Mode source of input `src` (Appendix A): the electric current J = n x h on
 * its plane, i.e. J_t1 = -h_t2, J_t2 = h_t1.  host_h is complex128 [2][n1][n0]
 * with h_t1 sampled at the E_t2 sites and h_t2 at the E_t1 sites. */
yo_status yo_set_source_mode(yo_plan *plan, int src, const double *host_h, yo_stream stream);

/* Output port `port` with mode (e, h) (Appendix A): monitor weights
 * w_t1 = conj(h_t2)/(2N), w_t2 = -conj(h_t1)/(2N), N = (1/2) sum (e_t1 conj(h_t2)
 * - e_t2 conj(h_t1)), so alpha = sum w . Ehat and alpha = 1 for Ehat = e.  The
 * unit-amplitude adjoint source of this port is jhat = w.  host_e, host_h:
 * complex128 [2][n1][n0] (e_t sampled at the E_t sites, h as above).
 * YO_EINVAL if N = 0. */
yo_status yo_set_port_mode(yo_plan *plan, int port, const double *host_e, const double *host_h,
                           yo_stream stream);

/* Parametrization (Sec. 3): dev_C FP32 [nc][mc] -> Eq. (2) level set with a
 * truncated Gaussian basis, tanh projection Eq. (3)/(6), the morphological
 * stages if any (yo_set_morphology) followed by the Eq. (6) projection,
 * density mix, Yee-cell averages Eq. (8), Sobel normals, Eq. (7), extrusion
 * through the slab; writes kappa on the design area plus a one-pixel ring.
 * Must follow yo_set_background.  Keeps what the gradient needs. */
yo_status yo_set_design(yo_plan *plan, const float *dev_C, double beta, yo_stream stream);

/* Time stepping.  `which` is YO_FORWARD, YO_ADJOINT or YO_BOTH.
 * yo_run: zero the selected right-hand sides' fields, step n_steps times in
 * one launch per step over all of them, then fit the steady-state phasors.
 * The step launches are replayed from a captured HIP graph of `chunk` steps
 * when use_graph != 0.
 *
 * Watchdog: yo_finalize (the end of yo_run) checks every fitted phasor of
 * the selected right-hand sides and synchronises `stream` to read the
 * result.  If any value is Inf or NaN (the fields diverged, e.g. from a
 * background kappa <= 0 or non-finite fields set through yo_set_fields) it
 * returns YO_EUNSTABLE, and yo_alpha, yo_gradient and yo_gradient_kappa
 * return YO_EUNSTABLE until the next yo_reset of that side; yo_get_dft still
 * returns the phasors for inspection.
 *
 * The forward and adjoint right-hand sides are independent: YO_BOTH steps
 * them in the same launches (sharing kappa), while a YO_FORWARD run followed
 * by a YO_ADJOINT run (or the reverse) gives bitwise the same phasors; a
 * reset of one side leaves the other side's phasors alone. */
yo_status yo_run(yo_plan *plan, int which, int chunk, int use_graph, yo_stream stream);

/* Lower-level pieces of yo_run (used by the batch executor and tests). */
yo_status yo_reset(yo_plan *plan, int which, yo_stream stream);
yo_status yo_advance(yo_plan *plan, int which, int n_steps, yo_stream stream);
yo_status yo_finalize(yo_plan *plan, int which, yo_stream stream);

/* Step several plans together: every launch covers every tile of every
 * plan's selected right-hand sides; each plan keeps its own step counter and
 * stops at its own n_steps.  Graph mode captures `chunk` launches once per
 * distinct plan list and relaunches them.  The plans must share their
 * yo_set_tiling flags except 1 and 128 (YO_EINVAL otherwise). */
yo_status yo_advance_many(yo_plan *const *plans, const int *which, int n_plans, int n_steps,
                          int chunk, int use_graph, yo_stream stream);

/* Host-side step count of the last reset/advance of `plan`. */
yo_status yo_steps_done(const yo_plan *plan, int *steps);

/* Work split of the time-stepping kernel.  Each step runs two launches: the
 * interior tiles (clear of every absorbing slab, no CPML code) and the CPML
 * shell.  rows: rows per wave, must be 4; zchunk: z-planes per tile, 4..63;
 * flags, a sum of:
 *    1  the CPML x-shell is cut into full 62-cell strips instead of just
 *       the absorbing columns
 *    2  8 waves per block instead of 4
 *    4  shell: cooperative blocks (the block's waves are stacked in y and
 *       pass the rows they share through LDS instead of each loading them)
 *    8  shell: each tile runs the code of its own CPML axes (else the code
 *       of all three axes)
 *   16  interior: cooperative blocks
 *   32  interior: no prefetch of the next plane's operands
 *   64  shell: no prefetch
 *  128  the CPML x-shell strips take what is left of each row once the
 *       interior is cut into whole 62-cell strips (overrides 1)
 *  256  tiles that meet only the x-slabs run in the interior launch, which
 *       then carries the x-axis CPML code
 *  512  two steps per launch over the two-step region where the run
 *       allows (needs yo_set_time_blocking(plan, 2); not with 16): its
 *       tiles are strips of at most 60 cells, 4 rows and zchunk planes, and
 *       the rest of the interior runs as single-step tiles around it (with
 *       256, together with the tiles that meet only the x-slabs).  The
 *       region clear of the slabs then starts two cells inside them (the
 *       two-step region's margin; the shell takes the layer between), and
 *       with 128 the two-step strips are whole 60-cell strips between the
 *       x-normal source and port planes, the shell strips the rest
 * 1024  with 512 (else YO_EINVAL): the two-step launch of a pair of steps
 *       runs on a second stream of the plan (created at its first advance,
 *       default priority), concurrently with the first step's other
 *       launches, and is joined back before the second step; advance calls
 *       on the caller's stream still complete in stream order, captured
 *       into a graph as well
 * 2048  with 512 (else YO_EINVAL): where the two-step region is the whole
 *       interior (no source or port plane cuts it, as with 128 when the
 *       planes lie in the shell strips), the z-slabs under it also go two
 *       steps per launch, with the z-axis CPML code; the shell launch of
 *       those steps then covers the x- and y-slabs only
 * 4096  with 512 (else YO_EINVAL): the two-step region's tiles have 6 rows
 *       instead of 4 (fewer halo rows re-read, fewer waves per SIMD)
 * 8192  with 512 (else YO_EINVAL): the two-step region in cooperative
 *       blocks (waves stacked in y pass the rows they share through LDS)
 * 16384 the CPML shell's tiles have 6 rows instead of 4 (not with 4:
 *       YO_EINVAL)
 * Other bits: YO_EINVAL.  Results do not depend on the split (bitwise).
 * With a workspace bound, synchronises the device. */
yo_status yo_set_tiling(yo_plan *plan, int rows, int zchunk, int flags);

/* Modal coefficients (Appendix A) of the forward right-hand sides:
 * dev_alpha complex64 [n_src][n_ports][n_freq]; may be null when n_src or
 * n_ports is 0 (nothing is written).  YO_ESTATE without a finished run of
 * the forward right-hand sides (YO_FORWARD or YO_BOTH), or when yo_set_design
 * or yo_set_background was called after that run's reset (its phasors belong
 * to another permittivity). */
yo_status yo_alpha(const yo_plan *plan, float *dev_alpha, yo_stream stream);

/* Gradient (Eq. (1) and the chain's VJP): dev_coef = dF/dalpha (holomorphic
 * Wirtinger derivative, e.g. conj(alpha) for F = |alpha|^2), complex64
 * [n_src][n_ports][n_freq]; dev_dFdC FP32 [nc][mc] receives
 * sum 2 Re(coef dalpha/dC).  Needs yo_set_design and finished forward and
 * adjoint runs: one YO_BOTH run, or a YO_FORWARD run and a YO_ADJOINT run in
 * either order (each side keeps its phasors until its own next reset);
 * YO_ESTATE if yo_set_design or yo_set_background was called after either
 * run's reset (Eq. (1) would pair one design's phasors with another's
 * permittivity and chain state).  With n_src or n_ports 0 there are no
 * coefficients: dev_coef may be null and the gradient is zero. */
yo_status yo_gradient(yo_plan *plan, const float *dev_coef, float *dev_dFdC, yo_stream stream);

/* Same, stopping after Eq. (1): dF/dkappa on the DFT box, FP32 [3][bz][by][bx]
 * (box = design area plus its one-pixel ring x E planes k_lo-1..k_hi). */
yo_status yo_gradient_kappa(yo_plan *plan, const float *dev_coef, float *dev_g, yo_stream stream);

/* The parametrization's VJP alone: dev_gkappa = dF/dkappa on the DFT box,
 * FP32 [3][bz][by][bx] (layout of yo_gradient_kappa) -> dev_dFdC FP32
 * [nc][mc] through the extrusion, Eq. (7), the normals, the averages, the
 * projection and the filter, for the design last set by yo_set_design. */
yo_status yo_chain_vjp(yo_plan *plan, const float *dev_gkappa, float *dev_dFdC, yo_stream stream);

/* Right-hand side numbering: forward (src s, freq f) -> f*n_src + s;
 * adjoint (port p, freq f) -> n_src*n_freq + f*n_ports + p. */
yo_status yo_rhs_count(const yo_plan *plan, int *n_rhs);

/* Steady-state phasors of right-hand side `rhs`: region 0 = DFT box,
 * complex64 [3][bz][by][bx]; region 1+p = plane of port p, complex64
 * [2][n1][n0].  Valid after yo_finalize. */
yo_status yo_get_dft(const yo_plan *plan, int rhs, int region, float *dev_out, yo_stream stream);

/* Test hooks: current fields of `rhs` as FP32 [3][nz][ny][nx] (E^n and
 * Ht^{n-1/2} after n steps); rhs counts the stepped right-hand sides (under
 * a pulse: the sources, then the ports). */
yo_status yo_set_fields(yo_plan *plan, int rhs, const float *dev_E, const float *dev_H,
                        yo_stream stream);
yo_status yo_get_fields(const yo_plan *plan, int rhs, float *dev_E, float *dev_H,
                        yo_stream stream);
/* Current kappa (background plus design), FP32 [3][nz][ny][nx]. */
yo_status yo_get_kappa(const yo_plan *plan, float *dev_kappa, yo_stream stream);

/* Bytes of the time-stepping kernel's traffic model per cell-update for
 * this plan (48 + 12/R + PML and DFT terms), host only. */
yo_status yo_model_bytes(const yo_plan *plan, int which, double *bytes_per_step,
                         double *cell_updates_per_step);

/* Measurement: time `n_launch` launches of one part of the time-stepping
 * kernel (cls 0: interior tiles, 1: CPML shell, 2: the two-step region's
 * launch, which advances its cells two steps (its bytes and cell-updates
 * count both; YO_ESTATE unless two steps remain in the run), 3: the interior
 * around it, 4: the two-step launch of the z-slabs under it (tiling flag
 * 2048; two steps like 2), 5: the CPML shell of the steps that go in pairs
 * (without the tiles of 4); other values YO_EINVAL; an empty part reports
 * zeros and launches nothing) over the
 * right-hand sides selected by the last yo_reset, at the current step, with
 * HIP events on `stream`; blocks until done.  The launches re-run the same
 * step (they read the current buffers and do not advance the counter), so
 * call it only outside the DFT window or after the results were read.
 * avg_ms: mean duration of one launch; bytes: algorithmic HBM bytes one
 * launch must move (48 per owned cell and right-hand side, plus 12 per
 * owned cell for kappa, plus 32 per CPML axis and right-hand side for cells
 * inside an absorbing slab); cells: owned cell-updates per launch. */
yo_status yo_time_kernel(yo_plan *plan, int cls, int n_launch, float *avg_ms, double *bytes,
                         double *cells, yo_stream stream);

/* The tiles of one launch part (as yo_time_kernel numbers them, 0 to 5)
 * under the plan's current tiling: *n = their number, and the first
 * min(n, cap) written to host memory `out` as 7 ints each: x0, x1, y0, y1,
 * z0, z1 (the cells [x0, x1) x [y0, y1) x [z0, z1) the tile owns) and its
 * CPML class (bit a: the tile meets the absorbing slab of axis a).  Host
 * only; needs no workspace.  For checking a split: in single steps parts 0
 * and 1 own every cell once, in steps that go in pairs parts 2 to 5. */
yo_status yo_tile_table(const yo_plan *plan, int part, int *out, int cap, int *n);

/* Unbinarity (Sec. 4): the fraction of the design area's high-resolution
 * sub-pixels whose final density rho lies strictly between lo and hi
 * (0 <= lo < hi <= 1), for the design last set; FP32 written to dev_u[0]
 * on `stream`.  YO_ESTATE before yo_set_design. */
yo_status yo_unbinarity(yo_plan *plan, double lo, double hi, float *dev_u, yo_stream stream);

/* One Adam step (Sec. 4, Eqs. (10)-(11)) on n controls, all FP32 device
 * arrays: M <- b1 M + (1-b1) G, V <- b2 V + (1-b2) G^2,
 * C <- C - lr (M / (1 - b1^step)) / (sqrt(V / (1 - b2^step)) + eps).
 * step counts from 1; M and V start at zero.  Needs no plan.  YO_EINVAL for
 * step < 1, b1 or b2 outside [0, 1), eps <= 0 or a null array. */
yo_status yo_adam_step(float *dev_C, const float *dev_G, float *dev_M, float *dev_V, int n, int step,
                       double lr, double b1, double b2, double eps, yo_stream stream);

/* Launch timing inside a solve: with n_last > 0, every later yo_advance,
 * yo_run or yo_advance_many (with this plan first in its list) runs its
 * last n_last steps with plain launches and records a pair of HIP events on
 * its stream around each launch of `part` (0 interior tiles, 1 CPML shell,
 * 2 every part, including the launches of the steps that go in pairs under
 * tiling flag 512: parts 2 to 5 of yo_time_kernel); the pairs accumulate over calls until
 * the next yo_set_timing with n_last > 0, which clears them.  n_last = 0
 * turns it off and keeps what was recorded.  n_last <= 4096; the events
 * are created as needed (outside graph capture: the timed steps are never
 * captured) and owned by the plan.  Host only.  YO_EINVAL on a bad part or
 * count. */
yo_status yo_set_timing(yo_plan *plan, int part, int n_last);

/* Mean duration of the launches of `part` (0 interior, 1 CPML shell, 2 the
 * two-step region, 3 the interior around it, 4 the z-slabs under it, 5 the
 * CPML shell of steps that go in pairs; see yo_time_kernel) timed since the last
 * yo_set_timing (waits for the last of them); count = how many (0: none,
 * avg_ms = 0). */
yo_status yo_get_timing(yo_plan *plan, int part, float *avg_ms, int *count);

const char *yo_last_error(void);
const char *yo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* YEEOPT_H */
