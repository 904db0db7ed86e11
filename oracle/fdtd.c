/*
 * FP64 reference FDTD: TEST INFRASTRUCTURE ONLY.
 *
 * This file is part of the oracle that checks the GPU path.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper Sec. 2: time-harmonic excitation, amplitude and
 * phase read from the steady state; Appendix A: electric-current mode
 * sources):
 *   - the standard Yee scheme with normalised magnetic field Ht = eta0*H and
 *     kappa = 1/eps_r per electric component (diagonal anisotropic medium):
 *       Ht^{n+1/2} = Ht^{n-1/2} - curl_e E^n
 *       E^{n+1}    = E^n + kappa * curl_h Ht^{n+1/2} - kappa * j^{n+1/2}
 *     where curl_e uses forward differences, curl_h backward differences and
 *     every difference along axis a is multiplied by S_a = c dt / d_a;
 *   - a PEC box: indices outside [0,n) read zero and the tangential E on the
 *     planes i=0, j=0, k=0 is held at zero;
 *   - a convolutional PML (recursive-convolution form) on any face with a
 *     polynomial grading: psi <- b psi + c D f, the curl uses D f / kp + psi;
 *   - one soft electric-current source plane,
 *       j^{n+1/2}(r) = ramp(t) Re( jhat(r) exp(-i w t) ),  t = (n+1/2) dt;
 *   - running DFT sums of E^n exp(+i w n dt) over the window, split into two
 *     halves so the caller can measure how steady the field is;
 *   - or (pulse excitation, the Fourier-transform-of-transients route of
 *     Sec. 2): the source current of a Gaussian pulse on the carrier w,
 *       j^{n+1/2}(r) = g(t) Re( jhat(r) exp(-i w t) ),
 *       g(t) = exp(-(t - t0)^2 / (2 sigma^2)),  t = (n+1/2) dt,
 *     and DFT sums of E^n exp(+i w_f n dt) over every step for each of
 *     n_dft frequencies w_f, split at win_start (steps from win_start on go
 *     to the second set, so the caller can see how much the late field
 *     still contributes);
 *   - optionally (the two-term modal coefficient of Appendix A): running DFT
 *     sums of the tangential Ht^{n+1/2} exp(+i w (n+1/2) dt) over the window
 *     on planes of H sites (half a cell past the plane's E sites along its
 *     normal), and one magnetic current plane,
 *       Ht^{n+1/2} -= ramp(n dt) Re( mhat(r) exp(-i w n dt) )
 *     on those tangential H sites, applied right after the H update;
 *   - optionally the discrete energy
 *       W^n = sum eps |E^n|^2 + sum Ht^{n-1/2} . Ht^{n+1/2},
 *     which the scheme conserves exactly in a closed lossless box.
 *
 * Loops are plain scalar loops, one component at a time, with OpenMP over
 * z-planes only.  Built without fast-math.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, nz;
    double sx, sy, sz;      /* c*dt/dx, c*dt/dy, c*dt/dz                       */
    int npml[6];            /* PML cells on faces -x,+x,-y,+y,-z,+z (0 = none)  */
    double pml_m;           /* grading exponent                                */
    double pml_sigma_scale; /* multiplies the classic optimum 0.8 (m+1) S_a     */
    double pml_kappa_max;   /* stretch at the outer wall (1 = none)            */
    double pml_a_max;       /* CFS shift at the inner edge (0 = none)          */
    int n_steps;
    double omega_dt;        /* angular frequency times dt                      */
    double ramp_steps;      /* raised-cosine ramp length in steps (0 = none)   */
    int win_start, win_len; /* E^n summed for n in [win_start, win_start+len)  */
    double pulse_sigma;     /* > 0: pulse excitation (steps); ramp and window unused */
    double pulse_t0;        /* pulse centre (steps)                            */
    int n_dft;              /* pulse excitation: number of DFT frequencies     */
    const double *dft_omega_dt;  /* [n_dft] angular frequencies times dt       */
} orc_sim;

/* plane normal to `axis` at cell index `index`; (c0, c1) are the two other
 * axes in increasing order, extents [lo0, lo0+n0) x [lo1, lo1+n1).  The two
 * tangential components are ordered cyclically: (t1, t2, axis) right-handed,
 * i.e. axis x -> (y, z), axis y -> (z, x), axis z -> (x, y). */
typedef struct { int axis, index, lo0, lo1, n0, n1; } orc_plane;
typedef struct { int x0, y0, z0, bx, by, bz; } orc_box;

/* H monitors and the magnetic current plane (NULL: none) */
typedef struct {
    int n_hmon;
    const orc_plane *hmon;   /* [n_hmon] */
    double *hmon_acc;        /* complex, [2 halves][sum of 2 n0 n1] like mon_acc */
    const orc_plane *msrc;   /* NULL: no magnetic source */
    const double *msrc_m;    /* complex [2][n1][n0]: mhat_t1, mhat_t2 */
} orc_ext;

#define IDX(i, j, k) (((size_t)(k) * ny + (size_t)(j)) * nx + (size_t)(i))

typedef struct { double *b, *c, *ki; } profile; /* per position along one axis */

/* depth into the PML at coordinate u (in cells) for an axis with n cells */
static double depth(double u, int n, int lo, int hi)
{
    double d = 0.0;
    if (lo > 0 && u < lo) d = (lo - u) / lo;
    if (hi > 0 && u > n - hi) d = (u - (n - hi)) / hi;
    return d;
}

static void make_profile(profile *p, int n, int lo, int hi, double shift,
                         double s_axis, const orc_sim *sim)
{
    p->b = malloc(sizeof(double) * n);
    p->c = malloc(sizeof(double) * n);
    p->ki = malloc(sizeof(double) * n);
    const double m = sim->pml_m;
    const double smax = sim->pml_sigma_scale * 0.8 * (m + 1.0) * s_axis;
    for (int u = 0; u < n; u++) {
        double xi = depth(u + shift, n, lo, hi);
        if (xi <= 0.0) { p->b[u] = 1.0; p->c[u] = 0.0; p->ki[u] = 1.0; continue; }
        double g = pow(xi, m);
        double sig = smax * g;
        double kp = 1.0 + (sim->pml_kappa_max - 1.0) * g;
        double a = sim->pml_a_max * (1.0 - xi);
        double b = exp(-(sig / kp + a));
        double c = (sig > 0.0) ? sig * (b - 1.0) / (kp * (sig + kp * a)) : 0.0;
        p->b[u] = b; p->c[u] = c; p->ki[u] = 1.0 / kp;
    }
}

static void free_profile(profile *p) { free(p->b); free(p->c); free(p->ki); }

/* one PML-modified difference: returns d/kp + psi after updating psi */
static inline double pml(double d, double *psi, const profile *p, int u)
{
    if (p->c[u] == 0.0 && p->ki[u] == 1.0) return d;
    *psi = p->b[u] * (*psi) + p->c[u] * d;
    return d * p->ki[u] + *psi;
}

static void plane_tangentials(int axis, int *t1, int *t2)
{
    *t1 = (axis + 1) % 3;
    *t2 = (axis + 2) % 3;
}

/* coordinates (i,j,k) of plane cell (a,b) along (c0,c1) */
static void plane_cell(const orc_plane *pl, int a, int b, int *i, int *j, int *k)
{
    int c[3];
    int c0 = pl->axis == 0 ? 1 : 0;
    int c1 = pl->axis == 2 ? 1 : 2;
    c[pl->axis] = pl->index;
    c[c0] = pl->lo0 + a;
    c[c1] = pl->lo1 + b;
    *i = c[0]; *j = c[1]; *k = c[2];
}

/* thread count of the OpenMP loops (n < 1: leave it); for timing the oracle
 * at a chosen core count */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_run(const orc_sim *sim, const double *kappa, double *E, double *H,
            const orc_plane *src, const double *src_j,
            const orc_box *box, double *box_acc,
            int n_mon, const orc_plane *mon, double *mon_acc,
            double *energy, const orc_ext *ext)
{
    const int nx = sim->nx, ny = sim->ny, nz = sim->nz;
    const size_t N = (size_t)nx * ny * nz;
    double *Ex = E, *Ey = E + N, *Ez = E + 2 * N;
    double *Hx = H, *Hy = H + N, *Hz = H + 2 * N;
    const double *kx = kappa, *ky = kappa + N, *kz = kappa + 2 * N;
    const double sx = sim->sx, sy = sim->sy, sz = sim->sz;

    /* psi for every (component, derivative axis); zero where unused */
    double *psi = calloc(12 * N, sizeof(double));
    if (!psi) return -1;
    double *pHxy = psi + 0 * N, *pHxz = psi + 1 * N, *pHyz = psi + 2 * N;
    double *pHyx = psi + 3 * N, *pHzx = psi + 4 * N, *pHzy = psi + 5 * N;
    double *pExy = psi + 6 * N, *pExz = psi + 7 * N, *pEyz = psi + 8 * N;
    double *pEyx = psi + 9 * N, *pEzx = psi + 10 * N, *pEzy = psi + 11 * N;

    /* E-derivative outputs sit at integer coordinates, H-derivative outputs
     * at half-integer ones */
    profile eX, eY, eZ, hX, hY, hZ;
    make_profile(&eX, nx, sim->npml[0], sim->npml[1], 0.0, sx, sim);
    make_profile(&eY, ny, sim->npml[2], sim->npml[3], 0.0, sy, sim);
    make_profile(&eZ, nz, sim->npml[4], sim->npml[5], 0.0, sz, sim);
    make_profile(&hX, nx, sim->npml[0], sim->npml[1], 0.5, sx, sim);
    make_profile(&hY, ny, sim->npml[2], sim->npml[3], 0.5, sy, sim);
    make_profile(&hZ, nz, sim->npml[4], sim->npml[5], 0.5, sz, sim);

    const int half = sim->win_len / 2;
    size_t mon_total = 0;
    for (int p = 0; p < n_mon; p++) mon_total += 2 * (size_t)mon[p].n0 * mon[p].n1;
    const size_t box_total = box ? 3 * (size_t)box->bx * box->by * box->bz : 0;

    const int pulse = sim->pulse_sigma > 0.0;
    /* optional progress lines on stderr for long runs (no effect on results) */
    const char *pe = getenv("ORC_PROGRESS_STEPS");
    const int progress = pe ? atoi(pe) : 0;
    for (int n = 0; n < sim->n_steps; n++) {
        if (progress > 0 && n > 0 && n % progress == 0) {
            fprintf(stderr, "oracle: step %d of %d\n", n, sim->n_steps);
            fflush(stderr);
        }
        /* ---- pulse excitation: DFT of E^n at every frequency, every step ---- */
        for (int f = 0; pulse && f < sim->n_dft; f++) {
            int h = (n < sim->win_start) ? 0 : 1;
            double cr = cos(sim->dft_omega_dt[f] * n), ci = sin(sim->dft_omega_dt[f] * n);
            const double *comp[3] = {Ex, Ey, Ez};
            if (box) {
                double *acc = box_acc + 2 * ((size_t)h * sim->n_dft + f) * box_total;
                for (int c = 0; c < 3; c++)
                    for (int k = 0; k < box->bz; k++)
                        for (int j = 0; j < box->by; j++)
                            for (int i = 0; i < box->bx; i++) {
                                size_t o = (((size_t)c * box->bz + k) * box->by + j) * box->bx + i;
                                double e = comp[c][IDX(box->x0 + i, box->y0 + j, box->z0 + k)];
                                acc[2 * o] += e * cr;
                                acc[2 * o + 1] += e * ci;
                            }
            }
            double *acc = mon_acc + 2 * ((size_t)h * sim->n_dft + f) * mon_total;
            size_t off = 0;
            for (int p = 0; p < n_mon; p++) {
                int t1, t2;
                plane_tangentials(mon[p].axis, &t1, &t2);
                for (int t = 0; t < 2; t++)
                    for (int b = 0; b < mon[p].n1; b++)
                        for (int a = 0; a < mon[p].n0; a++) {
                            int i, j, k;
                            plane_cell(&mon[p], a, b, &i, &j, &k);
                            double e = comp[t == 0 ? t1 : t2][IDX(i, j, k)];
                            size_t o = off + ((size_t)t * mon[p].n1 + b) * mon[p].n0 + a;
                            acc[2 * o] += e * cr;
                            acc[2 * o + 1] += e * ci;
                        }
                off += 2 * (size_t)mon[p].n0 * mon[p].n1;
            }
        }
        /* ---- running DFT of E^n over the window ---- */
        int w = n - sim->win_start;
        if (!pulse && w >= 0 && w < sim->win_len) {
            int h = (w < half) ? 0 : 1;
            double cr = cos(sim->omega_dt * n), ci = sin(sim->omega_dt * n);
            if (box) {
                double *acc = box_acc + 2 * h * box_total;
                const double *comp[3] = {Ex, Ey, Ez};
                for (int c = 0; c < 3; c++)
                    for (int k = 0; k < box->bz; k++)
                        for (int j = 0; j < box->by; j++)
                            for (int i = 0; i < box->bx; i++) {
                                size_t o = (((size_t)c * box->bz + k) * box->by + j) * box->bx + i;
                                double e = comp[c][IDX(box->x0 + i, box->y0 + j, box->z0 + k)];
                                acc[2 * o] += e * cr;
                                acc[2 * o + 1] += e * ci;
                            }
            }
            double *acc = mon_acc + 2 * h * mon_total;
            size_t off = 0;
            for (int p = 0; p < n_mon; p++) {
                int t1, t2;
                plane_tangentials(mon[p].axis, &t1, &t2);
                const double *comp[3] = {Ex, Ey, Ez};
                for (int t = 0; t < 2; t++)
                    for (int b = 0; b < mon[p].n1; b++)
                        for (int a = 0; a < mon[p].n0; a++) {
                            int i, j, k;
                            plane_cell(&mon[p], a, b, &i, &j, &k);
                            double e = comp[t == 0 ? t1 : t2][IDX(i, j, k)];
                            size_t o = off + ((size_t)t * mon[p].n1 + b) * mon[p].n0 + a;
                            acc[2 * o] += e * cr;
                            acc[2 * o + 1] += e * ci;
                        }
                off += 2 * (size_t)mon[p].n0 * mon[p].n1;
            }
        }

        double wsum_e = 0.0, wsum_h = 0.0;
        if (energy) {
            for (size_t q = 0; q < N; q++)
                wsum_e += Ex[q] * Ex[q] / kx[q] + Ey[q] * Ey[q] / ky[q] + Ez[q] * Ez[q] / kz[q];
        }

        /* ---- H update: Ht -= curl_e E (forward differences) ---- */
#pragma omp parallel for reduction(+ : wsum_h) schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t q = IDX(i, j, k);
                    double ez_j1 = (j + 1 < ny) ? Ez[IDX(i, j + 1, k)] : 0.0;
                    double ey_k1 = (k + 1 < nz) ? Ey[IDX(i, j, k + 1)] : 0.0;
                    double ex_k1 = (k + 1 < nz) ? Ex[IDX(i, j, k + 1)] : 0.0;
                    double ez_i1 = (i + 1 < nx) ? Ez[IDX(i + 1, j, k)] : 0.0;
                    double ey_i1 = (i + 1 < nx) ? Ey[IDX(i + 1, j, k)] : 0.0;
                    double ex_j1 = (j + 1 < ny) ? Ex[IDX(i, j + 1, k)] : 0.0;

                    double dyEz = pml(ez_j1 - Ez[q], &pHxy[q], &hY, j);
                    double dzEy = pml(ey_k1 - Ey[q], &pHxz[q], &hZ, k);
                    double dzEx = pml(ex_k1 - Ex[q], &pHyz[q], &hZ, k);
                    double dxEz = pml(ez_i1 - Ez[q], &pHyx[q], &hX, i);
                    double dxEy = pml(ey_i1 - Ey[q], &pHzx[q], &hX, i);
                    double dyEx = pml(ex_j1 - Ex[q], &pHzy[q], &hY, j);

                    double hx = Hx[q] - (sy * dyEz - sz * dzEy);
                    double hy = Hy[q] - (sz * dzEx - sx * dxEz);
                    double hz = Hz[q] - (sx * dxEy - sy * dyEx);
                    wsum_h += Hx[q] * hx + Hy[q] * hy + Hz[q] * hz;
                    Hx[q] = hx; Hy[q] = hy; Hz[q] = hz;
                }
        if (energy) energy[n] = wsum_e + wsum_h;

        /* ---- magnetic current on the tangential H sites of its plane ---- */
        if (ext && ext->msrc) {
            const orc_plane *mp = ext->msrc;
            double t = n;
            double r = 1.0;
            if (sim->ramp_steps > 0.0 && t < sim->ramp_steps)
                r = 0.5 * (1.0 - cos(M_PI * t / sim->ramp_steps));
            double ca = r * cos(sim->omega_dt * t), sa = r * sin(sim->omega_dt * t);
            int t1, t2;
            plane_tangentials(mp->axis, &t1, &t2);
            double *hcomp[3] = {Hx, Hy, Hz};
            for (int tt = 0; tt < 2; tt++)
                for (int b = 0; b < mp->n1; b++)
                    for (int a = 0; a < mp->n0; a++) {
                        int i, j, k;
                        plane_cell(mp, a, b, &i, &j, &k);
                        size_t o = ((size_t)tt * mp->n1 + b) * mp->n0 + a;
                        double mv = ext->msrc_m[2 * o] * ca + ext->msrc_m[2 * o + 1] * sa;
                        hcomp[tt == 0 ? t1 : t2][IDX(i, j, k)] -= mv;
                    }
        }

        /* ---- DFT of the tangential Ht^{n+1/2} on the H monitor planes ---- */
        if (ext && ext->n_hmon > 0 && w >= 0 && w < sim->win_len && !pulse) {
            int h = (w < half) ? 0 : 1;
            double cr = cos(sim->omega_dt * (n + 0.5)), ci = sin(sim->omega_dt * (n + 0.5));
            size_t htot = 0;
            for (int p = 0; p < ext->n_hmon; p++) htot += 2 * (size_t)ext->hmon[p].n0 * ext->hmon[p].n1;
            double *acc = ext->hmon_acc + 2 * h * htot;
            const double *hcomp[3] = {Hx, Hy, Hz};
            size_t off = 0;
            for (int p = 0; p < ext->n_hmon; p++) {
                const orc_plane *hp = &ext->hmon[p];
                int t1, t2;
                plane_tangentials(hp->axis, &t1, &t2);
                for (int tt = 0; tt < 2; tt++)
                    for (int b = 0; b < hp->n1; b++)
                        for (int a = 0; a < hp->n0; a++) {
                            int i, j, k;
                            plane_cell(hp, a, b, &i, &j, &k);
                            double hv = hcomp[tt == 0 ? t1 : t2][IDX(i, j, k)];
                            size_t o = off + ((size_t)tt * hp->n1 + b) * hp->n0 + a;
                            acc[2 * o] += hv * cr;
                            acc[2 * o + 1] += hv * ci;
                        }
                off += 2 * (size_t)hp->n0 * hp->n1;
            }
        }

        /* ---- E update: E += kappa curl_h Ht (backward differences) ---- */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t q = IDX(i, j, k);
                    double hz_jm = (j > 0) ? Hz[IDX(i, j - 1, k)] : 0.0;
                    double hy_km = (k > 0) ? Hy[IDX(i, j, k - 1)] : 0.0;
                    double hx_km = (k > 0) ? Hx[IDX(i, j, k - 1)] : 0.0;
                    double hz_im = (i > 0) ? Hz[IDX(i - 1, j, k)] : 0.0;
                    double hy_im = (i > 0) ? Hy[IDX(i - 1, j, k)] : 0.0;
                    double hx_jm = (j > 0) ? Hx[IDX(i, j - 1, k)] : 0.0;

                    double dyHz = pml(Hz[q] - hz_jm, &pExy[q], &eY, j);
                    double dzHy = pml(Hy[q] - hy_km, &pExz[q], &eZ, k);
                    double dzHx = pml(Hx[q] - hx_km, &pEyz[q], &eZ, k);
                    double dxHz = pml(Hz[q] - hz_im, &pEyx[q], &eX, i);
                    double dxHy = pml(Hy[q] - hy_im, &pEzx[q], &eX, i);
                    double dyHx = pml(Hx[q] - hx_jm, &pEzy[q], &eY, j);

                    double ex = Ex[q] + kx[q] * (sy * dyHz - sz * dzHy);
                    double ey = Ey[q] + ky[q] * (sz * dzHx - sx * dxHz);
                    double ez = Ez[q] + kz[q] * (sx * dxHy - sy * dyHx);
                    /* PEC: tangential E on the planes i=0, j=0, k=0 */
                    if (j == 0 || k == 0) ex = 0.0;
                    if (i == 0 || k == 0) ey = 0.0;
                    if (i == 0 || j == 0) ez = 0.0;
                    Ex[q] = ex; Ey[q] = ey; Ez[q] = ez;
                }

        /* ---- soft current source at t = (n + 1/2) dt ---- */
        if (src) {
            double t = n + 0.5;
            double r = 1.0;
            if (pulse) {
                double d = (t - sim->pulse_t0) / sim->pulse_sigma;
                r = exp(-0.5 * d * d);
            } else if (sim->ramp_steps > 0.0 && t < sim->ramp_steps)
                r = 0.5 * (1.0 - cos(M_PI * t / sim->ramp_steps));
            double ca = r * cos(sim->omega_dt * t), sa = r * sin(sim->omega_dt * t);
            int t1, t2;
            plane_tangentials(src->axis, &t1, &t2);
            double *comp[3] = {Ex, Ey, Ez};
            const double *kap[3] = {kx, ky, kz};
            for (int t = 0; t < 2; t++) {
                int c = t == 0 ? t1 : t2;
                for (int b = 0; b < src->n1; b++)
                    for (int a = 0; a < src->n0; a++) {
                        int i, j, k;
                        plane_cell(src, a, b, &i, &j, &k);
                        size_t o = ((size_t)t * src->n1 + b) * src->n0 + a;
                        double jv = src_j[2 * o] * ca + src_j[2 * o + 1] * sa;
                        size_t q = IDX(i, j, k);
                        comp[c][q] -= kap[c][q] * jv;
                    }
            }
        }
    }

    free_profile(&eX); free_profile(&eY); free_profile(&eZ);
    free_profile(&hX); free_profile(&hY); free_profile(&hZ);
    free(psi);
    return 0;
}
