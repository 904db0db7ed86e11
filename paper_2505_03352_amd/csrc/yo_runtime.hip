// Host runtime of libyeeopt: plan validation, workspace layout, FP64
// coefficient tables (CPML profiles, per-step source and DFT phases, the
// steady-state fit, filter taps), mode-to-source/monitor conversion
// (Appendix A), tile tables, HIP-graph capture of step chunks, and the C ABI.
// The library never allocates device memory: every device buffer lives in a
// caller-owned workspace.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "yeeopt.h"
#include "yo_internal.h"

namespace {

constexpr double kC0 = 299792458.0;
thread_local std::string g_err;

yo_status fail(yo_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(YO_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Region {
    size_t off = 0, bytes = 0;
};

struct Layout {
    Region fields, kappa, psi, dft_box, dft_mon, src_j, port_w, steptab, prof, desc_plan,
        desc_rhs, ctr, tiles, chain_f, chain_i, morph;
    size_t total = 0;
    size_t add(Region &r, size_t bytes)
    {
        r.off = total;
        r.bytes = bytes;
        total += align256(bytes);
        return r.off;
    }
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

std::mutex g_graph_mu;
std::map<std::string, GraphEntry> g_graphs;
int g_next_plan_id = 1;

// Static workspace for callers that cannot allocate (yo_bind_static_workspace).
// Each device the library runs on holds its own copy until the process
// ends.  Host code never uses the array's name as an address: its device
// address is looked up per device with hipGetSymbolAddress.
#define YO_STATIC_WS_BYTES ((size_t)32 << 20)
#define YO_MAX_DEVICES 64
static __device__ __align__(256) char scratch[YO_STATIC_WS_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[YO_MAX_DEVICES];
unsigned g_scratch_epoch[YO_MAX_DEVICES];

}  // namespace

// Tiling flags (yo_set_tiling)
enum {
    YO_TILE_XSTRIPS = 1,      // CPML x-shell as full 62-cell strips
    YO_TILE_WPB8 = 2,         // 8 waves per block (else 4)
    YO_TILE_COOP_SHELL = 4,   // CPML shell: cooperative blocks
    YO_TILE_CLASS_CODE = 8,   // CPML shell: each tile runs its own class's code
    YO_TILE_COOP_INT = 16,    // interior: cooperative blocks
    YO_TILE_NOPF_INT = 32,    // interior: no prefetch of the next plane
    YO_TILE_NOPF_SHELL = 64,  // CPML shell: no prefetch of the next plane
    YO_TILE_XFULL = 128,      // x-shell strips as narrow as whole 62-cell interior strips allow
    YO_TILE_XINT = 256,       // tiles inside the x-slabs only run in the interior launch (x CPML code)
    YO_TILE_PAIRS = 512,      // the two-step region advances two steps per sweep (yo_set_time_blocking)
    YO_TILE_OVERLAP = 1024,   // with 512: the two-step launch runs beside the first step's frame and shell
    YO_TILE_ZPAIRS = 2048,    // with 512: the z-slabs under the two-step region take two steps per launch too
    YO_TILE_PAIR6 = 4096,     // with 512: the two-step region's tiles have YO_TY2 rows (else YO_TY)
    YO_TILE_COOP_PAIRS = 8192,  // with 512: the two-step region in cooperative blocks
    YO_TILE_SHELL6 = 16384,   // the CPML shell's tiles have YO_TY2 rows (not with 4)
    YO_TILE_ALL = 32767
};

struct yo_plan {
    int id = 0;
    int generation = 0;
    yo_grid grid{};
    yo_design des{};
    int n_steps = 0, n_freq = 0, n_src = 0, n_ports = 0, n_rhs = 0, n_fwd = 0;
    // stepped right-hand sides: all of them, or under a pulse one per source
    // and one per port (each then accumulates every frequency's DFT)
    int n_phys = 0, n_pfwd = 0;
    bool pulse = false;
    double pulse_w = 0, pulse_sigma = 0, pulse_t0 = 0;
    int dft_stride = 1;          // under a pulse: the DFT samples every dft_stride-th step
    std::vector<float> fin;      // [n_freq][4] phasor matrices applied at finalize
    int mon_nc = 2;              // component planes per port (5: two-term coefficient)
    std::vector<yo_freq> freqs;
    std::vector<yo_plane> src_planes, port_planes;
    double dt = 0, sx = 0, sy = 0, sz = 0;
    int nxp = 0;
    int plo[3] = {0, 0, 0}, phi[3] = {0, 0, 0};
    size_t cells_p = 0;          // padded cells per component
    size_t psi_per_rhs = 0;      // floats
    size_t psi_axis_off[3] = {0, 0, 0}, psi_axis_n[3] = {0, 0, 0};   // per RHS, per axis slab size (floats per comp)
    size_t bsz = 0;              // box cells
    int box[6] = {0, 0, 0, 0, 0, 0};
    size_t mon_total = 0;        // complex entries per RHS
    std::vector<size_t> mon_off, src_off, port_off;
    size_t src_total = 0, port_total = 0;
    // chain sizes
    int S = 0, U = 0, V = 0, G0 = 0, G1 = 0, tmax = 0;
    size_t tiles_cap = 0;
    Layout L;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // host mirrors
    YoPlanD hplan{};
    std::vector<YoRhsD> hrhs;
    YoChainBufs chain{};
    std::vector<int> tap_lo_x, tap_n_x, tap_lo_y, tap_n_y, urange_x, urange_y;
    std::vector<float> tap_w_x, tap_w_y;
    std::string morph_ops;       // 'd'/'e' per stage, empty: no morphological filters
    double morph_d = 0, morph_alpha = 0;
    std::vector<int> mtaps;      // [n][2] dy, dx
    std::vector<float4> steptab;
    std::vector<float> prof;
    std::vector<float2> src_j_host, port_w_host;
    std::vector<int4> tiles_host;
    std::vector<float> ginv;     // [n_freq][4]
    std::vector<double> omega_dt;
    std::vector<char> src_set, port_set;
    int kc = 16, tflags = 0;     // z-planes per tile; tiling flags (YO_TILE_* below)
    int n_int = 0, n_tiles = 0;  // tile table: interior tiles [0, n_int), CPML shell [n_int, n_tiles)
    // temporal blocking (yo_set_time_blocking): steps per sweep the interior
    // may take, state buffers per right-hand side, the two-step region and
    // its tiles (after the shell: [n_tiles, n_tiles + n2)) and the single-step
    // tiles of the interior around it ([n_tiles + n2, n_tiles + n2 + nfr))
    int tsteps = 1, nbuf = 2;
    int r2[6] = {0, 0, 0, 0, 0, 0};
    int n2 = 0, nfr = 0;
    // YO_TILE_ZPAIRS: the z-slab tiles under R2 ([n_tiles + n2 + nfr, + nz2)),
    // and the shell's tiles they replace in steps that go in pairs (its last
    // n_c4 tiles, those of class 4)
    int nz2 = 0, n_c4 = 0;
    bool bg_set = false, design_set = false;
    double beta = 0;
    int steps_done = 0;
    int active = 0;              // which right-hand sides the last reset selected
    // per side (0 forward, 1 adjoint): phasors fitted by a finalize since
    // the side's last reset, and non-finite ones among them (watchdog)
    bool finalized[2] = {false, false};
    bool unstable[2] = {false, false};
    // material stamp: bumped by every change of kappa (background, design);
    // a reset records it, and results of a run whose kappa has changed since
    // (alpha, the Eq. (1) gradient) are refused
    int mat_gen = 0, run_mat_gen[2] = {-1, -1};
    // bound to the device's static workspace (yo_bind_static_workspace): the
    // device and the binding's epoch there; a later static binding on the
    // same device takes the memory over and this plan is refused
    int static_dev = -1;
    unsigned static_epoch = 0;
    hipStream_t cap_stream = nullptr;
    // YO_TILE_OVERLAP: the stream the two-step launch runs on, and the
    // events that fork it from the caller's stream and join it back
    hipStream_t side_stream = nullptr;
    hipEvent_t ov_fork = nullptr, ov_join = nullptr;
    // launch timing: the last tm_n steps of each advance run eagerly, with
    // HIP events around the launches of part tm_part (0 or 1, or 2 for
    // every part); tm_ev[q] holds the event pairs of part q (see part_range)
    // recorded since yo_set_timing (tm_done[q] of them), created as needed
    int tm_part = 0, tm_n = 0;
    int tm_done[6] = {0, 0, 0, 0, 0, 0};
    std::vector<hipEvent_t> tm_ev[6];
};

namespace {

// ------------------------------------------------------------------ helpers
// a workspace is bound and, for the static workspace, still this plan's
yo_status ws_check(const yo_plan *p)
{
    if (!p->ws) return fail(YO_EWORKSPACE, "no workspace bound");
    if (p->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_epoch[p->static_dev] != p->static_epoch)
            return fail(YO_EWORKSPACE, "another plan was bound to the static workspace of device %d "
                                       "since this one; bind again", p->static_dev);
    }
    return YO_OK;
}

template <class T>
T *wsp(yo_plan *p, const Region &r, size_t extra_bytes = 0)
{
    return reinterpret_cast<T *>(p->ws + r.off + extra_bytes);
}

bool plane_ok(const yo_plan *p, const yo_plane &pl)
{
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    if (pl.axis < 0 || pl.axis > 2 || pl.n0 <= 0 || pl.n1 <= 0) return false;
    const int c0 = pl.axis == 0 ? 1 : 0;
    const int c1 = pl.axis == 2 ? 1 : 2;
    auto inside = [&](int a, int lo, int cnt) {
        return lo >= p->plo[a] && lo + cnt <= n[a] - p->phi[a];
    };
    return inside(pl.axis, pl.index, 1) && inside(c0, pl.lo0, pl.n0) && inside(c1, pl.lo1, pl.n1);
}

// depth into the absorbing layer at coordinate u (cells)
double pml_depth(double u, int n, int lo, int hi)
{
    if (lo > 0 && u < lo) return (lo - u) / lo;
    if (hi > 0 && u > n - hi) return (u - (n - hi)) / hi;
    return 0.0;
}

void build_profiles(yo_plan *p)
{
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    const double s[3] = {p->sx, p->sy, p->sz};
    size_t tot = 6 * (size_t)(n[0] + n[1] + n[2]);
    p->prof.assign(tot, 0.0f);
    size_t off = 0;
    const double m = p->grid.pml_m;
    for (int a = 0; a < 3; ++a) {
        for (int which = 0; which < 2; ++which) {
            const double shift = which ? 0.5 : 0.0;
            const double smax = p->grid.pml_sigma_scale * 0.8 * (m + 1.0) * s[a];
            for (int u = 0; u < n[a]; ++u) {
                const double xi = pml_depth(u + shift, n[a], p->plo[a], p->phi[a]);
                double b = 1.0, c = 0.0, ki = 1.0;
                if (xi > 0.0) {
                    const double gr = std::pow(xi, m);
                    const double sig = smax * gr;
                    const double kp = 1.0 + (p->grid.pml_kappa_max - 1.0) * gr;
                    const double aa = p->grid.pml_a_max * (1.0 - xi);
                    b = std::exp(-(sig / kp + aa));
                    c = sig > 0.0 ? sig * (b - 1.0) / (kp * (sig + kp * aa)) : 0.0;
                    ki = 1.0 / kp;
                }
                p->prof[off + (3 * which + 0) * n[a] + u] = (float)b;
                p->prof[off + (3 * which + 1) * n[a] + u] = (float)c;
                p->prof[off + (3 * which + 2) * n[a] + u] = (float)ki;
            }
        }
        off += 6 * (size_t)n[a];
    }
}

size_t fields_per_rhs(const yo_plan *p);

// Port monitors and port weights: mon_nc component planes per port; the
// two-term weights depend on the frequency, so then each frequency has a
// block of port_total entries.
void build_port_tables(yo_plan *p)
{
    p->mon_off.clear();
    p->port_off.clear();
    p->mon_total = 0;
    p->port_total = 0;
    for (auto &pl : p->port_planes) {
        p->mon_off.push_back(p->mon_total);
        p->mon_total += (size_t)p->mon_nc * pl.n0 * pl.n1;
        p->port_off.push_back(p->port_total);
        p->port_total += (size_t)p->mon_nc * pl.n0 * pl.n1;
    }
}

size_t port_w_blocks(const yo_plan *p) { return p->mon_nc == 5 ? (size_t)p->n_freq : 1; }

// Bytes of the morphological region for n stages and t taps (each buffer
// padded to 64 floats, as set_chain_ptrs carves them).
size_t morph_bytes(const yo_plan *p, size_t n, size_t t)
{
    const size_t UV = (size_t)p->U * p->V;
    const size_t DD = (size_t)(p->S * p->des.md) * (p->S * p->des.nd);
    auto pad = [](size_t v) { return (v + 63) & ~(size_t)63; };
    return sizeof(float) * (pad((n + 1) * UV) + pad(n * DD) + pad(DD) + pad(2 * DD) + pad(DD) + pad(2 * t));
}


// CPML slabs (per right-hand side): per axis, 2 components per slot, three
// slots (E one, Ht two) with two state buffers, six (three each) with three;
// false when they would pass 2 GiB (32-bit buffer offsets).
static bool set_psi_layout(yo_plan *p)
{
    const yo_grid &g = p->grid;
    const size_t W[3] = {(size_t)p->plo[0] + p->phi[0], (size_t)p->plo[1] + p->phi[1],
                         (size_t)p->plo[2] + p->phi[2]};
    const size_t slab[3] = {(size_t)g.nz * g.ny * W[0], (size_t)g.nz * W[1] * p->nxp,
                            W[2] * g.ny * p->nxp};
    const size_t arrays = p->nbuf == 3 ? 12 : 6;
    size_t off = 0;
    for (int a = 0; a < 3; ++a) {
        p->psi_axis_off[a] = off;
        p->psi_axis_n[a] = slab[a];
        off += arrays * slab[a];
    }
    p->psi_per_rhs = off;
    return off * sizeof(float) < ((size_t)1 << 31);
}

// Workspace regions (fields, CPML memories and descriptors per stepped
// right-hand side; DFT results per output right-hand side).
void build_layout(yo_plan *p)
{
    const yo_design &d = p->des;
    const yo_grid &g = p->grid;
    Layout &L = p->L;
    L = Layout{};
    L.add(L.fields, sizeof(float) * fields_per_rhs(p) * p->n_phys);
    L.add(L.kappa, sizeof(float) * 3 * p->cells_p);
    L.add(L.psi, sizeof(float) * p->psi_per_rhs * p->n_phys);
    L.add(L.dft_box, sizeof(float2) * 3 * p->bsz * p->n_rhs);
    L.add(L.dft_mon, sizeof(float2) * std::max<size_t>(p->mon_total, 1) * p->n_rhs);
    L.add(L.src_j, sizeof(float2) * std::max<size_t>(p->src_total, 1));
    L.add(L.port_w, sizeof(float2) * std::max<size_t>(p->port_total, 1) * port_w_blocks(p));
    L.add(L.steptab, sizeof(float4) * (size_t)(p->n_freq + 1) * p->n_steps);
    L.add(L.prof, sizeof(float) * 6 * (size_t)(g.nx + g.ny + g.nz));
    L.add(L.desc_plan, sizeof(YoPlanD));
    L.add(L.desc_rhs, sizeof(YoRhsD) * p->n_phys);
    L.add(L.ctr, 256);
    L.add(L.tiles, sizeof(int4) * p->tiles_cap);
    const size_t G = (size_t)p->G0 * p->G1;
    const size_t UV = (size_t)p->U * p->V;
    const size_t DD = (size_t)(p->S * d.md) * (p->S * d.nd);
    const size_t nf = 2 * UV + DD /*tanh*/ + 9 * G + 6 * G + 4 * G + 6 * G + 4 * G + 2 * G + DD /*gphi*/ +
                      (size_t)(p->S * d.nd) * d.mc /*tmp*/ + (size_t)p->tmax * p->S * (d.md + d.nd);
    L.add(L.chain_f, sizeof(float) * (nf + 64 * 16));   // each of 15 buffers padded to 64 floats
    const size_t ni = 2 * (size_t)p->S * (d.md + d.nd) + 2 * (size_t)(d.mc + d.nc);
    L.add(L.chain_i, sizeof(int) * (ni + 64 * 8));     // each of 6 tables padded to 64 ints
    L.add(L.morph, p->morph_ops.empty() ? 0 : morph_bytes(p, p->morph_ops.size(), p->mtaps.size() / 2));
}

void build_steptab(yo_plan *p)
{
    p->steptab.resize((size_t)(p->n_freq + (p->pulse ? 1 : 0)) * p->n_steps);
    p->ginv.assign(4 * (size_t)p->n_freq, 0.0f);
    for (int f = 0; f < p->n_freq; ++f) {
        const double w = p->omega_dt[f];
        const double T = p->freqs[f].ramp_steps;
        for (int n = 0; n < p->n_steps; ++n) {
            const double t = n + 0.5;
            double r = 1.0;
            if (T > 0.0 && t < T) r = 0.5 * (1.0 - std::cos(M_PI * t / T));
            float4 v;
            v.x = (float)(r * std::cos(w * t));
            v.y = (float)(r * std::sin(w * t));
            v.z = (float)std::cos(w * n);
            v.w = (float)std::sin(w * n);
            p->steptab[(size_t)f * p->n_steps + n] = v;
        }
        double g00 = 0, g01 = 0, g11 = 0;
        for (int n = p->freqs[f].win_start; n < p->freqs[f].win_start + p->freqs[f].win_len; ++n) {
            const double c = std::cos(w * n), s = std::sin(w * n);
            g00 += c * c;
            g01 += c * s;
            g11 += s * s;
        }
        const double det = g00 * g11 - g01 * g01;
        p->ginv[4 * f + 0] = (float)(g11 / det);
        p->ginv[4 * f + 1] = (float)(-g01 / det);
        p->ginv[4 * f + 2] = (float)(-g01 / det);
        p->ginv[4 * f + 3] = (float)(g00 / det);
    }
    p->fin = p->ginv;
    if (!p->pulse) return;
    // Pulse excitation: the source signal g(t) e^{-i w0 t}, g a Gaussian, at
    // t = n + 1/2, stored like the ramped carrier (x = g cos, y = g sin, so
    // the current is Re(jhat (x - i y))).  The response to the real source is
    // the real part of the response to jhat s(t), whose DFT at w is
    // S(w) Ehat(w) with S(w) = sum_m s_m e^{+i w (m + 1/2)} (the conjugate part
    // lies at -w), so Ehat(w) = (2 / S(w)) DFT(w): applied at finalize as the
    // real 2 x 2 matrix of that complex factor.  S is summed over the stored
    // (rounded) samples, which are what the run injects.
    float4 *row = p->steptab.data() + (size_t)p->n_freq * p->n_steps;
    for (int n = 0; n < p->n_steps; ++n) {
        const double t = n + 0.5;
        const double d = (t - p->pulse_t0) / p->pulse_sigma;
        const double gt = std::exp(-0.5 * d * d);
        row[n] = make_float4((float)(gt * std::cos(p->pulse_w * t)), (float)(gt * std::sin(p->pulse_w * t)),
                             0.0f, 0.0f);
    }
    for (int f = 0; f < p->n_freq; ++f) {
        std::complex<double> S = 0.0;
        for (int n = 0; n < p->n_steps; ++n) {
            const std::complex<double> sm((double)row[n].x, -(double)row[n].y);
            S += sm * std::polar(1.0, p->omega_dt[f] * (n + 0.5));
        }
        // sampling every m-th step divides the sum by m (its aliases, at
        // w + 2 pi q / m, carry no pulse spectrum: yo_set_dft_stride checks)
        const std::complex<double> c = 2.0 * p->dft_stride / S;
        p->fin[4 * f + 0] = (float)c.real();
        p->fin[4 * f + 1] = (float)(-c.imag());
        p->fin[4 * f + 2] = (float)c.imag();
        p->fin[4 * f + 3] = (float)c.real();
    }
}

// Gaussian-basis taps of one axis: sub-pixel u of the design is centred at
// x = ((u + 1/2)/S) (n_ctl/n_px) - 1/2 control pixels; taps are the controls
// within distance r, weights exp(-d^2/(2 sigma^2)), sigma = r/2, normalised.
void build_taps(int S, int n_px, int n_ctl, double r, int tmax, std::vector<int> &lo,
                std::vector<int> &cnt, std::vector<float> &w, std::vector<int> &range)
{
    const int n = S * n_px;
    lo.assign(n, 0);
    cnt.assign(n, 0);
    w.assign((size_t)n * tmax, 0.0f);
    range.assign(2 * (size_t)n_ctl, 0);
    for (int a = 0; a < n_ctl; ++a) {
        range[2 * a] = n;
        range[2 * a + 1] = -1;
    }
    const double sigma = r / 2.0;
    for (int u = 0; u < n; ++u) {
        const double x = ((u + 0.5) / S) * (double)n_ctl / n_px - 0.5;
        const int l = (int)std::ceil(x - r), h = (int)std::floor(x + r);
        double z = 0.0;
        std::vector<double> g;
        for (int i = l; i <= h; ++i) {
            const double d = x - i;
            g.push_back(std::exp(-d * d / (2.0 * sigma * sigma)));
            z += g.back();
        }
        lo[u] = l;
        cnt[u] = h - l + 1;
        for (int t = 0; t <= h - l; ++t) {
            w[(size_t)u * tmax + t] = (float)(g[t] / z);
            const int a = std::min(std::max(l + t, 0), n_ctl - 1);
            range[2 * a] = std::min(range[2 * a], u);
            range[2 * a + 1] = std::max(range[2 * a + 1], u);
        }
    }
}

// Split [0, n) into pieces of at most `w`, with cuts at the two edges of the
// interior region [lo, hi) so that no piece straddles them.
void split_axis(int n, int lo, int hi, int w, std::vector<std::pair<int, int>> &out,
                std::vector<char> &interior)
{
    out.clear();
    interior.clear();
    const int cuts[4] = {0, lo, hi, n};
    for (int seg = 0; seg < 3; ++seg) {
        const int len = cuts[seg + 1] - cuts[seg];
        if (len <= 0) continue;
        // as few pieces as the width allows, sized as evenly as possible
        const int pieces = (len + w - 1) / w;
        int a = cuts[seg];
        for (int q = 0; q < pieces; ++q) {
            const int sz = len / pieces + (q < len % pieces ? 1 : 0);
            out.emplace_back(a, sz);
            interior.push_back(seg == 1);
            a += sz;
        }
    }
}

// Two-step region R2 inside the interior region [lo, hi) and its tiles.
// Along each axis R2 keeps two cells clear of the absorbing slabs (the
// two-step kernel recomputes step n+1's Ht two cells below and its E one
// cell on either side of its cells, all without CPML code) and clear of every
// source and port plane (whose currents enter E between the steps): the
// component planes a source writes, and one more on either side, stay
// outside the cells where the kernel computes step n+1's E.  Then the
// two-step tiles cover R2 (strips of at most 60 cells, YO_TY rows, kc
// planes), and single-step tiles cover the rest of the interior (the
// "frame"), cut at R2's faces.
// Keep the source and port planes normal to axis `a` out of [r0, r1) along
// it: step n+1's E is computed on [r0 - 1, r1] along the plane's normal and
// a plane's currents touch indices i .. i + (ncomp == 5); the range keeps
// the larger side of each plane that meets it.
static void cut_planes(const yo_plan *p, int a, int &r0, int &r1)
{
    auto cut = [&](const yo_plane &pl, int ncomp) {
        const int i = pl.index, i_end = pl.index + (ncomp == 5 ? 1 : 0);
        if (pl.axis != a || r1 <= r0 || i_end < r0 - 1 || i > r1) return;
        const int below = (i - 1) - r0, above = r1 - (i_end + 2);
        if (below >= above) r1 = i - 1;
        else r0 = i_end + 2;
    };
    for (const yo_plane &pl : p->src_planes) cut(pl, 2);
    for (const yo_plane &pl : p->port_planes) cut(pl, p->mon_nc);
}

void build_pair_tiles(yo_plan *p, const int lo[3], const int hi[3])
{
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    int r[6];
    for (int a = 0; a < 3; ++a) {
        r[2 * a] = std::max(lo[a], p->plo[a] + 2);
        r[2 * a + 1] = std::min(hi[a], n[a] - p->phi[a] - 1);
        cut_planes(p, a, r[2 * a], r[2 * a + 1]);
    }
    for (int a = 0; a < 3; ++a)
        if (r[2 * a + 1] - r[2 * a] < 4) return;   // too thin: no two-step region
    for (int i = 0; i < 6; ++i) p->r2[i] = r[i];
    // two-step tiles
    std::vector<std::pair<int, int>> ax, ay, az;
    std::vector<char> ix, iy, iz;
    split_axis(n[0], r[0], r[1], 60, ax, ix);
    // rows per tile: per wave (YO_TY or YO_TY2), times the waves of a
    // block in the cooperative layout
    const int wpb = (p->tflags & YO_TILE_WPB8) ? 8 : 4;
    split_axis(n[1], r[2], r[3],
               ((p->tflags & YO_TILE_PAIR6) ? YO_TY2 : YO_TY) * ((p->tflags & YO_TILE_COOP_PAIRS) ? wpb : 1),
               ay, iy);
    split_axis(n[2], r[4], r[5], p->kc, az, iz);
    for (size_t k = 0; k < az.size(); ++k)
        for (size_t j = 0; j < ay.size(); ++j)
            for (size_t i = 0; i < ax.size(); ++i) {
                if (!(ix[i] && iy[j] && iz[k])) continue;
                int4 t;
                t.x = ax[i].first | (ax[i].second << 16);
                t.y = ay[j].first | (ay[j].second << 16);
                t.z = az[k].first | ((az[k].first + az[k].second) << 16);
                t.w = 0;
                p->tiles_host.push_back(t);
            }
    p->n2 = (int)p->tiles_host.size() - p->n_tiles;
    // frame: the interior minus R2, single-step tiles cut at R2's faces
    auto pieces = [&](int a, int w, std::vector<std::pair<int, int>> &out, std::vector<char> &in_r2) {
        out.clear();
        in_r2.clear();
        const int cuts[4] = {lo[a], r[2 * a], r[2 * a + 1], hi[a]};
        for (int seg = 0; seg < 3; ++seg) {
            const int len = cuts[seg + 1] - cuts[seg];
            if (len <= 0) continue;
            const int np = (len + w - 1) / w;
            int st = cuts[seg];
            for (int q = 0; q < np; ++q) {
                const int sz = len / np + (q < len % np ? 1 : 0);
                out.emplace_back(st, sz);
                in_r2.push_back(seg == 1);
                st += sz;
            }
        }
    };
    pieces(0, YO_TX, ax, ix);
    pieces(1, YO_TY, ay, iy);
    pieces(2, p->kc, az, iz);
    for (size_t k = 0; k < az.size(); ++k)
        for (size_t j = 0; j < ay.size(); ++j)
            for (size_t i = 0; i < ax.size(); ++i) {
                if (ix[i] && iy[j] && iz[k]) continue;
                int4 t;
                t.x = ax[i].first | (ax[i].second << 16);
                t.y = ay[j].first | (ay[j].second << 16);
                t.z = az[k].first | ((az[k].first + az[k].second) << 16);
                t.w = 0;
                p->tiles_host.push_back(t);
            }
    // with YO_TILE_XINT the interior list also holds the tiles that meet
    // only the x-slabs (class 1); they join the frame, which then runs the
    // x-axis CPML code
    if (p->tflags & YO_TILE_XINT)
        for (int t = 0; t < p->n_int; ++t)
            if (p->tiles_host[t].w == 1) p->tiles_host.push_back(p->tiles_host[t]);
    p->nfr = (int)p->tiles_host.size() - p->n_tiles - p->n2;
    // YO_TILE_ZPAIRS: when R2 is the whole interior (no plane cuts it, so the
    // frame is empty and the shell's class-4 tiles are exactly the z-slabs
    // under R2), those z-slabs go two steps per launch too, in strips of 60
    // cells, YO_TY rows and at most kc planes
    bool whole = (p->tflags & YO_TILE_ZPAIRS) && (p->plo[2] > 0 || p->phi[2] > 0);
    for (int a = 0; a < 3; ++a) whole = whole && r[2 * a] == lo[a] && r[2 * a + 1] == hi[a];
    if (!whole) return;
    split_axis(n[0], r[0], r[1], 60, ax, ix);
    split_axis(n[1], r[2], r[3], YO_TY, ay, iy);
    az.clear();
    const int zs[2][2] = {{0, lo[2]}, {hi[2], n[2]}};
    for (const auto &z : zs) {
        const int len = z[1] - z[0];
        if (len <= 0) continue;
        const int np = (len + p->kc - 1) / p->kc;
        int st = z[0];
        for (int q = 0; q < np; ++q) {
            const int sz = len / np + (q < len % np ? 1 : 0);
            az.emplace_back(st, sz);
            st += sz;
        }
    }
    const size_t z2_0 = p->tiles_host.size();
    for (size_t k = 0; k < az.size(); ++k)
        for (size_t j = 0; j < ay.size(); ++j)
            for (size_t i = 0; i < ax.size(); ++i) {
                if (!(ix[i] && iy[j])) continue;
                int4 t;
                t.x = ax[i].first | (ax[i].second << 16);
                t.y = ay[j].first | (ay[j].second << 16);
                t.z = az[k].first | ((az[k].first + az[k].second) << 16);
                t.w = 4;
                p->tiles_host.push_back(t);
            }
    p->nz2 = (int)(p->tiles_host.size() - z2_0);
}

// Tile table: the interior tiles, then the CPML shell, each in space order
// (z, y, x fastest).  Along each axis the region clear of the absorbing
// slabs is [lo + 1, n - hi) for a CPML of lo/hi cells (no owned site and no
// recomputed halo site one below meets a CPML coefficient); a tile is
// interior when it lies in that region along all three axes (with
// YO_TILE_XINT also when it leaves it along x only: the interior launch then
// runs the x-axis CPML code, at the interior's register budget).  A shell tile's
// class (int4 .w) has bit a set when it is not clear along axis a.  The two
// parts may use different row counts (cooperative blocks take YO_TY rows per
// wave of the block).
// With two steps per launch (YO_TILE_PAIRS) the region clear of the slabs is
// [lo + 2, n - hi - 1), the two-step region's own margin, so that no
// single-step interior layer one cell thick lies between that region and
// the shell (the shell runs the layer, its CPML code idle there); and
// YO_TILE_XFULL then cuts whole 60-cell strips of the two-step launch out
// of the row between the x-normal source and port planes.
void build_tiles(yo_plan *p)
{
    const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
    const int wpb = (p->tflags & YO_TILE_WPB8) ? 8 : 4;
    const bool pr = p->tsteps == 2 && (p->tflags & YO_TILE_PAIRS);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = p->plo[a] > 0 ? p->plo[a] + (pr ? 2 : 1) : 0;
        hi[a] = n[a] - p->phi[a] - (pr && p->phi[a] > 0 ? 1 : 0);
        int a0 = lo[a], a1 = hi[a];
        if (a == 0 && pr) cut_planes(p, 0, a0, a1);
        if (a == 0 && pr && (p->tflags & YO_TILE_XFULL) && a1 - a0 >= 60) {
            // whole 60-cell two-step strips, centred in the row where the
            // planes allow; the shell strips take the rest
            const int whole = (a1 - a0) / 60 * 60;
            const int wlo = std::min(std::max((n[0] - whole) / 2, a0), a1 - whole);
            lo[0] = wlo;
            hi[0] = wlo + whole;
        } else if (a == 0 && (p->tflags & YO_TILE_XFULL) && hi[0] - lo[0] >= YO_TX) {
            // the interior takes as many whole strips as fit; the rest of the
            // row goes to the two shell strips (which then also carry
            // interior columns)
            const int whole = (hi[0] - lo[0]) / YO_TX * YO_TX;
            const int rest = n[0] - whole;
            int wlo = p->plo[0] > 0 ? (p->phi[0] > 0 ? rest / 2 : rest) : 0;
            wlo = std::max(wlo, lo[0]);
            wlo = std::min(wlo, n[0] - whole - (n[0] - hi[0]));
            lo[0] = wlo;
            hi[0] = wlo + whole;
        } else if (a == 0 && (p->tflags & YO_TILE_XSTRIPS)) {
            // full-width CPML strips: the shell strips also carry interior columns
            if (p->plo[0] > 0) lo[0] = std::max(lo[0], std::min(YO_TX, n[0]));
            if (p->phi[0] > 0) hi[0] = std::min(hi[0], n[0] - YO_TX);
        }
        hi[a] = std::max(hi[a], 0);
        lo[a] = std::min(lo[a], hi[a]);
    }
    std::vector<std::pair<int, int>> ax, ay, az;
    std::vector<char> ix, iy, iz;
    split_axis(n[0], lo[0], hi[0], YO_TX, ax, ix);
    split_axis(n[2], lo[2], hi[2], p->kc, az, iz);
    auto emit = [&](bool shell, int rows, std::vector<int4> &out) {
        split_axis(n[1], lo[1], hi[1], rows, ay, iy);
        for (size_t k = 0; k < az.size(); ++k)
            for (size_t j = 0; j < ay.size(); ++j)
                for (size_t i = 0; i < ax.size(); ++i) {
                    const int c = (ix[i] ? 0 : 1) | (iy[j] ? 0 : 2) | (iz[k] ? 0 : 4);
                    const bool in_shell = c != 0 && !(c == 1 && (p->tflags & YO_TILE_XINT));
                    if (in_shell != shell) continue;
                    int4 t;
                    t.x = ax[i].first | (ax[i].second << 16);
                    t.y = ay[j].first | (ay[j].second << 16);
                    t.z = az[k].first | ((az[k].first + az[k].second) << 16);
                    t.w = c;
                    out.push_back(t);
                }
    };
    p->tiles_host.clear();
    emit(false, (p->tflags & YO_TILE_COOP_INT) ? YO_TY * wpb : YO_TY, p->tiles_host);
    p->n_int = (int)p->tiles_host.size();
    emit(true, (p->tflags & YO_TILE_COOP_SHELL) ? YO_TY * wpb : ((p->tflags & YO_TILE_SHELL6) ? YO_TY2 : YO_TY),
         p->tiles_host);
    p->n_tiles = (int)p->tiles_host.size();
    p->n2 = p->nfr = p->nz2 = p->n_c4 = 0;
    if (pr && (p->tflags & YO_TILE_ZPAIRS)) {
        // the shell's class-4 tiles (z-slabs only) last, in order
        auto mid = std::stable_partition(p->tiles_host.begin() + p->n_int, p->tiles_host.end(),
                                         [](const int4 &t) { return t.w != 4; });
        p->n_c4 = (int)(p->tiles_host.end() - mid);
    }
    for (int i = 0; i < 6; ++i) p->r2[i] = 0;
    if (p->tsteps == 2 && (p->tflags & YO_TILE_PAIRS)) build_pair_tiles(p, lo, hi);
}

size_t tiles_capacity(const yo_grid &g, int ty_min, int kc_min)
{
    const size_t ntx = g.nx / YO_TX + 4;
    const size_t nty = g.ny / ty_min + 4;
    const size_t ntz = g.nz / kc_min + 4;
    return ntx * nty * ntz;
}

// Host tables go up with synchronous copies after the caller's stream has
// drained: pageable-memory copies are not reliably ordered behind kernels
// still running on the stream (a large workspace fill, or a solve that reads
// the descriptors being replaced).
yo_status upload(yo_plan *p, const Region &r, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes > r.bytes) return fail(YO_EWORKSPACE, "internal: region too small");
    if (!bytes) return YO_OK;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(p->ws + r.off, src, bytes, hipMemcpyHostToDevice));
    return YO_OK;
}

yo_status upload_to(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (!bytes) return YO_OK;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return YO_OK;
}

yo_status upload_desc(yo_plan *p, hipStream_t s)
{
    yo_status st = upload(p, p->L.desc_plan, &p->hplan, sizeof(YoPlanD), s);
    if (st) return st;
    return upload(p, p->L.desc_rhs, p->hrhs.data(), sizeof(YoRhsD) * p->hrhs.size(), s);
}

// stepped right-hand sides of `which`
void set_rhs_range(const yo_plan *p, int which, int &r0, int &r1)
{
    r0 = (which & YO_FORWARD) ? 0 : p->n_pfwd;
    r1 = (which & YO_ADJOINT) ? p->n_phys : p->n_pfwd;
}

// right-hand sides of `which` in the output numbering (DFT results)
void set_out_range(const yo_plan *p, int which, int &r0, int &r1)
{
    r0 = (which & YO_FORWARD) ? 0 : p->n_fwd;
    r1 = (which & YO_ADJOINT) ? p->n_rhs : p->n_fwd;
}

size_t fields_per_rhs(const yo_plan *p) { return 6 * (size_t)p->nbuf * p->cells_p; }   // buffers x (E, H) x 3

// DFT results of output right-hand side r (numbering of yo_rhs_count)
float2 *box_of(const yo_plan *p, int r)
{
    return reinterpret_cast<float2 *>(p->ws + p->L.dft_box.off) + 3 * p->bsz * r;
}
float2 *mon_of(const yo_plan *p, int r)
{
    return reinterpret_cast<float2 *>(p->ws + p->L.dft_mon.off) + std::max<size_t>(p->mon_total, 1) * r;
}

}  // namespace

static yo_status set_chain_ptrs(yo_plan *p);

// ====================================================================== ABI
extern "C" {

const char *yo_last_error(void) { return g_err.c_str(); }
const char *yo_version(void) { return "yeeopt 0.1 (gfx950)"; }

yo_status yo_plan_create(const yo_grid *grid, const yo_design *des, int n_steps, int n_freq,
                         const yo_freq *freqs, int n_src, const yo_plane *src_planes,
                         int n_ports, const yo_plane *port_planes, yo_plan **out)
{
    if (!grid || !des || !out || (n_freq > 0 && !freqs)) return fail(YO_EINVAL, "null argument");
    *out = nullptr;
    const yo_grid &g = *grid;
    if (g.nx < 4 || g.ny < 4 || g.nz < 4) return fail(YO_EINVAL, "grid must be at least 4^3");
    if ((size_t)3 * g.nz * g.ny * (size_t)(g.nx + 64) >= (1ull << 31))
        return fail(YO_EUNSUPPORTED, "grid too large for one right-hand side");
    if (!(g.dx > 0 && g.dy > 0 && g.dz > 0 && g.courant > 0)) return fail(YO_EINVAL, "bad spacing");
    for (int f = 0; f < 6; ++f)
        if (g.npml[f] < 0) return fail(YO_EINVAL, "negative npml");
    if (g.npml[0] + g.npml[1] >= g.nx || g.npml[2] + g.npml[3] >= g.ny || g.npml[4] + g.npml[5] >= g.nz)
        return fail(YO_EINVAL, "CPML fills the grid");
    if (g.nx > 65000 || g.ny > 65000 || g.nz > 65000)
        return fail(YO_EUNSUPPORTED, "grid too large for the tile encoding");
    const double dmin = std::min(g.dx, std::min(g.dy, g.dz));
    const double cdt = g.courant * dmin;
    const double lim = cdt * std::sqrt(1 / (g.dx * g.dx) + 1 / (g.dy * g.dy) + 1 / (g.dz * g.dz));
    if (!(lim < 1.0)) return fail(YO_EUNSTABLE, "Courant number %.4f above the limit (c dt |1/d| = %.4f)", g.courant, lim);
    if (n_steps < 1) return fail(YO_EINVAL, "n_steps < 1");
    if (n_freq < 1 || n_freq > YO_MAX_FREQ) return fail(n_freq < 1 ? YO_EINVAL : YO_EUNSUPPORTED, "n_freq out of range");
    if (n_src < 0 || n_ports < 0 || n_ports > YO_MAX_PORTS) return fail(YO_EUNSUPPORTED, "too many ports");
    if (n_src * n_freq > YO_MAX_GF || n_ports * n_freq > YO_MAX_GA)
        return fail(YO_EUNSUPPORTED, "too many right-hand sides");
    if (n_src + n_ports < 1) return fail(YO_EINVAL, "no sources and no ports");
    const yo_design &d = *des;
    if (d.supersample < 2 || (d.supersample & 1)) return fail(YO_EINVAL, "supersample must be even and >= 2");
    if (d.md < 1 || d.nd < 1 || d.mc < 1 || d.nc < 1 || !(d.filter_r > 0))
        return fail(YO_EINVAL, "bad design sizes");
    if (!(d.eps_core > 0 && d.eps_clad > 0 && d.sobel_delta > 0)) return fail(YO_EINVAL, "bad materials");
    if (d.k_hi < d.k_lo) return fail(YO_EINVAL, "empty slab");
    if (d.i0 - 1 < g.npml[0] || d.i0 + d.md + 1 > g.nx - g.npml[1] || d.j0 - 1 < g.npml[2] ||
        d.j0 + d.nd + 1 > g.ny - g.npml[3] || d.k_lo - 1 < g.npml[4] || d.k_hi + 1 > g.nz - g.npml[5])
        return fail(YO_EINVAL, "design region (plus its one-cell ring) must lie outside the CPML");
    for (int f = 0; f < n_freq; ++f) {
        const yo_freq &q = freqs[f];
        if (!(q.omega > 0) || q.ramp_steps < 0) return fail(YO_EINVAL, "bad frequency %d", f);
        if (q.win_len < 2 || q.win_start < 0 || q.win_start + q.win_len > n_steps)
            return fail(YO_EINVAL, "window of frequency %d outside [0, n_steps)", f);
    }

    yo_plan *p = new yo_plan();
    p->id = g_next_plan_id++;
    p->grid = g;
    p->des = d;
    p->n_steps = n_steps;
    p->n_freq = n_freq;
    p->n_src = n_src;
    p->n_ports = n_ports;
    p->n_fwd = n_src * n_freq;
    p->n_rhs = (n_src + n_ports) * n_freq;
    p->freqs.assign(freqs, freqs + n_freq);
    p->dt = cdt / kC0;
    p->sx = cdt / g.dx;
    p->sy = cdt / g.dy;
    p->sz = cdt / g.dz;
    for (int a = 0; a < 3; ++a) {
        p->plo[a] = g.npml[2 * a];
        p->phi[a] = g.npml[2 * a + 1];
    }
    p->omega_dt.resize(n_freq);
    for (int f = 0; f < n_freq; ++f) p->omega_dt[f] = freqs[f].omega * p->dt;
    for (int s = 0; s < n_src; ++s) {
        if (!src_planes || !plane_ok(p, src_planes[s])) {
            delete p;
            return fail(YO_EINVAL, "source plane %d outside the grid interior", s);
        }
        p->src_planes.push_back(src_planes[s]);
    }
    for (int q = 0; q < n_ports; ++q) {
        if (!port_planes || !plane_ok(p, port_planes[q])) {
            delete p;
            return fail(YO_EINVAL, "port plane %d outside the grid interior", q);
        }
        p->port_planes.push_back(port_planes[q]);
    }
    p->src_set.assign(n_src, 0);
    p->port_set.assign(n_ports, 0);

    // ghost layout: one zero layer on every face, rows padded to 128 bytes
    // ghosts at x = -1 and x = nx, rounded up to 32 floats
    p->nxp = (g.nx + 2 + 31) & ~31;
    p->cells_p = (size_t)(g.nz + 2) * (g.ny + 2) * p->nxp;
    if (6 * p->cells_p * sizeof(float) >= ((size_t)1 << 31)) {
        delete p;
        return fail(YO_EUNSUPPORTED, "one state array (6 components) must stay below 2 GiB");
    }
    if (!set_psi_layout(p)) {
        delete p;
        return fail(YO_EUNSUPPORTED, "the CPML memories of one right-hand side must stay below 2 GiB");
    }
    p->box[0] = d.i0 - 1;
    p->box[1] = d.j0 - 1;
    p->box[2] = d.k_lo - 1;
    p->box[3] = d.md + 2;
    p->box[4] = d.nd + 2;
    p->box[5] = d.k_hi - d.k_lo + 3;
    p->bsz = (size_t)p->box[3] * p->box[4] * p->box[5];
    build_port_tables(p);
    for (auto &pl : p->src_planes) {
        p->src_off.push_back(p->src_total);
        p->src_total += 2 * (size_t)pl.n0 * pl.n1;
    }
    p->S = d.supersample;
    p->U = p->S * (d.md + 4);
    p->V = p->S * (d.nd + 4);
    p->G0 = d.md + 4;
    p->G1 = d.nd + 4;
    p->tmax = 2 * (int)std::ceil(d.filter_r) + 2;
    p->tiles_cap = tiles_capacity(g, 4, 4);

    p->n_phys = p->n_rhs;
    p->n_pfwd = p->n_fwd;
    build_layout(p);

    build_profiles(p);
    build_steptab(p);
    build_taps(p->S, d.md, d.mc, d.filter_r, p->tmax, p->tap_lo_x, p->tap_n_x, p->tap_w_x, p->urange_x);
    build_taps(p->S, d.nd, d.nc, d.filter_r, p->tmax, p->tap_lo_y, p->tap_n_y, p->tap_w_y, p->urange_y);
    for (int v : p->tap_n_x)
        if (v > p->tmax) { delete p; return fail(YO_EINVAL, "internal: filter taps"); }
    for (int v : p->tap_n_y)
        if (v > p->tmax) { delete p; return fail(YO_EINVAL, "internal: filter taps"); }
    build_tiles(p);
    {
        // carve the parametrization buffers once against a stand-in base to
        // prove the layout holds them; the real pointers are set at bind time
        p->ws = reinterpret_cast<char *>((uintptr_t)1 << 20);
        const yo_status st = set_chain_ptrs(p);
        p->ws = nullptr;
        p->chain = YoChainBufs{};
        if (st) {
            delete p;
            return st;
        }
    }
    *out = p;
    return YO_OK;
}

void yo_plan_destroy(yo_plan *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        const std::string tag = "#" + std::to_string(p->id) + ":";
        for (auto it = g_graphs.begin(); it != g_graphs.end();) {
            if (it->first.find(tag) != std::string::npos) {
                if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
                if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
                it = g_graphs.erase(it);
            } else {
                ++it;
            }
        }
    }
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
    if (p->ov_fork) (void)hipEventDestroy(p->ov_fork);
    if (p->ov_join) (void)hipEventDestroy(p->ov_join);
    for (int q = 0; q < 6; ++q)
        for (hipEvent_t e : p->tm_ev[q]) (void)hipEventDestroy(e);
    delete p;
}

yo_status yo_workspace_bytes(const yo_plan *p, size_t *bytes)
{
    if (!p || !bytes) return fail(YO_EINVAL, "null argument");
    *bytes = p->L.total;
    return YO_OK;
}

yo_status yo_rhs_count(const yo_plan *p, int *n)
{
    if (!p || !n) return fail(YO_EINVAL, "null argument");
    *n = p->n_rhs;
    return YO_OK;
}

yo_status yo_steps_done(const yo_plan *p, int *steps)
{
    if (!p || !steps) return fail(YO_EINVAL, "null argument");
    *steps = p->steps_done;
    return YO_OK;
}

static yo_status rebuild_descriptors(yo_plan *p)
{
    const yo_grid &g = p->grid;
    YoPlanD &P = p->hplan;
    memset(&P, 0, sizeof P);
    P.nx = g.nx; P.ny = g.ny; P.nz = g.nz; P.nxp = p->nxp;
    P.sx = (float)p->sx; P.sy = (float)p->sy; P.sz = (float)p->sz;
    for (int a = 0; a < 3; ++a) { P.plo[a] = p->plo[a]; P.phi[a] = p->phi[a]; }
    P.kappa = wsp<float>(p, p->L.kappa);
    float *prof = wsp<float>(p, p->L.prof);
    P.prof[0] = prof;
    P.prof[1] = prof + 6 * (size_t)g.nx;
    P.prof[2] = prof + 6 * (size_t)(g.nx + g.ny);
    for (int i = 0; i < 6; ++i) P.box[i] = p->box[i];
    for (int a = 0; a < 3; ++a) {
        P.psi_off[a] = (int)p->psi_axis_off[a];
        P.psi_n[a] = (int)p->psi_axis_n[a];
    }
    P.psi_total = (int)p->psi_per_rhs;
    P.n_ports = p->n_ports;
    P.mon_nc = p->mon_nc;
    P.n_steps = p->n_steps;
    P.dft_stride = p->pulse ? p->dft_stride : 1;
    P.nbuf = p->nbuf;
    for (int i = 0; i < 6; ++i) P.r2[i] = p->r2[i];
    P.mon_total = (int)p->mon_total;
    for (int q = 0; q < p->n_ports; ++q) {
        const yo_plane &pl = p->port_planes[q];
        P.ports[q] = YoPlaneD{pl.axis, pl.index, pl.lo0, pl.lo1, pl.n0, pl.n1};
        P.mon_off[q] = (int)p->mon_off[q];
    }
    P.step_ctr = wsp<int>(p, p->L.ctr);
    P.n_rhs = p->n_phys;
    P.rhs = wsp<YoRhsD>(p, p->L.desc_rhs);

    p->hrhs.assign(p->n_phys, YoRhsD{});
    float *fields = wsp<float>(p, p->L.fields);
    float *psi = wsp<float>(p, p->L.psi);
    float2 *dbox = wsp<float2>(p, p->L.dft_box);
    float2 *dmon = wsp<float2>(p, p->L.dft_mon);
    const float2 *srcj = wsp<float2>(p, p->L.src_j);
    const float2 *portw = wsp<float2>(p, p->L.port_w);
    const float4 *stab = wsp<float4>(p, p->L.steptab);
    for (int r = 0; r < p->n_phys; ++r) {
        YoRhsD &R = p->hrhs[r];
        float *f = fields + fields_per_rhs(p) * r;
        R.F[0] = f;
        R.F[1] = f + 6 * p->cells_p;
        R.F[2] = p->nbuf == 3 ? f + 12 * p->cells_p : nullptr;
        R.psi = psi + p->psi_per_rhs * r;
        // under a pulse, stepped right-hand side r stands for the output
        // right-hand sides of its source or port at every frequency; its
        // DFT pointers are those of frequency 0
        const int ro = !p->pulse ? r : (r < p->n_pfwd ? r : p->n_fwd + (r - p->n_pfwd));
        R.dft_box = dbox + 3 * p->bsz * ro;
        R.dft_mon = dmon + std::max<size_t>(p->mon_total, 1) * ro;
        int f_idx, srcp;
        const float2 *jp;
        YoPlaneD pl;
        if (ro < p->n_fwd) {
            f_idx = ro / std::max(p->n_src, 1);
            srcp = ro % std::max(p->n_src, 1);
            const yo_plane &q = p->src_planes[srcp];
            pl = YoPlaneD{q.axis, q.index, q.lo0, q.lo1, q.n0, q.n1};
            jp = p->src_set[srcp] ? srcj + p->src_off[srcp] : nullptr;
        } else {
            const int ra = ro - p->n_fwd;
            f_idx = ra / p->n_ports;
            srcp = ra % p->n_ports;
            const yo_plane &q = p->port_planes[srcp];
            pl = YoPlaneD{q.axis, q.index, q.lo0, q.lo1, q.n0, q.n1};
            jp = p->port_set[srcp]
                     ? portw + (p->mon_nc == 5 ? (size_t)f_idx * p->port_total : 0) + p->port_off[srcp]
                     : nullptr;
        }
        R.steptab = stab + (size_t)f_idx * p->n_steps;
        R.src_j = jp;
        R.src = pl;
        R.win_start = p->freqs[f_idx].win_start;
        R.win_len = p->freqs[f_idx].win_len;
        for (int i = 0; i < 4; ++i) R.ginv[i] = p->ginv[4 * f_idx + i];
        R.freq = f_idx;
        R.src_nc = ro < p->n_fwd ? 2 : p->mon_nc;
        R.n_dft = 1;
        R.dfttab = R.steptab;
        R.box_fstride = 0;
        R.mon_fstride = 0;
        if (p->pulse) {
            const int per = ro < p->n_fwd ? p->n_src : p->n_ports;   // output RHS per frequency
            R.steptab = stab + (size_t)p->n_freq * p->n_steps;
            R.win_start = 0;
            R.win_len = p->n_steps;
            R.n_dft = p->n_freq;
            R.dfttab = stab;
            R.box_fstride = (int)(3 * p->bsz * per);
            R.mon_fstride = (int)(std::max<size_t>(p->mon_total, 1) * per);
        }
    }
    return YO_OK;
}

static yo_status set_chain_ptrs(yo_plan *p)
{
    YoChainBufs &c = p->chain;
    const yo_design &d = p->des;
    c.md = d.md; c.nd = d.nd; c.mc = d.mc; c.nc = d.nc; c.S = p->S; c.U = p->U; c.V = p->V;
    c.G0 = p->G0; c.G1 = p->G1; c.tmax = p->tmax;
    c.eps_core = (float)d.eps_core; c.eps_clad = (float)d.eps_clad; c.delta = (float)d.sobel_delta;
    const size_t G = (size_t)p->G0 * p->G1;
    const size_t UV = (size_t)p->U * p->V;
    const size_t DD = (size_t)(p->S * d.md) * (p->S * d.nd);
    float *f = wsp<float>(p, p->L.chain_f);
    auto take = [&](size_t n) {
        float *r = f;
        f += (n + 63) & ~(size_t)63;
        return r;
    };
    c.mask = take(UV);
    c.rho = take(UV);
    c.tanh_ = take(DD);
    c.P = take(3 * G);
    c.Q = take(3 * G);
    c.R = take(3 * G);
    c.aux = take(6 * G);
    c.gmap = take(4 * G);
    c.gPQ = take(6 * G);
    c.gG = take(4 * G);
    c.gR = take(2 * G);
    c.gphi = take(DD);
    c.tmp = take((size_t)(p->S * d.nd) * d.mc);
    c.tap_w_x = take((size_t)p->tmax * p->S * d.md);
    c.tap_w_y = take((size_t)p->tmax * p->S * d.nd);
    int *ip = wsp<int>(p, p->L.chain_i);
    auto takei = [&](size_t n) {
        int *r = ip;
        ip += (n + 63) & ~(size_t)63;
        return r;
    };
    c.tap_lo_x = takei(p->S * d.md);
    c.tap_n_x = takei(p->S * d.md);
    c.tap_lo_y = takei(p->S * d.nd);
    c.tap_n_y = takei(p->S * d.nd);
    c.urange_x = takei(2 * d.mc);
    c.urange_y = takei(2 * d.nc);
    if ((char *)f > p->ws + p->L.chain_f.off + p->L.chain_f.bytes ||
        (char *)ip > p->ws + p->L.chain_i.off + p->L.chain_i.bytes)
        return fail(YO_EWORKSPACE, "internal: parametrization buffers exceed their region");
    c.n_morph = (int)p->morph_ops.size();
    c.mdil = 0;
    for (int k = 0; k < c.n_morph; ++k)
        if (p->morph_ops[k] == 'd') c.mdil |= 1u << k;
    c.n_mtaps = (int)p->mtaps.size() / 2;
    c.malpha = (float)p->morph_alpha;
    c.minv = c.n_mtaps ? (float)(1.0 / c.n_mtaps) : 0.0f;
    c.mtap = nullptr;
    c.mcan = c.msum = c.tanh2 = c.mg = c.mq = nullptr;
    if (c.n_morph) {
        f = wsp<float>(p, p->L.morph);
        c.mcan = take((size_t)(c.n_morph + 1) * UV);
        c.msum = take((size_t)c.n_morph * DD);
        c.tanh2 = take(DD);
        c.mg = take(2 * DD);
        c.mq = take(DD);
        c.mtap = reinterpret_cast<int *>(take(p->mtaps.size()));
        if ((char *)f > p->ws + p->L.morph.off + p->L.morph.bytes)
            return fail(YO_EWORKSPACE, "internal: morphology buffers exceed their region");
    }
    return YO_OK;
}

yo_status yo_set_morphology(yo_plan *p, const char *ops, double diameter, double alpha)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->ws) return fail(YO_ESTATE, "set the morphological filters before binding a workspace");
    std::string seq = ops ? ops : "";
    if (seq.empty()) {
        p->morph_ops.clear();
        p->mtaps.clear();
        build_layout(p);
        return YO_OK;
    }
    if (seq.size() > 8) return fail(YO_EINVAL, "at most 8 morphological operations");
    for (char ch : seq)
        if (ch != 'd' && ch != 'e') return fail(YO_EINVAL, "operations are 'd' (dilate) and 'e' (erode)");
    if (!(diameter > 0)) return fail(YO_EINVAL, "the disc diameter must be positive");
    if (!(alpha > 0 && alpha <= 80)) return fail(YO_EINVAL, "alpha must be in (0, 80]");
    const double R = diameter * p->S / 2.0;
    if (R > 32.0) return fail(YO_EUNSUPPORTED, "disc radius above 32 sub-pixels");
    std::vector<int> taps;
    const int n = (int)std::floor(R);
    for (int dy = -n; dy <= n; ++dy)
        for (int dx = -n; dx <= n; ++dx)
            if ((double)(dx * dx + dy * dy) <= R * R) {
                taps.push_back(dy);
                taps.push_back(dx);
            }
    p->morph_ops = seq;
    p->morph_d = diameter;
    p->morph_alpha = alpha;
    p->mtaps = taps;
    build_layout(p);
    return YO_OK;
}

yo_status yo_set_alpha_terms(yo_plan *p, int terms)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->ws) return fail(YO_ESTATE, "choose the coefficient before binding a workspace");
    if (terms != 1 && terms != 2) return fail(YO_EINVAL, "terms must be 1 or 2");
    if (terms == 2) {
        if (p->pulse) return fail(YO_EUNSUPPORTED, "no two-term coefficient under a pulse");
        for (int q = 0; q < p->n_ports; ++q) {
            yo_plane next = p->port_planes[q];
            next.index += 1;
            if (!plane_ok(p, next))
                return fail(YO_EINVAL, "port %d: the plane after it leaves the grid interior", q);
        }
    }
    p->mon_nc = terms == 2 ? 5 : 2;
    // the two-step region keeps clear of every plane a port's currents touch
    build_tiles(p);
    build_port_tables(p);
    p->port_w_host.clear();
    std::fill(p->port_set.begin(), p->port_set.end(), 0);
    build_layout(p);
    return YO_OK;
}

yo_status yo_set_pulse(yo_plan *p, double omega0, double sigma_steps, double t0_steps)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->ws) return fail(YO_ESTATE, "set the pulse before binding a workspace");
    if (!(sigma_steps > 0)) {
        p->pulse = false;
        p->dft_stride = 1;
        p->n_phys = p->n_rhs;
        p->n_pfwd = p->n_fwd;
    } else {
        const double w = omega0 * p->dt;
        if (!(w > 0 && w < M_PI)) return fail(YO_EINVAL, "carrier outside (0, pi / dt)");
        if (p->mon_nc == 5)
            return fail(YO_EUNSUPPORTED, "the two-term coefficient's adjoint weights depend on the "
                                         "frequency; no pulse with it");
        if (!(t0_steps >= 0)) return fail(YO_EINVAL, "negative pulse centre");
        p->pulse = true;
        p->pulse_w = w;
        p->pulse_sigma = sigma_steps;
        p->pulse_t0 = t0_steps;
        p->n_phys = p->n_src + p->n_ports;
        p->n_pfwd = p->n_src;
    }
    build_steptab(p);
    build_layout(p);
    return YO_OK;
}

static yo_status bind_ws(yo_plan *p, void *dev, size_t bytes, hipStream_t s)
{
    p->ws = (char *)dev;
    p->ws_bytes = bytes;
    p->generation++;
    rebuild_descriptors(p);
    yo_status st = set_chain_ptrs(p);
    if (st) return st;
    // a fresh workspace holds garbage: clear the state and table regions first
    HIPCHK(yo_launch_fill((float *)p->ws, p->L.total / sizeof(float), 0.0f, s));
    if ((st = upload(p, p->L.prof, p->prof.data(), p->prof.size() * sizeof(float), s))) return st;
    if ((st = upload(p, p->L.steptab, p->steptab.data(), p->steptab.size() * sizeof(float4), s))) return st;
    if ((st = upload(p, p->L.tiles, p->tiles_host.data(), p->tiles_host.size() * sizeof(int4), s))) return st;
    const YoChainBufs &c = p->chain;
    if ((st = upload_to(c.tap_lo_x, p->tap_lo_x.data(), p->tap_lo_x.size() * 4, s))) return st;
    if ((st = upload_to(c.tap_n_x, p->tap_n_x.data(), p->tap_n_x.size() * 4, s))) return st;
    if ((st = upload_to(c.tap_lo_y, p->tap_lo_y.data(), p->tap_lo_y.size() * 4, s))) return st;
    if ((st = upload_to(c.tap_n_y, p->tap_n_y.data(), p->tap_n_y.size() * 4, s))) return st;
    if ((st = upload_to(c.urange_x, p->urange_x.data(), p->urange_x.size() * 4, s))) return st;
    if ((st = upload_to(c.urange_y, p->urange_y.data(), p->urange_y.size() * 4, s))) return st;
    if ((st = upload_to(c.tap_w_x, p->tap_w_x.data(), p->tap_w_x.size() * 4, s))) return st;
    if ((st = upload_to(c.tap_w_y, p->tap_w_y.data(), p->tap_w_y.size() * 4, s))) return st;
    if (c.n_morph && (st = upload_to(c.mtap, p->mtaps.data(), p->mtaps.size() * 4, s))) return st;
    if ((st = upload_desc(p, s))) return st;
    // copies from pageable host memory are staged; make them complete before
    // the host vectors can change
    HIPCHK(hipStreamSynchronize(s));
    p->bg_set = false;
    p->design_set = false;
    p->steps_done = 0;
    for (int q = 0; q < 2; ++q) p->finalized[q] = p->unstable[q] = false;
    return YO_OK;
}

yo_status yo_set_dft_stride(yo_plan *p, int stride)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->ws) return fail(YO_ESTATE, "set the DFT stride before binding a workspace");
    if (!p->pulse) return fail(YO_EINVAL, "a DFT stride needs pulse excitation (yo_set_pulse)");
    if (stride < 1 || stride > 64) return fail(YO_EINVAL, "stride must be in [1, 64]");
    // the sampled sum equals (1/m) sum_q DFT(w + 2 pi q / m); the pulse's own
    // spectrum S at every alias q != 0 (and that of its conjugate part, at
    // -w0) must be negligible against S(w) for the phasor to stay exact
    const float4 *row = p->steptab.data() + (size_t)p->n_freq * p->n_steps;
    auto spec = [&](double w, bool conj) {
        std::complex<double> S = 0.0;
        for (int n = 0; n < p->n_steps; ++n) {
            const std::complex<double> sm((double)row[n].x, (conj ? 1.0 : -1.0) * (double)row[n].y);
            S += sm * std::polar(1.0, w * (n + 0.5));
        }
        return std::abs(S);
    };
    for (int f = 0; f < p->n_freq && stride > 1; ++f) {
        const double w = p->omega_dt[f];
        const double s0 = spec(w, false);
        for (int q = 1; q < stride; ++q) {
            const double wa = w + 2.0 * M_PI * q / stride;
            const double leak = std::max(spec(wa, false), spec(wa, true));
            if (!(leak <= 1e-6 * s0))
                return fail(YO_EINVAL, "DFT stride %d: the pulse spectrum at the alias %d of wavelength %d "
                                       "is %.2e of its value there", stride, q, f, leak / s0);
        }
    }
    p->dft_stride = stride;
    build_steptab(p);
    return YO_OK;
}

yo_status yo_set_time_blocking(yo_plan *p, int steps)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->ws) return fail(YO_ESTATE, "set the time blocking before binding a workspace");
    if (steps != 1 && steps != 2) return fail(YO_EINVAL, "steps per sweep must be 1 or 2");
    const int nbuf_was = p->nbuf;
    p->nbuf = steps == 2 ? 3 : 2;
    if (!set_psi_layout(p)) {
        p->nbuf = nbuf_was;
        set_psi_layout(p);
        return fail(YO_EUNSUPPORTED, "the CPML memories of one right-hand side must stay below 2 GiB");
    }
    p->tsteps = steps;
    if (steps == 1)
        p->tflags &= ~(YO_TILE_PAIRS | YO_TILE_OVERLAP | YO_TILE_ZPAIRS | YO_TILE_PAIR6 | YO_TILE_COOP_PAIRS);
    // the two-step and frame tiles can add up to twice the single-step count
    p->tiles_cap = tiles_capacity(p->grid, 4, 4) * (steps == 2 ? 3 : 1);
    build_tiles(p);
    build_layout(p);
    return YO_OK;
}

yo_status yo_bind_workspace(yo_plan *p, void *dev, size_t bytes, yo_stream stream)
{
    if (!p || !dev) return fail(YO_EINVAL, "null argument");
    if (((uintptr_t)dev) & 255) return fail(YO_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < p->L.total)
        return fail(YO_EWORKSPACE, "workspace of %zu bytes, %zu needed", bytes, p->L.total);
    p->static_dev = -1;
    return bind_ws(p, dev, bytes, (hipStream_t)stream);
}

yo_status yo_bind_static_workspace(yo_plan *p, yo_stream stream)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (p->L.total > YO_STATIC_WS_BYTES)
        return fail(YO_EWORKSPACE, "the plan needs %zu workspace bytes; the static workspace holds %zu",
                    p->L.total, (size_t)YO_STATIC_WS_BYTES);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= YO_MAX_DEVICES) return fail(YO_EUNSUPPORTED, "device index %d", dev);
    void *ptr = nullptr;
    unsigned epoch = 0;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // once per device, with that device current: the array's address there
            void *q = nullptr;
            const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !q)
                return fail(YO_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_scratch_ptr[dev] = q;
        }
        ptr = g_scratch_ptr[dev];
        epoch = ++g_scratch_epoch[dev];
    }
    p->static_dev = dev;
    p->static_epoch = epoch;
    // bind_ws clears the whole region the plan uses (the last binding's
    // contents stay in the array) and uploads the tables
    return bind_ws(p, ptr, YO_STATIC_WS_BYTES, (hipStream_t)stream);
}

yo_status yo_set_tiling(yo_plan *p, int rows, int zchunk, int flags)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (rows != YO_TY) return fail(YO_EINVAL, "rows per wave must be %d", YO_TY);
    // a tile's planes and the halo plane below are at most one per lane
    if (zchunk < 4 || zchunk > 63) return fail(YO_EINVAL, "zchunk must be in [4, 63]");
    if (flags & ~YO_TILE_ALL) return fail(YO_EINVAL, "unknown tiling flags");
    if ((flags & YO_TILE_PAIRS) && p->tsteps != 2)
        return fail(YO_EINVAL, "flag 512 needs yo_set_time_blocking(plan, 2) before binding");
    if ((flags & YO_TILE_PAIRS) && (flags & YO_TILE_COOP_INT))
        return fail(YO_EINVAL, "flag 512 does not combine with flag 16");
    if ((flags & YO_TILE_OVERLAP) && !(flags & YO_TILE_PAIRS))
        return fail(YO_EINVAL, "flag 1024 needs flag 512");
    if ((flags & YO_TILE_ZPAIRS) && !(flags & YO_TILE_PAIRS))
        return fail(YO_EINVAL, "flag 2048 needs flag 512");
    if ((flags & YO_TILE_PAIR6) && !(flags & YO_TILE_PAIRS))
        return fail(YO_EINVAL, "flag 4096 needs flag 512");
    if ((flags & YO_TILE_COOP_PAIRS) && !(flags & YO_TILE_PAIRS))
        return fail(YO_EINVAL, "flag 8192 needs flag 512");
    if ((flags & YO_TILE_SHELL6) && (flags & YO_TILE_COOP_SHELL))
        return fail(YO_EINVAL, "flag 16384 does not combine with flag 4");
    p->kc = zchunk;
    p->tflags = flags;
    build_tiles(p);
    if (p->tiles_host.size() > p->tiles_cap) return fail(YO_EINVAL, "internal: tile table");
    if (p->ws) {
        // synchronous: the graph cache keys on the tiling, and old graphs may still run
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemcpy(p->ws + p->L.tiles.off, p->tiles_host.data(), p->tiles_host.size() * sizeof(int4),
                         hipMemcpyHostToDevice));
        // the plan descriptor carries the two-step region, which the split sets
        rebuild_descriptors(p);
        if (yo_status st = upload_desc(p, nullptr)) return st;
        HIPCHK(hipDeviceSynchronize());
    }
    return YO_OK;
}

yo_status yo_set_background(yo_plan *p, const float *kappa, const float *mask, yo_stream stream)
{
    if (!p || !kappa || !mask) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    hipStream_t s = (hipStream_t)stream;
    const yo_grid &g = p->grid;
    HIPCHK(yo_launch_to_ghost(kappa, wsp<float>(p, p->L.kappa), 3, 0, 3, g.nz, g.ny, g.nx, p->nxp, s));
    HIPCHK(hipMemcpyAsync(p->chain.mask, mask, sizeof(float) * p->U * p->V, hipMemcpyDeviceToDevice, s));
    p->bg_set = true;
    p->design_set = false;
    p->mat_gen++;
    return YO_OK;
}

static std::complex<double> cget(const double *a, size_t i) { return {a[2 * i], a[2 * i + 1]}; }

yo_status yo_set_source_mode(yo_plan *p, int src, const double *h, yo_stream stream)
{
    if (!p || !h) return fail(YO_EINVAL, "null argument");
    if (src < 0 || src >= p->n_src) return fail(YO_EINVAL, "source index out of range");
    if (yo_status st_ = ws_check(p)) return st_;
    const yo_plane &pl = p->src_planes[src];
    const size_t n = (size_t)pl.n0 * pl.n1;
    if (p->src_j_host.size() < p->src_total) p->src_j_host.assign(p->src_total, float2{0, 0});
    // J = n x h: J_t1 = -h_t2 (h_t2 stored at the E_t1 sites), J_t2 = h_t1
    for (size_t i = 0; i < n; ++i) {
        const auto h1 = cget(h, i), h2 = cget(h, n + i);
        p->src_j_host[p->src_off[src] + i] = float2{(float)-h2.real(), (float)-h2.imag()};
        p->src_j_host[p->src_off[src] + n + i] = float2{(float)h1.real(), (float)h1.imag()};
    }
    hipStream_t s = (hipStream_t)stream;
    yo_status st0 = upload_to(p->ws + p->L.src_j.off + sizeof(float2) * p->src_off[src],
                              p->src_j_host.data() + p->src_off[src], sizeof(float2) * 2 * n, s);
    if (st0) return st0;
    p->src_set[src] = 1;
    rebuild_descriptors(p);
    yo_status st = upload_desc(p, s);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(s));
    return YO_OK;
}

yo_status yo_set_port_mode(yo_plan *p, int port, const double *e, const double *h, yo_stream stream)
{
    if (!p || !e || !h) return fail(YO_EINVAL, "null argument");
    if (port < 0 || port >= p->n_ports) return fail(YO_EINVAL, "port index out of range");
    if (yo_status st_ = ws_check(p)) return st_;
    const yo_plane &pl = p->port_planes[port];
    const size_t n = (size_t)pl.n0 * pl.n1;
    // N = 1/2 sum (e_t1 conj(h_t2) - e_t2 conj(h_t1)); cell area cancels
    std::complex<double> N = 0.0;
    for (size_t i = 0; i < n; ++i)
        N += cget(e, i) * std::conj(cget(h, n + i)) - cget(e, n + i) * std::conj(cget(h, i));
    N *= 0.5;
    if (std::abs(N) == 0.0) return fail(YO_EINVAL, "mode normalisation N is zero");
    const size_t blocks = port_w_blocks(p);
    if (p->port_w_host.size() < p->port_total * blocks)
        p->port_w_host.assign(p->port_total * blocks, float2{0, 0});
    auto put = [&](size_t k, std::complex<double> v) {
        p->port_w_host[k] = float2{(float)v.real(), (float)v.imag()};
    };
    hipStream_t s = (hipStream_t)stream;
    if (p->mon_nc == 2) {
        for (size_t i = 0; i < n; ++i) {
            put(p->port_off[port] + i, std::conj(cget(h, n + i)) / (2.0 * N));
            put(p->port_off[port] + n + i, -std::conj(cget(h, i)) / (2.0 * N));
        }
        yo_status st0 = upload_to(p->ws + p->L.port_w.off + sizeof(float2) * p->port_off[port],
                                  p->port_w_host.data() + p->port_off[port], sizeof(float2) * 2 * n, s);
        if (st0) return st0;
    } else {
        // Two-term coefficient (App. A): alpha = 1/4 (1/N sum E x h* + 1/N* sum e* x H)
        // = wE . E + u . H with wE half the E-only weights, u_t1 = -conj(e_t2)/(4 conj N),
        // u_t2 = conj(e_t1)/(4 conj N) on the tangential H sites half a cell past the
        // plane.  The Yee update's H step gives Hhat = curl_e Ehat / (2 i sin theta), so
        // u . H is a sum over E sites: the tangential E on this plane and the next and
        // the normal E between them.  u is dropped where its curl would reach past the
        // plane (last row along t2 for u_t1, last column along t1 for u_t2).
        const int a = pl.axis, t1 = (a + 1) % 3, t2 = (a + 2) % 3;
        const bool t1_cols = t1 < t2;            // t1 runs along the plane's columns (index % n0)
        const double S[3] = {p->sx, p->sy, p->sz};
        std::vector<std::complex<double>> u0(n), u1(n);
        const std::complex<double> cN = std::conj(N);
        for (size_t i = 0; i < n; ++i) {
            const int col = (int)(i % pl.n0), row = (int)(i / pl.n0);
            const bool last_t2 = t1_cols ? row == pl.n1 - 1 : col == pl.n0 - 1;
            const bool last_t1 = t1_cols ? col == pl.n0 - 1 : row == pl.n1 - 1;
            u0[i] = last_t2 ? 0.0 : -std::conj(cget(e, n + i)) / (4.0 * cN);
            u1[i] = last_t1 ? 0.0 : std::conj(cget(e, i)) / (4.0 * cN);
        }
        // index of the cell one step back along t1 / t2, or -1 at the first one
        auto back = [&](size_t i, bool along_t1) -> long {
            const int col = (int)(i % pl.n0), row = (int)(i / pl.n0);
            const bool cols = along_t1 == t1_cols;
            if (cols) return col > 0 ? (long)i - 1 : -1;
            return row > 0 ? (long)i - pl.n0 : -1;
        };
        for (int f = 0; f < p->n_freq; ++f) {
            const std::complex<double> fac = 1.0 / std::complex<double>(0.0, 2.0 * std::sin(0.5 * p->omega_dt[f]));
            const size_t base = (size_t)f * p->port_total + p->port_off[port];
            for (size_t i = 0; i < n; ++i) {
                const std::complex<double> w1 = std::conj(cget(h, n + i)) / (4.0 * N);
                const std::complex<double> w2 = -std::conj(cget(h, i)) / (4.0 * N);
                put(base + i, w1 - S[a] * u1[i] * fac);
                put(base + n + i, w2 + S[a] * u0[i] * fac);
                std::complex<double> qn = (-S[t2] * u0[i] + S[t1] * u1[i]) * fac;
                const long i2 = back(i, false), i1 = back(i, true);
                if (i2 >= 0) qn += S[t2] * u0[i2] * fac;
                if (i1 >= 0) qn -= S[t1] * u1[i1] * fac;
                put(base + 2 * n + i, qn);
                put(base + 3 * n + i, S[a] * u1[i] * fac);
                put(base + 4 * n + i, -S[a] * u0[i] * fac);
            }
            yo_status st0 = upload_to(p->ws + p->L.port_w.off + sizeof(float2) * base,
                                      p->port_w_host.data() + base, sizeof(float2) * 5 * n, s);
            if (st0) return st0;
        }
    }
    p->port_set[port] = 1;
    rebuild_descriptors(p);
    yo_status st = upload_desc(p, s);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(s));
    return YO_OK;
}

yo_status yo_set_design(yo_plan *p, const float *C, double beta, yo_stream stream)
{
    if (!p || !C) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->bg_set) return fail(YO_ESTATE, "yo_set_background first");
    if (!(beta > 0)) return fail(YO_EINVAL, "beta must be positive");
    const yo_design &d = p->des;
    HIPCHK(yo_launch_chain_forward(p->chain, C, (float)beta, wsp<float>(p, p->L.kappa), p->grid.nx,
                                   p->grid.ny, p->grid.nz, p->nxp, d.i0, d.j0, d.k_lo, d.k_hi,
                                   (hipStream_t)stream));
    p->beta = beta;
    p->design_set = true;
    p->mat_gen++;
    return YO_OK;
}

yo_status yo_reset(yo_plan *p, int which, yo_stream stream)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (which < 1 || which > 3) return fail(YO_EINVAL, "which must be YO_FORWARD, YO_ADJOINT or YO_BOTH");
    hipStream_t s = (hipStream_t)stream;
    int r0, r1;
    set_rhs_range(p, which, r0, r1);
    if (r1 > r0) {
        HIPCHK(yo_launch_fill(wsp<float>(p, p->L.fields) + fields_per_rhs(p) * r0,
                              fields_per_rhs(p) * (r1 - r0), 0.0f, s));
        HIPCHK(yo_launch_fill(wsp<float>(p, p->L.psi) + p->psi_per_rhs * r0,
                              p->psi_per_rhs * (r1 - r0), 0.0f, s));
    }
    int o0, o1;
    set_out_range(p, which, o0, o1);
    if (o1 > o0) {
        HIPCHK(yo_launch_fill(wsp<float>(p, p->L.dft_box) + 6 * p->bsz * o0, 6 * p->bsz * (o1 - o0),
                              0.0f, s));
        const size_t mt = std::max<size_t>(p->mon_total, 1);
        HIPCHK(yo_launch_fill(wsp<float>(p, p->L.dft_mon) + 2 * mt * o0, 2 * mt * (o1 - o0), 0.0f, s));
    }
    YoCtrArgs ca{};
    ca.n = 1;
    ca.add = 0;
    ca.ctr[0] = wsp<int>(p, p->L.ctr);
    HIPCHK(yo_launch_ctr(ca, 1, s));
    p->steps_done = 0;
    p->active = which;
    for (int q = 0; q < 2; ++q)
        if (which & (1 << q)) {
            p->finalized[q] = p->unstable[q] = false;
            p->run_mat_gen[q] = p->mat_gen;
        }
    return YO_OK;
}

// Work lists of the per-step DFT and source kernels for a group of plans.
static void aux_args(yo_plan *const *plans, const int *which, int cnt, bool dft, YoAuxArgs &a)
{
    memset(&a, 0, sizeof a);
    a.n_slots = cnt;
    int tot = 0;
    for (int i = 0; i < cnt; ++i) {
        yo_plan *p = plans[i];
        int r0, r1;
        set_rhs_range(p, which[i], r0, r1);
        int npts = 0;
        if (dft) {
            npts = (int)(3 * p->bsz + p->mon_total);
        } else {
            for (int r = r0; r < r1; ++r)
                npts = std::max(npts, p->hrhs[r].src_nc * p->hrhs[r].src.n0 * p->hrhs[r].src.n1);
        }
        a.plan[i] = wsp<YoPlanD>(p, p->L.desc_plan);
        a.rhs0[i] = r0;
        a.nrhs[i] = std::max(r1 - r0, 0);
        a.npts[i] = npts;
        a.prefix[i] = tot;
        tot += (int)(((long)npts * a.nrhs[i] + 255) / 256);
    }
    a.prefix[cnt] = tot;
    a.total_blocks = tot;
}

// Fill the step-kernel arguments of tile class `cls` for a plan list;
// returns the number of blocks (0: no plan has tiles of that class).
// tiles of launch part `part`: 0 interior, 1 CPML shell, 2 two-step region,
// 3 the interior around it (single steps), 4 the z-slabs under the two-step
// region (two steps, YO_TILE_ZPAIRS), 5 the CPML shell of steps that go in
// pairs (without the tiles of part 4)
static void part_range(const yo_plan *p, int part, int &t0, int &t1)
{
    switch (part) {
    case 0: t0 = 0; t1 = p->n_int; break;
    case 1: t0 = p->n_int; t1 = p->n_tiles; break;
    case 2: t0 = p->n_tiles; t1 = p->n_tiles + p->n2; break;
    case 3: t0 = p->n_tiles + p->n2; t1 = t0 + p->nfr; break;
    case 4: t0 = p->n_tiles + p->n2 + p->nfr; t1 = t0 + p->nz2; break;
    default: t0 = p->n_int; t1 = p->n_tiles - (p->nz2 ? p->n_c4 : 0); break;
    }
}

// Step-kernel arguments of one part (see part_range) for a plan list;
// returns the number of blocks (0: no plan has tiles there).
static int step_args(yo_plan *const *plans, const int *which, int cnt, int part, YoStepArgs &a)
{
    memset(&a, 0, sizeof(YoStepArgs));
    a.n_slots = cnt;
    const int wpb = (plans[0]->tflags & YO_TILE_WPB8) ? 8 : 4;
    const int f = plans[0]->tflags;
    const bool coop = part == 0   ? (f & YO_TILE_COOP_INT) != 0
                      : part == 2 ? (f & YO_TILE_COOP_PAIRS) != 0
                                  : (part == 1 || part == 5) && (f & YO_TILE_COOP_SHELL) != 0;
    int tot = 0;
    for (int i = 0; i < cnt; ++i) {
        yo_plan *p = plans[i];
        int r0, r1;
        set_rhs_range(p, which[i], r0, r1);
        YoSlot &sl = a.slot[i];
        int t0, t1;
        part_range(p, part, t0, t1);
        sl.plan = wsp<YoPlanD>(p, p->L.desc_plan);
        sl.tiles = wsp<int4>(p, p->L.tiles) + t0;
        sl.rhs0 = r0;
        sl.nrhs = std::max(r1 - r0, 1);
        sl.ntile = (r1 > r0) ? t1 - t0 : 0;
        a.prefix[i] = tot;
        // waves come in groups of wpb per right-hand side: wpb tiles, or in
        // the cooperative layout one tile
        const int groups = coop ? sl.ntile : (sl.ntile + wpb - 1) / wpb;
        tot += sl.nrhs * groups * wpb;
    }
    a.prefix[cnt] = tot;
    a.total_waves = tot;
    a.wpb = wpb;
    return (tot + wpb - 1) / wpb;
}

// Launch one part's step kernel (the variant its tiling flags choose).
static hipError_t launch_part(const yo_plan *p0, int part, const YoStepArgs &a, int blocks, hipStream_t s)
{
    const int f = p0->tflags;
    if (part == 2)
        return yo_launch_step2(false, (f & YO_TILE_PAIR6) ? YO_TY2 : YO_TY, (f & YO_TILE_COOP_PAIRS) != 0, a,
                               blocks, s);
    if (part == 4) return yo_launch_step2(true, YO_TY, false, a, blocks, s);
    if (part == 3)
        return yo_launch_step((f & YO_TILE_XINT) ? 1 : 0, false, !(f & YO_TILE_NOPF_INT), a, blocks, s);
    if (part == 0)
        return yo_launch_step((f & YO_TILE_XINT) ? 1 : 0, (f & YO_TILE_COOP_INT) != 0,
                              !(f & YO_TILE_NOPF_INT), a, blocks, s);
    return yo_launch_step((f & YO_TILE_CLASS_CODE) ? 8 : 7, (f & YO_TILE_COOP_SHELL) != 0,
                          !(f & YO_TILE_NOPF_SHELL), a, blocks, s, (f & YO_TILE_SHELL6) ? YO_TY2 : YO_TY);
}

// Launch `n_launch` steps (k_offset 0..n_launch-1) of a plan list, then add
// n_launch to every plan's counter.  Per step: DFT of E^n (when `with_dft`),
// the step launches (interior, CPML shell), the source.  Plans must share
// every tiling flag but the x-split ones.
// DFT launches: at the steps k of the call with k % dft_every == 0 (the
// kernel itself skips steps its plan does not sample).  pairs: the steps go
// two at a time where two remain (the two-step region in one launch for
// both, the interior around it and the CPML shell one step at a time, the
// source after each step); the caller guarantees no DFT at the second step
// of a pair.  With YO_TILE_OVERLAP the two-step launch of a pair goes on
// the first plan's side stream, forked after the launches before it and
// joined before the pair's second step: the first step's frame, shell and
// source read only step n's buffer and write cells of step n+1's buffer that
// the two-step launch does not (it reads step n's and writes R2's rim of
// step n+1's and R2 of step n+2's), so the two may run at once.
static yo_status launch_steps(yo_plan *const *plans, const int *which, int n, int n_launch,
                              bool with_dft, hipStream_t s, yo_plan *timed = nullptr,
                              int dft_every = 1, bool pairs = false)
{
    yo_plan *const p0 = plans[0];
    const bool overlap = pairs && (p0->tflags & YO_TILE_OVERLAP) && p0->side_stream;
    for (int base = 0; base < n; base += YO_MAX_SLOTS) {
        const int cnt = std::min(YO_MAX_SLOTS, n - base);
        static thread_local YoStepArgs A[6];
        int blocks[6] = {0, 0, 0, 0, 0, 0};
        for (int part = 0; part < (pairs ? 6 : 2); ++part)
            blocks[part] = step_args(plans + base, which + base, cnt, part, A[part]);
        YoAuxArgs ad, as;
        aux_args(plans + base, which + base, cnt, true, ad);
        aux_args(plans + base, which + base, cnt, false, as);
        auto launch = [&](int part, int k, hipStream_t on) -> yo_status {
            A[part].k_offset = k;
            const bool tm = timed && base == 0 && blocks[part] &&
                            (timed->tm_part == part || timed->tm_part == 2);
            if (tm) {
                std::vector<hipEvent_t> &ev = timed->tm_ev[part];
                const size_t need = 2 * (size_t)timed->tm_done[part] + 2;
                while (ev.size() < need) {
                    hipEvent_t e;
                    HIPCHK(hipEventCreate(&e));
                    ev.push_back(e);
                }
                HIPCHK(hipEventRecord(ev[need - 2], on));
                HIPCHK(launch_part(plans[base], part, A[part], blocks[part], on));
                HIPCHK(hipEventRecord(ev[need - 1], on));
                timed->tm_done[part]++;
            } else {
                HIPCHK(launch_part(plans[base], part, A[part], blocks[part], on));
            }
            return YO_OK;
        };
        yo_status st;
        for (int k = 0; k < n_launch;) {
            if (with_dft && k % dft_every == 0) {
                ad.k_offset = k;
                HIPCHK(yo_launch_dft(ad, s));
            }
            if (pairs && k + 1 < n_launch) {
                // the two-step launches (R2, and with YO_TILE_ZPAIRS the
                // z-slabs under it: part 5 is then the shell without them)
                hipStream_t s2 = overlap ? p0->side_stream : s;
                if (overlap) {
                    HIPCHK(hipEventRecord(p0->ov_fork, s));
                    HIPCHK(hipStreamWaitEvent(s2, p0->ov_fork, 0));
                }
                if ((st = launch(2, k, s2))) return st;
                if ((st = launch(4, k, s2))) return st;
                if (overlap) HIPCHK(hipEventRecord(p0->ov_join, s2));
                for (int q = 0; q < 2; ++q) {
                    if (q == 1 && overlap) HIPCHK(hipStreamWaitEvent(s, p0->ov_join, 0));
                    if ((st = launch(3, k + q, s))) return st;
                    if ((st = launch(5, k + q, s))) return st;
                    as.k_offset = k + q;
                    HIPCHK(yo_launch_source(as, s));
                }
                k += 2;
            } else {
                for (int part = 0; part < 2; ++part)
                    if ((st = launch(part, k, s))) return st;
                as.k_offset = k;
                HIPCHK(yo_launch_source(as, s));
                k += 1;
            }
        }
        YoCtrArgs ca{};
        ca.n = cnt;
        ca.add = n_launch;
        for (int i = 0; i < cnt; ++i) ca.ctr[i] = wsp<int>(plans[base + i], plans[base + i]->L.ctr);
        HIPCHK(yo_launch_ctr(ca, 0, s));
    }
    return YO_OK;
}

// Steps of a call may go two at a time when every plan has the two-step
// layout and the count left in its run, and no DFT falls on a pair's second
// step (no DFT in the call, or pulse DFTs on even steps only).
static bool pairs_ok(yo_plan *const *plans, int n, int n_launch, bool with_dft, int every)
{
    for (int i = 0; i < n; ++i) {
        const yo_plan *p = plans[i];
        // (a plan whose two-step region came out empty has no frame tiles either)
        if (!(p->tflags & YO_TILE_PAIRS) || p->tsteps != 2 || p->n2 == 0) return false;
        if (p->steps_done + n_launch > p->n_steps) return false;
    }
    if (with_dft) {
        if (every % 2) return false;
        for (int i = 0; i < n; ++i)
            if (!plans[i]->pulse) return false;
    }
    return true;
}

// The DFT stride every plan of the list samples, when they share one and all
// stand at a step it divides (then the DFT kernel need only be launched on
// every stride-th step of a call); else 1.
static int dft_every(yo_plan *const *plans, int n)
{
    const int st = plans[0]->pulse ? plans[0]->dft_stride : 1;
    if (st <= 1) return 1;
    for (int i = 0; i < n; ++i)
        if (!plans[i]->pulse || plans[i]->dft_stride != st || plans[i]->steps_done % st) return 1;
    return st;
}

// does any plan's DFT window meet the steps [steps_done, steps_done + count)?
static bool chunk_needs_dft(yo_plan *const *plans, const int *which, int n, int count)
{
    for (int i = 0; i < n; ++i) {
        const yo_plan *p = plans[i];
        const int a = p->steps_done, b = std::min(p->steps_done + count, p->n_steps);
        if (p->pulse && b > a) return true;
        for (int f = 0; f < p->n_freq; ++f) {
            const int ws = p->freqs[f].win_start, we = ws + p->freqs[f].win_len;
            if (a < we && b > ws) return true;
        }
        (void)which;
    }
    return false;
}

yo_status yo_advance_many(yo_plan *const *plans, const int *which, int n, int n_steps, int chunk,
                          int use_graph, yo_stream stream)
{
    if (!plans || !which || n < 1) return fail(YO_EINVAL, "empty plan list");
    if (n_steps < 0) return fail(YO_EINVAL, "negative step count");
    for (int i = 0; i < n; ++i) {
        yo_plan *p = plans[i];
        if (!p) return fail(YO_EINVAL, "plan %d is null", i);
        if (yo_status st_ = ws_check(p)) return st_;
        if (which[i] != p->active) return fail(YO_ESTATE, "plan %d: which differs from its reset", i);
        // the x-split flags only shape each plan's own tile table; the others
        // pick the kernel variant, which one launch shares
        const int own = YO_TILE_XSTRIPS | YO_TILE_XFULL;
        if ((p->tflags & ~own) != (plans[0]->tflags & ~own))
            return fail(YO_EINVAL, "plans in one call must share the tiling flags (but the x-split ones)");
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) return fail(YO_EINVAL, "plan listed twice");
    }
    hipStream_t s = (hipStream_t)stream;
    if (chunk < 1) chunk = 1;
    if ((plans[0]->tflags & YO_TILE_OVERLAP) && !plans[0]->side_stream) {
        yo_plan *p0 = plans[0];
        HIPCHK(hipEventCreateWithFlags(&p0->ov_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&p0->ov_join, hipEventDisableTiming));
        HIPCHK(hipStreamCreateWithFlags(&p0->side_stream, hipStreamNonBlocking));
    }
    // launch timing (yo_set_timing on the first plan): the last tm_n steps
    // of this call run eagerly with events around the timed part
    yo_plan *timed = plans[0]->tm_n > 0 ? plans[0] : nullptr;
    const int tail = timed ? std::min(timed->tm_n, n_steps) : 0;
    // steps_done is advanced per chunk so chunk_needs_dft sees the current steps
    std::vector<int> start(n);
    for (int i = 0; i < n; ++i) start[i] = plans[i]->steps_done;
    auto bump = [&](int k) {
        for (int i = 0; i < n; ++i) plans[i]->steps_done += k;
    };
    int done = 0;
    if (use_graph && n_steps - tail >= chunk) {
        std::string key = "c" + std::to_string(chunk);
        for (int i = 0; i < n; ++i)
            key += "#" + std::to_string(plans[i]->id) + ":" + std::to_string(plans[i]->generation) +
                   "w" + std::to_string(which[i]) + "k" + std::to_string(plans[i]->kc) + "f" +
                   std::to_string(plans[i]->tflags);
        // a graph launching the DFT only on every stride-th step is replayed
        // only at steps the stride divides: its chunk must be a multiple
        int every = dft_every(plans, n);
        if (chunk % every) every = 1;
        key += "e" + std::to_string(every);
        GraphEntry ge[4];
        while (n_steps - tail - done >= chunk) {
            const bool need_dft = chunk_needs_dft(plans, which, n, chunk);
            const bool pairs = pairs_ok(plans, n, chunk, need_dft, every) && chunk % 2 == 0;
            const int variant = (need_dft ? 1 : 0) | (pairs ? 2 : 0);
            const std::string kv = key + (need_dft ? "|dft" : "|nodft") + (pairs ? "|pairs" : "");
            if (!ge[variant].exec) {
                std::lock_guard<std::mutex> lk(g_graph_mu);
                auto it = g_graphs.find(kv);
                if (it != g_graphs.end()) ge[variant] = it->second;
            }
            if (!ge[variant].exec) {
                yo_plan *p0 = plans[0];
                if (!p0->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p0->cap_stream, hipStreamNonBlocking));
                HIPCHK(hipStreamBeginCapture(p0->cap_stream, hipStreamCaptureModeThreadLocal));
                yo_status st = launch_steps(plans, which, n, chunk, need_dft, p0->cap_stream, nullptr,
                                            every, pairs);
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamEndCapture(p0->cap_stream, &graph);
                if (st) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return st;
                }
                if (e != hipSuccess) return fail(YO_EHIP, "graph capture: %s", hipGetErrorString(e));
                hipGraphExec_t exec = nullptr;
                HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                ge[variant].graph = graph;
                ge[variant].exec = exec;
                std::lock_guard<std::mutex> lk(g_graph_mu);
                g_graphs[kv] = ge[variant];
            }
            HIPCHK(hipGraphLaunch(ge[variant].exec, s));
            done += chunk;
            bump(chunk);
        }
    }
    while (done < n_steps) {
        const bool in_tail = done >= n_steps - tail;
        const int lim = in_tail ? n_steps - done : n_steps - tail - done;
        const int k = std::min(chunk, lim);
        const bool need_dft = chunk_needs_dft(plans, which, n, k);
        const int every = dft_every(plans, n);
        yo_status st = launch_steps(plans, which, n, k, need_dft, s, in_tail ? timed : nullptr, every,
                                    pairs_ok(plans, n, k, need_dft, every));
        if (st) return st;
        done += k;
        bump(k);
    }
    for (int i = 0; i < n; ++i)
        plans[i]->steps_done = std::min(plans[i]->n_steps, start[i] + n_steps);
    return YO_OK;
}

yo_status yo_advance(yo_plan *p, int which, int n_steps, yo_stream stream)
{
    return yo_advance_many(&p, &which, 1, n_steps, std::max(n_steps, 1), 0, stream);
}

yo_status yo_finalize(yo_plan *p, int which, yo_stream stream)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (which != p->active) return fail(YO_ESTATE, "finalize: which differs from the reset");
    if (p->steps_done < p->n_steps) return fail(YO_ESTATE, "finalize before all steps ran");
    hipStream_t s = (hipStream_t)stream;
    int r0, r1;
    set_out_range(p, which, r0, r1);
    const size_t mt = std::max<size_t>(p->mon_total, 1);
    // watchdog word of the counter region (after the step counter and the
    // unbinarity counter); zero bits are the float 0
    int *bad = wsp<int>(p, p->L.ctr) + 32;
    HIPCHK(yo_launch_fill(reinterpret_cast<float *>(bad), 1, 0.0f, s));
    for (int r = r0; r < r1; ++r) {
        const int f = r < p->n_fwd ? r / std::max(p->n_src, 1) : (r - p->n_fwd) / p->n_ports;
        const float *m = p->fin.data() + 4 * f;
        HIPCHK(yo_launch_finalize(box_of(p, r), 3 * p->bsz, m[0], m[1], m[2], m[3], bad, s));
        HIPCHK(yo_launch_finalize(mon_of(p, r), mt, m[0], m[1], m[2], m[3], bad, s));
    }
    int host_bad = 0;
    HIPCHK(hipMemcpyAsync(&host_bad, bad, sizeof host_bad, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < 2; ++q)
        if (which & (1 << q)) {
            p->finalized[q] = true;
            p->unstable[q] = host_bad != 0;
        }
    if (host_bad)
        return fail(YO_EUNSTABLE, "non-finite phasors after %d steps: the fields diverged", p->steps_done);
    return YO_OK;
}

yo_status yo_run(yo_plan *p, int which, int chunk, int use_graph, yo_stream stream)
{
    yo_status st = yo_reset(p, which, stream);
    if (st) return st;
    st = yo_advance_many(&p, &which, 1, p->n_steps, chunk, use_graph, stream);
    if (st) return st;
    return yo_finalize(p, which, stream);
}

yo_status yo_alpha(const yo_plan *p, float *alpha, yo_stream stream)
{
    // with no sources or no ports the array is empty and may be null
    if (!p || (!alpha && p->n_src > 0 && p->n_ports > 0)) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->finalized[0]) return fail(YO_ESTATE, "no finished forward run");
    if (p->run_mat_gen[0] != p->mat_gen)
        return fail(YO_ESTATE, "the design or background changed after the forward run started");
    if (p->unstable[0]) return fail(YO_EUNSTABLE, "the forward run diverged (non-finite phasors)");
    hipStream_t s = (hipStream_t)stream;
    const float2 *w = reinterpret_cast<const float2 *>(p->ws + p->L.port_w.off);
    for (int sidx = 0; sidx < p->n_src; ++sidx)
        for (int q = 0; q < p->n_ports; ++q) {
            if (!p->port_set[q]) return fail(YO_ESTATE, "port %d mode not set", q);
            for (int f = 0; f < p->n_freq; ++f) {
                const int r = f * p->n_src + sidx;
                const yo_plane &pl = p->port_planes[q];
                float2 *out = reinterpret_cast<float2 *>(alpha) + ((size_t)sidx * p->n_ports + q) * p->n_freq + f;
                const size_t wb = p->mon_nc == 5 ? (size_t)f * p->port_total : 0;
                HIPCHK(yo_launch_alpha(mon_of(p, r) + p->mon_off[q], w + wb + p->port_off[q],
                                       p->mon_nc * pl.n0 * pl.n1, out, s));
            }
        }
    return YO_OK;
}

static yo_status grad_common(yo_plan *p, const float *coef, float *gbox, float *gmap, hipStream_t s)
{
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->finalized[0] || !p->finalized[1])
        return fail(YO_ESTATE, "needs finished forward and adjoint runs (together or one after the other)");
    if (p->run_mat_gen[0] != p->mat_gen || p->run_mat_gen[1] != p->mat_gen)
        return fail(YO_ESTATE, "the design or background changed after a run started");
    if (p->unstable[0] || p->unstable[1])
        return fail(YO_EUNSTABLE, "a run diverged (non-finite phasors)");
    YoGradArgs a;
    memset(&a, 0, sizeof a);
    for (int f = 0; f < p->n_freq; ++f) {
        for (int si = 0; si < p->n_src; ++si) a.EF[f * p->n_src + si] = box_of(p, f * p->n_src + si);
        for (int q = 0; q < p->n_ports; ++q) a.EA[f * p->n_ports + q] = box_of(p, p->n_fwd + f * p->n_ports + q);
        a.sinth[f] = (float)std::sin(0.5 * p->omega_dt[f]);
    }
    a.coef = reinterpret_cast<const float2 *>(coef);
    a.kappa = wsp<float>(p, p->L.kappa);
    a.gbox = gbox;
    a.gmap = gmap;
    a.n_src = p->n_src;
    a.n_ports = p->n_ports;
    a.n_freq = p->n_freq;
    a.nxp = p->nxp;
    a.ny = p->grid.ny;
    a.nz = p->grid.nz;
    for (int i = 0; i < 6; ++i) a.box[i] = p->box[i];
    a.k_lo = p->des.k_lo;
    a.k_hi = p->des.k_hi;
    a.G0 = p->G0;
    a.G1 = p->G1;
    HIPCHK(yo_launch_grad_assemble(a, s));
    return YO_OK;
}

yo_status yo_gradient_kappa(yo_plan *p, const float *coef, float *g, yo_stream stream)
{
    if (!p || !g || (!coef && p->n_src > 0 && p->n_ports > 0)) return fail(YO_EINVAL, "null argument");
    return grad_common(p, coef, g, nullptr, (hipStream_t)stream);
}

yo_status yo_gradient(yo_plan *p, const float *coef, float *dFdC, yo_stream stream)
{
    // with no sources or no ports there is no coefficient (the gradient is 0)
    if (!p || !dFdC || (!coef && p->n_src > 0 && p->n_ports > 0)) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->design_set) return fail(YO_ESTATE, "yo_set_design first");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(yo_launch_fill(p->chain.gmap, 4 * (size_t)p->G0 * p->G1, 0.0f, s));
    yo_status st = grad_common(p, coef, nullptr, p->chain.gmap, s);
    if (st) return st;
    HIPCHK(yo_launch_chain_vjp(p->chain, (float)p->beta, dFdC, s));
    return YO_OK;
}

yo_status yo_chain_vjp(yo_plan *p, const float *gk, float *dFdC, yo_stream stream)
{
    if (!p || !gk || !dFdC) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->design_set) return fail(YO_ESTATE, "yo_set_design first");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(yo_launch_fill(p->chain.gmap, 4 * (size_t)p->G0 * p->G1, 0.0f, s));
    HIPCHK(yo_launch_zsum(gk, p->box, p->des.k_lo, p->des.k_hi, p->chain.gmap, p->G0, p->G1, s));
    HIPCHK(yo_launch_chain_vjp(p->chain, (float)p->beta, dFdC, s));
    return YO_OK;
}

yo_status yo_unbinarity(yo_plan *p, double lo, double hi, float *dev_u, yo_stream stream)
{
    if (!p || !dev_u) return fail(YO_EINVAL, "null argument");
    if (!(lo >= 0.0 && lo < hi && hi <= 1.0)) return fail(YO_EINVAL, "need 0 <= lo < hi <= 1");
    if (yo_status st_ = ws_check(p)) return st_;
    if (!p->design_set) return fail(YO_ESTATE, "yo_set_design first");
    // the counter sits after the step counter in the counter region
    int *count = wsp<int>(p, p->L.ctr) + 16;
    HIPCHK(yo_launch_unbinarity(p->chain, (float)(2.0 * lo - 1.0), (float)(2.0 * hi - 1.0), count, dev_u,
                                (hipStream_t)stream));
    return YO_OK;
}

yo_status yo_adam_step(float *dev_C, const float *dev_G, float *dev_M, float *dev_V, int n, int step,
                       double lr, double b1, double b2, double eps, yo_stream stream)
{
    if (n < 0 || (n > 0 && (!dev_C || !dev_G || !dev_M || !dev_V))) return fail(YO_EINVAL, "bad arrays");
    if (step < 1) return fail(YO_EINVAL, "steps count from 1");
    if (!(b1 >= 0.0 && b1 < 1.0 && b2 >= 0.0 && b2 < 1.0 && eps > 0.0))
        return fail(YO_EINVAL, "need 0 <= b1, b2 < 1 and eps > 0");
    const double inv1 = 1.0 / (1.0 - std::pow(b1, step));
    const double inv2 = 1.0 / (1.0 - std::pow(b2, step));
    HIPCHK(yo_launch_adam(dev_C, dev_G, dev_M, dev_V, n, (float)lr, (float)b1, (float)b2, (float)eps,
                          (float)inv1, (float)inv2, (hipStream_t)stream));
    return YO_OK;
}

yo_status yo_set_timing(yo_plan *p, int part, int n_last)
{
    if (!p) return fail(YO_EINVAL, "null argument");
    if (part < 0 || part > 2 || n_last < 0 || n_last > 4096) return fail(YO_EINVAL, "bad part or count");
    p->tm_part = part;
    p->tm_n = n_last;
    // starting clears what was recorded; stopping (n_last = 0) keeps it for
    // yo_get_timing
    if (n_last > 0)
        for (int q = 0; q < 6; ++q) p->tm_done[q] = 0;
    return YO_OK;
}

yo_status yo_get_timing(yo_plan *p, int part, float *avg_ms, int *count)
{
    if (!p || !avg_ms || !count) return fail(YO_EINVAL, "null argument");
    if (part < 0 || part > 5) return fail(YO_EINVAL, "part must be 0 to 5");
    *avg_ms = 0.0f;
    const int n = p->tm_done[part];
    *count = n;
    if (!n) return YO_OK;
    const std::vector<hipEvent_t> &ev = p->tm_ev[part];
    HIPCHK(hipEventSynchronize(ev[2 * n - 1]));
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        tot += ms;
    }
    *avg_ms = (float)(tot / n);
    return YO_OK;
}

yo_status yo_tile_table(const yo_plan *p, int part, int *out, int cap, int *n)
{
    if (!p || !n || (cap > 0 && !out)) return fail(YO_EINVAL, "null argument");
    if (part < 0 || part > 5) return fail(YO_EINVAL, "part must be 0 to 5");
    int t0, t1;
    part_range(p, part, t0, t1);
    *n = t1 - t0;
    for (int t = t0; t < t1 && t - t0 < cap; ++t) {
        const int4 tt = p->tiles_host[t];
        int *o = out + 7 * (t - t0);
        o[0] = tt.x & 0xffff;
        o[1] = o[0] + (tt.x >> 16);
        o[2] = tt.y & 0xffff;
        o[3] = o[2] + (tt.y >> 16);
        o[4] = tt.z & 0xffff;
        o[5] = tt.z >> 16;
        o[6] = tt.w;
    }
    return YO_OK;
}

yo_status yo_time_kernel(yo_plan *p, int cls, int n_launch, float *avg_ms, double *bytes,
                         double *cells, yo_stream stream)
{
    if (!p || !avg_ms || !bytes || !cells) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    if (cls < 0 || cls > 5 || n_launch < 1) return fail(YO_EINVAL, "bad part or count");
    if (!p->active) return fail(YO_ESTATE, "yo_reset first");
    if ((cls == 2 || cls == 4) && p->steps_done + 2 > p->n_steps)
        return fail(YO_ESTATE, "the two-step launch needs two steps left in the run");
    hipStream_t s = (hipStream_t)stream;
    int r0, r1;
    set_rhs_range(p, p->active, r0, r1);
    static thread_local YoStepArgs A;
    const int blocks = step_args(&p, &p->active, 1, cls, A);
    // owned cells of the part and (cell, axis) pairs inside an absorbing slab
    const yo_grid &g = p->grid;
    double own = 0.0, in_pml = 0.0;
    int ta, tb;
    part_range(p, cls, ta, tb);
    for (int t = ta; t < tb; ++t) {
        const int4 tt = p->tiles_host[t];
        const int x0 = tt.x & 0xffff, x1 = x0 + (tt.x >> 16);
        const int y0 = tt.y & 0xffff, y1 = y0 + (tt.y >> 16);
        const int z0 = tt.z & 0xffff, z1 = tt.z >> 16;
        own += (double)(x1 - x0) * (y1 - y0) * (z1 - z0);
        if (tt.w) {
            for (int z = z0; z < z1; ++z)
                for (int y = y0; y < y1; ++y)
                    for (int x = x0; x < x1; ++x) {
                        in_pml += (x < p->plo[0] || x >= g.nx - p->phi[0]);
                        in_pml += (y < p->plo[1] || y >= g.ny - p->phi[1]);
                        in_pml += (z < p->plo[2] || z >= g.nz - p->phi[2]);
                    }
        }
    }
    const double R = r1 - r0;
    // the two-step launch advances its cells two steps: twice the bytes
    // two one-step sweeps must move
    const double steps = (cls == 2 || cls == 4) ? 2.0 : 1.0;
    *bytes = steps * (own * (48.0 * R + 12.0) + 32.0 * R * in_pml);
    *cells = steps * own * R;
    if (!blocks || r1 <= r0) {
        *avg_ms = 0.0f;
        *bytes = *cells = 0.0;
        return YO_OK;
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    for (int k = 0; k < n_launch; ++k) HIPCHK(launch_part(p, cls, A, blocks, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / n_launch;
    return YO_OK;
}

yo_status yo_get_dft(const yo_plan *p, int rhs, int region, float *out, yo_stream stream)
{
    if (!p || !out) return fail(YO_EINVAL, "null argument");
    if (rhs < 0 || rhs >= p->n_rhs) return fail(YO_EINVAL, "rhs out of range");
    if (region < 0 || region > p->n_ports) return fail(YO_EINVAL, "region out of range");
    if (yo_status st_ = ws_check(p)) return st_;
    const void *src;
    size_t bytes;
    if (region == 0) {
        src = box_of(p, rhs);
        bytes = sizeof(float2) * 3 * p->bsz;
    } else {
        const yo_plane &pl = p->port_planes[region - 1];
        src = mon_of(p, rhs) + p->mon_off[region - 1];
        bytes = sizeof(float2) * p->mon_nc * pl.n0 * pl.n1;
    }
    HIPCHK(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return YO_OK;
}

yo_status yo_set_fields(yo_plan *p, int rhs, const float *E, const float *H, yo_stream stream)
{
    if (!p || !E || !H) return fail(YO_EINVAL, "null argument");
    if (rhs < 0 || rhs >= p->n_phys) return fail(YO_EINVAL, "rhs out of range");
    if (yo_status st_ = ws_check(p)) return st_;
    const yo_grid &g = p->grid;
    const YoRhsD &R = p->hrhs[rhs];
    const int par = p->steps_done % p->nbuf;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(yo_launch_to_ghost(E, R.F[par], 3, 0, 6, g.nz, g.ny, g.nx, p->nxp, s));
    HIPCHK(yo_launch_to_ghost(H, R.F[par], 3, 3, 6, g.nz, g.ny, g.nx, p->nxp, s));
    return YO_OK;
}

yo_status yo_get_fields(const yo_plan *p, int rhs, float *E, float *H, yo_stream stream)
{
    if (!p || !E || !H) return fail(YO_EINVAL, "null argument");
    if (rhs < 0 || rhs >= p->n_phys) return fail(YO_EINVAL, "rhs out of range");
    if (yo_status st_ = ws_check(p)) return st_;
    const yo_grid &g = p->grid;
    const YoRhsD &R = p->hrhs[rhs];
    const int par = p->steps_done % p->nbuf;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(yo_launch_from_ghost(R.F[par], E, 3, 0, 6, g.nz, g.ny, g.nx, p->nxp, s));
    HIPCHK(yo_launch_from_ghost(R.F[par], H, 3, 3, 6, g.nz, g.ny, g.nx, p->nxp, s));
    return YO_OK;
}

yo_status yo_get_kappa(const yo_plan *p, float *kappa, yo_stream stream)
{
    if (!p || !kappa) return fail(YO_EINVAL, "null argument");
    if (yo_status st_ = ws_check(p)) return st_;
    const yo_grid &g = p->grid;
    HIPCHK(yo_launch_from_ghost(reinterpret_cast<const float *>(p->ws + p->L.kappa.off), kappa, 3,
                                0, 3, g.nz, g.ny, g.nx, p->nxp, (hipStream_t)stream));
    return YO_OK;
}

yo_status yo_model_bytes(const yo_plan *p, int which, double *bytes, double *cells)
{
    if (!p || !bytes || !cells) return fail(YO_EINVAL, "null argument");
    int r0, r1;
    set_rhs_range(p, which, r0, r1);
    const double R = r1 - r0;
    const yo_grid &g = p->grid;
    const double N = (double)g.nx * g.ny * g.nz;
    // cells inside each axis' absorbing slabs
    const double pml = (double)(p->plo[0] + p->phi[0]) * g.ny * g.nz +
                       (double)(p->plo[1] + p->phi[1]) * g.nx * g.nz +
                       (double)(p->plo[2] + p->phi[2]) * g.nx * g.ny;
    double win = 0.0;
    for (auto &f : p->freqs) win += (double)f.win_len / p->n_steps;
    win /= p->n_freq;
    if (p->pulse) win = p->n_freq;   // every step, every frequency
    *bytes = R * (48.0 * N + 32.0 * pml + 48.0 * (double)p->bsz * win) + 12.0 * N;
    *cells = R * N;
    return YO_OK;
}

}  // extern "C"
