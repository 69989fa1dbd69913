// api.hip -- host side of the libtdgl C ABI (see include/tdgl.h).
//
// The host validates parameters, lays out the caller's workspace, builds the
// small coefficient tables of the multigrid hierarchy in double precision,
// and enqueues the kernels of each step.  Convergence of the Jacobi and
// multigrid loops is decided on the device (every launch first checks the
// previous iteration's residual word and exits when the solve has
// finished); the host only decides how many launches to enqueue, reading the
// residual words one iteration behind the device so that the GPU never waits
// for the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "tdgl.h"

using namespace tdgl;

namespace {

thread_local std::string g_err;

tdgl_status fail(tdgl_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(TDGL_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

#define LAUNCHCHK()                                                                    \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return fail(TDGL_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr float kOmega = 6.0f / 7.0f;  // smoother damping (pseudo time step)
constexpr int kCoarsestMax = 4096;     // nodes the one-work-group coarse solve accepts

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// multigrid hierarchy (host description)
struct AxisLevel {
    int n = 0;
    bool per = false;
    std::vector<double> pos;  // node positions (open axes)
    std::vector<double> am, ap, vol;
    bool can = false;         // can be coarsened further
};

// One axis through all levels: periodic axes halve while even and >= 4;
// open axes keep nodes {0, 2, 4, ...} plus the last one while n >= 3.
std::vector<AxisLevel> axis_levels(int n, double h, bool per, double cf) {
    std::vector<AxisLevel> out;
    std::vector<double> pos(n);
    for (int i = 0; i < n; ++i) pos[i] = i * h;
    const double Lp = n * h;
    for (;;) {
        AxisLevel a;
        a.n = (int)pos.size();
        a.per = per;
        a.pos = pos;
        a.am.assign(a.n, 0.0);
        a.ap.assign(a.n, 0.0);
        a.vol.assign(a.n, 0.0);
        if (per) {
            const double hl = Lp / a.n;
            for (int i = 0; i < a.n; ++i) { a.am[i] = a.ap[i] = cf / (hl * hl); a.vol[i] = hl; }
            a.can = (a.n % 2 == 0) && a.n >= 4;
        } else {
            if (a.n == 1) {
                a.vol[0] = 1.0;
            } else {
                for (int i = 0; i < a.n; ++i) {
                    const double dm = i > 0 ? pos[i] - pos[i - 1] : 0.0;
                    const double dp = i < a.n - 1 ? pos[i + 1] - pos[i] : 0.0;
                    a.vol[i] = 0.5 * (dm + dp);
                    a.am[i] = dm > 0 ? cf / (dm * a.vol[i]) : 0.0;
                    a.ap[i] = dp > 0 ? cf / (dp * a.vol[i]) : 0.0;
                }
            }
            a.can = a.n >= 3;
        }
        out.push_back(a);
        if (!a.can) break;
        std::vector<double> np;
        if (per) {
            for (int i = 0; i < a.n; i += 2) np.push_back(pos[i]);
        } else {
            for (int i = 0; i < a.n; i += 2) np.push_back(pos[i]);
            if ((a.n - 1) % 2 != 0) np.push_back(pos[a.n - 1]);
        }
        pos = np;
    }
    return out;
}

// 1D transfer between a fine and a coarse axis level (coarse == fine when
// the axis is not coarsened at this level).
struct Transfer1D {
    std::vector<int> pk;    // 2 per fine index
    std::vector<float> pw;
    std::vector<int> rk;    // 3 per coarse index
    std::vector<float> rw;
};

Transfer1D make_transfer(const AxisLevel &f, const AxisLevel &c, bool coarsened) {
    Transfer1D t;
    const int nf = f.n, nc = c.n;
    std::vector<std::vector<std::pair<int, double>>> P(nf);  // fine -> (coarse, w)
    if (!coarsened) {
        for (int k = 0; k < nf; ++k) P[k].push_back({k, 1.0});
    } else if (f.per) {
        for (int k = 0; k < nf; ++k) {
            const int K = k / 2;
            if (k % 2 == 0) P[k].push_back({K, 1.0});
            else { P[k].push_back({K, 0.5}); P[k].push_back({(K + 1) % nc, 0.5}); }
        }
    } else {
        for (int k = 0; k < nf; ++k) {
            const double x = f.pos[k];
            int j = (int)(std::lower_bound(c.pos.begin(), c.pos.end(), x - 1e-12) - c.pos.begin());
            if (j < nc && std::fabs(c.pos[j] - x) < 1e-9) {
                P[k].push_back({j, 1.0});
            } else {
                const int K0 = j - 1, K1 = j;
                const double w1 = (x - c.pos[K0]) / (c.pos[K1] - c.pos[K0]);
                P[k].push_back({K0, 1.0 - w1});
                P[k].push_back({K1, w1});
            }
        }
    }
    t.pk.resize(2 * nf);
    t.pw.resize(2 * nf);
    for (int k = 0; k < nf; ++k) {
        t.pk[2 * k] = P[k][0].first;
        t.pw[2 * k] = (float)P[k][0].second;
        t.pk[2 * k + 1] = P[k].size() > 1 ? P[k][1].first : P[k][0].first;
        t.pw[2 * k + 1] = P[k].size() > 1 ? (float)P[k][1].second : 0.f;
    }
    // restriction R[K][k] = P[k][K] V_f[k] / V_c[K]
    std::vector<std::vector<std::pair<int, double>>> R(nc);
    for (int k = 0; k < nf; ++k)
        for (auto &e : P[k]) R[e.first].push_back({k, e.second * f.vol[k] / c.vol[e.first]});
    t.rk.resize(3 * nc);
    t.rw.resize(3 * nc);
    for (int K = 0; K < nc; ++K) {
        if (R[K].size() > 3) { /* cannot happen for factor-2 coarsening */ }
        for (int a = 0; a < 3; ++a) {
            if (a < (int)R[K].size()) { t.rk[3 * K + a] = R[K][a].first; t.rw[3 * K + a] = (float)R[K][a].second; }
            else { t.rk[3 * K + a] = R[K].empty() ? 0 : R[K][0].first; t.rw[3 * K + a] = 0.f; }
        }
    }
    return t;
}

struct LevelHost {
    int n[3];
    AxisLevel ax[3];
    Transfer1D tr[3];  // to the next coarser level
    long N;
};

struct Hierarchy {
    std::vector<LevelHost> lev;
    bool ok = true;
};

Hierarchy build_hierarchy(const tdgl_params &p) {
    Hierarchy H;
    const int ns[3] = {p.nx, p.ny, p.nz};
    const double hs[3] = {p.hx, p.hy, p.hz};
    const double cf[3] = {1.0, 1.0, 1.0 / (p.g * p.g)};
    std::vector<AxisLevel> A[3];
    for (int a = 0; a < 3; ++a) A[a] = axis_levels(ns[a], hs[a], p.bc[a] == TDGL_PERIODIC, cf[a]);
    int li[3] = {0, 0, 0};
    for (;;) {
        LevelHost L;
        for (int a = 0; a < 3; ++a) { L.ax[a] = A[a][li[a]]; L.n[a] = L.ax[a].n; }
        L.N = (long)L.n[0] * L.n[1] * L.n[2];
        bool can[3];
        bool any = false;
        for (int a = 0; a < 3; ++a) { can[a] = L.ax[a].can; any = any || can[a]; }
        if (!any || L.N <= 512 || (int)H.lev.size() == kMaxLevels - 1) {
            H.lev.push_back(L);
            break;
        }
        int nl[3];
        for (int a = 0; a < 3; ++a) {
            nl[a] = li[a] + (can[a] ? 1 : 0);
            L.tr[a] = make_transfer(A[a][li[a]], A[a][nl[a]], can[a]);
        }
        H.lev.push_back(L);
        for (int a = 0; a < 3; ++a) li[a] = nl[a];
    }
    if (H.lev.back().N > kCoarsestMax) H.ok = false;
    return H;
}

// Radix plan of an FFT length (radices 4, 2, 3, 5); false if n has another
// prime factor.
bool radix_plan(int n, int *rad, int *nrad) {
    int k = 0;
    while (n % 4 == 0 && k < 16) { rad[k++] = 4; n /= 4; }
    while (n % 2 == 0 && k < 16) { rad[k++] = 2; n /= 2; }
    while (n % 3 == 0 && k < 16) { rad[k++] = 3; n /= 3; }
    while (n % 5 == 0 && k < 16) { rad[k++] = 5; n /= 5; }
    *nrad = k;
    return n == 1;
}

// The direct spectral Poisson solve applies to periodic x and y, open z,
// FFT-friendly x and y sizes and nz within the z-solve's tile.
bool fft_eligible(const tdgl_params &p) {
    int r[16], k;
    return p.driven && p.poisson == 0 && p.bc[0] == TDGL_PERIODIC && p.bc[1] == TDGL_PERIODIC &&
           p.bc[2] == TDGL_OPEN && p.nz <= FFT_ZMAX && p.nx <= FFT_MAXN / 2 && p.ny <= FFT_MAXN &&
           radix_plan(p.nx, r, &k) && radix_plan(p.ny, r, &k);
}

// ---------------------------------------------------------------------------
// validation and layout
tdgl_status validate(const tdgl_params &p, int idx) {
    if (p.nx < 1 || p.ny < 1 || p.nz < 1)
        return fail(TDGL_EINVAL, "instance %d: grid sizes must be >= 1", idx);
    if ((long)p.nx * p.ny * p.nz >= (1L << 31))
        return fail(TDGL_EINVAL, "instance %d: nx*ny*nz must be < 2^31", idx);
    if (!(p.hx > 0) || !(p.hy > 0) || !(p.hz > 0))
        return fail(TDGL_EINVAL, "instance %d: mesh spacings must be > 0", idx);
    for (int a = 0; a < 3; ++a)
        if (p.bc[a] != TDGL_PERIODIC && p.bc[a] != TDGL_OPEN)
            return fail(TDGL_EINVAL, "instance %d: bc[%d] must be TDGL_PERIODIC or TDGL_OPEN", idx, a);
    if (!(p.g > 0) || !(p.u > 0) || !(p.dt > 0))
        return fail(TDGL_EINVAL, "instance %d: g, u and dt must be > 0", idx);
    if (!(p.tol > 0)) return fail(TDGL_EINVAL, "instance %d: tol must be > 0", idx);
    if (p.max_iter < 1 || p.max_iter > TDGL_MAX_ITER)
        return fail(TDGL_EINVAL, "instance %d: max_iter must be in [1, %d]", idx, TDGL_MAX_ITER);
    if (p.driven != 0 && p.driven != 1) return fail(TDGL_EINVAL, "instance %d: driven must be 0 or 1", idx);
    if (p.driven) {
        if (p.bc[0] == TDGL_OPEN)
            return fail(TDGL_EINVAL,
                        "instance %d: a current along x needs a periodic x axis (open x with driven=1)", idx);
        if (!(p.mu_tol > 0)) return fail(TDGL_EINVAL, "instance %d: mu_tol must be > 0", idx);
        if (!(p.mu_rtol >= 0 && p.mu_rtol < 1)) return fail(TDGL_EINVAL, "instance %d: mu_rtol must be in [0, 1)", idx);
        if (p.mu_max_cycles < 1 || p.mu_max_cycles > TDGL_MAX_CYCLES)
            return fail(TDGL_EINVAL, "instance %d: mu_max_cycles must be in [1, %d]", idx, TDGL_MAX_CYCLES);
        if (p.poisson != 0 && p.poisson != 1)
            return fail(TDGL_EINVAL, "instance %d: poisson must be 0 (auto) or 1 (multigrid)", idx);
        Hierarchy H = build_hierarchy(p);
        if (!fft_eligible(p) && !H.ok)
            return fail(TDGL_EINVAL,
                        "instance %d: the grid cannot be coarsened below %d nodes for the Poisson "
                        "multigrid (periodic axes need even sizes)", idx, kCoarsestMax);
    }
    if (p.tile_cz < 0 || p.tile_cz > 1024) return fail(TDGL_EINVAL, "instance %d: tile_cz out of range", idx);
    if (p.tile_rows != 0 && p.tile_rows != 1 && p.tile_rows != 2 && p.tile_rows != 4)
        return fail(TDGL_EINVAL, "instance %d: tile_rows must be 0, 1, 2 or 4", idx);
    if (p.strict != 0 && p.strict != 1) return fail(TDGL_EINVAL, "instance %d: strict must be 0 or 1", idx);
    if (!(p.noise_T >= 0 && std::isfinite(p.noise_T)))
        return fail(TDGL_EINVAL, "instance %d: noise_T must be finite and >= 0", idx);
    if (p.reserved0 != 0) return fail(TDGL_EINVAL, "instance %d: reserved fields must be zero", idx);
    for (size_t r = 0; r < sizeof(p.reserved) / sizeof(p.reserved[0]); ++r)
        if (p.reserved[r] != 0) return fail(TDGL_EINVAL, "instance %d: reserved fields must be zero", idx);
    return TDGL_OK;
}

int auto_chunk(long tiles_xy, int nz, int req) {
    if (req > 0) return std::min(req, nz);
    // about 1024 or more work-groups (four per CU) where the grid allows,
    // and z runs of at least two planes so the two halo planes a run
    // re-reads stay a bounded overhead
    long c = (long)nz * tiles_xy / 1024;
    c = std::max(2L, std::min(32L, c));
    return (int)std::min<long>(c, nz);
}

// Rows per thread of the stencil tiles, shared by every instance of a
// context (one launch covers them all): the first non-zero request, else 4.
int ctx_rows(int n, const tdgl_params *params) {
    for (int i = 0; i < n; ++i)
        if (params[i].tile_rows) return params[i].tile_rows;
    return 2;
}

// Largest stencil grid of one instance over every tiling (one row per
// thread, one-plane z runs): the partial-sum buffer is sized for it so that
// re-tiling allocates nothing.
long max_st_blocks(const tdgl_params &p) { return (long)cdiv(p.nx, TX) * cdiv(p.ny, 4) * p.nz; }

// Carves one context's workspace.  With base == nullptr only sizes are
// computed.  Fills the host copies of the device descriptors.
struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

struct InstHost {
    tdgl_params p;
    Inst d;
    Hierarchy H;
    int st_blocks = 0, flat_blocks = 0;
    int r4_blocks = 0;  // blocks of the four-row Poisson right-side pass
    float2 *edge_buf = nullptr;  // side copies of b/M for two-sweep super-tiles (Inst::edge when in use)
    int mg_blocks[kMaxLevels] = {0};
    int fx_blocks = 0, fy_blocks = 0, fz_blocks = 0;  // spectral Poisson passes
    double Bx = 0, Bz = 0, J = 0;
    double By = 0;
    bool yz = false;  // field in the yz plane (tdgl_set_field_yz)
    bool insulated = false;  // eps holds the cut shares of tdgl_set_insulators
};

// Stencil tiling of one instance: work-groups of 64 x 4 rows columns
// marching through z runs of `chunk` planes (chunk_req = 0: heuristic); the
// two-sweep super-tile kernel marches through z runs of its own
// (chunk2_req = 0: the stencil's).
void set_tiling(InstHost &h, int rows, int chunk_req, int chunk2_req, int tys) {
    Inst &d = h.d;
    const tdgl_params &p = h.p;
    d.rows = rows;
    d.tys = tys > 0 ? tys : tys_default(rows);
    d.tiles_x = cdiv(p.nx, TX);
    d.tiles_y = cdiv(p.ny, 4 * rows);
    const long txy = (long)d.tiles_x * d.tiles_y;
    d.chunk = auto_chunk(txy, p.nz, chunk_req);
    d.tiles_z = cdiv(p.nz, d.chunk);
    d.chunk2 = chunk2_req > 0 ? std::min(chunk2_req, p.nz) : d.chunk;
    d.tiles_z2 = cdiv(p.nz, d.chunk2);
    h.st_blocks = (int)(txy * d.tiles_z);
    // the four-row right-side tiling (the stencil's own when rows = 4)
    d.tiles_y4 = cdiv(p.ny, 16);
    const long txy4 = (long)d.tiles_x * d.tiles_y4;
    d.chunk4 = auto_chunk(txy4, p.nz, chunk_req);
    d.tiles_z4 = cdiv(p.nz, d.chunk4);
    h.r4_blocks = (int)(txy4 * d.tiles_z4);
}

}  // namespace

struct tdgl_ctx {
    int n = 0;
    std::vector<InstHost> inst;
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Inst *d_inst = nullptr;
    // prefix tables of the batched launches; multigrid ones per level:
    // "all" = instances that have level l, "mid" = instances for which level
    // l is not the coarsest (kMaxLevels * (n+1) each)
    int *d_pref_st = nullptr, *d_pref_flat = nullptr, *d_pref_mg = nullptr, *d_pref_mid = nullptr;
    int *d_pref_b = nullptr;  // blocks of the two-sweep boundary kernel per instance
    int *d_pref_i = nullptr;  // ... and of the interior (super-tile) kernel
    int *d_pref_sr = nullptr;  // ... and of the seam-ring pre-pass (seam2 instances)
    int *d_pref_r4 = nullptr;  // blocks of the four-row Poisson right-side pass
    int tot_b = 0, tot_i = 0, tot_sr = 0, tot_r4 = 0;
    int rhs_rows = 0;  // rows per thread of the Poisson right side (0: rows)
    int *d_np_st = nullptr, *d_np_flat = nullptr, *d_np_mg0 = nullptr;
    int *d_np_r4 = nullptr;  // per instance: blocks of the four-row right-side pass
    unsigned *d_res = nullptr, *d_mures = nullptr;
    unsigned *h_mures = nullptr;  // pinned copy of the Poisson rows
    // Jacobi convergence words handed over by the sweeps themselves (pinned,
    // mapped): word (row, inst) at h_pub[row * n + inst] for rows 0 ..
    // max_iter - 1, then the finalize kernel's iteration counts and last
    // residuals (2n words).  The high half of a word is the solve's sequence
    // number pub_seq.
    unsigned long long *h_pub = nullptr, *d_pub = nullptr;
    unsigned pub_seq = 0;
    bool pub_on = false;  // sweeps being launched belong to a host-driven solve
    int poll_lag = 1;     // launches between the newest one and the one whose row the host waits for
    int npad = 64;        // instance stride of a convergence row
    size_t row_words() const { return (size_t)NSLOT * npad; }
    // max over the slots of one polled row for one instance
    float host_row_max(const unsigned *rows, int row, int inst) const {
        unsigned m = 0;
        for (int s = 0; s < NSLOT; ++s) m = std::max(m, rows[((size_t)row * NSLOT + s) * npad + inst]);
        float f;
        memcpy(&f, &m, 4);
        return f;
    }
    std::vector<hipEvent_t> evc;
    int tot_st = 0, tot_flat = 0, tot_mg[kMaxLevels] = {0}, tot_mid[kMaxLevels] = {0};
    int nlev_max = 0;
    // spectral Poisson path: prefix tables of its three kernels and LDS sizes
    int *d_pref_fx = nullptr, *d_pref_fy = nullptr, *d_pref_fz = nullptr;
    int tot_fx = 0, tot_fy = 0, tot_fz = 0;
    size_t fx_lds = 0, fy_lds = 0, fz_lds = 0;
    int fz_nzmax = 0;  // deepest z over the instances: scan rows per lane of the z solve
    bool fx_p2 = true, fy_p2 = true;  // every spectral instance has power-of-two nx (ny)
    bool fx_long = false;             // some spectral instance has nx > FFT_X_PTS
    bool noisy = false;               // some instance has a Langevin term
    bool any_yz = false;              // some instance has a yz-plane field
    bool any_zseam = false;           // ... with By != 0 on a periodic z axis (single sweeps, no adjoint)
    bool any_fft = false, any_mg = false;
    bool any_driven = false;
    int max_iter = 1, max_cycles = 1;
    int rows = 2;     // stencil rows per thread
    bool nt = false;  // streaming (non-temporal) hints in the sweep and assemble passes
    bool fused = false;  // Jacobi sweeps after the first run as two-sweep passes
    // the last kHist sweep counts of every instance's host-driven solves
    // (0: time steps, 1: the adjoint's systems; -1 = none yet), from which
    // each solve picks the pass schedule with the fewer expected passes
    std::vector<int> sweep_hist[2];
    int hist_pos[2] = {0, 0};
    // sweep count of instance 0's last host-driven solve (-1: the host did
    // not see it: a persistent solve, or one decided on the device)
    int last_sweeps = -1;
    bool persist = false;  // the Jacobi solve as one cooperative launch
    int num_cu = 0;        // compute units of the device
    // captured step of tdgl_step_graph (rebuilt when the budget or the
    // tiling changes)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_budget = 0;
    hipStream_t cap_stream = nullptr;  // private stream the step is captured on
    // per-kernel-class timing (tdgl_profile_start/stop)
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> prof_pool;
    std::vector<std::pair<int, int>> prof_recs;  // (class, index of the first event of the pair)
    size_t prof_used = 0;
    long long prof_launches[TDGL_K_COUNT] = {0};
    double prof_ms[TDGL_K_COUNT] = {0};
};

namespace {

size_t layout(int n, const tdgl_params *params, char *base, tdgl_ctx *ctx) {
    Carver cv{base};
    std::vector<InstHost> local;
    std::vector<InstHost> &ih = ctx ? ctx->inst : local;
    ih.assign(n, InstHost());
    int max_iter = 1, max_cycles = 1;
    for (int i = 0; i < n; ++i) {
        max_iter = std::max(max_iter, params[i].max_iter);
        if (params[i].driven) max_cycles = std::max(max_cycles, params[i].mu_max_cycles);
    }
    // context-level arrays
    Inst *d_inst = cv.take<Inst>(n);
    int *pref_st = cv.take<int>(n + 1);
    int *pref_flat = cv.take<int>(n + 1);
    int *pref_mg = cv.take<int>((size_t)kMaxLevels * (n + 1));
    int *pref_mid = cv.take<int>((size_t)kMaxLevels * (n + 1));
    int *pref_fx = cv.take<int>(n + 1);
    int *pref_fy = cv.take<int>(n + 1);
    int *pref_fz = cv.take<int>(n + 1);
    int *pref_b = cv.take<int>(n + 1);
    int *pref_i = cv.take<int>(n + 1);
    int *pref_sr = cv.take<int>(n + 1);
    int *pref_r4 = cv.take<int>(n + 1);
    int *np_st = cv.take<int>(n);
    int *np_r4 = cv.take<int>(n);
    int *np_flat = cv.take<int>(n);
    int *np_mg0 = cv.take<int>(n);
    const int npad = (n + 63) / 64 * 64;
    unsigned *res = cv.take<unsigned>((size_t)max_iter * NSLOT * npad);
    unsigned *mures = cv.take<unsigned>((size_t)max_cycles * NSLOT * npad);
    for (int i = 0; i < n; ++i) {
        const tdgl_params &p = params[i];
        InstHost &h = ih[i];
        h.p = p;
        Inst &d = h.d;
        memset(&d, 0, sizeof d);
        d.nx = p.nx; d.ny = p.ny; d.nz = p.nz;
        const long N = (long)p.nx * p.ny * p.nz;
        d.N = (int)N;
        for (int a = 0; a < 3; ++a) d.per[a] = p.bc[a] == TDGL_PERIODIC;
        d.driven = p.driven;
        const bool dx = !(p.bc[0] == TDGL_OPEN && p.nx == 1), dy = !(p.bc[1] == TDGL_OPEN && p.ny == 1),
                   dz = !(p.bc[2] == TDGL_OPEN && p.nz == 1);
        d.cx = dx ? (float)(1.0 / (p.hx * p.hx)) : 0.f;
        d.cy = dy ? (float)(1.0 / (p.hy * p.hy)) : 0.f;
        d.cz = dz ? (float)(1.0 / (p.g * p.g * p.hz * p.hz)) : 0.f;
        const double S = (dx ? 1.0 / (p.hx * p.hx) : 0) + (dy ? 1.0 / (p.hy * p.hy) : 0) +
                         (dz ? 1.0 / (p.g * p.g * p.hz * p.hz) : 0);
        d.S2 = (float)(2.0 * S);
        d.ht2 = (float)(0.5 * p.dt / p.u);
        d.u = (float)p.u;
        d.tol = (float)p.tol;
        // Langevin amplitude (Sec. 3.1.2): zeta_max^2 = 3 T u / (2 dt hx hy hz)
        d.zeta_max = p.noise_T > 0 ? (float)std::sqrt(3.0 * p.noise_T * p.u / (2.0 * p.dt * p.hx * p.hy * p.hz))
                                   : 0.f;
        d.seed0 = (unsigned)(p.noise_seed & 0xffffffffull);
        d.seed1 = (unsigned)(p.noise_seed >> 32);
        d.mu_tol = (float)p.mu_tol;
        d.hx = p.hx; d.hy = p.hy; d.hz = p.hz; d.dt = p.dt;
        {
            auto wsum = [](int nn, bool open) { return open && nn > 1 ? nn - 1.0 : (double)nn; };
            d.w_sum = wsum(p.nx, p.bc[0] == TDGL_OPEN) * wsum(p.ny, p.bc[1] == TDGL_OPEN) *
                      wsum(p.nz, p.bc[2] == TDGL_OPEN);
        }
        d.psi[0] = cv.take<float2>(N);
        d.psi[1] = cv.take<float2>(N);
        d.bh = cv.take<float2>(N);
        d.dh = cv.take<float2>(N);
        h.edge_buf = cv.take<float2>((size_t)4 * cdiv(p.nx, TX) * p.ny * p.nz);
        d.eps = cv.take<float>(N);
        d.ux = cv.take<float2>(p.ny);
        d.uz = cv.take<float2>(p.ny);
        d.P = cv.take<float2>((size_t)p.nx * p.nz);
        d.wz = cv.take<float2>(p.nz);
        d.zs = cv.take<float2>(p.nx);
        d.btile = cv.take<int>((size_t)cdiv(p.nx, TX) * cdiv(p.ny, 4));  // room for any rows per thread
        if (p.bc[1] == TDGL_PERIODIC && p.ny % TYS_MIN == 0) d.sring = cv.take<float2>((size_t)2 * p.nz * p.nx);
        d.st = cv.take<DevState>(1);
        d.res = res ? res + i : nullptr;
        d.mures = mures ? mures + i : nullptr;
        d.rstride = npad;
        d.mu_rtol = (float)p.mu_rtol;
        d.max_iter = p.max_iter;
        d.mu_max_cycles = p.driven ? p.mu_max_cycles : 1;
        // stencil tiling
        set_tiling(h, ctx_rows(n, params), p.tile_cz, 0, 0);
        // longer runs per thread where the grid is large: a work-group's
        // fixed costs (descriptor loads, the FP64 reduction) are paid once
        // for more cells
        d.fcpt = (int)std::max<long>(JAV_CPT, std::min<long>(JAV_CPT_MAX, N / (256L * 2048) / 8 * 8));
        h.flat_blocks = cdiv(N, 256L * d.fcpt);
        int part_cap = (int)std::max<long>(max_st_blocks(p), h.flat_blocks);
        // multigrid
        if (p.driven) {
            h.H = build_hierarchy(p);
            if (fft_eligible(p)) h.H.lev.resize(1);  // level 0 arrays only
            d.nlev = (int)h.H.lev.size();
            for (int l = 0; l < d.nlev; ++l) {
                LevelHost &LH = h.H.lev[l];
                MGLevel &L = d.lev[l];
                L.nx = LH.n[0]; L.ny = LH.n[1]; L.nz = LH.n[2];
                L.N = (int)LH.N;
                for (int a = 0; a < 3; ++a) {
                    L.per[a] = LH.ax[a].per;
                    L.am[a] = cv.take<float>(LH.n[a]);
                    L.ap[a] = cv.take<float>(LH.n[a]);
                    L.vol[a] = cv.take<float>(LH.n[a]);
                }
                double vs = 1.0;
                for (int a = 0; a < 3; ++a) {
                    double s = 0;
                    for (double v : LH.ax[a].vol) s += v;
                    vs *= s;
                }
                L.vsum = vs;
                if (l == 0) {
                    L.rhs = cv.take<float>(N);
                    L.mu[0] = cv.take<float>(N);
                    L.mu[1] = cv.take<float>(N);
                    L.r = cv.take<float>(N);
                } else {
                    L.rhs = cv.take<float>(LH.N);
                    L.mu[0] = cv.take<float>(LH.N);
                    L.mu[1] = cv.take<float>(LH.N);
                    L.r = cv.take<float>(LH.N);
                }
                if (l + 1 < d.nlev) {
                    for (int a = 0; a < 3; ++a) {
                        L.pk[a] = cv.take<int>(2 * LH.n[a]);
                        L.pw[a] = cv.take<float>(2 * LH.n[a]);
                        L.rk[a] = cv.take<int>(3 * h.H.lev[l + 1].n[a]);
                        L.rw[a] = cv.take<float>(3 * h.H.lev[l + 1].n[a]);
                    }
                }
                const long mtxy = (long)cdiv(L.nx, MTX) * cdiv(L.ny, MTY);
                L.tiles_x = cdiv(L.nx, MTX);
                L.tiles_y = cdiv(L.ny, MTY);
                L.chunk = auto_chunk(mtxy, L.nz, 0);
                // a spectral instance uses its level-0 tiles only for the
                // mean of mu: z runs of at least one batch of loads (eight
                // planes), so that a batch of small instances does not
                // become a swarm of work-groups that each sum two planes
                if (l == 0 && fft_eligible(p)) L.chunk = std::min(L.nz, std::max(L.chunk, 8));
                L.tiles_z = cdiv(L.nz, L.chunk);
                h.mg_blocks[l] = (int)(mtxy * L.tiles_z);
            }
            d.mu = d.lev[0].mu[0];
            d.f = d.lev[0].rhs;
            if (fft_eligible(p)) {
                d.fft = 1;
                radix_plan(p.nx, d.xrad, &d.nxrad);
                radix_plan(p.ny, d.yrad, &d.nyrad);
                const int P = p.nx / 2 + 1;
                d.sp = fft_pitch(p.nx);
                d.spec = cv.take<float2>((size_t)p.nz * p.ny * d.sp);
                d.twx = cv.take<float2>(p.nx);
                d.twy = cv.take<float2>(p.ny);
                d.zip = cv.take<double>((size_t)p.ny * P * p.nz);
                {
                    // groups of fft_x_pairs row pairs; up to eight per
                    // work-group while at least 2048 groups' work remain
                    const long groups = cdiv((long)p.ny * p.nz, 2L * fft_x_pairs(p.nx));
                    d.fxg = (int)std::max(1L, std::min(8L, groups / 2048));
                    h.fx_blocks = (int)cdiv(groups, (long)d.fxg);
                }
                h.fy_blocks = fft_y_plan(p.nx, p.ny, p.nz).blocks;
                h.fz_blocks = p.nz <= FFT_ZSERIAL ? cdiv(p.ny * P, 256) : p.ny * cdiv(P, FFT_ZTK);
            }
            part_cap = std::max(part_cap, h.mg_blocks[0]);
        }
        d.part = cv.take<double>(part_cap);
        d.part_cap = part_cap;
    }
    if (ctx) {
        ctx->n = n;
        ctx->d_inst = d_inst;
        ctx->d_pref_st = pref_st;
        ctx->d_pref_flat = pref_flat;
        ctx->d_pref_mg = pref_mg;
        ctx->d_pref_mid = pref_mid;
        ctx->d_pref_fx = pref_fx;
        ctx->d_pref_fy = pref_fy;
        ctx->d_pref_fz = pref_fz;
        ctx->d_pref_b = pref_b;
        ctx->d_pref_i = pref_i;
        ctx->d_pref_sr = pref_sr;
        ctx->d_pref_r4 = pref_r4;
        ctx->d_np_st = np_st;
        ctx->d_np_r4 = np_r4;
        ctx->d_np_flat = np_flat;
        ctx->d_np_mg0 = np_mg0;
        ctx->d_res = res;
        ctx->d_mures = mures;
        ctx->npad = npad;
        ctx->rows = ctx_rows(n, params);
        // streaming hints by default when the sweep's arrays (32 B per node)
        // exceed the 256 MB last-level cache; tdgl_autotune measures it
        double bytes = 0.0;
        for (int i = 0; i < n; ++i) bytes += 32.0 * params[i].nx * params[i].ny * params[i].nz;
        ctx->nt = bytes > 256.0 * 1024 * 1024;
        ctx->max_iter = max_iter;
        ctx->max_cycles = max_cycles;
    }
    return cv.off;
}

tdgl_status check_ctx(tdgl_ctx *ctx, int inst) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (inst < 0 || inst >= ctx->n) return fail(TDGL_EINVAL, "instance index %d out of range [0, %d)", inst, ctx->n);
    return TDGL_OK;
}

int fill_grid(long n) { return (int)std::min<long>(std::max<long>(cdiv(n, 256), 1), 8192); }

tdgl_status upload_tables(tdgl_ctx *ctx) {
    for (int i = 0; i < ctx->n; ++i) {
        InstHost &h = ctx->inst[i];
        if (!h.p.driven) continue;
        for (int l = 0; l < h.d.nlev; ++l) {
            LevelHost &LH = h.H.lev[l];
            MGLevel &L = h.d.lev[l];
            for (int a = 0; a < 3; ++a) {
                std::vector<float> am(LH.ax[a].am.begin(), LH.ax[a].am.end());
                std::vector<float> ap(LH.ax[a].ap.begin(), LH.ax[a].ap.end());
                std::vector<float> vol(LH.ax[a].vol.begin(), LH.ax[a].vol.end());
                HIPCHK(hipMemcpy((void *)L.am[a], am.data(), am.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy((void *)L.ap[a], ap.data(), ap.size() * 4, hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy((void *)L.vol[a], vol.data(), vol.size() * 4, hipMemcpyHostToDevice));
                if (l + 1 < h.d.nlev) {
                    Transfer1D &t = LH.tr[a];
                    HIPCHK(hipMemcpy((void *)L.pk[a], t.pk.data(), t.pk.size() * 4, hipMemcpyHostToDevice));
                    HIPCHK(hipMemcpy((void *)L.pw[a], t.pw.data(), t.pw.size() * 4, hipMemcpyHostToDevice));
                    HIPCHK(hipMemcpy((void *)L.rk[a], t.rk.data(), t.rk.size() * 4, hipMemcpyHostToDevice));
                    HIPCHK(hipMemcpy((void *)L.rw[a], t.rw.data(), t.rw.size() * 4, hipMemcpyHostToDevice));
                }
            }
        }
    }
    // prefix tables
    const int n = ctx->n;
    std::vector<int> ps(n + 1, 0), pf(n + 1, 0), pm((size_t)kMaxLevels * (n + 1), 0),
        pmid((size_t)kMaxLevels * (n + 1), 0), pfx(n + 1, 0), pfy(n + 1, 0), pfz(n + 1, 0);
    std::vector<int> nps(n), npf(n), npm(n);
    for (int i = 0; i < n; ++i) {
        InstHost &h = ctx->inst[i];
        ps[i + 1] = ps[i] + h.st_blocks;
        pf[i + 1] = pf[i] + h.flat_blocks;
        nps[i] = h.st_blocks;
        npf[i] = h.flat_blocks;
        npm[i] = h.p.driven ? h.mg_blocks[0] : 0;
        const bool mg = h.p.driven && !h.d.fft;
        for (int l = 0; l < kMaxLevels; ++l) {
            const size_t o = (size_t)l * (n + 1) + i;
            // level 0 "all" also drives the mean of mu for every driven instance
            const int b = (h.p.driven && l < h.d.nlev && (mg || l == 0)) ? h.mg_blocks[l] : 0;
            const int bm = (mg && l + 1 < h.d.nlev) ? h.mg_blocks[l] : 0;
            pm[o + 1] = pm[o] + b;
            pmid[o + 1] = pmid[o] + bm;
        }
        pfx[i + 1] = pfx[i] + h.fx_blocks;
        pfy[i + 1] = pfy[i] + h.fy_blocks;
        pfz[i + 1] = pfz[i] + h.fz_blocks;
        ctx->noisy = ctx->noisy || h.d.zeta_max > 0.f;
        ctx->fz_nzmax = std::max(ctx->fz_nzmax, h.p.nz);
        if (h.d.fft) {
            ctx->any_fft = true;
            ctx->fx_lds = std::max(ctx->fx_lds, (size_t)(fft_x_pairs(h.p.nx) + 1) * h.p.nx * 8);
            ctx->fy_lds = std::max(ctx->fy_lds, ((size_t)fft_y_plan(h.p.nx, h.p.ny, h.p.nz).TK *
                                                      fft_y_stride(h.p.ny) + h.p.ny) * 8);
            ctx->fx_p2 = ctx->fx_p2 && (h.p.nx & (h.p.nx - 1)) == 0;
            ctx->fx_long = ctx->fx_long || h.p.nx > FFT_X_PTS;
            ctx->fy_p2 = ctx->fy_p2 && (h.p.ny & (h.p.ny - 1)) == 0;
            ctx->fz_lds = std::max(ctx->fz_lds, fft_z_lds(h.p.nz));
        } else if (h.p.driven) {
            ctx->any_mg = true;
        }
    }
    ctx->tot_st = ps[n];
    ctx->tot_flat = pf[n];
    for (int l = 0; l < kMaxLevels; ++l) {
        ctx->tot_mg[l] = pm[(size_t)l * (n + 1) + n];
        ctx->tot_mid[l] = pmid[(size_t)l * (n + 1) + n];
    }
    HIPCHK(hipMemcpy(ctx->d_pref_mid, pmid.data(), pmid.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_fx, pfx.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_fy, pfy.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_fz, pfz.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    ctx->tot_fx = pfx[n];
    ctx->tot_fy = pfy[n];
    ctx->tot_fz = pfz[n];
    if (ctx->any_fft) {
        for (const void *fn : {(const void *)k_fft_x<false, FFT_X_PTS>, (const void *)k_fft_x<true, FFT_X_PTS>,
                                (const void *)k_fft_x<false, 4 * FFT_X_PTS>, (const void *)k_fft_x<true, 4 * FFT_X_PTS>})
            HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->fx_lds));
        HIPCHK(hipFuncSetAttribute((const void *)k_fft_y<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)ctx->fy_lds));
        HIPCHK(hipFuncSetAttribute((const void *)k_fft_y<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)ctx->fy_lds));
        for (const void *fn : {(const void *)k_fft_zsolve<2>, (const void *)k_fft_zsolve<4>})
            HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->fz_lds));
    }
    HIPCHK(hipMemcpy(ctx->d_pref_st, ps.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_flat, pf.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_mg, pm.data(), pm.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_np_st, nps.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_np_flat, npf.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_np_mg0, npm.data(), n * 4, hipMemcpyHostToDevice));
    std::vector<Inst> di(n);
    for (int i = 0; i < n; ++i) di[i] = ctx->inst[i].d;
    HIPCHK(hipMemcpy(ctx->d_inst, di.data(), n * sizeof(Inst), hipMemcpyHostToDevice));
    return TDGL_OK;
}

const int *pref_mg(tdgl_ctx *c, int l) { return c->d_pref_mg + (size_t)l * (c->n + 1); }
const int *pref_mid(tdgl_ctx *c, int l) { return c->d_pref_mid + (size_t)l * (c->n + 1); }

// Resolve the recorded event pairs into the per-class sums (waits for the
// last recorded event).
tdgl_status prof_flush(tdgl_ctx *c) {
    if (c->prof_recs.empty()) return TDGL_OK;
    HIPCHK(hipEventSynchronize(c->prof_pool[c->prof_recs.back().second + 1]));
    for (auto &r : c->prof_recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->prof_pool[r.second], c->prof_pool[r.second + 1]));
        c->prof_ms[r.first] += ms;
        c->prof_launches[r.first] += 1;
    }
    c->prof_recs.clear();
    c->prof_used = 0;
    return TDGL_OK;
}

// Bracket one launch of kernel class `cls` (no-op unless profiled).
struct ProfScope {
    tdgl_ctx *c;
    int cls;
    int idx = -1;
    ProfScope(tdgl_ctx *c_, int cls_) : c(c_), cls(cls_) {
        if (!(c->prof_mask & (1u << cls))) return;
        if (c->prof_used + 2 > c->prof_pool.size()) prof_flush(c);
        idx = (int)c->prof_used;
        c->prof_used += 2;
        (void)hipEventRecord(c->prof_pool[idx], c->stream);
    }
    ~ProfScope() {
        if (idx < 0) return;
        (void)hipEventRecord(c->prof_pool[idx + 1], c->stream);
        c->prof_recs.push_back({cls, idx});
    }
};

// Launch one stencil pass over every instance with the context's tile
// (rows per thread; streaming hints for the sweep and assemble passes).
template <int MODE, int R>
void launch_stencil_r(tdgl_ctx *c, int l, const float2 *in, float2 *out) {
    constexpr bool can_nt = (MODE == MODE_SWEEP || is_first_mode(MODE));
    unsigned long long *pub = (MODE == MODE_SWEEP && c->pub_on && l > 0) ? c->d_pub : nullptr;
    // a yz-plane field takes the variant with per-plane x links
    if (c->any_yz) {
        if (can_nt && c->nt)
            hipLaunchKernelGGL((k_stencil<MODE, R, can_nt, true>), dim3(c->tot_st), dim3(WG), 0, c->stream,
                               c->d_inst, c->d_pref_st, c->n, l, in, out, pub, c->pub_seq);
        else
            hipLaunchKernelGGL((k_stencil<MODE, R, false, true>), dim3(c->tot_st), dim3(WG), 0, c->stream,
                               c->d_inst, c->d_pref_st, c->n, l, in, out, pub, c->pub_seq);
    } else if (can_nt && c->nt) {
        hipLaunchKernelGGL((k_stencil<MODE, R, can_nt, false>), dim3(c->tot_st), dim3(WG), 0, c->stream, c->d_inst,
                           c->d_pref_st, c->n, l, in, out, pub, c->pub_seq);
    } else {
        hipLaunchKernelGGL((k_stencil<MODE, R, false, false>), dim3(c->tot_st), dim3(WG), 0, c->stream, c->d_inst,
                           c->d_pref_st, c->n, l, in, out, pub, c->pub_seq);
    }
}
template <int R, bool NT, bool YZ>
void launch_sweep2_v(tdgl_ctx *c, int l, unsigned long long *pub) {
    if (c->tot_b > 0)
        hipLaunchKernelGGL((k_sweep2<R, NT, YZ>), dim3(c->tot_b), dim3(WG), 0, c->stream, c->d_inst, c->d_pref_b,
                           c->n, l, pub, c->pub_seq);
    if (c->tot_i > 0) {
        // the super-tiles on the quasi-periodic seam read their ring slots
        // beyond it from this pre-pass
        if (c->tot_sr > 0)
            hipLaunchKernelGGL((k_seam_ring<YZ>), dim3(c->tot_sr), dim3(256), 0, c->stream, c->d_inst, c->d_pref_sr,
                               c->n, l);
        const int tys = c->inst[0].d.tys;
        if constexpr (R > 1) {
            if (tys == 32) {
                hipLaunchKernelGGL((k_sweep2i<R, NT, YZ, 32>), dim3(c->tot_i), dim3(WG * sweep2i_mult(R, 32)), 0,
                                   c->stream, c->d_inst, c->d_pref_i, c->n, l, pub, c->pub_seq);
                return;
            }
        }
        hipLaunchKernelGGL((k_sweep2i<R, NT, YZ, 16>), dim3(c->tot_i), dim3(WG * sweep2i_mult(R, 16)), 0,
                           c->stream, c->d_inst, c->d_pref_i, c->n, l, pub, c->pub_seq);
    }
}
// One two-sweep pass (l odd; l = -1: timing pass).
template <int R>
void launch_sweep2_r(tdgl_ctx *c, int l) {
    // boundary tiles by the general kernel (which also hands the rows
    // over), then interior super-tiles by the plain-load kernel.  The two
    // write disjoint tiles and read only psi^(l), b/M and (ht/2)/M; run
    // side by side on two streams they were slower than in sequence, the
    // boundary groups taking CU slots from the interior kernel for longer
    // than the boundary kernel takes alone.  Either grid can be empty (no
    // boundary tiles when super-tiles cover every tile, no super-tile on
    // grids too small for one); an instance without boundary tiles hands its
    // rows over from the interior kernel.  YZ: a yz-plane field in the
    // context (per-plane x-link factor).
    unsigned long long *pub = (c->pub_on && l > 0) ? c->d_pub : nullptr;
    if (c->any_yz) {
        if (c->nt) launch_sweep2_v<R, true, true>(c, l, pub);
        else launch_sweep2_v<R, false, true>(c, l, pub);
    } else {
        if (c->nt) launch_sweep2_v<R, true, false>(c, l, pub);
        else launch_sweep2_v<R, false, false>(c, l, pub);
    }
}
void launch_sweep2(tdgl_ctx *c, int l) {
    if (c->rows == 1) launch_sweep2_r<1>(c, l);
    else if (c->rows == 2) launch_sweep2_r<2>(c, l);
    else launch_sweep2_r<4>(c, l);
}

// The whole Jacobi solve (sweeps 1 .. max_iter-1 of every instance) as one
// cooperative launch: as many work-groups as can be resident at once (a
// multiple of 8 for the XCD-aware tile order), never more than tiles.
// l0 = -1: lcap timing sweeps instead (state untouched).
template <int R, bool NT>
tdgl_status launch_persist_r(tdgl_ctx *c, int l0, int lcap) {
    const void *fn = (const void *)k_jacobi_persist<R, NT>;
    int per_cu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WG, 0));
    if (per_cu < 1) return fail(TDGL_EDEVICE, "the persistent Jacobi kernel cannot be resident");
    int grid = std::min(per_cu * c->num_cu, c->tot_st);
    if (grid >= 8) grid -= grid % 8;
    grid = std::max(grid, 1);
    const Inst *ins = c->d_inst;
    const int *pref = c->d_pref_st;
    int n = c->n, nt = c->tot_st;
    void *args[] = {(void *)&ins, (void *)&pref, (void *)&n, (void *)&l0, (void *)&lcap, (void *)&nt};
    HIPCHK(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(WG), args, 0, c->stream));
    return TDGL_OK;
}
tdgl_status launch_persist(tdgl_ctx *c, int l0, int lcap) {
    if (c->rows == 1)
        return c->nt ? launch_persist_r<1, true>(c, l0, lcap) : launch_persist_r<1, false>(c, l0, lcap);
    if (c->rows == 2)
        return c->nt ? launch_persist_r<2, true>(c, l0, lcap) : launch_persist_r<2, false>(c, l0, lcap);
    return c->nt ? launch_persist_r<4, true>(c, l0, lcap) : launch_persist_r<4, false>(c, l0, lcap);
}

template <int MODE>
void launch_stencil(tdgl_ctx *c, int l, const float2 *in = nullptr, float2 *out = nullptr) {
    if (c->rows == 1) launch_stencil_r<MODE, 1>(c, l, in, out);
    else if (c->rows == 2) launch_stencil_r<MODE, 2>(c, l, in, out);
    else launch_stencil_r<MODE, 4>(c, l, in, out);
}
// The Poisson right-side pass: with the context's tile, or on 64 x 16
// tiles with four rows per thread (its own block table) when the tiling
// asks for them.
void launch_rhs(tdgl_ctx *c) {
    if (c->rhs_rows != 4) {
        launch_stencil<MODE_RHS>(c, 0);
        return;
    }
    if (c->any_yz)
        hipLaunchKernelGGL((k_stencil<MODE_RHS, 4, false, true>), dim3(c->tot_r4), dim3(WG), 0, c->stream,
                           c->d_inst, c->d_pref_r4, c->n, 0, nullptr, nullptr, nullptr, 0u);
    else
        hipLaunchKernelGGL((k_stencil<MODE_RHS, 4, false, false>), dim3(c->tot_r4), dim3(WG), 0, c->stream,
                           c->d_inst, c->d_pref_r4, c->n, 0, nullptr, nullptr, nullptr, 0u);
}

// Per-instance counts of the partial sums the right-side pass writes.
const int *rhs_parts(const tdgl_ctx *c) { return c->rhs_rows == 4 ? c->d_np_r4 : c->d_np_st; }

// The assemble pass, with the Langevin draws where some instance has them.
void launch_assemble(tdgl_ctx *c, int l = 0) {
    if (c->noisy)
        launch_stencil<MODE_FIRSTN>(c, l);
    else
        launch_stencil<MODE_FIRST>(c, l);
}

// One multigrid V-cycle for every driven instance (cycle index cyc).
// Instances may have hierarchies of different depth: each per-level launch
// covers only the instances the operation applies to (prefix tables with
// zero blocks for the others), and the one-group coarse solve runs every
// instance on its own coarsest level.  Per instance and level the sequence
// is V(2,2) with damped-Jacobi smoothing; the finest level starts a cycle
// with its residual (the convergence test) and ends it with four sweeps.
tdgl_status enqueue_vcycle(tdgl_ctx *c, int cyc) {
    hipStream_t s = c->stream;
    const int n = c->n;
    const int L = c->nlev_max;
    auto grid = [](int b) { return dim3(std::max(b, 1)); };
    {
        ProfScope ps(c, TDGL_K_MG_FINE);
        hipLaunchKernelGGL(k_mg_residual, grid(c->tot_mg[0]), dim3(256), 0, s, c->d_inst, pref_mg(c, 0), n, 0,
                           0, cyc);
    }
    for (int l = 0; l + 1 < L; ++l) {
        ProfScope ps(c, TDGL_K_MG_COARSE);
        if (l >= 1) {
            hipLaunchKernelGGL(k_mg_smooth, grid(c->tot_mid[l]), dim3(256), 0, s, c->d_inst, pref_mid(c, l), n,
                               l, 0, 1, cyc, kOmega);
            hipLaunchKernelGGL(k_mg_residual, grid(c->tot_mid[l]), dim3(256), 0, s, c->d_inst, pref_mid(c, l),
                               n, l, 1, cyc);
        }
        // restrict into level l+1 for the instances that have it
        hipLaunchKernelGGL(k_mg_restrict, grid(c->tot_mg[l + 1]), dim3(256), 0, s, c->d_inst,
                           pref_mg(c, l + 1), n, l, cyc, kOmega);
    }
    {
        ProfScope ps(c, TDGL_K_MG_COARSE);
        hipLaunchKernelGGL(k_mg_coarsest, dim3(n), dim3(CO_THREADS), 0, s, c->d_inst, n, cyc);
    }
    for (int l = L - 2; l >= 0; --l) {
        ProfScope ps(c, l == 0 ? TDGL_K_MG_FINE : TDGL_K_MG_COARSE);
        const int ifine = (l == 0) ? 0 : 1;
        hipLaunchKernelGGL(k_mg_prolong, grid(c->tot_mid[l]), dim3(256), 0, s, c->d_inst, pref_mid(c, l), n, l,
                           ifine, cyc);
        const int nsm = (l == 0) ? 4 : 2;
        for (int it = 0; it < nsm; ++it) {
            const int a = (l == 0) ? (it & 1) : ((it & 1) ^ 1);
            hipLaunchKernelGGL(k_mg_smooth, grid(c->tot_mid[l]), dim3(256), 0, s, c->d_inst, pref_mid(c, l), n,
                               l, a, a ^ 1, cyc, kOmega);
        }
    }
    LAUNCHCHK();
    return TDGL_OK;
}

// Contexts with fewer nodes than this keep two sweep launches in flight.
constexpr long long kPollLag2Nodes = 4ll << 20;

// Host wait for the word of this solve at w: spins on the pinned word and,
// now and then, asks whether the stream has drained or failed, so a word
// that can no longer come ends in an error instead of a hang.
tdgl_status wait_pub(tdgl_ctx *ctx, const unsigned long long *w, unsigned *bits) {
    for (unsigned it = 1;; ++it) {
        const unsigned long long v = __atomic_load_n(w, __ATOMIC_ACQUIRE);
        if ((unsigned)(v >> 32) == ctx->pub_seq) {
            *bits = (unsigned)v;
            return TDGL_OK;
        }
        if ((it & 255u) == 0u) {
            const hipError_t q = hipStreamQuery(ctx->stream);
            if (q == hipSuccess) {
                const unsigned long long v2 = __atomic_load_n(w, __ATOMIC_ACQUIRE);
                if ((unsigned)(v2 >> 32) == ctx->pub_seq) {
                    *bits = (unsigned)v2;
                    return TDGL_OK;
                }
                return fail(TDGL_EDEVICE, "a convergence word was never handed over");
            }
            if (q != hipErrorNotReady) return fail(TDGL_EDEVICE, "HIP error: %s", hipGetErrorString(q));
        }
        __builtin_ia32_pause();
    }
}

constexpr int kHist = 4;

// Passes (corrective sweep included) a solve of s sweeps costs under
// schedule 1 (two-sweep passes from l = 1) or 2 (one single sweep, then
// two-sweep passes from l = 2): a solve that ends on the first sweep of a
// pair pays a corrective single sweep.
int sched_cost(int sched, int s) {
    if (sched == 1) return pass_count(1, s) + ((s > 1 && !(s & 1)) ? 1 : 0);
    return pass_count(2, s) + ((s > 1 && (s & 1)) ? 1 : 0);
}

// Pass schedule of the next two-sweep solve of kind `kind`: the one with
// the smaller cost over the recent sweep counts, weighted by the instances'
// node counts (schedule 1 without history).
int pick_schedule(tdgl_ctx *ctx, int kind) {
    const std::vector<int> &h = ctx->sweep_hist[kind];
    if ((int)h.size() != ctx->n * kHist) return 1;
    double c1 = 0.0, c2 = 0.0;
    for (int i = 0; i < ctx->n; ++i)
        for (int q = 0; q < kHist; ++q) {
            const int sw = h[(size_t)i * kHist + q];
            if (sw <= 0) continue;
            const double w = (double)ctx->inst[i].d.N;
            c1 += w * sched_cost(1, sw);
            c2 += w * sched_cost(2, sw);
        }
    return c2 < c1 ? 2 : 1;
}

// The Jacobi iterations after the first sweep (already enqueued, its input
// residual in row 0): sweep l reads row l-1 on the device and is a no-op
// for instances whose solve has ended.  The work-group of each instance's
// first tile also hands the row it read to pinned host memory, so row r
// reaches the host when the launch after the one that wrote it starts; the
// host waits for the rows of the launch poll_lag launches behind the newest
// and stops enqueueing once every instance has met its stop rule.  A row that
// no sweep hands over (an instance's cap row, the last rows before the
// context's cap) leaves that instance to the finalize kernel, which fixes the
// per-instance result buffer on the device (count_step: also advances the
// step counters) and hands its iteration count and last residual over;
// the host waits for those only when statistics or a strict stop need them.
tdgl_status jacobi_loop(tdgl_ctx *ctx, tdgl_step_stats *acc, bool *strict_fail, int count_step) {
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    if (ctx->persist) {
        // one launch, no host round trip; the statistics come from the
        // device counters (tdgl_step reads them)
        {
            ProfScope ps(ctx, TDGL_K_SWEEP);
            tdgl_status e = launch_persist(ctx, 1, ctx->max_iter);
            if (e) return e;
        }
        ProfScope ps(ctx, TDGL_K_OTHER);
        hipLaunchKernelGGL(k_solve_finalize, dim3(n), dim3(FIN_THREADS), 0, s, ctx->d_inst, n, count_step,
                           ctx->max_iter, 0, nullptr, 0u);
        LAUNCHCHK();
        ctx->last_sweeps = -1;
        return TDGL_OK;
    }
    ++ctx->pub_seq;
    ctx->pub_on = true;
    struct PubOff {  // sweeps launched after this loop hand nothing over
        tdgl_ctx *c;
        ~PubOff() { c->pub_on = false; }
    } pub_off{ctx};
    // per instance: the row that ended the solve (-1: undecided), or
    // deferred to the finalize kernel's report
    std::vector<int> conv_at(n, -1);
    std::vector<float> conv_r(n, 0.f);
    std::vector<char> deferred(n, 0);
    const int MI = ctx->max_iter;
    // start index of every launch so far (0: the assemble kernel); launch k
    // hands over the rows below starts[k] not handed over before
    std::vector<int> starts{0};
    starts.reserve(MI + 1);
    int remaining = n, launched = 1, polled = 0;
    // two-sweep passes from l = 1 (schedule 1) or after one single sweep
    // from l = 2 (schedule 2), whichever the recent sweep counts favour
    const int kind = count_step ? 0 : 1;
    const int sched = ctx->fused ? pick_schedule(ctx, kind) : 0;
    for (;;) {
        // rows handed over by launches at least poll_lag behind the newest
        // (all of them once no launch can follow)
        const int nk = (int)starts.size();
        const int kk = (launched >= MI) ? nk - 1 : nk - ctx->poll_lag;
        const int avail = (kk >= 1) ? starts[kk] : 0;  // rows < avail are handed over
        while (remaining > 0 && polled < avail) {
            for (int i = 0; i < n; ++i) {
                if (conv_at[i] >= 0 || deferred[i]) continue;
                const InstHost &h = ctx->inst[i];
                if (polled + 1 >= h.p.max_iter) {  // the cap row: no sweep hands it over
                    deferred[i] = 1;
                    --remaining;
                    continue;
                }
                unsigned bits;
                tdgl_status e = wait_pub(ctx, ctx->h_pub + (size_t)polled * n + i, &bits);
                if (e) return e;
                float r;
                memcpy(&r, &bits, 4);
                if (r < (float)h.p.tol) {
                    conv_at[i] = polled;
                    conv_r[i] = r;
                    --remaining;
                }
            }
            ++polled;
        }
        if (remaining == 0 || launched >= MI) break;
        const int l = launched;
        const bool pair = ctx->fused && !(sched == 2 && l == 1);
        const int nr = pair ? std::min(2, MI - l) : 1;
        {
            ProfScope ps(ctx, TDGL_K_SWEEP);
            if (pair) launch_sweep2(ctx, l);
            else launch_stencil<MODE_SWEEP>(ctx, l);
        }
        LAUNCHCHK();
        starts.push_back(l);
        launched += nr;
    }
    for (int i = 0; i < n; ++i)
        if (conv_at[i] < 0 && !deferred[i]) deferred[i] = 1;  // rows past the last hand-over
    unsigned long long *fin = ctx->d_pub + (size_t)MI * n;
    {
        ProfScope ps(ctx, TDGL_K_OTHER);
        hipLaunchKernelGGL(k_solve_finalize, dim3(n), dim3(FIN_THREADS), 0, s, ctx->d_inst, n, count_step,
                           launched, sched, fin, ctx->pub_seq);
        if (ctx->fused) launch_stencil<MODE_SWEEP>(ctx, -2);  // corrective sweep where needed
    }
    LAUNCHCHK();
    if (acc && sched == 2) acc->single_first_steps++;
    ctx->last_sweeps = deferred[0] ? -1 : conv_at[0] + 1;
    if (ctx->fused) {
        // sweep counts the host has seen (capped or deferred solves left out)
        std::vector<int> &h = ctx->sweep_hist[kind];
        if ((int)h.size() != n * kHist) h.assign((size_t)n * kHist, -1);
        const int q = ctx->hist_pos[kind];
        for (int i = 0; i < n; ++i) h[(size_t)i * kHist + q] = deferred[i] ? -1 : conv_at[i] + 1;
        ctx->hist_pos[kind] = (q + 1) % kHist;
    }
    bool need_strict = false;
    for (int i = 0; i < n; ++i) need_strict = need_strict || (deferred[i] && ctx->inst[i].p.strict);
    if (!acc && !(need_strict && strict_fail)) return TDGL_OK;
    for (int i = 0; i < n; ++i) {
        const InstHost &h = ctx->inst[i];
        int sw;
        float r;
        if (!deferred[i]) {
            sw = conv_at[i] + 1;
            r = conv_r[i];
        } else {
            unsigned sb, rb;
            tdgl_status e = wait_pub(ctx, ctx->h_pub + (size_t)MI * n + i, &sb);
            if (!e) e = wait_pub(ctx, ctx->h_pub + (size_t)MI * n + n + i, &rb);
            if (e) return e;
            sw = (int)sb;
            memcpy(&r, &rb, 4);
        }
        const bool capped = !(r < (float)h.p.tol);
        if (capped && h.p.strict && strict_fail) *strict_fail = true;
        if (!acc) continue;
        acc->sweep_passes += pass_count(sched, sw);
        acc->sweeps_min = std::min(acc->sweeps_min, sw);
        acc->sweeps_max = std::max(acc->sweeps_max, sw);
        acc->sweeps_sum += sw;
        acc->last_res2 = r;
        if (capped) acc->capped_steps++;
    }
    return TDGL_OK;
}

// Solve the Poisson equation of every driven instance: right side I.f,
// solution into I.mu (level-0 mu[0]), then the weighted mean of mu.  Spectral
// instances take the five FFT / z-solve passes; multigrid instances take
// V-cycles until their stop rule, decided on the device and polled by the
// host one cycle behind.  Statistics are accumulated into acc.
// The five passes of the spectral solve for every instance that uses it.
tdgl_status enqueue_fft(tdgl_ctx *ctx) {
    if (!ctx->any_fft) return TDGL_OK;
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    ProfScope ps(ctx, TDGL_K_MG_FINE);
    const float *nf = nullptr;
    float *nm = nullptr;
    const dim3 gx(std::max(ctx->tot_fx, 1)), gy(std::max(ctx->tot_fy, 1)), bt(FFT_XY_THREADS), bx(FFT_X_THREADS);
    auto xpass = [&](int dir) {
        const void *fn = ctx->fx_long ? (ctx->fx_p2 ? (const void *)k_fft_x<true, 4 * FFT_X_PTS>
                                                    : (const void *)k_fft_x<false, 4 * FFT_X_PTS>)
                                      : (ctx->fx_p2 ? (const void *)k_fft_x<true, FFT_X_PTS>
                                                    : (const void *)k_fft_x<false, FFT_X_PTS>);
        const Inst *ins = ctx->d_inst;
        const int *pref = ctx->d_pref_fx;
        int nn = n, d = dir;
        void *args[] = {(void *)&ins, (void *)&pref, (void *)&nn, (void *)&d, (void *)&nf, (void *)&nm};
        (void)hipLaunchKernel(fn, gx, bx, args, ctx->fx_lds, s);
    };
    auto ypass = [&](int dir) {
        if (ctx->fy_p2) hipLaunchKernelGGL(k_fft_y<true>, gy, bt, ctx->fy_lds, s, ctx->d_inst, ctx->d_pref_fy, n, dir);
        else hipLaunchKernelGGL(k_fft_y<false>, gy, bt, ctx->fy_lds, s, ctx->d_inst, ctx->d_pref_fy, n, dir);
    };
    xpass(-1);
    ypass(-1);
    // up to 64 planes two rows per lane, else four (32-lane segments up to
    // 128 planes, 64-lane ones beyond)
    if (ctx->fz_nzmax <= 64)
        hipLaunchKernelGGL(k_fft_zsolve<2>, dim3(std::max(ctx->tot_fz, 1)), dim3(256), ctx->fz_lds, s, ctx->d_inst,
                           ctx->d_pref_fz, n);
    else
        hipLaunchKernelGGL(k_fft_zsolve<4>, dim3(std::max(ctx->tot_fz, 1)), dim3(256), ctx->fz_lds, s, ctx->d_inst,
                           ctx->d_pref_fz, n);
    ypass(+1);
    xpass(+1);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status enqueue_poisson(tdgl_ctx *ctx, tdgl_step_stats *acc) {
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    const size_t RW = ctx->row_words();
    tdgl_status fe = enqueue_fft(ctx);
    if (fe) return fe;
    std::vector<int> mconv_at(n, 0);
    if (ctx->any_mg) {
        int mrem = 0;
        for (int i = 0; i < n; ++i) {
            const InstHost &h = ctx->inst[i];
            if (h.p.driven && !h.d.fft) { ++mrem; mconv_at[i] = -1; }
        }
        int mlaunched = 0, mpolled = 0;
        for (;;) {
            while (mrem > 0 && (mpolled < mlaunched - 1 || mlaunched == ctx->max_cycles) && mpolled < mlaunched) {
                HIPCHK(hipEventSynchronize(ctx->evc[mpolled]));
                for (int i = 0; i < n; ++i) {
                    if (mconv_at[i] >= 0) continue;
                    const InstHost &h = ctx->inst[i];
                    const float r = ctx->host_row_max(ctx->h_mures, mpolled, i);
                    const float thr = std::max((float)h.p.mu_tol,
                                               (float)h.p.mu_rtol * ctx->host_row_max(ctx->h_mures, 0, i));
                    if (r < thr || mpolled + 1 >= h.p.mu_max_cycles) {
                        mconv_at[i] = mpolled;
                        --mrem;
                    }
                }
                ++mpolled;
            }
            if (mrem == 0 || mlaunched == ctx->max_cycles) break;
            tdgl_status e = enqueue_vcycle(ctx, mlaunched);
            if (e) return e;
            HIPCHK(hipMemcpyAsync(ctx->h_mures + (size_t)mlaunched * RW, ctx->d_mures + (size_t)mlaunched * RW,
                                  RW * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ctx->evc[mlaunched], s));
            ++mlaunched;
        }
    }
    {
        ProfScope ps(ctx, TDGL_K_OTHER);
        if (ctx->any_mg)
            hipLaunchKernelGGL(k_mg_finalize, dim3(n), dim3(FIN_THREADS), 0, s, ctx->d_inst, n, acc ? 1 : 0);
        hipLaunchKernelGGL(k_mu_mean_partial, dim3(std::max(ctx->tot_mg[0], 1)), dim3(256), 0, s, ctx->d_inst,
                           pref_mg(ctx, 0), n, 0);
        hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, s, ctx->d_inst, ctx->d_np_mg0, 1, 1);
    }
    LAUNCHCHK();
    if (acc && ctx->any_mg) {
        for (int i = 0; i < n; ++i) {
            const InstHost &h = ctx->inst[i];
            if (!h.p.driven || h.d.fft) continue;
            const float r = ctx->host_row_max(ctx->h_mures, mconv_at[i], i);
            const float thr = std::max((float)h.p.mu_tol,
                                       (float)h.p.mu_rtol * ctx->host_row_max(ctx->h_mures, 0, i));
            const bool capped = !(r < thr);
            acc->mu_cycles_sum += capped ? h.p.mu_max_cycles : mconv_at[i];
            if (capped) acc->mu_capped_steps++;
            acc->mu_last_res = r;
        }
    }
    return TDGL_OK;
}

// Releases the captured step (after a change of the launch sequence).
void drop_graph(tdgl_ctx *ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_budget = 0;
}

// Recompute whether some instance has a yz-plane field.  The stencil passes
// then take their per-plane x-link variants (the persistent solve has none
// and is switched off), and a captured step graph is dropped because its
// launches change.
void update_any_yz(tdgl_ctx *ctx) {
    bool any = false;
    bool zs = false;
    for (const auto &h : ctx->inst) {
        any = any || h.yz;
        zs = zs || (h.yz && h.By != 0.0 && h.p.bc[2] != TDGL_OPEN);
    }
    if (any != ctx->any_yz) drop_graph(ctx);
    ctx->any_yz = any;
    ctx->any_zseam = zs;
    if (any && ctx->persist) {
        drop_graph(ctx);
        ctx->persist = false;
    }
}

// One whole step of every instance as a fixed launch sequence with no host
// synchronisation, for graph capture: the assemble kernel and budget - 1
// sweep launches (a launch whose instance has converged or reached its cap
// exits at once; the finalize kernel picks the first converged sweep), the
// current and K update, the Poisson right side and a solve with every
// multigrid cycle launched (each instance's cycles stop by themselves).
tdgl_status enqueue_step_fixed(tdgl_ctx *ctx, int budget) {
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    launch_assemble(ctx);
    if (ctx->fused)
        for (int l = 1; l < budget; l += 2) launch_sweep2(ctx, l);
    else
        for (int l = 1; l < budget; ++l) launch_stencil<MODE_SWEEP>(ctx, l);
    hipLaunchKernelGGL(k_solve_finalize, dim3(n), dim3(FIN_THREADS), 0, s, ctx->d_inst, n, 1, budget,
                       ctx->fused ? 1 : 0, nullptr, 0u);
    if (ctx->fused) launch_stencil<MODE_SWEEP>(ctx, -2);
    LAUNCHCHK();
    if (!ctx->any_driven) return TDGL_OK;
    hipLaunchKernelGGL(k_jav_partial, dim3(ctx->tot_flat), dim3(256), 0, s, ctx->d_inst, ctx->d_pref_flat, n);
    hipLaunchKernelGGL(k_kupdate, dim3(n), dim3(256), 0, s, ctx->d_inst, ctx->d_np_flat);
    launch_rhs(ctx);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, s, ctx->d_inst, rhs_parts(ctx), 0, 1);
    LAUNCHCHK();
    tdgl_status e = enqueue_fft(ctx);
    if (e) return e;
    if (ctx->any_mg) {
        for (int cyc = 0; cyc < ctx->max_cycles; ++cyc) {
            e = enqueue_vcycle(ctx, cyc);
            if (e) return e;
        }
        hipLaunchKernelGGL(k_mg_finalize, dim3(n), dim3(FIN_THREADS), 0, s, ctx->d_inst, n, 1);
    }
    hipLaunchKernelGGL(k_mu_mean_partial, dim3(std::max(ctx->tot_mg[0], 1)), dim3(256), 0, s, ctx->d_inst,
                       pref_mg(ctx, 0), n, 0);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, s, ctx->d_inst, ctx->d_np_mg0, 1, 1);
    LAUNCHCHK();
    return TDGL_OK;
}

// defined with the tiling entry points below
tdgl_status upload_tiling(tdgl_ctx *ctx);

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

const char *tdgl_last_error(void) { return g_err.c_str(); }

tdgl_status tdgl_plan(int n, const tdgl_params *params, size_t *ws_bytes) {
    if (n < 1 || !params || !ws_bytes) return fail(TDGL_EINVAL, "tdgl_plan: need n >= 1 and non-null pointers");
    for (int i = 0; i < n; ++i) {
        tdgl_status s = validate(params[i], i);
        if (s) return s;
        if (params[i].tile_rows && params[i].tile_rows != ctx_rows(n, params))
            return fail(TDGL_EINVAL, "instances of one context must request the same tile_rows");
    }
    *ws_bytes = layout(n, params, nullptr, nullptr);
    return TDGL_OK;
}

tdgl_status tdgl_create(int n, const tdgl_params *params, void *ws, size_t ws_bytes, void *stream,
                        tdgl_ctx **out) {
    if (!out) return fail(TDGL_EINVAL, "tdgl_create: null output pointer");
    *out = nullptr;
    size_t need = 0;
    tdgl_status s = tdgl_plan(n, params, &need);
    if (s) return s;
    if (!ws || ((uintptr_t)ws % kAlign) != 0)
        return fail(TDGL_EWS, "tdgl_create: workspace missing or not %zu-byte aligned", kAlign);
    if (ws_bytes < need) return fail(TDGL_EWS, "tdgl_create: workspace has %zu bytes, needs %zu", ws_bytes, need);
    tdgl_ctx *c = new tdgl_ctx();
    c->ws = (char *)ws;
    c->ws_bytes = ws_bytes;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fail(TDGL_EDEVICE, "hipGetDevice failed"); }
    if (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        c->num_cu < 1) {
        delete c;
        return fail(TDGL_EDEVICE, "cannot read the number of compute units");
    }
    layout(n, params, (char *)ws, c);
    c->nlev_max = 0;
    for (auto &h : c->inst) {
        c->any_driven = c->any_driven || h.p.driven;
        if (!h.d.fft) c->nlev_max = std::max(c->nlev_max, h.d.nlev);
    }
    auto bail = [&](tdgl_status st) { tdgl_destroy(c); return st; };
    // sweeps of a few microseconds finish before the host has reacted to a
    // launch's start: keep one more launch queued for small contexts
    {
        long long nodes = 0;
        for (auto &h : c->inst) nodes += (long long)h.d.N;
        c->poll_lag = nodes < kPollLag2Nodes ? 2 : 1;
    }
    const size_t pub_words = ((size_t)c->max_iter + 2) * n;
    if (hipHostMalloc((void **)&c->h_pub, pub_words * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_mures, c->max_cycles * c->row_words() * 4, hipHostMallocDefault) !=
            hipSuccess)
        return bail(fail(TDGL_EDEVICE, "hipHostMalloc of the polling buffers failed"));
    memset(c->h_pub, 0, pub_words * 8);  // sequence 0 is never a solve's
    if (hipHostGetDevicePointer((void **)&c->d_pub, c->h_pub, 0) != hipSuccess)
        return bail(fail(TDGL_EDEVICE, "hipHostGetDevicePointer of the convergence words failed"));
    c->evc.resize(c->max_cycles);
    for (auto &e : c->evc)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(TDGL_EDEVICE, "hipEventCreate failed"));
    if ((s = upload_tables(c))) return bail(s);
    if ((s = upload_tiling(c))) return bail(s);
    // initial state: psi = 1, eps = 1, mu = 0, B = 0, K = 0
    hipStream_t st = c->stream;
    for (int i = 0; i < n; ++i) {
        Inst &d = c->inst[i].d;
        const long N = d.N;
        hipLaunchKernelGGL(k_fill_c, dim3(fill_grid(N)), dim3(256), 0, st, d.psi[0], N, 1.f, 0.f);
        hipLaunchKernelGGL(k_fill_c, dim3(fill_grid(N)), dim3(256), 0, st, d.psi[1], N, 1.f, 0.f);
        hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(N)), dim3(256), 0, st, d.eps, N, 1.f);
        if (d.driven)
            for (int l = 0; l < d.nlev; ++l) {
                MGLevel &L = d.lev[l];
                hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(L.N)), dim3(256), 0, st, L.mu[0], (long)L.N, 0.f);
                hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(L.N)), dim3(256), 0, st, L.mu[1], (long)L.N, 0.f);
                hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(L.N)), dim3(256), 0, st, L.rhs, (long)L.N, 0.f);
                hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(L.N)), dim3(256), 0, st, L.r, (long)L.N, 0.f);
            }
        HIPCHK(hipMemsetAsync(d.st, 0, sizeof(DevState), st));
        hipLaunchKernelGGL(k_acc_reset, dim3(1), dim3(64), 0, st, c->d_inst + i, 1);
        hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, st, c->d_inst, i, 11, 1.0);  // in window
    }
    hipLaunchKernelGGL(k_fill_u, dim3(64), dim3(256), 0, st, c->d_res, (long)(c->max_iter * c->row_words()), 0u);
    hipLaunchKernelGGL(k_fill_u, dim3(64), dim3(256), 0, st, c->d_mures, (long)(c->max_cycles * c->row_words()),
                       0u);
    hipLaunchKernelGGL(k_links, dim3(n), dim3(256), 0, st, c->d_inst, 0, (const double *)nullptr);
    for (int i = 0; i < n; ++i) {
        const tdgl_params &p = c->inst[i].p;
        if (!c->inst[i].d.fft) continue;
        const long cols = std::max<long>(std::max(p.nx, p.ny), (long)p.ny * (p.nx / 2 + 1));
        hipLaunchKernelGGL(k_fft_tables, dim3((unsigned)cdiv(cols, 256L)), dim3(256), 0, st, c->d_inst, i);
    }
    LAUNCHCHK();
    if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(TDGL_EDEVICE, "initialisation failed"));
    *out = c;
    return TDGL_OK;
}

tdgl_status tdgl_destroy(tdgl_ctx *ctx) {
    if (!ctx) return TDGL_OK;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->evc) if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->prof_pool) if (e) (void)hipEventDestroy(e);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->h_pub) (void)hipHostFree(ctx->h_pub);
    if (ctx->h_mures) (void)hipHostFree(ctx->h_mures);
    delete ctx;
    return TDGL_OK;
}

tdgl_status tdgl_size(const tdgl_ctx *ctx, int *n) {
    if (!ctx || !n) return fail(TDGL_EINVAL, "null argument");
    *n = ctx->n;
    return TDGL_OK;
}

tdgl_status tdgl_quantize_field(const tdgl_params *p, double Bx, double Bz, double *Bx_eff, double *Bz_eff) {
    if (!p || !Bx_eff || !Bz_eff) return fail(TDGL_EINVAL, "null argument");
    const double twopi = 6.283185307179586476925286766559;
    auto len = [](int n, double h, int bc) { return bc == TDGL_OPEN ? (n - 1) * h : n * h; };
    const double Lx = len(p->nx, p->hx, p->bc[0]), Ly = len(p->ny, p->hy, p->bc[1]),
                 Lz = len(p->nz, p->hz, p->bc[2]);
    if (p->bc[0] == TDGL_PERIODIC && p->bc[1] == TDGL_PERIODIC)
        Bz = twopi * std::nearbyint(Bz * Lx * Ly / twopi) / (Lx * Ly);
    if (p->bc[1] == TDGL_PERIODIC && p->bc[2] == TDGL_PERIODIC)
        Bx = twopi * std::nearbyint(Bx * Ly * Lz / twopi) / (Ly * Lz);
    *Bx_eff = Bx;
    *Bz_eff = Bz;
    return TDGL_OK;
}

tdgl_status tdgl_quantize_field_yz(const tdgl_params *p, double By, double Bz, double *By_eff, double *Bz_eff) {
    if (!p || !By_eff || !Bz_eff) return fail(TDGL_EINVAL, "null argument");
    const double twopi = 6.283185307179586476925286766559;
    auto len = [](int n, double h, int bc) { return bc == TDGL_OPEN ? (n - 1) * h : n * h; };
    const double Lx = len(p->nx, p->hx, p->bc[0]), Ly = len(p->ny, p->hy, p->bc[1]);
    if (p->bc[0] == TDGL_PERIODIC && p->bc[1] == TDGL_PERIODIC)
        Bz = twopi * std::nearbyint(Bz * Lx * Ly / twopi) / (Lx * Ly);
    if (p->bc[0] == TDGL_PERIODIC && p->bc[2] == TDGL_PERIODIC) {
        const double Lz = len(p->nz, p->hz, p->bc[2]);
        By = twopi * std::nearbyint(By * Lx * Lz / twopi) / (Lx * Lz);
    }
    *By_eff = By;
    *Bz_eff = Bz;
    return TDGL_OK;
}

tdgl_status tdgl_set_field_yz(tdgl_ctx *ctx, int inst, double By, double Bz, int quantize, double *By_eff,
                              double *Bz_eff) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!std::isfinite(By) || !std::isfinite(Bz)) return fail(TDGL_EINVAL, "field must be finite");
    InstHost &h = ctx->inst[inst];
    double qy, qz;
    tdgl_quantize_field_yz(&h.p, By, Bz, &qy, &qz);
    if (!quantize) {
        auto off = [](double a, double b) { return std::fabs(a - b) > 1e-9 * std::max(1.0, std::fabs(b)); };
        if (off(By, qy) || off(Bz, qz))
            return fail(TDGL_EINVAL,
                        "field (%.9g, %.9g) is not a whole number of flux quanta through the periodic "
                        "cross sections (nearest: %.9g, %.9g); pass quantize=1", By, Bz, qy, qz);
        qy = By;
        qz = Bz;
    }
    if (qy != 0.0 && h.p.bc[2] != TDGL_OPEN && ctx->fused)
        return fail(TDGL_EINVAL, "a yz-plane field with By != 0 on a periodic z axis needs single-sweep "
                                 "tiling (set fused = 0 first)");
    h.Bx = 0.0;
    h.By = qy;
    h.Bz = qz;
    h.yz = true;
    update_any_yz(ctx);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 8, 0.0);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 9, qz);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 13, qy);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 14, 1.0);
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, ctx->stream, ctx->d_inst + inst, 0, (const double *)nullptr);
    LAUNCHCHK();
    if (By_eff) *By_eff = qy;
    if (Bz_eff) *Bz_eff = qz;
    return TDGL_OK;
}

tdgl_status tdgl_set_field(tdgl_ctx *ctx, int inst, double Bx, double Bz, int quantize, double *Bx_eff,
                           double *Bz_eff) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!std::isfinite(Bx) || !std::isfinite(Bz)) return fail(TDGL_EINVAL, "field must be finite");
    double qx, qz;
    tdgl_quantize_field(&ctx->inst[inst].p, Bx, Bz, &qx, &qz);
    if (!quantize) {
        auto off = [](double a, double b) { return std::fabs(a - b) > 1e-9 * std::max(1.0, std::fabs(b)); };
        if (off(Bx, qx) || off(Bz, qz))
            return fail(TDGL_EINVAL,
                        "field (%.9g, %.9g) is not a whole number of flux quanta through the periodic "
                        "cross sections (nearest: %.9g, %.9g); pass quantize=1", Bx, Bz, qx, qz);
        qx = Bx;
        qz = Bz;
    }
    ctx->inst[inst].Bx = qx;
    ctx->inst[inst].Bz = qz;
    ctx->inst[inst].By = 0.0;
    ctx->inst[inst].yz = false;
    update_any_yz(ctx);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 8, qx);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 9, qz);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 13, 0.0);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 14, 0.0);
    // rebuild the tables of this instance only: launch over all with a
    // single-instance view (the kernel reads the descriptor by block index)
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, ctx->stream, ctx->d_inst + inst, 0, (const double *)nullptr);
    LAUNCHCHK();
    if (Bx_eff) *Bx_eff = qx;
    if (Bz_eff) *Bz_eff = qz;
    return TDGL_OK;
}

tdgl_status tdgl_set_current(tdgl_ctx *ctx, int inst, double J) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!std::isfinite(J)) return fail(TDGL_EINVAL, "current must be finite");
    if (J != 0.0 && !ctx->inst[inst].p.driven)
        return fail(TDGL_EINVAL, "instance %d is not driven (driven=0): only J_ext = 0 is allowed", inst);
    ctx->inst[inst].J = J;
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 7, J);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_set_eps(tdgl_ctx *ctx, int inst, const float *eps) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!eps) return fail(TDGL_EINVAL, "null eps");
    const Inst &d = ctx->inst[inst].d;
    HIPCHK(hipMemcpyAsync(d.eps, eps, (size_t)d.N * 4, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->inst[inst].insulated = false;
    return TDGL_OK;
}

tdgl_status tdgl_get_eps(tdgl_ctx *ctx, int inst, float *eps) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!eps) return fail(TDGL_EINVAL, "null eps");
    const Inst &d = ctx->inst[inst].d;
    HIPCHK(hipMemcpyAsync(eps, d.eps, (size_t)d.N * 4, hipMemcpyDeviceToDevice, ctx->stream));
    return TDGL_OK;
}

tdgl_status tdgl_gen_inclusions(tdgl_ctx *ctx, int inst, const double *centres, const double *diameters,
                                int nc, double target, float eps_in, float eps_out, int *n_used,
                                double *fraction) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    const Inst &d = ctx->inst[inst].d;
    if (nc < 0 || nc > d.N) return fail(TDGL_EINVAL, "candidate count must be in [0, N]");
    if (nc > 0 && (!centres || !diameters)) return fail(TDGL_EINVAL, "null candidate arrays");
    if (!(target >= 0.0 && target <= 1.0)) return fail(TDGL_EINVAL, "target fraction must be in [0, 1]");
    // scratch: first covering index (N words) and histogram (nc words) in bh
    unsigned *first = reinterpret_cast<unsigned *>(d.bh);
    unsigned *cnt = first + d.N;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_fill_u, dim3(fill_grid(d.N)), dim3(256), 0, st, first, (long)d.N, 0xffffffffu);
    if (nc > 0) {
        hipLaunchKernelGGL(k_fill_u, dim3(fill_grid(nc)), dim3(256), 0, st, cnt, (long)nc, 0u);
        hipLaunchKernelGGL(k_incl_first, dim3(nc), dim3(256), 0, st, ctx->d_inst, inst, centres, diameters, nc,
                           first);
        hipLaunchKernelGGL(k_incl_count, dim3(fill_grid(d.N)), dim3(256), 0, st, first, (long)d.N, nc, cnt);
    }
    hipLaunchKernelGGL(k_incl_scan, dim3(1), dim3(1024), 0, st, ctx->d_inst, inst, cnt, nc, target);
    hipLaunchKernelGGL(k_incl_write, dim3(fill_grid(d.N)), dim3(256), 0, st, ctx->d_inst, inst, first, eps_in,
                       eps_out);
    LAUNCHCHK();
    ctx->inst[inst].insulated = false;
    DevState h;
    HIPCHK(hipMemcpyAsync(&h, d.st, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (n_used) *n_used = h.n_used;
    if (fraction) *fraction = h.frac;
    return TDGL_OK;
}

tdgl_status tdgl_set_insulators(tdgl_ctx *ctx, int inst, const unsigned char *mask) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!mask) return fail(TDGL_EINVAL, "null mask");
    if (ctx->inst[inst].insulated)
        return fail(TDGL_ESTATE, "instance %d: eps already holds insulators; set eps (or generate it) again first",
                    inst);
    const Inst &d = ctx->inst[inst].d;
    hipLaunchKernelGGL(k_insulate, dim3(fill_grid(d.N)), dim3(256), 0, ctx->stream, ctx->d_inst, inst, mask);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->inst[inst].insulated = true;
    return TDGL_OK;
}

tdgl_status tdgl_gen_voronoi(tdgl_ctx *ctx, int inst, const double *seeds, const float *values, int ns,
                             int metric, int axes) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    const Inst &d = ctx->inst[inst].d;
    if (ns < 0) return fail(TDGL_EINVAL, "seed count must be >= 0");
    if (ns > 0 && (!seeds || !values)) return fail(TDGL_EINVAL, "null seed or value array");
    if (metric < 0 || metric > 2) return fail(TDGL_EINVAL, "metric must be 0 (Euclidean), 1 (absolute) or 2 (maximum)");
    if (axes < 1 || axes > 7) return fail(TDGL_EINVAL, "axes must be a non-empty mask of bits 1 (x), 2 (y), 4 (z)");
    if (ns == 0) return TDGL_OK;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_voronoi, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, st, ctx->d_inst, inst, seeds,
                       values, ns, metric, axes);
    LAUNCHCHK();
    ctx->inst[inst].insulated = false;
    HIPCHK(hipStreamSynchronize(st));
    return TDGL_OK;
}

tdgl_status tdgl_gen_shapes(tdgl_ctx *ctx, int inst, const double *shapes, int nc, double target, float eps_in,
                            float eps_out, int *n_used, double *fraction) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    const Inst &d = ctx->inst[inst].d;
    if (nc < 0 || nc > d.N) return fail(TDGL_EINVAL, "candidate count must be in [0, N]");
    if (nc > 0 && !shapes) return fail(TDGL_EINVAL, "null shape array");
    if (!(target >= 0.0 && target <= 1.0)) return fail(TDGL_EINVAL, "target fraction must be in [0, 1]");
    // scratch as for spheres: first covering index (N words), histogram (nc words)
    unsigned *first = reinterpret_cast<unsigned *>(d.bh);
    unsigned *cnt = first + d.N;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_fill_u, dim3(fill_grid(d.N)), dim3(256), 0, st, first, (long)d.N, 0xffffffffu);
    if (nc > 0) {
        hipLaunchKernelGGL(k_fill_u, dim3(fill_grid(nc)), dim3(256), 0, st, cnt, (long)nc, 0u);
        hipLaunchKernelGGL(k_incl_first_q, dim3(nc), dim3(256), 0, st, ctx->d_inst, inst, shapes, nc, first);
        hipLaunchKernelGGL(k_incl_count, dim3(fill_grid(d.N)), dim3(256), 0, st, first, (long)d.N, nc, cnt);
    }
    hipLaunchKernelGGL(k_incl_scan, dim3(1), dim3(1024), 0, st, ctx->d_inst, inst, cnt, nc, target);
    hipLaunchKernelGGL(k_incl_write, dim3(fill_grid(d.N)), dim3(256), 0, st, ctx->d_inst, inst, first, eps_in,
                       eps_out);
    LAUNCHCHK();
    ctx->inst[inst].insulated = false;
    DevState h;
    HIPCHK(hipMemcpyAsync(&h, d.st, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (n_used) *n_used = h.n_used;
    if (fraction) *fraction = h.frac;
    return TDGL_OK;
}

tdgl_status tdgl_set_psi(tdgl_ctx *ctx, int inst, const void *psi) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!psi) return fail(TDGL_EINVAL, "null psi");
    hipLaunchKernelGGL(k_psi_io, dim3(fill_grid(ctx->inst[inst].d.N)), dim3(256), 0, ctx->stream, ctx->d_inst,
                       inst, (float2 *)psi, 0);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_get_psi(tdgl_ctx *ctx, int inst, void *psi) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!psi) return fail(TDGL_EINVAL, "null psi");
    hipLaunchKernelGGL(k_psi_io, dim3(fill_grid(ctx->inst[inst].d.N)), dim3(256), 0, ctx->stream, ctx->d_inst,
                       inst, (float2 *)psi, 1);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_set_mu(tdgl_ctx *ctx, int inst, const float *mu) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!mu) return fail(TDGL_EINVAL, "null mu");
    if (!ctx->inst[inst].p.driven) return fail(TDGL_ESTATE, "instance %d is not driven: mu is identically 0", inst);
    hipLaunchKernelGGL(k_mu_io, dim3(fill_grid(ctx->inst[inst].d.N)), dim3(256), 0, ctx->stream, ctx->d_inst,
                       inst, (float *)mu, 0);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 10, 0.0);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_get_mu(tdgl_ctx *ctx, int inst, float *mu) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!mu) return fail(TDGL_EINVAL, "null mu");
    const Inst &d = ctx->inst[inst].d;
    if (!d.driven) {
        hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(d.N)), dim3(256), 0, ctx->stream, mu, (long)d.N, 0.f);
    } else {
        hipLaunchKernelGGL(k_mu_io, dim3(fill_grid(d.N)), dim3(256), 0, ctx->stream, ctx->d_inst, inst, mu, 1);
    }
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_get_scalars(tdgl_ctx *ctx, int inst, tdgl_scalars *sc) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!sc) return fail(TDGL_EINVAL, "null scalars");
    DevState h;
    HIPCHK(hipMemcpyAsync(&h, ctx->inst[inst].d.st, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    sc->K = h.K;
    sc->t = h.t;
    sc->V_sum = h.V_sum;
    sc->n = (long long)h.n;
    sc->n_avg = (long long)h.n_avg;
    sc->E_last = h.E_last;
    sc->J_av_last = h.J_last;
    return TDGL_OK;
}

tdgl_status tdgl_set_scalars(tdgl_ctx *ctx, int inst, const tdgl_scalars *sc) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!sc) return fail(TDGL_EINVAL, "null scalars");
    if (!ctx->inst[inst].p.driven && sc->K != 0.0) return fail(TDGL_EINVAL, "undriven instance: K must be 0");
    const double v[7] = {sc->K, sc->t, sc->V_sum, (double)sc->n, (double)sc->n_avg, sc->E_last, sc->J_av_last};
    for (int f = 0; f < 7; ++f)
        hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, f, v[f]);
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, ctx->stream, ctx->d_inst + inst, 1, (const double *)nullptr);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_voltage_window_reset(tdgl_ctx *ctx, int inst) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 2, 0.0);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, ctx->stream, ctx->d_inst, inst, 4, 0.0);
    LAUNCHCHK();
    return TDGL_OK;
}

tdgl_status tdgl_step(tdgl_ctx *ctx, int nsteps, tdgl_step_stats *stats) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (nsteps < 0) return fail(TDGL_EINVAL, "nsteps must be >= 0");
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    tdgl_step_stats acc;
    memset(&acc, 0, sizeof acc);
    acc.sweeps_min = 1 << 30;
    bool strict_fail = false;
    bool any_strict = false;
    for (int i = 0; i < n; ++i) any_strict = any_strict || ctx->inst[i].p.strict;
    const bool dev_stats = ctx->persist && (stats || any_strict);
    if (dev_stats) {
        hipLaunchKernelGGL(k_acc_reset, dim3(cdiv(n, 64)), dim3(64), 0, s, ctx->d_inst, n);
        LAUNCHCHK();
    }
    for (int step = 0; step < nsteps; ++step) {
        // ---- Jacobi solve (all instances) --------------------------------
        {
            ProfScope ps(ctx, TDGL_K_ASSEMBLE);
            launch_assemble(ctx);
        }
        LAUNCHCHK();
        tdgl_status e = jacobi_loop(ctx, &acc, &strict_fail, 1);
        if (e) return e;
        // ---- current, K and the scalar potential (driven instances) -------
        if (ctx->any_driven) {
            {
                ProfScope ps(ctx, TDGL_K_CURRENT);
                hipLaunchKernelGGL(k_jav_partial, dim3(ctx->tot_flat), dim3(256), 0, s, ctx->d_inst,
                                   ctx->d_pref_flat, n);
                hipLaunchKernelGGL(k_kupdate, dim3(n), dim3(256), 0, s, ctx->d_inst, ctx->d_np_flat);
            }
            {
                ProfScope ps(ctx, TDGL_K_RHS);
                launch_rhs(ctx);
                hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, s, ctx->d_inst, rhs_parts(ctx), 0, 1);
            }
            LAUNCHCHK();
            tdgl_status e = enqueue_poisson(ctx, &acc);
            if (e) return e;
        }
        acc.steps++;
        if (strict_fail) break;
    }
    if (dev_stats) {
        // persistent solves: the sweep statistics of the call from the
        // device counters; a strict instance's capped solve shows here
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) {
            DevState d;
            HIPCHK(hipMemcpy(&d, ctx->inst[i].d.st, sizeof d, hipMemcpyDeviceToHost));
            acc.sweeps_sum += (long long)d.acc_sweeps;
            acc.sweep_passes += (long long)d.acc_passes;
            acc.capped_steps += (int)d.acc_capped;
            acc.sweeps_min = std::min(acc.sweeps_min, d.acc_sw_min);
            acc.sweeps_max = std::max(acc.sweeps_max, d.acc_sw_max);
            acc.last_res2 = d.last_res2;
            if (ctx->inst[i].p.strict && d.acc_capped > 0) strict_fail = true;
        }
    }
    if (stats) {
        HIPCHK(hipStreamSynchronize(s));
        if (acc.steps == 0) acc.sweeps_min = 0;
        *stats = acc;
    }
    if (strict_fail) return fail(TDGL_ENOCONV, "a Jacobi solve reached max_iter without meeting tol");
    return TDGL_OK;
}

tdgl_status tdgl_step_graph(tdgl_ctx *ctx, int nsteps, int budget, tdgl_step_stats *stats) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (nsteps < 0) return fail(TDGL_EINVAL, "nsteps must be >= 0");
    if (budget < 1 || budget > ctx->max_iter)
        return fail(TDGL_EINVAL, "sweep budget must be in [1, %d] (the largest max_iter)", ctx->max_iter);
    if (ctx->prof_mask)
        return fail(TDGL_ESTATE, "per-kernel profiling is active; graph-replayed steps are not profiled");
    const int n = ctx->n;
    hipStream_t s = ctx->stream;
    if (!ctx->graph_exec || ctx->graph_budget != budget) {
        drop_graph(ctx);
        if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamSynchronize(s));
        ctx->stream = ctx->cap_stream;
        hipError_t be = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (be != hipSuccess) {
            ctx->stream = s;
            return fail(TDGL_EDEVICE, "hipStreamBeginCapture failed: %s", hipGetErrorString(be));
        }
        tdgl_status e = enqueue_step_fixed(ctx, budget);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
        ctx->stream = s;
        if (e || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return e ? e : fail(TDGL_EDEVICE, "step capture failed: %s", hipGetErrorString(ce));
        }
        hipGraphExec_t ge = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(TDGL_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
        }
        ctx->graph = g;
        ctx->graph_exec = ge;
        ctx->graph_budget = budget;
    }
    if (stats) {
        hipLaunchKernelGGL(k_acc_reset, dim3(cdiv(n, 64)), dim3(64), 0, s, ctx->d_inst, n);
        LAUNCHCHK();
    }
    for (int q = 0; q < nsteps; ++q) HIPCHK(hipGraphLaunch(ctx->graph_exec, s));
    if (stats) {
        HIPCHK(hipStreamSynchronize(s));
        tdgl_step_stats a;
        memset(&a, 0, sizeof a);
        a.steps = nsteps;
        a.sweeps_min = 1 << 30;
        for (int i = 0; i < n; ++i) {
            DevState d;
            HIPCHK(hipMemcpy(&d, ctx->inst[i].d.st, sizeof d, hipMemcpyDeviceToHost));
            a.sweeps_sum += (long long)d.acc_sweeps;
            a.sweep_passes += (long long)d.acc_passes;
            a.capped_steps += (int)d.acc_capped;
            a.mu_cycles_sum += (int)d.acc_mu_cycles;
            a.mu_capped_steps += (int)d.acc_mu_capped;
            a.sweeps_min = std::min(a.sweeps_min, d.acc_sw_min);
            a.sweeps_max = std::max(a.sweeps_max, d.acc_sw_max);
            a.last_res2 = d.last_res2;
            a.mu_last_res = d.mu_last_res;
        }
        if (nsteps == 0) a.sweeps_min = 0;
        *stats = a;
    }
    return TDGL_OK;
}

tdgl_status tdgl_poisson_solve(tdgl_ctx *ctx, const float *f, float *mu) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (ctx->n != 1) return fail(TDGL_EINVAL, "tdgl_poisson_solve needs a context with one instance");
    if (!f || !mu) return fail(TDGL_EINVAL, "null array");
    const Inst &d = ctx->inst[0].d;
    if (!d.driven) return fail(TDGL_ESTATE, "the instance is not driven: it has no Poisson solver");
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemcpyAsync(d.f, f, (size_t)d.N * 4, hipMemcpyDeviceToDevice, s));
    // weighted mean of f for the multigrid right side
    hipLaunchKernelGGL(k_mu_mean_partial, dim3(std::max(ctx->tot_mg[0], 1)), dim3(256), 0, s, ctx->d_inst,
                       pref_mg(ctx, 0), 1, 1);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(1), dim3(256), 0, s, ctx->d_inst, ctx->d_np_mg0, 4, 1);
    LAUNCHCHK();
    tdgl_status e = enqueue_poisson(ctx, nullptr);
    if (e) return e;
    hipLaunchKernelGGL(k_mu_io, dim3(fill_grid(d.N)), dim3(256), 0, s, ctx->d_inst, 0, mu, 1);
    LAUNCHCHK();
    return TDGL_OK;
}

}  // extern "C"

namespace {

// Re-uploads what a change of stencil tiling touches: the instance
// descriptors and the stencil prefix and partial-count tables.  The stream
// must be idle.
// Z planes per work-group of the two-sweep boundary kernel.  Measured at
// 1024 x 1024 x 128 (boundary kernel alone before the interior one): 1, 2,
// 4, 8, 16, 32 planes gave passes of 1057, 1007, 1001, 981, 1014, 1112 us.
constexpr int kBoundaryChunk = 8;

tdgl_status upload_tiling(tdgl_ctx *ctx) {
    const int n = ctx->n;
    std::vector<int> ps(n + 1, 0), nps(n), pb(n + 1, 0), pi(n + 1, 0), psr(n + 1, 0), pr4(n + 1, 0), npr4(n);
    std::vector<Inst> di(n);
    for (int i = 0; i < n; ++i) {
        InstHost &h = ctx->inst[i];
        Inst &d = h.d;
        // the 64 x 4R tiles of the super-tiles (M of them stacked in y) that
        // the plain-load two-sweep kernel does not take
        std::vector<int> bt;
        const int M = sweep2i_mult(d.rows, d.tys);
        d.seam2 = seam2_ok(d.per[1] != 0, d.ny, d.tys) ? 1 : 0;
        const bool seam = d.seam2 != 0;
        const int nsy = sweep2i_rows(d.ny, d.rows, d.tys, seam);
        for (int ty = 0; ty < d.tiles_y; ++ty)
            for (int tx = 0; tx < d.tiles_x; ++tx) {
                // tile row ty lies in super-tile row ty / M (seam2) or, one
                // tile row in, (ty - 1) / M
                const int tr = seam ? ty : ty - 1;
                const int j = tr / M;
                const bool inner = tr >= 0 && j < nsy &&
                                   tile_interior2(tx * TX, sweep2i_y0(j, d.rows, d.tys, seam), d.tys, d.nx, d.ny,
                                                  d.per[0] != 0, seam);
                if (!inner) bt.push_back(tx + d.tiles_x * ty);
            }
        pi[i + 1] = pi[i] + d.tiles_x * nsy * d.tiles_z2;
        // rows ny-1 and 0 of every plane, for the super-tiles on the seam
        psr[i + 1] = psr[i] + ((seam && nsy > 0) ? cdiv(2L * d.nz * d.nx, 256L) : 0);
        if (!bt.empty()) HIPCHK(hipMemcpy(d.btile, bt.data(), bt.size() * 4, hipMemcpyHostToDevice));
        d.nbt = (int)bt.size();
        d.bchunk = std::min(d.chunk, kBoundaryChunk);
        // side copies of b/M for the super-tiles' ring, addressed from bh and
        // dh with 32-bit offsets
        {
            const size_t esz = (size_t)4 * d.tiles_x * d.ny * d.nz;
            const bool fit = h.edge_buf > d.dh && d.dh > d.bh &&
                             (size_t)(h.edge_buf - d.bh) + esz < (size_t(1) << 32);
            d.edge = (ctx->fused && fit && nsy > 0) ? h.edge_buf : nullptr;
            d.edge_r = (unsigned)(esz / 2);
            d.edge_ob = fit ? (unsigned)(h.edge_buf - d.bh) : 0u;
            d.edge_od = fit ? (unsigned)(h.edge_buf - d.dh) : 0u;
        }
        ps[i + 1] = ps[i] + h.st_blocks;
        nps[i] = h.st_blocks;
        pr4[i + 1] = pr4[i] + h.r4_blocks;
        npr4[i] = h.r4_blocks;
        pb[i + 1] = pb[i] + d.nbt * cdiv(d.nz, d.bchunk);
        di[i] = d;
    }
    HIPCHK(hipMemcpy(ctx->d_pref_st, ps.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_np_st, nps.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_b, pb.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_i, pi.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_sr, psr.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pref_r4, pr4.data(), (n + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_np_r4, npr4.data(), n * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_inst, di.data(), n * sizeof(Inst), hipMemcpyHostToDevice));
    ctx->tot_st = ps[n];
    ctx->tot_b = pb[n];
    ctx->tot_i = pi[n];
    ctx->tot_sr = psr[n];
    ctx->tot_r4 = pr4[n];
    return TDGL_OK;
}

struct Tiling {
    int rows = 2;
    int chunk = 0;  // 0: heuristic
    int chunk2 = 0;  // z run of the two-sweep super-tile kernel; 0: chunk
    int nt = 0;       // streaming hints
    int fused = 0;    // two-sweep passes
    int persist = 0;  // one cooperative launch per Jacobi solve
    int rhs4 = 0;     // Poisson right side on 64 x 16 tiles (four rows per thread)
    int tys = 0;      // rows of the two-sweep super-tiles (0: tys_default(rows))
};

tdgl_status apply_tiling(tdgl_ctx *ctx, const Tiling &t) {
    drop_graph(ctx);
    ctx->rows = t.rows;
    ctx->rhs_rows = (t.rhs4 && t.rows != 4) ? 4 : 0;
    ctx->nt = t.nt != 0;
    ctx->fused = t.fused != 0 && !ctx->any_zseam;  // the two-sweep kernels have no z-seam phase
    ctx->persist = t.persist != 0 && !ctx->fused && !ctx->any_yz;
    for (auto &h : ctx->inst) set_tiling(h, t.rows, t.chunk, t.chunk2, t.tys);
    return upload_tiling(ctx);
}

// Key of a context's shape for the tiling cache: every instance's grid,
// boundary kinds and driven flag.
std::string tiling_key(const tdgl_ctx *ctx) {
    std::string k;
    char buf[96];
    for (const auto &h : ctx->inst) {
        snprintf(buf, sizeof buf, "%dx%dx%d/%d%d%d/%d%s;", h.p.nx, h.p.ny, h.p.nz, h.p.bc[0], h.p.bc[1], h.p.bc[2],
                 h.p.driven, h.yz ? "/yz" : "");
        k += buf;
    }
    return k;
}

std::mutex g_tune_mu;
std::map<std::string, std::pair<Tiling, double>> g_tune_cache;

bool tune_file_lookup(const char *path, const std::string &key, Tiling *t, double *us) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[4000];
        int r, c, nt, fu, pe, c2 = 0, r4 = 0, ty = 0;
        double u;
        // key rows chunk streaming fused persistent us [chunk2 [rhs4 [super-tile rows]]]
        const int got =
            sscanf(line, "%3999s %d %d %d %d %d %lf %d %d %d", k, &r, &c, &nt, &fu, &pe, &u, &c2, &r4, &ty);
        if (got >= 7 && key == k && (r == 1 || r == 2 || r == 4) && c >= 0 && c2 >= 0 &&
            (nt == 0 || nt == 1) && (fu == 0 || fu == 1) && (pe == 0 || pe == 1) && (r4 == 0 || r4 == 1) &&
            (ty == 0 || ty == 16 || (ty == 32 && r >= 2))) {
            t->rows = r;
            t->chunk = c;
            t->chunk2 = got >= 8 ? c2 : 0;
            t->rhs4 = got >= 9 ? r4 : 0;
            t->tys = got >= 10 ? ty : 0;
            t->nt = nt;
            t->fused = fu;
            t->persist = pe;
            *us = u;
            found = true;  // the last entry wins
        }
    }
    fclose(f);
    return found;
}

}  // namespace

extern "C" {

tdgl_status tdgl_autotune(tdgl_ctx *ctx, const char *cache_path, tdgl_tiling *chosen) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    hipStream_t s = ctx->stream;
    HIPCHK(hipStreamSynchronize(s));
    const std::string key = tiling_key(ctx);
    Tiling best;
    double best_us = 0.0;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best = it->second.first;
            best_us = it->second.second;
            have = true;
        }
    }
    if (!have) have = tune_file_lookup(cache_path, key, &best, &best_us);
    if (!have) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // z runs up to the deepest instance's whole z (a run re-reads the
        // planes around its ends); longer requests would repeat a candidate
        const int chunks[] = {0, 4, 8, 16, 32, 64, 128, 256};
        int nzmax = 1;
        for (const auto &h : ctx->inst) nzmax = std::max(nzmax, h.p.nz);
        const int rows[] = {1, 2, 4};
        best_us = 1e300;
        // single sweeps first: their best z run per (streaming, rows) is
        // also the z run of the stencil passes (assemble, Poisson right
        // side, single sweeps) under the two-sweep candidates, which vary
        // only the super-tile kernel's own z run
        int stencil_chunk[2][5] = {};
        double stencil_us[2][5];
        for (auto &a : stencil_us) for (double &v : a) v = 1e300;
        for (int fu = 0; fu < 2; ++fu)
        for (int nt = 0; nt < 2; ++nt)
        for (int r : rows)
        for (int c : chunks)
            for (int ty : {0, 16, 32}) {
                if (c > 4 && c / 2 >= nzmax) continue;
                // super-tile heights are a two-sweep notion; 32 rows need R >= 2
                if ((fu == 0) != (ty == 0) || (ty == 32 && r == 1)) continue;
                // the two-sweep kernels have no z-seam phase
                if (fu && ctx->any_zseam) continue;
                Tiling t;
                t.rows = r;
                t.chunk = fu ? stencil_chunk[nt][r] : c;
                t.chunk2 = fu ? std::max(c, 1) : 0;
                if (fu && c == 0) continue;  // the heuristic z run is a single-sweep notion
                t.nt = nt;
                t.fused = fu;
                t.tys = ty;
                tdgl_status e = apply_tiling(ctx, t);
                if (e) return e;
                auto pass = [&]() {
                    if (fu) launch_sweep2(ctx, -1);
                    else launch_stencil<MODE_SWEEP>(ctx, -1);
                };
                pass();  // warm-up
                HIPCHK(hipEventRecord(e0, s));
                const int reps = 4;
                for (int q = 0; q < reps; ++q) pass();
                HIPCHK(hipEventRecord(e1, s));
                LAUNCHCHK();
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                // time per Jacobi iteration (a two-sweep pass makes two)
                const double us = 1e3 * ms / reps / (fu ? 2 : 1);
                if (!fu && us < stencil_us[nt][r]) {
                    stencil_us[nt][r] = us;
                    stencil_chunk[nt][r] = c;
                }
                if (us < best_us) {
                    best_us = us;
                    best = t;
                }
            }
        // two-sweep passes: the stencil passes that remain (the assemble
        // every step, the Poisson right side, an occasional single sweep)
        // take the z run under which the assemble is fastest
        if (best.fused) {
            double best_a = 1e300;
            int best_c = best.chunk;
            for (int c : chunks) {
                if (c > 4 && c / 2 >= nzmax) continue;
                Tiling t = best;
                t.chunk = c;
                tdgl_status e = apply_tiling(ctx, t);
                if (e) return e;
                launch_assemble(ctx, -1);  // warm-up
                HIPCHK(hipEventRecord(e0, s));
                const int reps = 4;
                for (int q = 0; q < reps; ++q) launch_assemble(ctx, -1);
                HIPCHK(hipEventRecord(e1, s));
                LAUNCHCHK();
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_a) {
                    best_a = ms;
                    best_c = c;
                }
            }
            best.chunk = best_c;
        }
        // the best single-sweep tiling as one persistent launch: chosen when
        // its sweeps, barrier included, beat separate launches by 10 %
        if (!best.fused && !ctx->any_yz) {
            tdgl_status e = apply_tiling(ctx, best);
            if (e) return e;
            const int K = 16;
            e = launch_persist(ctx, -1, K);  // warm-up
            if (e) return e;
            HIPCHK(hipEventRecord(e0, s));
            e = launch_persist(ctx, -1, K);
            if (e) return e;
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            const double pus = 1e3 * ms / K;
            if (pus < 0.9 * best_us) {
                best.persist = 1;
                best_us = pus;
            }
        }
        // the Poisson right side on the chosen tile or on 64 x 16 tiles with
        // four rows per thread, whichever runs faster
        bool any_driven = false;
        for (const auto &h : ctx->inst) any_driven = any_driven || h.p.driven;
        if (any_driven && best.rows != 4) {
            float rms[2];
            for (int q4 = 0; q4 < 2; ++q4) {
                Tiling t = best;
                t.rhs4 = q4;
                tdgl_status e = apply_tiling(ctx, t);
                if (e) return e;
                launch_rhs(ctx);  // warm-up
                HIPCHK(hipEventRecord(e0, s));
                for (int q = 0; q < 4; ++q) launch_rhs(ctx);
                HIPCHK(hipEventRecord(e1, s));
                LAUNCHCHK();
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&rms[q4], e0, e1));
            }
            best.rhs4 = rms[1] < rms[0] ? 1 : 0;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s %d %d %d %d %d %.3f %d %d %d\n", key.c_str(), best.rows, best.chunk, best.nt,
                        best.fused, best.persist, best_us, best.chunk2, best.rhs4, best.tys);
                fclose(f);
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best, best_us};
    }
    tdgl_status e = apply_tiling(ctx, best);
    if (e) return e;
    if (chosen) {
        chosen->rows = best.rows;
        chosen->chunk = ctx->inst[0].d.chunk;
        chosen->chunk2 = ctx->inst[0].d.chunk2;
        chosen->streaming = best.nt;
        chosen->fused = best.fused;
        chosen->persistent = ctx->persist ? 1 : 0;
        chosen->sweep_us = best_us;
        chosen->rhs_rows = ctx->rhs_rows;
        chosen->super_rows = ctx->inst[0].d.tys;
    }
    return TDGL_OK;
}

tdgl_status tdgl_set_tiling(tdgl_ctx *ctx, const tdgl_tiling *t) {
    if (!ctx || !t) return fail(TDGL_EINVAL, "null argument");
    if (t->rows != 1 && t->rows != 2 && t->rows != 4) return fail(TDGL_EINVAL, "rows must be 1, 2 or 4");
    if (t->chunk < 0 || t->chunk > 1024) return fail(TDGL_EINVAL, "chunk must be in [0, 1024]");
    if (t->chunk2 < 0 || t->chunk2 > 1024) return fail(TDGL_EINVAL, "chunk2 must be in [0, 1024]");
    if (t->rhs_rows != 0 && t->rhs_rows != 4 && t->rhs_rows != t->rows)
        return fail(TDGL_EINVAL, "rhs_rows must be 0, 4 or rows");
    if (t->super_rows != 0 && t->super_rows != 16 && t->super_rows != 32)
        return fail(TDGL_EINVAL, "super_rows must be 0, 16 or 32");
    if (t->super_rows == 32 && t->rows == 1)
        return fail(TDGL_EINVAL, "32-row super-tiles need rows 2 or 4");
    if ((t->streaming != 0 && t->streaming != 1) || (t->fused != 0 && t->fused != 1) ||
        (t->persistent != 0 && t->persistent != 1))
        return fail(TDGL_EINVAL, "streaming, fused and persistent must be 0 or 1");
    if (t->fused && t->persistent) return fail(TDGL_EINVAL, "persistent solves use single sweeps (fused = 0)");
    if (ctx->any_yz && t->persistent)
        return fail(TDGL_EINVAL, "a context with a yz-plane field has no persistent solve (persistent = 0)");
    if (ctx->any_zseam && t->fused)
        return fail(TDGL_EINVAL, "a yz-plane field with By != 0 on a periodic z axis has no two-sweep passes "
                                 "(fused = 0)");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    Tiling s;
    s.rows = t->rows;
    s.chunk = t->chunk;
    s.chunk2 = t->chunk2;
    s.nt = t->streaming;
    s.fused = t->fused;
    s.persist = t->persistent;
    s.rhs4 = t->rhs_rows == 4 ? 1 : 0;
    s.tys = t->super_rows;
    return apply_tiling(ctx, s);
}

tdgl_status tdgl_get_tiling(const tdgl_ctx *ctx, int inst, tdgl_tiling *out) {
    if (!ctx || !out) return fail(TDGL_EINVAL, "null argument");
    if (inst < 0 || inst >= ctx->n) return fail(TDGL_EINVAL, "instance %d out of range", inst);
    out->rows = ctx->rows;
    out->chunk = ctx->inst[inst].d.chunk;
    out->chunk2 = ctx->inst[inst].d.chunk2;
    out->streaming = ctx->nt ? 1 : 0;
    out->fused = ctx->fused ? 1 : 0;
    out->persistent = ctx->persist ? 1 : 0;
    out->sweep_us = 0.0;
    out->rhs_rows = ctx->rhs_rows;
    out->super_rows = ctx->inst[inst].d.tys;
    return TDGL_OK;
}

}  // extern "C"

namespace {

struct AdjLayout {
    float2 *ck_psi, *seg_psi, *fin_psi, *psibar, *t1, *t2, *t3, *lamW, *lamW2;
    float *ck_mu, *seg_mu, *fin_mu, *mubar;
    double *ck_K, *seg_K, *fin_K, *Elog, *vbar;
    DevState *fin_st;
    AdjState *adj;
};

size_t adj_layout(long N, int nsteps, int C, char *base, AdjLayout *L) {
    Carver cv{base};
    const int ncp = (nsteps + C - 1) / C;
    AdjLayout l;
    l.ck_psi = cv.take<float2>((size_t)ncp * N);
    l.ck_mu = cv.take<float>((size_t)ncp * N);
    l.ck_K = cv.take<double>(3 * (size_t)ncp);  // K, mean of mu, step counter
    l.seg_psi = cv.take<float2>((size_t)(C + 1) * N);
    l.seg_mu = cv.take<float>((size_t)(C + 1) * N);
    l.seg_K = cv.take<double>(C + 1);
    l.fin_psi = cv.take<float2>(N);
    l.fin_mu = cv.take<float>(N);
    l.fin_K = cv.take<double>(3);
    l.fin_st = cv.take<DevState>(1);
    l.psibar = cv.take<float2>(N);
    l.mubar = cv.take<float>(N);
    l.t1 = cv.take<float2>(N);
    l.t2 = cv.take<float2>(N);
    l.t3 = cv.take<float2>(N);
    l.lamW = cv.take<float2>(N);
    l.lamW2 = cv.take<float2>(N);
    l.Elog = cv.take<double>(nsteps);
    l.vbar = cv.take<double>(1);
    l.adj = cv.take<AdjState>(1);
    if (L) *L = l;
    return cv.off;
}

// Reverse of one step: prev = state n-1, nxt = state n (segment slots).
// k: reverse steps done before this one.  The last two reverse steps'
// solutions (lambda / W) alternate between lamW and lamW2: the newest warm
// starts this step's M^H solve (extrapolated with the older from the third
// reverse step on), and this step's solution replaces the older.
tdgl_status adjoint_step(tdgl_ctx *c, const AdjLayout &L, int iprev, int inext, double ew, float *grad, int k) {
    float2 *newest = (k & 1) ? L.lamW2 : L.lamW, *older = (k & 1) ? L.lamW : L.lamW2;
    const Inst &d = c->inst[0].d;
    const long N = d.N;
    hipStream_t s = c->stream;
    const int G = std::max(1, std::min(d.part_cap, 2048));
    const float2 *psim = L.seg_psi + (size_t)iprev * N, *psin = L.seg_psi + (size_t)inext * N;
    const float *mum = L.seg_mu + (size_t)iprev * N;
    const double *Km = L.seg_K + iprev, *Kn = L.seg_K + inext;
    // Poisson transpose: fbar = W G(W^-1 mubar)
    hipLaunchKernelGGL(k_adj_prep_f, dim3(G), dim3(256), 0, s, c->d_inst, L.mubar);
    hipLaunchKernelGGL(k_mu_mean_partial, dim3(std::max(c->tot_mg[0], 1)), dim3(256), 0, s, c->d_inst,
                       pref_mg(c, 0), 1, 1);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(1), dim3(256), 0, s, c->d_inst, c->d_np_mg0, 4, 1);
    LAUNCHCHK();
    tdgl_status e = enqueue_poisson(c, nullptr);
    if (e) return e;
    // adjoint of the Poisson right side, links at K_n
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, s, c->d_inst, 1, Kn);
    hipLaunchKernelGGL(k_adj_g, dim3(G), dim3(256), 0, s, c->d_inst, psin, L.t1);
    launch_stencil<MODE_NS>(c, 0, psin, L.t2);
    launch_stencil<MODE_NS>(c, 0, L.t1, L.t3);
    hipLaunchKernelGGL(k_adj_facc, dim3(G), dim3(256), 0, s, c->d_inst, L.psibar, L.t2, L.t3);
    hipLaunchKernelGGL(k_adj_edge_f, dim3(G), dim3(256), 0, s, c->d_inst, psin);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, c->d_inst, G, 0, ew, L.adj);
    // J_av(psi_n, K_{n-1}) and the K update
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, s, c->d_inst, 1, Km);
    hipLaunchKernelGGL(k_adj_jterm, dim3(G), dim3(256), 0, s, c->d_inst, L.psibar, psin, L.adj);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, c->d_inst, G, 1, 0.0, L.adj);
    // the Crank-Nicolson system transposed
    hipLaunchKernelGGL(k_adj_maxabs, dim3(G), dim3(256), 0, s, c->d_inst, L.psibar);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, c->d_inst, G, 3, 0.0, L.adj);
    hipLaunchKernelGGL(k_adj_assemble, dim3(G), dim3(256), 0, s, c->d_inst, L.psibar, psim, mum, newest, older, k >= 2 ? 1 : 0, L.adj);
    LAUNCHCHK();
    e = jacobi_loop(c, nullptr, nullptr, 0);
    if (e) return e;
    // sources: eps gradient, mubar^-, K terms and psibar^-
    hipLaunchKernelGGL(k_adj_scale_nu, dim3(G), dim3(256), 0, s, c->d_inst, L.adj, older);
    launch_stencil<MODE_NS>(c, 0, older, L.t2);
    hipLaunchKernelGGL(k_adj_edge_s, dim3(G), dim3(256), 0, s, c->d_inst, psim, psin, L.adj);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, c->d_inst, G, 2, 0.0, L.adj);
    hipLaunchKernelGGL(k_adj_sources, dim3(G), dim3(256), 0, s, c->d_inst, L.psibar, L.mubar, grad, psim, psin,
                       mum, L.t2, L.adj);
    LAUNCHCHK();
    return TDGL_OK;
}

// Arguments of both adjoint entry points.
tdgl_status voltage_grad_check(tdgl_ctx *ctx, int nsteps, int window_begin, int ckpt_every, double *vbar,
                               float *grad) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (ctx->n != 1) return fail(TDGL_EINVAL, "tdgl_voltage_grad needs a context with one instance");
    if (!ctx->inst[0].p.driven) return fail(TDGL_EINVAL, "the voltage needs a driven instance (driven = 1)");
    if (nsteps < 1 || window_begin < 0 || window_begin >= nsteps || ckpt_every < 1)
        return fail(TDGL_EINVAL, "need nsteps >= 1, 0 <= window_begin < nsteps, ckpt_every >= 1");
    if (!grad || !vbar) return fail(TDGL_EINVAL, "null output");
    return TDGL_OK;
}

// Forward with checkpoints, then the reverse sweep, on the adjoint buffers
// carved from ws (adj_layout(N, nsteps, C) bytes, 256-byte aligned).
tdgl_status voltage_grad_run(tdgl_ctx *ctx, int nsteps, int window_begin, int C, char *ws, double *vbar,
                             float *grad) {
    const InstHost &h = ctx->inst[0];
    const long N = h.d.N;
    AdjLayout L;
    adj_layout(N, nsteps, C, ws, &L);
    hipStream_t s = ctx->stream;
    const int G = std::max(1, std::min(h.d.part_cap, 2048));
    hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(N)), dim3(256), 0, s, grad, N, 0.f);
    hipLaunchKernelGGL(k_fill_c, dim3(fill_grid(N)), dim3(256), 0, s, L.psibar, N, 0.f, 0.f);
    hipLaunchKernelGGL(k_fill_c, dim3(fill_grid(N)), dim3(256), 0, s, L.lamW, N, 0.f, 0.f);
    hipLaunchKernelGGL(k_fill_c, dim3(fill_grid(N)), dim3(256), 0, s, L.lamW2, N, 0.f, 0.f);
    hipLaunchKernelGGL(k_fill_f, dim3(fill_grid(N)), dim3(256), 0, s, L.mubar, N, 0.f);
    hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(64), 0, s, L.adj);
    LAUNCHCHK();
    // forward with checkpoints; the states of the last segment go straight
    // into the segment buffer, so that segment is not recomputed (with
    // ckpt_every >= nsteps nothing is)
    const int ncp = (nsteps + C - 1) / C;
    const int s0_last = (ncp - 1) * C;
    // each forward solve's sweep count, for the replays (-1: not seen by
    // the host)
    std::vector<int> fw_sweeps(nsteps, -1);
    for (int n = 0; n < nsteps; ++n) {
        if (n % C == 0) {
            const int q = n / C;
            hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.ck_psi + (size_t)q * N,
                               L.ck_mu + (size_t)q * N, L.ck_K + 3 * q, 1);
        }
        if (n == s0_last)
            hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.seg_psi, L.seg_mu, L.seg_K, 0);
        tdgl_status e = tdgl_step(ctx, 1, nullptr);
        if (e) return e;
        fw_sweeps[n] = ctx->last_sweeps;
        hipLaunchKernelGGL(k_adj_logE, dim3(1), dim3(64), 0, s, ctx->d_inst, L.Elog, n);
        if (n >= s0_last) {
            const int j = n + 1 - s0_last;
            hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.seg_psi + (size_t)j * N,
                               L.seg_mu + (size_t)j * N, L.seg_K + j, 0);
        }
    }
    hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.fin_psi, L.fin_mu, L.fin_K, 1);
    HIPCHK(hipMemcpyAsync(L.fin_st, h.d.st, sizeof(DevState), hipMemcpyDeviceToDevice, s));
    LAUNCHCHK();
    // reverse sweep, segment by segment (the last one is already stored)
    const double W = (double)(nsteps - window_begin);
    for (int q = ncp - 1; q >= 0; --q) {
        const int s0 = q * C, s1 = std::min(s0 + C, nsteps);
        if (q != ncp - 1) {
            hipLaunchKernelGGL(k_adj_load, dim3(G), dim3(256), 0, s, ctx->d_inst, L.ck_psi + (size_t)q * N,
                               L.ck_mu + (size_t)q * N, L.ck_K + 3 * q);
            hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, s, ctx->d_inst, 1, (const double *)nullptr);
            hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.seg_psi, L.seg_mu, L.seg_K,
                               0);
            LAUNCHCHK();
            for (int j = 1; j <= s1 - s0; ++j) {
                // a replayed step whose forward solve took sw sweeps runs
                // the fixed launch sequence of sw sweeps (the same iterates,
                // with no host round trip); spectral Poisson only, where the
                // rest of the step is a fixed sequence too
                const int sw = fw_sweeps[s0 + j - 1];
                tdgl_status e = (sw > 0 && !ctx->any_mg && !ctx->persist) ? enqueue_step_fixed(ctx, sw)
                                                                           : tdgl_step(ctx, 1, nullptr);
                if (e) return e;
                hipLaunchKernelGGL(k_adj_save, dim3(G), dim3(256), 0, s, ctx->d_inst, L.seg_psi + (size_t)j * N,
                                   L.seg_mu + (size_t)j * N, L.seg_K + j, 0);
            }
        }
        for (int n = s1; n > s0; --n) {
            const double ew = (n - 1 >= window_begin) ? 1.0 / W : 0.0;
            tdgl_status e = adjoint_step(ctx, L, n - 1 - s0, n - s0, ew, grad, nsteps - n);
            if (e) return e;
        }
    }
    // back to the state after the forward run
    HIPCHK(hipMemcpyAsync(h.d.st, L.fin_st, sizeof(DevState), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_adj_load, dim3(G), dim3(256), 0, s, ctx->d_inst, L.fin_psi, L.fin_mu, L.fin_K);
    hipLaunchKernelGGL(k_links, dim3(1), dim3(256), 0, s, ctx->d_inst, 1, (const double *)nullptr);
    hipLaunchKernelGGL(k_adj_vbar, dim3(1), dim3(64), 0, s, L.Elog, window_begin, nsteps, L.vbar);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(vbar, L.vbar, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return TDGL_OK;
}

// Scratch of tdgl_voltage_grad_noalloc: a fixed device array in place of a
// caller workspace, for callers that cannot allocate.  Each device the
// library runs on holds its own copy for the life of the process; its
// address on a device comes from hipGetSymbolAddress, taken once per device
// with that device current (the array's name in host code is not a device
// address).  Calls that overlap on one device share it and race.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

tdgl_status scratch_of(int device, char **out) {
    if (device < 0 || device >= kMaxDevices) return fail(TDGL_EDEVICE, "device %d beyond the scratch table", device);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != device) HIPCHK(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(TDGL_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                        hipGetErrorString(e));
        if ((uintptr_t)p % kAlign != 0) return fail(TDGL_EDEVICE, "scratch array not %zu-byte aligned", kAlign);
        g_scratch_ptr[device] = (char *)p;
    }
    *out = g_scratch_ptr[device];
    return TDGL_OK;
}

}  // namespace

extern "C" {

tdgl_status tdgl_adjoint_plan(const tdgl_ctx *ctx, int nsteps, int ckpt_every, size_t *bytes) {
    if (!ctx || !bytes) return fail(TDGL_EINVAL, "null argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(TDGL_EINVAL, "nsteps and ckpt_every must be >= 1");
    *bytes = adj_layout(ctx->inst[0].d.N, nsteps, std::min(ckpt_every, nsteps), nullptr, nullptr);
    return TDGL_OK;
}

tdgl_status tdgl_voltage_grad(tdgl_ctx *ctx, int nsteps, int window_begin, int ckpt_every, void *ws,
                              size_t ws_bytes, double *vbar, float *grad) {
    tdgl_status e = voltage_grad_check(ctx, nsteps, window_begin, ckpt_every, vbar, grad);
    if (e) return e;
    const int C = std::min(ckpt_every, nsteps);
    const size_t need = adj_layout(ctx->inst[0].d.N, nsteps, C, nullptr, nullptr);
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < need)
        return fail(TDGL_EWS, "adjoint workspace missing, misaligned or below %zu bytes", need);
    return voltage_grad_run(ctx, nsteps, window_begin, C, (char *)ws, vbar, grad);
}

tdgl_status tdgl_voltage_grad_noalloc(tdgl_ctx *ctx, int nsteps, int window_begin, int ckpt_every, double *vbar,
                                      float *grad) {
    tdgl_status e = voltage_grad_check(ctx, nsteps, window_begin, ckpt_every, vbar, grad);
    if (e) return e;
    const int C = std::min(ckpt_every, nsteps);
    const size_t need = adj_layout(ctx->inst[0].d.N, nsteps, C, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(TDGL_EWS,
                    "tdgl_voltage_grad_noalloc: %d steps with a checkpoint every %d on %ld nodes need %zu bytes of "
                    "scratch, above its fixed %zu bytes (use tdgl_voltage_grad with a workspace)",
                    nsteps, C, (long)ctx->inst[0].d.N, need, kScratchBytes);
    char *ws = nullptr;
    if ((e = scratch_of(ctx->device, &ws))) return e;
    return voltage_grad_run(ctx, nsteps, window_begin, C, ws, vbar, grad);
}

tdgl_status tdgl_profile_start(tdgl_ctx *ctx, unsigned mask) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    if (mask >> TDGL_K_COUNT) return fail(TDGL_EINVAL, "profile mask has bits beyond TDGL_K_COUNT");
    if (ctx->prof_pool.empty()) {
        ctx->prof_pool.resize(8192);
        for (auto &e : ctx->prof_pool) HIPCHK(hipEventCreate(&e));
    }
    ctx->prof_recs.clear();
    ctx->prof_used = 0;
    for (int k = 0; k < TDGL_K_COUNT; ++k) { ctx->prof_ms[k] = 0; ctx->prof_launches[k] = 0; }
    ctx->prof_mask = mask;
    return TDGL_OK;
}

tdgl_status tdgl_profile_stop(tdgl_ctx *ctx, tdgl_prof *out) {
    if (!ctx) return fail(TDGL_EINVAL, "null context");
    tdgl_status s = prof_flush(ctx);
    if (s) return s;
    ctx->prof_mask = 0;
    if (out)
        for (int k = 0; k < TDGL_K_COUNT; ++k) { out->launches[k] = ctx->prof_launches[k]; out->ms[k] = ctx->prof_ms[k]; }
    return TDGL_OK;
}

tdgl_status tdgl_observables(tdgl_ctx *ctx, int inst, tdgl_obs *obs) {
    tdgl_status s = check_ctx(ctx, inst);
    if (s) return s;
    if (!obs) return fail(TDGL_EINVAL, "null observables");
    const int n = ctx->n;
    hipStream_t st = ctx->stream;
    launch_stencil<MODE_ENERGY>(ctx, 0);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, st, ctx->d_inst, ctx->d_np_st, 2, 0);
    hipLaunchKernelGGL(k_psi2_partial, dim3(ctx->tot_flat), dim3(256), 0, st, ctx->d_inst, ctx->d_pref_flat, n);
    hipLaunchKernelGGL(k_reduce_to_state, dim3(n), dim3(256), 0, st, ctx->d_inst, ctx->d_np_flat, 3, 0);
    LAUNCHCHK();
    DevState h;
    HIPCHK(hipMemcpyAsync(&h, ctx->inst[inst].d.st, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const tdgl_params &p = ctx->inst[inst].p;
    const double Lx = p.bc[0] == TDGL_OPEN ? (p.nx - 1) * p.hx : p.nx * p.hx;
    obs->F = h.F;
    obs->E_last = h.E_last;
    obs->E_mean = h.n_avg > 0 ? h.V_sum / h.n_avg : 0.0;
    obs->V_mean = Lx * obs->E_mean;
    obs->J_av = h.J_last;
    obs->K = h.K;
    obs->res2_last = h.last_res2;
    obs->mu_mean_w = h.mu_mean;
    obs->psi2_mean = h.psi2;
    obs->n = (long long)h.n;
    obs->n_avg = (long long)h.n_avg;
    return TDGL_OK;
}

}  // extern "C"
