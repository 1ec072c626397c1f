// C ABI of the NPCF library (include/npcf.h): plan lifecycle, device
// workspace, and the per-call orchestration of
//   quantise -> cell list -> primary list -> [harmonic -> coupling -> FP64 reduce] per chunk
// on the plan's stream.  No exception crosses the ABI.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "npcf_internal.h"

using namespace npcf;

namespace {

constexpr int64_t kADefaultBudget = 3LL << 30;  // bytes of per-chunk a^b storage

struct DevAlloc {
    std::vector<void *> ptrs;
    bool ok = true;
    template <class T>
    T *get(size_t count)
    {
        if (!ok) return nullptr;
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
    void release()
    {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

struct StageTimer {
    hipEvent_t a = nullptr, b = nullptr;
};

struct BatchState;

// Device buffers of one flat-catalogue accumulation: the catalogue's cell
// list, the rows of a of one chunk of primaries and the coupling partials.
// The plan owns one set (allocated at plan time); npcf_accumulate_static
// carves another from the static workspace for each call.
struct Workspace {
    uint32_t *qtmp[kMaxD] = {};
    uint4 *rec = nullptr;
    uint32_t *cell = nullptr;
    int32_t *perm = nullptr, *perm_sorted = nullptr, *orig = nullptr, *prim = nullptr;
    float *ws = nullptr;
    double *w64s = nullptr;
    uint32_t *flag = nullptr, *flagpos = nullptr;
    uint32_t *count = nullptr, *cell_start = nullptr, *cursor = nullptr;
    uint32_t *scan_scratch = nullptr;
    int64_t scan_scratch_len = 0;
    float *A = nullptr, *wrow = nullptr;
    double *partial = nullptr;
    int64_t partial_len = 0;
    unsigned int *work = nullptr;
    // curved spaces: the secondaries in spatial order and their tile caps
    double *pos64 = nullptr;  // [4][max_points]
    float *caps = nullptr;    // [tiles][8]
    unsigned *bbox = nullptr; // [8] key-axis bounds, [8] the largest x0 (H^D)
    int64_t rows_cap = 0;    // primaries per chunk (rows of a held at once)
    bool growable = true;    // the partial buffer may be re-allocated (plan-owned set only)
    bool timed = true;       // record stage events (the static path creates none)
};

// Gridded data (npcf_accumulate_grid): the kernel spectra of one grid shape
// and the per-call buffers.
struct GridState {
    int dims[3] = {0, 0, 0};
    int64_t ng = 0;
    int nbs = 0;                          // bins x stored states
    DevAlloc mem;
    double2 *khat = nullptr;              // [nbs][ng] FFT of K'_{b,s}
    double2 *work = nullptr;              // [nbs][ng] a_{b,s} on the grid
    double2 *xhat = nullptr;              // [ng] FFT of the weights
    double *w64 = nullptr;
    float *w32 = nullptr;
    uint8_t *sreal = nullptr;             // [nstate] states with l1 = 0 (real a)
    double2 *tw[3] = {nullptr, nullptr, nullptr};   // twiddles e^{-2 pi i j / n} per axis
    unsigned long long offsets_in_range = 0;        // grid offsets with e_0 <= r < e_nb
};

}  // namespace

struct npcf_plan_s {
    npcf_config cfg{};
    std::vector<double> edges;
    hipStream_t stream = nullptr;
    int64_t max_points = 0;
    Tables t;
    int D = 0, N = 0, L = 0, nb = 0;
    int cell_subdiv = 3;
    int couple_rows = 0;  // 0: automatic
    int harm_bpc = 0;     // persistent harmonic grid: blocks per compute unit (0: automatic, 8)
    int ncs[kMaxD] = {1, 1, 1, 1};
    int64_t ncell = 1;
    int curved_bits = 0;       // curved spaces: bits per axis of the Hilbert cells of the spatial sort
    int curved_group = 0;      // curved spaces: bins per pass of the all-pairs kernel (a sph_group value)
    int harm_pass = 0;         // flat harmonic stage: 1 = one pass per radial bin, 0 = bin-sorted staging
    int64_t rows_cap_max = 0;  // rows the a buffer was sized for
    int njobs = 0;
    int max_block_terms = 0;  // N = 4: coupling terms one coupling block copies to LDS
    bool term_coupling = false;  // force the term-by-term N = 4 kernel (NPCF_COUPLING=terms)
    bool failed = false;

    DevAlloc mem;
    DevAlloc cellmem;  // cell arrays (re-allocated when the cell grid changes)
    Workspace wk;      // the plan's own catalogue workspace and stage buffers
    void *static_ws = nullptr;  // this device's static workspace (npcf_accumulate_static)
    double *acc[2] = {nullptr, nullptr};
    double *out_dev = nullptr;
    unsigned long long *pairs = nullptr;  // [2]
    int *bad = nullptr;
    // tables
    double *d_e2 = nullptr;
    uint8_t *d_bucket = nullptr;
    CoupleTerm *d_terms = nullptr;
    CoupleGroup *d_groups = nullptr;
    int *d_lam_group_begin = nullptr, *d_lam_part = nullptr;
    int2 *d_row_pairs = nullptr;
    float *d_sfac = nullptr;
    int *d_bt_row = nullptr, *d_bt_col = nullptr;
    double *d_bt_scale = nullptr;
    FPair *d_fpairs = nullptr;
    FGroup *d_fgroups = nullptr;
    FProd *d_fprods = nullptr;
    float *d_fcoef = nullptr;
    int2 *d_ftasks = nullptr;
    C5Job *d_c5jobs = nullptr;
    C5Label *d_c5labels = nullptr;
    int *d_c5mterm = nullptr;
    uint2 *d_c5terms = nullptr;
    int2 *d_c5pairs = nullptr;
    int *d_c5idx = nullptr;
    double *d_c5sign = nullptr;
    // stage timing (harmonic, coupling, prep) in ms, accumulated since reset
    std::vector<StageTimer> timers[3];
    int ncu = 256;  // compute units of the plan's device
    // batched accumulation (npcf_accumulate_batch); owned
    BatchState *batch = nullptr;
    // gridded accumulation (npcf_accumulate_grid); owned
    GridState *grid = nullptr;
};

namespace {

// The last HIP failure seen on this thread (npcf_last_error_detail).
thread_local char g_last_error[256] = "";

npcf_status dev_err(hipError_t e) { return e == hipSuccess ? NPCF_OK : (e == hipErrorOutOfMemory ? NPCF_E_NOMEM : NPCF_E_DEVICE); }

npcf_status dev_err_at(hipError_t e, const char *what, int line)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d) from %s at npcf_abi.cpp:%d", hipGetErrorName(e),
                  (int)e, what, line);
    return dev_err(e);
}

#define NPCF_TRY(expr)                                                      \
    do {                                                                    \
        hipError_t e__ = (expr);                                            \
        if (e__ != hipSuccess) return dev_err_at(e__, #expr, __LINE__);     \
    } while (0)

template <class T>
hipError_t upload(T *dst, const std::vector<T> &src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

void compute_grid(npcf_plan_s *p)
{
    if (p->t.sphere) {
        // no cell list: the Hilbert cells that put the secondaries in spatial
        // order, 2^20 or 2^21 of them over the key axes (all D + 1
        // coordinates on the sphere, the D spatial ones in H^D): about one
        // point per occupied cell at 1e5-1e6 points, so the order within a
        // cell hardly matters
        const int axes = p->t.curv > 0 ? p->D + 1 : p->D;
        p->curved_bits = axes == 2 ? 10 : (axes == 3 ? 7 : 5);
        // the narrow kernel by default: it won on every curved workload measured
        if (p->curved_group == 0) p->curved_group = sph_group(p->D, p->L, true);
        p->ncell = (int64_t)1 << (p->curved_bits * axes);
        for (int k = 0; k < kMaxD; k++) p->ncs[k] = 1;
        return;
    }
    // Cells of side about rmax / s, except along x, the axis a stencil row
    // of cells runs along: there they are kCellXSub times thinner, so a
    // row's x range is cut to the sphere (and the inner sphere's cells left
    // out) more tightly, with the same number of rows and the same per-row
    // work.  c2 harmonic stage, s = 4: 87.3 ms with cubic cells, 82.5 / 80.2 /
    // 78.7 / 77.9 ms at 2 / 4 / 8 / 16 thinner x cells (pair counts equal).
    // Over 2^24 cells the x factor halves first, then s drops.
    constexpr int kCellXSub = 8;
    const double rmax = p->edges[p->nb];
    int64_t total = 1;
    for (int k = 0; k < kMaxD; k++) p->ncs[k] = 1;
    int s = p->cell_subdiv, xs = kCellXSub;
    for (;;) {
        total = 1;
        for (int k = 0; k < p->D; k++) {
            double c = std::floor(p->cfg.box[k] / (rmax / s));
            if (c < 1) c = 1;
            if (k == 0) c *= xs;
            if (c > 4096) c = 4096;
            p->ncs[k] = (int)c;
            total *= p->ncs[k];
        }
        if (total <= (1LL << 24) || (s == 1 && xs == 1)) break;
        if (xs > 1) xs /= 2;
        else s--;
    }
    p->ncell = total;
}

npcf_status alloc_cells(npcf_plan_s *p)
{
    p->cellmem.release();
    p->cellmem.ok = true;
    p->wk.count = p->cellmem.get<uint32_t>(p->ncell + 1);
    p->wk.cell_start = p->cellmem.get<uint32_t>(p->ncell + 1);
    p->wk.cursor = p->cellmem.get<uint32_t>(p->ncell + 1);
    int64_t m = std::max<int64_t>(p->ncell + 1, p->max_points);
    p->wk.scan_scratch_len = (m + 1023) / 1024 + 1;
    p->wk.scan_scratch = p->cellmem.get<uint32_t>(p->wk.scan_scratch_len);
    return p->cellmem.ok ? NPCF_OK : NPCF_E_NOMEM;
}

int couple_rows_per_block(const npcf_plan_s *p, int64_t nrows)
{
    if (p->couple_rows > 0) return ((p->couple_rows + 15) / 16) * 16;
    if (p->N == 5) {
        // about 32k blocks in all, at least 256 primaries each (measured on the
        // 5PCF workload: 256-512 beat 1024-4096, whose long blocks leave the
        // chip idle in the tail), and no more row blocks than keep the per-block
        // partials (one accumulator set each) within 1 GiB
        int64_t rpb = nrows * (int64_t)p->t.c5jobs.size() / 32768;
        rpb = std::max<int64_t>(256, ((rpb + 15) / 16) * 16);
        const int64_t max_nrb = std::max<int64_t>(8, (1LL << 30) / ((int64_t)p->t.c5tiles * 256 * 8));
        if ((nrows + rpb - 1) / rpb > max_nrb) rpb = ((nrows + max_nrb - 1) / max_nrb + 15) / 16 * 16;
        return (int)rpb;
    }
    if (p->N == 4) {
        // about 32k blocks in all, 256 to 1024 primaries each (measured at
        // full size on 800k clustered D = 3 and 500k D = 2 points: fastest at
        // 512-1024, slower at 64 and 2048)
        const int jpb = couple_jobs_per_block();
        const int bpr = (!p->t.fpairs.empty() && !p->term_coupling) ? couple_ftask_groups((int)p->t.ftasks.size())
                                                                     : (p->njobs + jpb - 1) / jpb;
        int64_t rpb = nrows * bpr / 32768;
        rpb = ((rpb + 15) / 16) * 16;
        return (int)std::min<int64_t>(1024, std::max<int64_t>(256, rpb));
    }
    const int njg = (p->njobs + 31) / 32;
    int64_t want_rb = std::max<int64_t>(8, (2048 + njg - 1) / njg);
    int64_t rpb = (nrows + want_rb - 1) / want_rb;
    rpb = ((rpb + 15) / 16) * 16;
    if (rpb < 64) rpb = 64;
    return (int)rpb;
}

float elapsed(const StageTimer &t)
{
    float ms = 0.f;
    if (hipEventSynchronize(t.b) != hipSuccess) return 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) return 0.f;
    return ms;
}

npcf_status timer_begin(npcf_plan_s *p, int stage, StageTimer &t)
{
    NPCF_TRY(hipEventCreate(&t.a));
    NPCF_TRY(hipEventCreate(&t.b));
    NPCF_TRY(hipEventRecord(t.a, p->stream));
    (void)stage;
    return NPCF_OK;
}

void clear_timers(npcf_plan_s *p)
{
    for (auto &v : p->timers) {
        for (auto &t : v) {
            if (t.a) (void)hipEventDestroy(t.a);
            if (t.b) (void)hipEventDestroy(t.b);
        }
        v.clear();
    }
}

// Build the cell list of a catalogue: sorted SoA lattice coordinates and weights.
npcf_status build_cells(npcf_plan_s *p, Workspace &W, const double *pos, const double *w, int64_t n)
{
    hipStream_t s = p->stream;
    NPCF_TRY(launch_fill_u32(W.count, 0u, p->ncell + 1, s));
    NPCF_TRY(launch_quantize(p->D, p->cfg.periodic, pos, w, n, p->cfg.box, p->ncs, W.qtmp, W.cell, W.count, p->bad, s));
    NPCF_TRY(launch_exclusive_scan(W.count, W.cell_start, p->ncell + 1, W.scan_scratch, W.scan_scratch_len, s));
    NPCF_TRY(launch_copy_u32(W.cursor, W.cell_start, p->ncell + 1, s));
    NPCF_TRY(launch_scatter_perm(n, W.cell, W.cursor, W.perm, s));
    NPCF_TRY(launch_cellsort(n, W.cell, W.cell_start, W.perm, W.perm_sorted, s));
    NPCF_TRY(launch_gather(p->D, n, W.perm_sorted, W.qtmp, w, W.rec, W.ws, W.w64s, W.orig, s));
    return NPCF_OK;
}

HarmArgs harm_args(const npcf_plan_s *p, const Workspace &W, int rows, const int32_t *prim, unsigned long long *pairs)
{
    HarmArgs a{};
    a.rec = W.rec;
    for (int k = 0; k < kMaxD; k++) {
        a.ncs[k] = p->ncs[k];
        a.cell_len[k] = 4294967296.0 / p->ncs[k];
        a.inv_cell_len[k] = p->ncs[k] / 4294967296.0;
        double sc = (k < p->D) ? p->cfg.box[k] / 4294967296.0 : 1.0;
        a.scale64[k] = sc;
        a.scale[k] = (float)sc;
        a.rmax_lat[k] = p->edges[p->nb] / sc;
    }
    a.cube = 1;
    for (int k = 1; k < p->D; k++) a.cube = a.cube && a.scale64[k] == a.scale64[0];
    a.w = W.ws;
    a.cell_start = W.cell_start;
    a.prim = prim;
    a.nrows = rows;
    a.nb = p->nb;
    a.e2lo_f = p->t.e2lo_f;
    a.e2hi_f = p->t.e2hi_f;
    a.bucket_lo = p->t.bucket_lo;
    a.bucket_inv = p->t.bucket_inv;
    a.nbucket = (int)p->t.bucket_bin.size();
    a.e2 = p->d_e2;
    a.bucket_bin = p->d_bucket;
    a.A = W.A;
    a.wrow = W.wrow;
    a.pairs = pairs;
    a.work = W.work;
    a.periodic = p->cfg.periodic;
    a.per_bin = p->harm_pass;
    return a;
}

// Persistent harmonic launch over a.nrows rows (rows handed out dynamically
// through a.work, which is cleared first).
hipError_t launch_harmonic(const npcf_plan_s *p, const HarmArgs &a, hipStream_t s)
{
    hipError_t e = launch_fill_u32(a.work, 0u, 1, s);
    if (e != hipSuccess) return e;
    // persistent grid: blocks of 4 waves per CU (tuned, default 8), no more
    // blocks than rows / 4; rows are handed out dynamically
    int grid = p->ncu * (p->harm_bpc > 0 ? p->harm_bpc : 8);
    const int64_t need = ((int64_t)a.nrows + 3) / 4;
    if (grid > need) grid = (int)std::max<int64_t>(1, need);
    switch (p->D) {
    case 2: return launch_harmonic_d2(p->L, a, grid, s);
    case 3: return launch_harmonic_d3(p->L, a, grid, s);
    default: return launch_harmonic_d4(p->L, a, grid, s);
    }
}

npcf_status run_harmonic(npcf_plan_s *p, Workspace &W, int rows, const int32_t *prim, unsigned long long *pairs)
{
    hipStream_t s = p->stream;
    HarmArgs a = harm_args(p, W, rows, prim, pairs);
    StageTimer t;
    if (W.timed) {
        npcf_status st = timer_begin(p, 0, t);
        if (st != NPCF_OK) return st;
    }
    NPCF_TRY(launch_harmonic(p, a, s));
    if (W.timed) {
        NPCF_TRY(hipEventRecord(t.b, s));
        p->timers[0].push_back(t);
    }
    return NPCF_OK;
}

CoupleArgs couple_args(const npcf_plan_s *p, const Workspace &W, int rows)
{
    const Tables &t = p->t;
    CoupleArgs a{};
    a.A = W.A;
    a.wrow = W.wrow;
    a.nrows = rows;
    a.nb = p->nb;
    a.nstate = t.nstate;
    a.rows_per_block = couple_rows_per_block(p, rows);
    a.n_rowblocks = (int)((rows + a.rows_per_block - 1) / a.rows_per_block);
    a.nlam = t.nlam;
    a.terms = p->d_terms;
    a.groups = p->d_groups;
    a.lam_group_begin = p->d_lam_group_begin;
    a.lam_part = p->d_lam_part;
    a.row_pairs = p->d_row_pairs;
    a.mrows = t.mrows;
    a.mtiles = t.mtiles;
    a.max_block_terms = p->max_block_terms;
    a.n3_terms = t.n3_terms ? 1 : 0;
    if (p->N == 5) {
        a.c5jobs = p->d_c5jobs;
        a.nc5jobs = (int)t.c5jobs.size();
        a.c5labels = p->d_c5labels;
        a.c5mterm = p->d_c5mterm;
        a.c5terms = p->d_c5terms;
        a.c5pairs = p->d_c5pairs;
        a.c5_lds_extra = t.c5_lds_extra;
    }
    if (p->d_fpairs && !p->term_coupling) {
        a.fpairs = p->d_fpairs;
        a.fgroups = p->d_fgroups;
        a.fprods = p->d_fprods;
        a.fcoef = p->d_fcoef;
        a.ftasks = p->d_ftasks;
        a.nftasks = (int)t.ftasks.size();
    }
    return a;
}

npcf_status run_couple(npcf_plan_s *p, Workspace &W, int rows, double *acc)
{
    hipStream_t s = p->stream;
    const Tables &t = p->t;
    CoupleArgs a = couple_args(p, W, rows);
    const int64_t len = (int64_t)p->njobs * 256;
    if ((int64_t)a.n_rowblocks * len > W.partial_len) {
        // the static workspace was carved for this call's block count
        if (!W.growable) return NPCF_E_INVALID;
        // grow the partial buffer (rare: only with small custom block sizes)
        void *np = nullptr;
        NPCF_TRY(hipStreamSynchronize(s));
        NPCF_TRY(hipMalloc(&np, (size_t)a.n_rowblocks * len * sizeof(double)));
        p->mem.ptrs.push_back(np);
        W.partial = (double *)np;
        W.partial_len = (int64_t)a.n_rowblocks * len;
    }
    a.partial = W.partial;
    StageTimer tm;
    if (W.timed) {
        npcf_status st = timer_begin(p, 1, tm);
        if (st != NPCF_OK) return st;
    }
    NPCF_TRY(launch_couple_kernel(p->N, p->cfg.precision, a, p->njobs, t.nparts, p->d_sfac, s));
    NPCF_TRY(launch_reduce_partials(W.partial, a.n_rowblocks, len, acc, s));
    if (W.timed) {
        NPCF_TRY(hipEventRecord(tm.b, s));
        p->timers[1].push_back(tm);
    }
    return NPCF_OK;
}

npcf_status check_inputs(npcf_plan_s *p, const double *pos, const double *w, int64_t n, int64_t p0, int64_t p1)
{
    if (!p) return NPCF_E_INVALID;
    if (p->failed) return NPCF_E_STATE;
    if (!pos || !w || n < 1 || n > p->max_points) return NPCF_E_INVALID;
    if (p0 < 0 || p1 > n || p0 >= p1) return NPCF_E_INVALID;
    return NPCF_OK;
}

npcf_status prepare(npcf_plan_s *p, Workspace &W, const double *pos, const double *w, int64_t n, int64_t p0, int64_t p1)
{
    StageTimer t;
    if (W.timed) {
        npcf_status st = timer_begin(p, 2, t);
        if (st != NPCF_OK) return st;
    }
    npcf_status st = build_cells(p, W, pos, w, n);
    if (st != NPCF_OK) return st;
    NPCF_TRY(launch_primlist(n, W.orig, p0, p1, W.flag, W.flagpos, W.prim, W.scan_scratch, W.scan_scratch_len,
                             p->stream));
    if (W.timed) {
        NPCF_TRY(hipEventRecord(t.b, p->stream));
        p->timers[2].push_back(t);
    }
    return NPCF_OK;
}

// Sphere harmonic stage for rows [0, rows) = primaries p0 + [0, rows): every
// secondary, no cell list.
npcf_status run_sphere(npcf_plan_s *p, Workspace &W, const double *pos, const double *w, int64_t n, int64_t p0, int rows,
                       unsigned long long *pairs)
{
    SphereArgs a{};
    a.pos = pos;
    a.w = w;
    a.pf = reinterpret_cast<float4 *>(W.rec);   // the flat path's record buffer (max_points x 16 B), unused here
    a.x0max = W.bbox + 8;
    a.spos = W.pos64;
    a.sw = W.w64s;
    a.sorig = W.orig;
    a.caps = W.caps;
    a.key = W.cell;
    a.count = W.count;
    a.cell_start = W.cell_start;
    a.cursor = W.cursor;
    a.scan = W.scan_scratch;
    a.scan_len = W.scan_scratch_len;
    a.perm = W.perm;
    a.bbox = W.bbox;
    a.prim = W.prim;
    a.pflag = W.flag;
    a.ppos = W.flagpos;
    a.ncell_bits = p->curved_bits;
    for (int b = 0; b <= p->nb; b++) a.erad[b] = (float)p->edges[b];
    a.n = n;
    a.p0 = p0;
    a.rows = rows;
    a.nb = p->nb;
    a.group = p->curved_group;
    for (int b = 0; b <= p->nb; b++) a.cedge[b] = p->t.cedge[b];
    a.A = W.A;
    a.wrow = W.wrow;
    a.pairs = pairs;
    StageTimer t;
    if (W.timed) {
        npcf_status st = timer_begin(p, 0, t);
        if (st != NPCF_OK) return st;
    }
    NPCF_TRY(launch_sphere(p->D, p->L, p->t.curv, a, p->stream));
    if (W.timed) {
        NPCF_TRY(hipEventRecord(t.b, p->stream));
        p->timers[0].push_back(t);
    }
    return NPCF_OK;
}

npcf_status accumulate_impl(npcf_plan_s *p, Workspace &W, const double *pos, const double *w, int64_t n, int64_t p0,
                            int64_t p1, double *acc, unsigned long long *pairs)
{
    if (p->t.sphere) {
        for (int64_t c0 = p0; c0 < p1; c0 += W.rows_cap) {
            const int rows = (int)std::min<int64_t>(W.rows_cap, p1 - c0);
            npcf_status st = run_sphere(p, W, pos, w, n, c0, rows, pairs);
            if (st != NPCF_OK) return st;
            st = run_couple(p, W, rows, acc);
            if (st != NPCF_OK) return st;
        }
        return NPCF_OK;
    }
    npcf_status st = prepare(p, W, pos, w, n, p0, p1);
    if (st != NPCF_OK) return st;
    const int64_t nprim = p1 - p0;
    for (int64_t c0 = 0; c0 < nprim; c0 += W.rows_cap) {
        const int rows = (int)std::min<int64_t>(W.rows_cap, nprim - c0);
        st = run_harmonic(p, W, rows, W.prim + c0, pairs);
        if (st != NPCF_OK) return st;
        st = run_couple(p, W, rows, acc);
        if (st != NPCF_OK) return st;
    }
    return NPCF_OK;
}


// ---------------------------------------------------------------------------
// Batches: ncat independent catalogues in one captured launch sequence.
//   quantise all catalogues into one array with cell key c * ncell + cell ->
//   one counting sort (catalogue-major, so catalogue c occupies sorted
//   positions [off[c], off[c+1]) and cells [c * ncell, (c+1) * ncell)) ->
//   rows (primaries) taken catalogue by catalogue, smallest catalogue first
//   (shortest job first: a catalogue's pair count grows as the square of its
//   size, so most catalogues finish early in the batch) ->
//   per chunk of rows: persistent harmonic launch over rows of any catalogue,
//   coupling with row blocks cut at catalogue boundaries, FP64 reduction of
//   each catalogue's blocks into its own accumulator, and a device-clock
//   timestamp for every catalogue whose last row the chunk holds.
// The sequence is captured once per shape (sizes and input pointers) as a HIP
// graph on an internal stream and replayed; it is ordered after the plan's
// stream by events, and the plan's stream waits for it.
// ---------------------------------------------------------------------------
struct BatchSeg {
    int cat, rb0, rb1;  // catalogue and its row blocks [rb0, rb1) in the chunk
};

struct BatchChunk {
    int64_t r0 = 0;       // first global row
    int rows = 0;
    int rb_off = 0;       // into the row-block tables
    int nrb = 0;
    std::vector<BatchSeg> segs;
    std::vector<int> ends;  // catalogues whose last row is in this chunk
};

struct BatchState {
    int ncat = 0;
    int64_t ntot = 0;
    std::vector<int64_t> n, off;
    std::vector<int> order;             // catalogues in processing order (ascending size)
    std::vector<int64_t> roff;          // rows of order[i] are [roff[i], roff[i+1]) of the row list
    std::vector<const double *> pos, w;
    int ncs[kMaxD] = {1, 1, 1, 1};
    int64_t ncell_cat = 1, ncell_tot = 1;
    int rpb = 64;
    std::vector<BatchChunk> chunks;
    DevAlloc mem;
    const double **d_pos = nullptr, **d_w = nullptr;
    int64_t *d_off = nullptr;
    uint32_t *qtmp[kMaxD] = {};
    double *wall = nullptr, *w64s = nullptr;
    uint32_t *cell = nullptr, *count = nullptr, *cell_start = nullptr, *cursor = nullptr, *scan = nullptr;
    int64_t scan_len = 0;
    int32_t *perm = nullptr, *perm_sorted = nullptr, *orig = nullptr;
    int32_t *rowlist = nullptr;         // sorted positions of the primaries in processing order
    uint4 *rec = nullptr;
    float *ws = nullptr;
    double *acc = nullptr, *partial = nullptr;
    unsigned long long *pairs = nullptr, *ts = nullptr;
    int *rb_begin = nullptr, *rb_end = nullptr;
    hipStream_t cs = nullptr;           // capture / replay stream (default priority)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double clock_khz = 0.0;
    bool done = false;                  // a batch has been launched on this shape
};

void batch_release(npcf_plan_s *p)
{
    BatchState *b = p->batch;
    if (!b) return;
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    b->mem.release();
    delete b;
    p->batch = nullptr;
}

bool batch_same_shape(const BatchState *b, int ncat, const double *const *pos, const double *const *w,
                      const int64_t *n, const int *ncs)
{
    if (!b || b->ncat != ncat) return false;
    for (int k = 0; k < kMaxD; k++)
        if (b->ncs[k] != ncs[k]) return false;
    for (int c = 0; c < ncat; c++)
        if (b->n[c] != n[c] || b->pos[c] != pos[c] || b->w[c] != w[c]) return false;
    return true;
}

npcf_status batch_setup(npcf_plan_s *p, int ncat, const double *const *pos, const double *const *w,
                        const int64_t *n)
{
    batch_release(p);
    BatchState *b = new (std::nothrow) BatchState();
    if (!b) return NPCF_E_NOMEM;
    p->batch = b;
    b->ncat = ncat;
    b->n.assign(n, n + ncat);
    b->pos.assign(pos, pos + ncat);
    b->w.assign(w, w + ncat);
    b->off.assign(ncat + 1, 0);
    for (int c = 0; c < ncat; c++) b->off[c + 1] = b->off[c] + n[c];
    b->ntot = b->off[ncat];
    if (b->ntot > (int64_t)INT32_MAX) return NPCF_E_INVALID;
    b->ncell_cat = 1;
    for (int k = 0; k < kMaxD; k++) b->ncs[k] = p->ncs[k];
    for (int k = 0; k < p->D; k++) b->ncell_cat *= p->ncs[k];
    b->ncell_tot = b->ncell_cat * ncat;
    if (b->ncell_tot + 1 >= (int64_t)UINT32_MAX) return NPCF_E_UNSUPPORTED;  // 32-bit cell keys

    // processing order: ascending size (stable), and the row list in that
    // order (catalogue c's primaries are the sorted positions off[c] ..)
    b->order.resize(ncat);
    for (int c = 0; c < ncat; c++) b->order[c] = c;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return n[x] < n[y]; });
    b->roff.assign(ncat + 1, 0);
    for (int i = 0; i < ncat; i++) b->roff[i + 1] = b->roff[i] + n[b->order[i]];
    std::vector<int32_t> rows_h((size_t)b->ntot);
    for (int i = 0; i < ncat; i++)
        for (int64_t k = 0; k < n[b->order[i]]; k++) rows_h[(size_t)(b->roff[i] + k)] = (int32_t)(b->off[b->order[i]] + k);

    // chunks of rows and their row blocks (never straddling a catalogue)
    const int64_t cap = p->wk.rows_cap;
    b->rpb = couple_rows_per_block(p, std::min<int64_t>(cap, b->ntot));
    std::vector<int> rbb, rbe;
    for (int64_t r0 = 0; r0 < b->ntot; r0 += cap) {
        BatchChunk ch;
        ch.r0 = r0;
        ch.rows = (int)std::min<int64_t>(cap, b->ntot - r0);
        ch.rb_off = (int)rbb.size();
        for (int i = 0; i < ncat; i++) {
            const int c = b->order[i];
            const int64_t lo = std::max<int64_t>(b->roff[i], r0), hi = std::min<int64_t>(b->roff[i + 1], r0 + ch.rows);
            if (lo >= hi) continue;
            BatchSeg sg{c, (int)rbb.size() - ch.rb_off, 0};
            for (int64_t r = lo; r < hi; r += b->rpb) {
                rbb.push_back((int)(r - r0));
                rbe.push_back((int)(std::min<int64_t>(r + b->rpb, hi) - r0));
            }
            sg.rb1 = (int)rbb.size() - ch.rb_off;
            ch.segs.push_back(sg);
            if (b->roff[i + 1] <= r0 + ch.rows) ch.ends.push_back(c);
        }
        ch.nrb = (int)rbb.size() - ch.rb_off;
        b->chunks.push_back(ch);
    }
    int max_nrb = 1;
    for (auto &ch : b->chunks) max_nrb = std::max(max_nrb, ch.nrb);

    DevAlloc &m = b->mem;
    const int64_t N = std::max<int64_t>(b->ntot, 1);
    const int64_t len = (int64_t)p->njobs * 256;
    b->d_pos = m.get<const double *>(ncat);
    b->d_w = m.get<const double *>(ncat);
    b->d_off = m.get<int64_t>(ncat + 1);
    for (int k = 0; k < p->D; k++) b->qtmp[k] = m.get<uint32_t>(N);
    b->wall = m.get<double>(N);
    b->w64s = m.get<double>(N);
    b->cell = m.get<uint32_t>(N);
    b->count = m.get<uint32_t>(b->ncell_tot + 1);
    b->cell_start = m.get<uint32_t>(b->ncell_tot + 1);
    b->cursor = m.get<uint32_t>(b->ncell_tot + 1);
    b->scan_len = (std::max<int64_t>(b->ncell_tot + 1, N) + 1023) / 1024 + 1;
    b->scan = m.get<uint32_t>(b->scan_len);
    b->perm = m.get<int32_t>(N);
    b->perm_sorted = m.get<int32_t>(N);
    b->orig = m.get<int32_t>(N);
    b->rowlist = m.get<int32_t>(N);
    b->rec = m.get<uint4>(N);
    b->ws = m.get<float>(N);
    b->acc = m.get<double>((size_t)ncat * len);
    b->partial = m.get<double>((size_t)max_nrb * len);
    b->pairs = m.get<unsigned long long>(ncat);
    b->ts = m.get<unsigned long long>(ncat + 1);
    b->rb_begin = m.get<int>(std::max<size_t>(1, rbb.size()));
    b->rb_end = m.get<int>(std::max<size_t>(1, rbe.size()));
    if (!m.ok) return NPCF_E_NOMEM;
    NPCF_TRY(hipStreamCreate(&b->cs));
    NPCF_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    NPCF_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    int dev = 0, khz = 0;
    NPCF_TRY(hipGetDevice(&dev));
    NPCF_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    b->clock_khz = khz > 0 ? (double)khz : 100000.0;
    hipStream_t s = b->cs;
    NPCF_TRY(hipMemcpyAsync(b->d_pos, pos, ncat * sizeof(double *), hipMemcpyHostToDevice, s));
    NPCF_TRY(hipMemcpyAsync(b->d_w, w, ncat * sizeof(double *), hipMemcpyHostToDevice, s));
    NPCF_TRY(hipMemcpyAsync(b->d_off, b->off.data(), (ncat + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (!rbb.empty()) {
        NPCF_TRY(hipMemcpyAsync(b->rb_begin, rbb.data(), rbb.size() * sizeof(int), hipMemcpyHostToDevice, s));
        NPCF_TRY(hipMemcpyAsync(b->rb_end, rbe.data(), rbe.size() * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (b->ntot > 0)
        NPCF_TRY(hipMemcpyAsync(b->rowlist, rows_h.data(), (size_t)b->ntot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    NPCF_TRY(hipStreamSynchronize(s));
    return NPCF_OK;
}

// Every launch of one batch, in order, on stream s (captured into the graph).
npcf_status batch_record(npcf_plan_s *p, hipStream_t s)
{
    BatchState *b = p->batch;
    const int64_t len = (int64_t)p->njobs * 256;
    NPCF_TRY(launch_timestamp(b->ts + b->ncat, s));
    NPCF_TRY(launch_fill_f64(b->acc, 0.0, (int64_t)b->ncat * len, s));
    NPCF_TRY(launch_fill_u32((uint32_t *)b->pairs, 0u, 2 * (int64_t)b->ncat, s));
    NPCF_TRY(launch_fill_u32(b->count, 0u, b->ncell_tot + 1, s));
    // cell list of every catalogue at once
    NPCF_TRY(launch_quantize_batch(p->D, p->cfg.periodic, b->ncat, b->d_pos, b->d_w, b->d_off, b->ntot, p->cfg.box,
                                   b->ncs, b->ncell_cat, b->qtmp, b->wall, b->cell, b->count, p->bad, s));
    NPCF_TRY(launch_exclusive_scan(b->count, b->cell_start, b->ncell_tot + 1, b->scan, b->scan_len, s));
    NPCF_TRY(launch_copy_u32(b->cursor, b->cell_start, b->ncell_tot + 1, s));
    NPCF_TRY(launch_scatter_perm(b->ntot, b->cell, b->cursor, b->perm, s));
    NPCF_TRY(launch_cellsort(b->ntot, b->cell, b->cell_start, b->perm, b->perm_sorted, s));
    NPCF_TRY(launch_gather(p->D, b->ntot, b->perm_sorted, b->qtmp, b->wall, b->rec, b->ws, b->w64s, b->orig, s));
    // chunks: harmonic over rows of any catalogue, coupling per catalogue
    for (const BatchChunk &ch : b->chunks) {
        HarmArgs ha = harm_args(p, p->wk, ch.rows, b->rowlist + ch.r0, b->pairs);
        ha.rec = b->rec;
        ha.w = b->ws;
        ha.cell_start = b->cell_start;
        ha.cat_begin = b->d_off;
        ha.ncat = b->ncat;
        ha.ncell_cat = b->ncell_cat;
        NPCF_TRY(launch_harmonic(p, ha, s));
        CoupleArgs ca = couple_args(p, p->wk, ch.rows);
        ca.rows_per_block = b->rpb;
        ca.n_rowblocks = ch.nrb;
        ca.rb_begin = b->rb_begin + ch.rb_off;
        ca.rb_end = b->rb_end + ch.rb_off;
        ca.partial = b->partial;
        NPCF_TRY(launch_couple_kernel(p->N, p->cfg.precision, ca, p->njobs, p->t.nparts, p->d_sfac, s));
        for (const BatchSeg &sg : ch.segs)
            NPCF_TRY(launch_reduce_partials(b->partial + (size_t)sg.rb0 * len, sg.rb1 - sg.rb0, len,
                                            b->acc + (size_t)sg.cat * len, s));
        for (int c : ch.ends) NPCF_TRY(launch_timestamp(b->ts + c, s));
    }
    return NPCF_OK;
}
void grid_release(npcf_plan_s *p)
{
    if (!p->grid) return;
    (void)hipStreamSynchronize(p->stream);
    p->grid->mem.release();
    delete p->grid;
    p->grid = nullptr;
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

// Kernel spectra for a grid shape: K'_{b,s} on the grid, then its FFT.
npcf_status grid_setup(npcf_plan_s *p, const int *dims)
{
    grid_release(p);
    GridState *g = new (std::nothrow) GridState();
    if (!g) return NPCF_E_NOMEM;
    p->grid = g;
    const int D = p->D;
    g->ng = 1;
    for (int k = 0; k < D; k++) {
        g->dims[k] = dims[k];
        g->ng *= dims[k];
    }
    g->nbs = p->nb * p->t.nstate;
    DevAlloc &m = g->mem;
    g->khat = m.get<double2>((size_t)g->nbs * g->ng);
    g->work = m.get<double2>((size_t)g->nbs * g->ng);
    g->xhat = m.get<double2>(g->ng);
    g->w64 = m.get<double>(g->ng);
    g->w32 = m.get<float>(g->ng);
    g->sreal = m.get<uint8_t>(p->t.nstate);
    for (int k = 0; k < D; k++) g->tw[k] = m.get<double2>(dims[k] / 2);
    if (!m.ok) return NPCF_E_NOMEM;
    hipStream_t s = p->stream;
    std::vector<uint8_t> sreal(p->t.nstate);
    for (int st = 0; st < p->t.nstate; st++) sreal[st] = p->t.state_lab[3 * st] == 0;
    NPCF_TRY(hipMemcpyAsync(g->sreal, sreal.data(), sreal.size(), hipMemcpyHostToDevice, s));
    std::vector<std::vector<double2>> tws(D);
    for (int k = 0; k < D; k++) {
        const int n = dims[k];
        tws[k].resize(n / 2);
        for (int j = 0; j < n / 2; j++) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * j / n;
            tws[k][j] = make_double2((double)cosl(a), (double)-sinl(a));
        }
        NPCF_TRY(hipMemcpyAsync(g->tw[k], tws[k].data(), tws[k].size() * sizeof(double2), hipMemcpyHostToDevice, s));
    }
    GridArgs ga{};
    ga.ng = g->ng;
    for (int k = 0; k < 3; k++) {
        ga.dims[k] = k < D ? dims[k] : 1;
        ga.h[k] = k < D ? p->cfg.box[k] / dims[k] : 1.0;
    }
    ga.e2 = p->d_e2;
    ga.nb = p->nb;
    NPCF_TRY(launch_grid_kernel(D, p->L, ga, g->khat, (int64_t)g->nbs * g->ng, s));
    int64_t stride = g->ng;
    for (int k = 0; k < D; k++) {
        stride /= dims[k];
        NPCF_TRY(launch_fft(g->khat, g->khat, g->tw[k], dims[k], stride, (int64_t)g->nbs * g->ng, 0, nullptr, g->ng, s));
    }
    // in-range offsets (the same FP64 arithmetic as the kernel grid)
    const double *e2 = p->t.e2.data();
    int R[3] = {0, 0, 0};
    for (int k = 0; k < D; k++) R[k] = (int)std::ceil(p->edges[p->nb] / ga.h[k]) + 1;
    unsigned long long cnt = 0;
    for (int a0 = -R[0]; a0 <= R[0]; a0++)
        for (int a1 = -R[1]; a1 <= R[1]; a1++)
            for (int a2 = (D == 3 ? -R[2] : 0); a2 <= (D == 3 ? R[2] : 0); a2++) {
                const int mm[3] = {a0, a1, a2};
                double r2 = 0.0;
                for (int k = 0; k < D; k++) {
                    const double d = (double)mm[k] * ga.h[k];
                    r2 += d * d;
                }
                if (r2 >= e2[0] && r2 < e2[p->nb]) cnt++;
            }
    g->offsets_in_range = cnt;
    NPCF_TRY(hipStreamSynchronize(s));
    return NPCF_OK;
}

// a on every node of the grid (g->work), counting the primaries' pairs into
// the role's pair counter
npcf_status grid_harmonics(npcf_plan_s *p, const double *field, int64_t p0, int64_t p1, int role)
{
    GridState *g = p->grid;
    hipStream_t s = p->stream;
    const int D = p->D;
    double dV = 1.0;
    for (int k = 0; k < D; k++) dV *= p->cfg.box[k] / g->dims[k];
    StageTimer th;
    npcf_status st = timer_begin(p, 0, th);
    if (st != NPCF_OK) return st;
    NPCF_TRY(launch_grid_weights(field, g->ng, dV, g->w64, g->w32, g->xhat, p->bad, s));
    int64_t stride = g->ng;
    for (int k = 0; k < D; k++) {
        stride /= g->dims[k];
        NPCF_TRY(launch_fft(g->xhat, g->xhat, g->tw[k], g->dims[k], stride, g->ng, 0, nullptr, g->ng, s));
    }
    // a = FFT^-1[FFT(w) FFT(K')]: the product is taken as the first inverse pass loads
    stride = g->ng;
    for (int k = 0; k < D; k++) {
        stride /= g->dims[k];
        NPCF_TRY(launch_fft(k == 0 ? g->khat : g->work, g->work, g->tw[k], g->dims[k], stride,
                            (int64_t)g->nbs * g->ng, 1, k == 0 ? g->xhat : nullptr, g->ng, s));
    }
    NPCF_TRY(launch_add_u64(p->pairs + role, (unsigned long long)(p1 - p0) * g->offsets_in_range, s));
    NPCF_TRY(hipEventRecord(th.b, s));
    p->timers[0].push_back(th);
    return NPCF_OK;
}

npcf_status grid_accumulate(npcf_plan_s *p, const double *field, int64_t p0, int64_t p1, int role)
{
    GridState *g = p->grid;
    hipStream_t s = p->stream;
    npcf_status st = grid_harmonics(p, field, p0, p1, role);
    if (st != NPCF_OK) return st;
    for (int64_t c0 = p0; c0 < p1; c0 += p->wk.rows_cap) {
        const int rows = (int)std::min<int64_t>(p->wk.rows_cap, p1 - c0);
        StageTimer tr;
        st = timer_begin(p, 0, tr);
        if (st != NPCF_OK) return st;
        NPCF_TRY(launch_grid_rows(g->work, g->ng, g->nbs, p->t.nstate, g->sreal, g->w32, c0, rows, p->wk.A, p->wk.wrow, s));
        NPCF_TRY(hipEventRecord(tr.b, s));
        p->timers[0].push_back(tr);
        st = run_couple(p, p->wk, rows, p->acc[role]);
        if (st != NPCF_OK) return st;
    }
    return NPCF_OK;
}

// ---------------------------------------------------------------------------
// Autotuner cache: a JSON file of tuned knobs keyed by the problem's shape
//   {"npcf_tuning": 1, "entries": {"<key>": {"cell_subdiv": s, "couple_block": b,
//    "chunk_rows": r, "harmonic_blocks_per_cu": g, "curved_bins_per_pass": c, "ms": t}, ...}}
// ---------------------------------------------------------------------------
std::string tune_key(const npcf_plan_s *p, int64_t n)
{
    char buf[256];
    std::snprintf(buf, sizeof(buf), "D%d-N%d-L%d-nb%d-n%lld-box%.9g", p->D, p->N, p->L, p->nb, (long long)n,
                  p->cfg.box[0]);
    std::string k(buf);
    for (int d = 1; d < p->D; d++) {
        std::snprintf(buf, sizeof(buf), "x%.9g", p->cfg.box[d]);
        k += buf;
    }
    std::snprintf(buf, sizeof(buf), "-rmax%.9g-prec%d-mode%d-basis%d-per%d-geo%d-cu%d", p->edges[p->nb],
                  p->cfg.precision, p->cfg.btuple_mode, p->cfg.basis, p->cfg.periodic, (int)p->cfg.geometry, p->ncu);
    return k + buf;
}

std::string read_file(const char *path)
{
    std::string out;
    if (FILE *f = std::fopen(path, "rb")) {
        char buf[4096];
        size_t k;
        while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) out.append(buf, k);
        std::fclose(f);
    }
    return out;
}

// The entries of a cache file as (key, object text) pairs; malformed text gives none.
std::vector<std::pair<std::string, std::string>> tune_cache_entries(const std::string &text)
{
    std::vector<std::pair<std::string, std::string>> out;
    size_t at = text.find("\"entries\"");
    if (at == std::string::npos) return out;
    at = text.find('{', at);
    if (at == std::string::npos) return out;
    at++;
    for (;;) {
        const size_t k0 = text.find('"', at);
        const size_t close = text.find('}', at);
        if (k0 == std::string::npos || (close != std::string::npos && close < k0)) break;
        const size_t k1 = text.find('"', k0 + 1);
        const size_t o0 = text.find('{', k1);
        const size_t o1 = text.find('}', o0);
        if (k1 == std::string::npos || o0 == std::string::npos || o1 == std::string::npos) break;
        out.push_back({text.substr(k0 + 1, k1 - k0 - 1), text.substr(o0, o1 - o0 + 1)});
        at = o1 + 1;
    }
    return out;
}

double json_number(const std::string &obj, const char *field, double dflt)
{
    const std::string f = std::string("\"") + field + "\"";
    size_t at = obj.find(f);
    if (at == std::string::npos) return dflt;
    at = obj.find(':', at);
    if (at == std::string::npos) return dflt;
    return std::strtod(obj.c_str() + at + 1, nullptr);
}

bool tune_cache_lookup(const char *path, const std::string &key, npcf_tuning &t, double &ms)
{
    for (const auto &e : tune_cache_entries(read_file(path))) {
        if (e.first != key) continue;
        t.cell_subdiv = (int)json_number(e.second, "cell_subdiv", 0);
        t.couple_block = (int)json_number(e.second, "couple_block", 0);
        t.chunk_rows = (int64_t)json_number(e.second, "chunk_rows", 0);
        t.harmonic_blocks_per_cu = (int)json_number(e.second, "harmonic_blocks_per_cu", 0);
        t.curved_bins_per_pass = (int)json_number(e.second, "curved_bins_per_pass", 0);
        ms = json_number(e.second, "ms", 0.0);
        return t.cell_subdiv > 0;
    }
    return false;
}

void tune_cache_store(const char *path, const std::string &key, const npcf_tuning &t, double ms)
{
    auto entries = tune_cache_entries(read_file(path));
    char obj[256];
    std::snprintf(obj, sizeof(obj),
                  "{\"cell_subdiv\": %d, \"couple_block\": %d, \"chunk_rows\": %lld, \"harmonic_blocks_per_cu\": %d, "
                  "\"curved_bins_per_pass\": %d, \"ms\": %.6g}",
                  t.cell_subdiv, t.couple_block, (long long)t.chunk_rows, t.harmonic_blocks_per_cu,
                  t.curved_bins_per_pass, ms);
    bool found = false;
    for (auto &e : entries) {
        if (e.first == key) {
            e.second = obj;
            found = true;
        }
    }
    if (!found) entries.push_back({key, obj});
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\"npcf_tuning\": 1, \"entries\": {\n");
    for (size_t i = 0; i < entries.size(); i++)
        std::fprintf(f, "  \"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                     i + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

// ---------------------------------------------------------------------------
// Static workspace (npcf_accumulate_static).  Callers that cannot allocate
// device memory (code under stream capture, serving loops) get their per-call
// buffers from one file-scope device array.  The loader gives every device
// the library runs on its own copy at its own address, held until the process
// ends; host code never passes the array's name to a kernel (in host code it
// is a stand-in, not a device address): npcf_plan looks up this device's
// address once with hipGetSymbolAddress and every call uses that pointer.
// ---------------------------------------------------------------------------
constexpr size_t kStaticBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// This device's address of the static workspace (the device must be current).
npcf_status static_workspace(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return NPCF_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return dev_err_at(e, "hipGetSymbolAddress(scratch)", __LINE__);
        if (!ptr) return NPCF_E_DEVICE;
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return NPCF_OK;
}

// Coupling row blocks of a chunk of `rows` primaries.
int64_t couple_row_blocks(const npcf_plan_s *p, int64_t rows)
{
    const int64_t rpb = couple_rows_per_block(p, rows);
    return (rows + rpb - 1) / rpb;
}

// Cut the static workspace into the buffers of one flat accumulation of a
// catalogue of n points with nprim primaries: per-point arrays, the cell
// arrays of the plan's cell grid, the harmonic work counter, then the rows of
// a, row weights and coupling partials of the largest chunk of primaries that
// fits (at most the plan's chunk size).  *need receives the bytes the
// smallest layout (16-row chunks) would take.  False when even that does not fit.
bool carve_static(const npcf_plan_s *p, unsigned char *base, int64_t n, int64_t nprim, Workspace &W, size_t *need)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        return o;
    };
    const int D = p->D;
    size_t o_q[kMaxD] = {};
    for (int k = 0; k < D; k++) o_q[k] = take((size_t)n * 4);
    const size_t o_rec = take((size_t)n * 16), o_cell = take((size_t)n * 4);
    const size_t o_perm = take((size_t)n * 4), o_ps = take((size_t)n * 4), o_orig = take((size_t)n * 4),
                 o_prim = take((size_t)n * 4);
    const size_t o_ws = take((size_t)n * 4), o_w64 = take((size_t)n * 8);
    const size_t o_flag = take((size_t)n * 4), o_flagpos = take((size_t)n * 4);
    const int64_t nc = p->ncell + 1;
    const size_t o_count = take((size_t)nc * 4), o_cs = take((size_t)nc * 4), o_cur = take((size_t)nc * 4);
    const int64_t scan_len = (std::max<int64_t>(nc, n) + 1023) / 1024 + 1;
    const size_t o_scan = take((size_t)scan_len * 4);
    const size_t o_work = take(4);
    const size_t fixed = off;
    const int64_t rowbytes = (int64_t)p->nb * 2 * p->t.nstate * 4;
    const int64_t len = (int64_t)p->njobs * 256;
    auto chunk_bytes = [&](int64_t R) {
        // the largest block count over the full chunks and the last one
        int64_t nrb = couple_row_blocks(p, std::min(R, nprim));
        if (nprim % R) nrb = std::max(nrb, couple_row_blocks(p, nprim % R));
        return ((size_t)(R * rowbytes) + 255) / 256 * 256 + ((size_t)R * 4 + 255) / 256 * 256 +
               (size_t)nrb * len * 8;
    };
    int64_t R = std::min<int64_t>(p->wk.rows_cap, nprim);
    while (R > 16 && fixed + chunk_bytes(R) > kStaticBytes) R = std::max<int64_t>(16, (R / 2 + 15) / 16 * 16);
    *need = fixed + chunk_bytes(std::min<int64_t>(16, nprim));
    if (fixed + chunk_bytes(R) > kStaticBytes) return false;
    const size_t o_A = take((size_t)R * rowbytes), o_wrow = take((size_t)R * 4);
    int64_t nrb = couple_row_blocks(p, R);
    if (nprim % R) nrb = std::max(nrb, couple_row_blocks(p, nprim % R));
    const size_t o_part = take((size_t)nrb * len * 8);
    if (off > kStaticBytes) return false;
    for (int k = 0; k < D; k++) W.qtmp[k] = reinterpret_cast<uint32_t *>(base + o_q[k]);
    W.rec = reinterpret_cast<uint4 *>(base + o_rec);
    W.cell = reinterpret_cast<uint32_t *>(base + o_cell);
    W.perm = reinterpret_cast<int32_t *>(base + o_perm);
    W.perm_sorted = reinterpret_cast<int32_t *>(base + o_ps);
    W.orig = reinterpret_cast<int32_t *>(base + o_orig);
    W.prim = reinterpret_cast<int32_t *>(base + o_prim);
    W.ws = reinterpret_cast<float *>(base + o_ws);
    W.w64s = reinterpret_cast<double *>(base + o_w64);
    W.flag = reinterpret_cast<uint32_t *>(base + o_flag);
    W.flagpos = reinterpret_cast<uint32_t *>(base + o_flagpos);
    W.count = reinterpret_cast<uint32_t *>(base + o_count);
    W.cell_start = reinterpret_cast<uint32_t *>(base + o_cs);
    W.cursor = reinterpret_cast<uint32_t *>(base + o_cur);
    W.scan_scratch = reinterpret_cast<uint32_t *>(base + o_scan);
    W.scan_scratch_len = scan_len;
    W.work = reinterpret_cast<unsigned int *>(base + o_work);
    W.A = reinterpret_cast<float *>(base + o_A);
    W.wrow = reinterpret_cast<float *>(base + o_wrow);
    W.partial = reinterpret_cast<double *>(base + o_part);
    W.partial_len = nrb * len;
    W.rows_cap = R;
    W.growable = false;
    W.timed = false;
    return true;
}

}  // namespace

extern "C" {

const char *npcf_strerror(npcf_status status)
{
    switch (status) {
    case NPCF_OK: return "ok";
    case NPCF_E_INVALID: return "invalid argument or configuration";
    case NPCF_E_UNSUPPORTED: return "unsupported configuration";
    case NPCF_E_NOMEM: return "out of memory";
    case NPCF_E_DEVICE: return "HIP device error";
    case NPCF_E_STATE: return "call out of order (plan in failed state)";
    }
    return "unknown status";
}

const char *npcf_last_error_detail(void) { return g_last_error; }

const char *npcf_version(void) { return "npcf-mi355x 0.1 (gfx950)"; }

npcf_status npcf_plan(const npcf_config *cfg, void *stream, int64_t max_points, npcf_plan_t *out)
{
    if (!out) return NPCF_E_INVALID;
    *out = nullptr;
    g_last_error[0] = '\0';
    if (!cfg || max_points < 1 || max_points > (int64_t)INT32_MAX) return NPCF_E_INVALID;
    npcf_plan_s *p = new (std::nothrow) npcf_plan_s();
    if (!p) return NPCF_E_NOMEM;
    p->cfg = *cfg;
    std::string err;
    npcf_config c = *cfg;
    npcf_status st = build_tables(c, p->t, err);
    if (st != NPCF_OK) {
        delete p;
        return st;
    }
    if (p->t.nbt == 0) {
        // b1 < b2 < ... < b_{N-1} needs at least N - 1 bins: nothing to estimate
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "no radial tuple: %d bins with b1 < ... < b%d (btuple_mode 0) needs at least %d bins", cfg->nbins,
                      cfg->N - 1, cfg->N - 1);
        delete p;
        return NPCF_E_INVALID;
    }
    p->edges.assign(cfg->edges, cfg->edges + cfg->nbins + 1);
    p->cfg.edges = p->edges.data();
    for (int k = cfg->D; k < 4; k++) p->cfg.box[k] = 1.0;
    p->stream = (hipStream_t)stream;
    p->max_points = max_points;
    p->D = cfg->D;
    p->N = cfg->N;
    p->L = cfg->lmax;
    p->nb = cfg->nbins;
    p->cell_subdiv = (p->D == 4) ? 2 : 3;
    const Tables &t = p->t;
    p->njobs = p->N == 5 ? t.c5tiles : couple_njobs(p->N, t.nlam, t.nparts, t.mtiles);
    if (p->N == 4) {
        // a block's jobs are consecutive and span the Lambdas [lam(first), lam(last)]
        const int jpb = couple_jobs_per_block();
        for (int j0 = 0; j0 < p->njobs; j0 += jpb) {
            const int j1 = std::min(j0 + jpb, p->njobs) - 1;
            const int l0 = j0 / t.mtiles / t.nparts, l1 = j1 / t.mtiles / t.nparts;
            const int gb = t.lam_group_begin[l0], ge = t.lam_group_begin[l1 + 1];
            if (gb < ge)
                p->max_block_terms = std::max(p->max_block_terms, t.groups[ge - 1].term_end - t.groups[gb].term_begin);
        }
    } else if (p->N == 3 && t.n3_terms) {
        // line-of-sight basis: a block's jobs are up to jpb consecutive Lambdas,
        // one group each; the block copies the span of their term ranges
        const int jpb = couple_jobs_per_block();
        for (int j0 = 0; j0 < p->njobs; j0 += jpb) {
            int tb = INT_MAX, te = 0;
            for (int j = j0; j < std::min(j0 + jpb, p->njobs); j++) {
                const CoupleGroup &g = t.groups[t.lam_group_begin[j]];
                tb = std::min(tb, g.term_begin);
                te = std::max(te, g.term_end);
            }
            if (te > tb) p->max_block_terms = std::max(p->max_block_terms, te - tb);
        }
    }

    int dev = 0;
    if (const hipError_t eg = hipGetDevice(&dev); eg != hipSuccess) {
        delete p;
        return dev_err_at(eg, "hipGetDevice", __LINE__);
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            p->ncu = ncu;
    }
    // set-up of npcf_accumulate_static: this device's static workspace (a
    // failed lookup only disables that entry point, which then reports it)
    if (static_workspace(dev, &p->static_ws) != NPCF_OK) {
        p->static_ws = nullptr;
        g_last_error[0] = '\0';
    }
    compute_grid(p);
    {
        const char *cv = std::getenv("NPCF_COUPLING");
        p->term_coupling = cv && std::strcmp(cv, "terms") == 0;
        // the per-bin queue harmonic kernel is switched off (its first run
        // did not finish; no cause found yet): asking for it is an error
        const char *hv = std::getenv("NPCF_HARMONIC");
        if (hv && std::strcmp(hv, "stage") != 0 && std::strcmp(hv, "pass") != 0) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "NPCF_HARMONIC=%s: 'stage' (bin-sorted staging) or 'pass' (one pass per bin)", hv);
            delete p;
            return NPCF_E_UNSUPPORTED;
        }
        // one pass per bin by default for D = 2 and 3; D = 4 takes the staging
        // kernel unless asked (on the c5 catalogue the staging kernel was the
        // faster: lmax 4 92.2 against 99.8 ms, lmax 5 128.2 against 141.1 ms;
        // at lmax 6 the per-bin kernel does not exist)
        p->harm_pass = hv ? std::strcmp(hv, "pass") == 0 : p->D <= 3;
    }
    {
        const int L = p->L;
        const int lds = p->D == 2 ? harmonic_lds_bytes_d2(L) : (p->D == 3 ? harmonic_lds_bytes_d3(L) : harmonic_lds_bytes_d4(L));
        if (lds <= 0 || lds > 160 * 1024 || (p->N == 5 && couple5_lds_bytes(p->nb, t.nstate, t.c5_lds_extra) > 160 * 1024)) {
            delete p;
            return NPCF_E_UNSUPPORTED;
        }
    }
    DevAlloc &m = p->mem;
    for (int k = 0; k < p->D; k++) p->wk.qtmp[k] = m.get<uint32_t>(max_points);
    p->wk.rec = m.get<uint4>(max_points);
    p->wk.cell = m.get<uint32_t>(max_points);
    p->wk.perm = m.get<int32_t>(max_points);
    p->wk.perm_sorted = m.get<int32_t>(max_points);
    p->wk.orig = m.get<int32_t>(max_points);
    p->wk.prim = m.get<int32_t>(max_points);
    p->wk.ws = m.get<float>(max_points);
    p->wk.w64s = m.get<double>(max_points);
    if (t.sphere) {
        p->wk.pos64 = m.get<double>((size_t)4 * max_points);
        p->wk.caps = m.get<float>((size_t)8 * ((max_points + kSphChunk - 1) / kSphChunk + 1));
        p->wk.bbox = m.get<unsigned>(12);   // key-axis bounds [8], then the largest x0
    }
    p->wk.flag = m.get<uint32_t>(max_points);
    p->wk.flagpos = m.get<uint32_t>(max_points);
    const int64_t rowbytes = (int64_t)p->nb * 2 * t.nstate * sizeof(float);
    p->wk.rows_cap = std::min<int64_t>(max_points, std::max<int64_t>(1024, kADefaultBudget / rowbytes));
    p->rows_cap_max = p->wk.rows_cap;
    p->wk.A = m.get<float>((size_t)p->wk.rows_cap * p->nb * 2 * t.nstate);
    p->wk.wrow = m.get<float>(p->wk.rows_cap);
    // partials for the automatic coupling block size
    {
        int rpb = couple_rows_per_block(p, p->wk.rows_cap);
        int64_t nrb = (p->wk.rows_cap + rpb - 1) / rpb;
        p->wk.partial_len = nrb * (int64_t)p->njobs * 256;
        p->wk.partial = m.get<double>(p->wk.partial_len);
    }
    p->acc[0] = m.get<double>((size_t)p->njobs * 256);
    p->acc[1] = m.get<double>((size_t)p->njobs * 256);
    p->out_dev = m.get<double>((size_t)t.nlam * t.nparts * t.nbt);
    p->pairs = m.get<unsigned long long>(2);
    p->wk.work = m.get<unsigned int>(1);
    p->bad = m.get<int>(1);
    p->d_e2 = m.get<double>(t.e2.size());
    p->d_bucket = m.get<uint8_t>(t.bucket_bin.size());
    p->d_terms = m.get<CoupleTerm>(t.terms.size());
    p->d_groups = m.get<CoupleGroup>(std::max<size_t>(1, t.groups.size()));
    p->d_lam_group_begin = m.get<int>(t.lam_group_begin.size());
    p->d_lam_part = m.get<int>(t.lam_part.size());
    p->d_row_pairs = m.get<int2>(t.row_pairs.size());
    p->d_sfac = m.get<float>(t.sfac.size());
    p->d_bt_row = m.get<int>(t.bt_row.size());
    p->d_bt_col = m.get<int>(t.bt_col.size());
    p->d_bt_scale = m.get<double>(t.bt_scale.size());
    if (!t.fpairs.empty()) {
        p->d_fpairs = m.get<FPair>(t.fpairs.size());
        p->d_fgroups = m.get<FGroup>(t.fgroups.size());
        p->d_fprods = m.get<FProd>(t.fprods.size());
        p->d_fcoef = m.get<float>(t.fcoef.size());
        p->d_ftasks = m.get<int2>(t.ftasks.size());
    }
    if (p->N == 5) {
        p->d_c5jobs = m.get<C5Job>(t.c5jobs.size());
        p->d_c5labels = m.get<C5Label>(t.c5labels.size());
        p->d_c5mterm = m.get<int>(t.c5mterm.size());
        p->d_c5terms = m.get<uint2>(t.c5packed.size());
        p->d_c5pairs = m.get<int2>(t.c5pairs.size());
        p->d_c5idx = m.get<int>(t.c5idx.size());
        p->d_c5sign = m.get<double>(t.c5sign.size());
    }
    if (!m.ok || alloc_cells(p) != NPCF_OK) {
        p->mem.release();
        p->cellmem.release();
        delete p;
        return NPCF_E_NOMEM;
    }
    hipStream_t s = p->stream;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(p->d_e2, t.e2, s);
    if (e == hipSuccess) e = upload(p->d_bucket, t.bucket_bin, s);
    if (e == hipSuccess) e = upload(p->d_terms, t.terms, s);
    if (e == hipSuccess) e = upload(p->d_groups, t.groups, s);
    if (e == hipSuccess) e = upload(p->d_lam_group_begin, t.lam_group_begin, s);
    if (e == hipSuccess) e = upload(p->d_lam_part, t.lam_part, s);
    if (e == hipSuccess) e = upload(p->d_row_pairs, t.row_pairs, s);
    if (e == hipSuccess) e = upload(p->d_sfac, t.sfac, s);
    if (e == hipSuccess) e = upload(p->d_bt_row, t.bt_row, s);
    if (e == hipSuccess) e = upload(p->d_bt_col, t.bt_col, s);
    if (e == hipSuccess) e = upload(p->d_bt_scale, t.bt_scale, s);
    if (!t.fpairs.empty()) {
        if (e == hipSuccess) e = upload(p->d_fpairs, t.fpairs, s);
        if (e == hipSuccess) e = upload(p->d_fgroups, t.fgroups, s);
        if (e == hipSuccess) e = upload(p->d_fprods, t.fprods, s);
        if (e == hipSuccess) e = upload(p->d_fcoef, t.fcoef, s);
        if (e == hipSuccess) e = upload(p->d_ftasks, t.ftasks, s);
    }
    if (p->N == 5) {
        if (e == hipSuccess) e = upload(p->d_c5jobs, t.c5jobs, s);
        if (e == hipSuccess) e = upload(p->d_c5labels, t.c5labels, s);
        if (e == hipSuccess) e = upload(p->d_c5mterm, t.c5mterm, s);
        if (e == hipSuccess) e = upload(p->d_c5terms, t.c5packed, s);
        if (e == hipSuccess) e = upload(p->d_c5pairs, t.c5pairs, s);
        if (e == hipSuccess) e = upload(p->d_c5idx, t.c5idx, s);
        if (e == hipSuccess) e = upload(p->d_c5sign, t.c5sign, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        p->mem.release();
        p->cellmem.release();
        delete p;
        return dev_err_at(e, "table upload", __LINE__);
    }
    *out = p;
    st = npcf_reset(p);
    if (st != NPCF_OK) {
        npcf_destroy(p);
        *out = nullptr;
        return st;
    }
    return NPCF_OK;
}

npcf_status npcf_reset(npcf_plan_t p)
{
    if (!p) return NPCF_E_INVALID;
    hipStream_t s = p->stream;
    NPCF_TRY(launch_fill_f64(p->acc[0], 0.0, (int64_t)p->njobs * 256, s));
    NPCF_TRY(launch_fill_f64(p->acc[1], 0.0, (int64_t)p->njobs * 256, s));
    NPCF_TRY(launch_fill_u32((uint32_t *)p->pairs, 0u, 4, s));
    NPCF_TRY(launch_fill_u32((uint32_t *)p->bad, 0u, 1, s));
    NPCF_TRY(hipStreamSynchronize(s));
    clear_timers(p);
    p->failed = false;
    return NPCF_OK;
}

npcf_status npcf_destroy(npcf_plan_t p)
{
    if (!p) return NPCF_OK;
    (void)hipStreamSynchronize(p->stream);
    clear_timers(p);
    batch_release(p);
    grid_release(p);
    p->mem.release();
    p->cellmem.release();
    delete p;
    return NPCF_OK;
}

npcf_status npcf_set_tuning(npcf_plan_t p, int cell_subdiv, int couple_block, int64_t chunk_rows)
{
    if (!p) return NPCF_E_INVALID;
    if (cell_subdiv < 0 || cell_subdiv > 8 || couple_block < 0 || chunk_rows < 0 || chunk_rows > p->rows_cap_max)
        return NPCF_E_INVALID;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return NPCF_E_DEVICE;
    batch_release(p);  // the captured batch depends on every knob
    if (chunk_rows > 0) p->wk.rows_cap = chunk_rows;
    if (cell_subdiv > 0 && cell_subdiv != p->cell_subdiv) {
        p->cell_subdiv = cell_subdiv;
        compute_grid(p);
        npcf_status st = alloc_cells(p);
        if (st != NPCF_OK) {
            p->failed = true;
            return st;
        }
    }
    if (couple_block > 0) p->couple_rows = couple_block;
    return NPCF_OK;
}

npcf_status npcf_accumulate(npcf_plan_t p, const double *pos, const double *w, int64_t n, int64_t prim_begin,
                            int64_t prim_end, int role)
{
    npcf_status st = check_inputs(p, pos, w, n, prim_begin, prim_end);
    if (st != NPCF_OK) return st;
    if (role != NPCF_ROLE_DATA && role != NPCF_ROLE_RANDOMS) return NPCF_E_INVALID;
    st = accumulate_impl(p, p->wk, pos, w, n, prim_begin, prim_end, p->acc[role], p->pairs + role);
    if (st != NPCF_OK) p->failed = true;
    return st;
}

static npcf_status grid_check(npcf_plan_t p, const double *field, const int *dims, int64_t prim_begin,
                              int64_t prim_end)
{
    if (!p || !field || !dims) return NPCF_E_INVALID;
    if (p->failed) return NPCF_E_STATE;
    if (p->t.sphere) {
        std::snprintf(g_last_error, sizeof(g_last_error), "gridded data needs flat geometry");
        return NPCF_E_UNSUPPORTED;
    }
    if (p->D > 3) {
        std::snprintf(g_last_error, sizeof(g_last_error), "gridded data needs D = 2 or 3");
        return NPCF_E_UNSUPPORTED;
    }
    if (!p->cfg.periodic) {
        std::snprintf(g_last_error, sizeof(g_last_error), "gridded data needs a periodic box");
        return NPCF_E_INVALID;
    }
    int64_t ng = 1;
    for (int k = 0; k < p->D; k++) {
        if (!pow2_in(dims[k], 2, 2048)) {
            std::snprintf(g_last_error, sizeof(g_last_error), "grid dims must be powers of two in 2..2048");
            return NPCF_E_INVALID;
        }
        ng *= dims[k];
    }
    if (ng > (int64_t)INT32_MAX || prim_begin < 0 || prim_end > ng || prim_begin >= prim_end) return NPCF_E_INVALID;
    bool same = p->grid != nullptr;
    for (int k = 0; k < p->D && same; k++) same = p->grid->dims[k] == dims[k];
    npcf_status st = NPCF_OK;
    if (!same) st = grid_setup(p, dims);
    if (st != NPCF_OK) p->failed = true;
    return st;
}

npcf_status npcf_accumulate_grid(npcf_plan_t p, const double *field, const int *dims, int64_t prim_begin,
                                 int64_t prim_end, int role)
{
    if (p && role != NPCF_ROLE_DATA && role != NPCF_ROLE_RANDOMS) return NPCF_E_INVALID;
    npcf_status st = grid_check(p, field, dims, prim_begin, prim_end);
    if (st != NPCF_OK) return st;
    st = grid_accumulate(p, field, prim_begin, prim_end, role);
    if (st != NPCF_OK) p->failed = true;
    return st;
}

npcf_status npcf_alm_grid(npcf_plan_t p, const double *field, const int *dims, int64_t prim_begin, int64_t prim_end,
                          double *out, size_t out_len)
{
    npcf_status st = grid_check(p, field, dims, prim_begin, prim_end);
    if (st != NPCF_OK) return st;
    const Tables &t = p->t;
    const int64_t nprim = prim_end - prim_begin;
    const int64_t per = (int64_t)p->nb * t.nstate * 2;
    if (!out || out_len != (size_t)(nprim * per)) return NPCF_E_INVALID;
    st = grid_harmonics(p, field, prim_begin, prim_end, NPCF_ROLE_DATA);
    if (st != NPCF_OK) {
        p->failed = true;
        return st;
    }
    GridState *g = p->grid;
    std::vector<float> Ah;
    for (int64_t c0 = prim_begin; c0 < prim_end; c0 += p->wk.rows_cap) {
        const int rows = (int)std::min<int64_t>(p->wk.rows_cap, prim_end - c0);
        NPCF_TRY(launch_grid_rows(g->work, g->ng, g->nbs, t.nstate, g->sreal, g->w32, c0, rows, p->wk.A, p->wk.wrow,
                                  p->stream));
        Ah.resize((size_t)rows * per);
        NPCF_TRY(hipMemcpyAsync(Ah.data(), p->wk.A, (size_t)rows * per * sizeof(float), hipMemcpyDeviceToHost, p->stream));
        NPCF_TRY(hipStreamSynchronize(p->stream));
        for (int r = 0; r < rows; r++)
            for (int b = 0; b < p->nb; b++)
                for (int64_t k = 0; k < 2 * t.nstate; k++)
                    out[(c0 - prim_begin + r) * per + b * 2 * t.nstate + k] =
                        (double)Ah[(size_t)r * per + b * 2 * t.nstate + k] / t.vb[b];
    }
    return NPCF_OK;
}

npcf_status npcf_describe(npcf_plan_t p, int *n_lambda, int *lambda_labels, int *n_bt, int *btuples, size_t *out_len)
{
    if (!p) return NPCF_E_INVALID;
    const Tables &t = p->t;
    if (n_lambda) *n_lambda = t.nlam;
    if (lambda_labels) std::memcpy(lambda_labels, t.lam_lab.data(), t.lam_lab.size() * sizeof(int));
    if (n_bt) *n_bt = t.nbt;
    if (btuples) std::memcpy(btuples, t.bt_lab.data(), t.bt_lab.size() * sizeof(int));
    if (out_len) *out_len = (size_t)t.nlam * t.nbt * t.nparts;
    return NPCF_OK;
}

static npcf_status finalize_from(npcf_plan_t p, const double *acc, const double *acc_rand, double *out, size_t out_len)
{
    const Tables &t = p->t;
    if (!out || out_len != (size_t)t.nlam * t.nbt * t.nparts) return NPCF_E_INVALID;
    hipStream_t s = p->stream;
    if (p->N == 5)
        NPCF_TRY(launch_finalize_idx(acc, acc_rand, p->d_c5idx, p->d_c5sign, p->d_bt_scale, t.nlam, t.nbt,
                                     p->cfg.norm == NPCF_NORM_BY_RANDOMS, t.lam0, p->out_dev, p->bad, s));
    else
        NPCF_TRY(launch_finalize2(acc, acc_rand, t.nlam, t.nparts, t.mtiles, p->d_bt_row, p->d_bt_col, p->d_bt_scale,
                                  t.nbt, p->cfg.norm == NPCF_NORM_BY_RANDOMS, t.lam0, p->out_dev, p->bad, s));
    NPCF_TRY(hipMemcpyAsync(out, p->out_dev, out_len * sizeof(double), hipMemcpyDeviceToHost, s));
    int bad = 0;
    NPCF_TRY(hipMemcpyAsync(&bad, p->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    NPCF_TRY(hipStreamSynchronize(s));
    if (bad) return NPCF_E_INVALID;
    return NPCF_OK;
}

npcf_status npcf_finalize(npcf_plan_t p, double *out, size_t out_len)
{
    if (!p) return NPCF_E_INVALID;
    if (p->failed) return NPCF_E_STATE;
    return finalize_from(p, p->acc[0], p->acc[1], out, out_len);
}

npcf_status npcf_pair_count(npcf_plan_t p, int64_t *pairs_data, int64_t *pairs_randoms)
{
    if (!p) return NPCF_E_INVALID;
    unsigned long long h[2] = {0, 0};
    NPCF_TRY(hipMemcpyAsync(h, p->pairs, sizeof(h), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipStreamSynchronize(p->stream));
    if (pairs_data) *pairs_data = (int64_t)h[0];
    if (pairs_randoms) *pairs_randoms = (int64_t)h[1];
    return NPCF_OK;
}

npcf_status npcf_alm(npcf_plan_t p, const double *pos, const double *w, int64_t n, int64_t prim_begin,
                     int64_t prim_end, double *out, size_t out_len)
{
    npcf_status st = check_inputs(p, pos, w, n, prim_begin, prim_end);
    if (st != NPCF_OK) return st;
    const Tables &t = p->t;
    const int64_t nprim = prim_end - prim_begin;
    const int64_t per = (int64_t)p->nb * t.nstate * 2;
    if (!out || out_len != (size_t)(nprim * per)) return NPCF_E_INVALID;
    if (t.sphere) {
        std::vector<float> Ah;
        for (int64_t c0 = prim_begin; c0 < prim_end; c0 += p->wk.rows_cap) {
            const int rows = (int)std::min<int64_t>(p->wk.rows_cap, prim_end - c0);
            st = run_sphere(p, p->wk, pos, w, n, c0, rows, p->pairs);
            if (st != NPCF_OK) {
                p->failed = true;
                return st;
            }
            Ah.resize((size_t)rows * per);
            NPCF_TRY(hipMemcpyAsync(Ah.data(), p->wk.A, (size_t)rows * per * sizeof(float), hipMemcpyDeviceToHost, p->stream));
            NPCF_TRY(hipStreamSynchronize(p->stream));
            for (int r = 0; r < rows; r++)
                for (int b = 0; b < p->nb; b++)
                    for (int64_t k = 0; k < 2 * t.nstate; k++)
                        out[(c0 - prim_begin + r) * per + b * 2 * t.nstate + k] =
                            (double)Ah[(size_t)r * per + b * 2 * t.nstate + k] / t.vb[b];
        }
        return NPCF_OK;
    }
    st = prepare(p, p->wk, pos, w, n, prim_begin, prim_end);
    if (st != NPCF_OK) {
        p->failed = true;
        return st;
    }
    std::vector<int32_t> prim(nprim), orig(n);
    NPCF_TRY(hipMemcpyAsync(prim.data(), p->wk.prim, nprim * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipMemcpyAsync(orig.data(), p->wk.orig, n * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    std::vector<float> Ah;
    unsigned long long *scratch_pairs = p->pairs;  // counted as data pairs
    for (int64_t c0 = 0; c0 < nprim; c0 += p->wk.rows_cap) {
        const int rows = (int)std::min<int64_t>(p->wk.rows_cap, nprim - c0);
        st = run_harmonic(p, p->wk, rows, p->wk.prim + c0, scratch_pairs);
        if (st != NPCF_OK) {
            p->failed = true;
            return st;
        }
        Ah.resize((size_t)rows * per);
        NPCF_TRY(hipMemcpyAsync(Ah.data(), p->wk.A, (size_t)rows * per * sizeof(float), hipMemcpyDeviceToHost, p->stream));
        NPCF_TRY(hipStreamSynchronize(p->stream));
        for (int r = 0; r < rows; r++) {
            const int64_t o = orig[prim[c0 + r]] - prim_begin;
            for (int b = 0; b < p->nb; b++)
                for (int64_t k = 0; k < 2 * t.nstate; k++)
                    out[o * per + b * 2 * t.nstate + k] = (double)Ah[(size_t)r * per + b * 2 * t.nstate + k] / t.vb[b];
        }
    }
    return NPCF_OK;
}

npcf_status npcf_accumulate_batch(npcf_plan_t p, int ncat, const double *const *pos, const double *const *w,
                                  const int64_t *n)
{
    if (p && p->t.sphere) {
        std::snprintf(g_last_error, sizeof(g_last_error), "batches are for flat geometry");
        return NPCF_E_UNSUPPORTED;
    }
    if (!p || ncat < 1 || !pos || !w || !n) return NPCF_E_INVALID;
    if (p->failed) return NPCF_E_STATE;
    if (p->cfg.norm == NPCF_NORM_BY_RANDOMS) return NPCF_E_UNSUPPORTED;
    for (int c = 0; c < ncat; c++)
        if (!pos[c] || !w[c] || n[c] < 1) return NPCF_E_INVALID;
    npcf_status st = NPCF_OK;
    if (!batch_same_shape(p->batch, ncat, pos, w, n, p->ncs)) {
        NPCF_TRY(hipStreamSynchronize(p->stream));
        st = batch_setup(p, ncat, pos, w, n);
        if (st != NPCF_OK) {
            batch_release(p);
            return st;
        }
    }
    BatchState *b = p->batch;
    // order after the caller's stream, capture once, replay
    NPCF_TRY(hipEventRecord(b->ev_in, p->stream));
    NPCF_TRY(hipStreamWaitEvent(b->cs, b->ev_in, 0));
    if (!b->exec) {
        NPCF_TRY(hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed));
        st = batch_record(p, b->cs);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->cs, &g);
        if (st != NPCF_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            batch_release(p);
            return st != NPCF_OK ? st : dev_err_at(ec, "hipStreamEndCapture", __LINE__);
        }
        b->graph = g;
        const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            batch_release(p);
            return dev_err_at(ei, "hipGraphInstantiate", __LINE__);
        }
    }
    NPCF_TRY(hipGraphLaunch(b->exec, b->cs));
    NPCF_TRY(hipEventRecord(b->ev_out, b->cs));
    NPCF_TRY(hipStreamWaitEvent(p->stream, b->ev_out, 0));
    b->done = true;
    return NPCF_OK;
}

npcf_status npcf_finalize_batch(npcf_plan_t p, int cat, double *out, size_t out_len, double *done_ms,
                                int64_t *pairs)
{
    if (!p) return NPCF_E_INVALID;
    if (p->failed) return NPCF_E_STATE;
    BatchState *b = p->batch;
    if (!b || !b->done) return NPCF_E_STATE;
    if (cat < 0 || cat >= b->ncat) return NPCF_E_INVALID;
    const int64_t len = (int64_t)p->njobs * 256;
    npcf_status st = finalize_from(p, b->acc + (size_t)cat * len, nullptr, out, out_len);
    if (st != NPCF_OK) return st;
    unsigned long long h[2] = {0, 0}, pc = 0;
    NPCF_TRY(hipMemcpyAsync(&h[0], b->ts + cat, sizeof(unsigned long long), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipMemcpyAsync(&h[1], b->ts + b->ncat, sizeof(unsigned long long), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipMemcpyAsync(&pc, b->pairs + cat, sizeof(unsigned long long), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipStreamSynchronize(p->stream));
    if (done_ms) *done_ms = (double)(int64_t)(h[0] - h[1]) / b->clock_khz;
    if (pairs) *pairs = (int64_t)pc;
    return NPCF_OK;
}

npcf_status npcf_get_tuning(npcf_plan_t p, npcf_tuning *out)
{
    if (!p || !out) return NPCF_E_INVALID;
    out->cell_subdiv = p->cell_subdiv;
    out->couple_block = p->couple_rows;
    out->chunk_rows = p->wk.rows_cap;
    out->harmonic_blocks_per_cu = p->harm_bpc > 0 ? p->harm_bpc : 8;
    out->curved_bins_per_pass = p->t.sphere ? p->curved_group : 0;
    return NPCF_OK;
}

npcf_status npcf_apply_tuning(npcf_plan_t p, const npcf_tuning *t)
{
    if (!p || !t) return NPCF_E_INVALID;
    if (t->harmonic_blocks_per_cu < 0 || t->harmonic_blocks_per_cu > 32) return NPCF_E_INVALID;
    const int g = t->curved_bins_per_pass;
    if (g != 0 && (!p->t.sphere || (g != sph_group(p->D, p->L, false) && g != sph_group(p->D, p->L, true)))) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "npcf_apply_tuning: curved_bins_per_pass %d is not one of the kernel's widths for this plan", g);
        return NPCF_E_INVALID;
    }
    npcf_status st = npcf_set_tuning(p, t->cell_subdiv, t->couple_block, t->chunk_rows);
    if (st != NPCF_OK) return st;
    if (t->harmonic_blocks_per_cu > 0) p->harm_bpc = t->harmonic_blocks_per_cu;
    if (g != 0) p->curved_group = g;
    return NPCF_OK;
}

npcf_status npcf_autotune(npcf_plan_t p, const double *pos, const double *w, int64_t n, int64_t sample,
                          int *cell_subdiv, int *couple_block, double *best_ms)
{
    npcf_status st = check_inputs(p, pos, w, n, 0, n);
    if (st != NPCF_OK) return st;
    const std::string key = tune_key(p, n);
    const char *cache = std::getenv("NPCF_TUNE_CACHE");
    npcf_tuning cached{};
    double cached_ms = 0.0;
    if (cache && *cache && tune_cache_lookup(cache, key, cached, cached_ms)) {
        st = npcf_apply_tuning(p, &cached);
        if (st != NPCF_OK) return st;
        if (cell_subdiv) *cell_subdiv = p->cell_subdiv;
        if (couple_block) *couple_block = p->couple_rows;
        if (best_ms) *best_ms = cached_ms;
        return npcf_reset(p);
    }
    if (sample < 4) sample = 4;
    if (sample > n) sample = n;
    // time the stages over primary ranges spread over the catalogue (data and
    // randoms alike), best of two
    auto spread = [&](int64_t per_range) {
        std::vector<std::pair<int64_t, int64_t>> r;
        for (int k = 0; k < 4; k++) {
            const int64_t a = n * k / 4, b = std::min<int64_t>(n, a + std::max<int64_t>(1, per_range));
            if (a < b) r.push_back({a, b});
        }
        return r;
    };
    auto measure = [&](const std::vector<std::pair<int64_t, int64_t>> &ranges, double &harm, double &coup) -> npcf_status {
        double bh = 1e300, bc = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            npcf_status s2 = npcf_reset(p);
            if (s2 != NPCF_OK) return s2;
            for (auto &r : ranges) {
                s2 = npcf_accumulate(p, pos, w, n, r.first, r.second, NPCF_ROLE_DATA);
                if (s2 != NPCF_OK) return s2;
            }
            double ms3[3];
            s2 = npcf_stage_ms(p, ms3);
            if (s2 != NPCF_OK) return s2;
            bh = std::min(bh, ms3[0] + ms3[2]);
            bc = std::min(bc, ms3[1]);
        }
        harm = bh;
        coup = bc;
        return NPCF_OK;
    };
    const auto small = spread(sample / 4);
    const std::vector<std::pair<int64_t, int64_t>> whole{{0, n}};
    double h = 0.0, c = 0.0;
    st = measure(small, h, c);  // first launches (code loading) out of the way
    if (st != NPCF_OK) return st;
    int best_s = p->cell_subdiv;
    double best_h = 1e300;
    if (p->t.sphere) {
        // curved spaces (no cell grid): the all-pairs kernel's two widths,
        // on the whole catalogue (which of them wins depends on the share of
        // visited pairs in the bins, which a part of the catalogue need not
        // have); the narrow one (the default) unless the wide one wins by 2%
        const int gw = sph_group(p->D, p->L, false), gn = sph_group(p->D, p->L, true);
        std::vector<int> widths{gn};
        if (gw != gn) widths.push_back(gw);
        int best_w = gn;
        for (int g : widths) {
            p->curved_group = g;
            st = measure(whole, h, c);
            if (st != NPCF_OK) return st;
            if (h < best_h * (g == gn ? 1.0 : 0.98)) {
                best_h = h;
                best_w = g;
            }
        }
        p->curved_group = best_w;
    } else {
        // harmonic stage with its cell list: the cell subdivision, then the
        // persistent grid's blocks per CU, on four spread ranges of up to 128k
        // primaries (a quarter of the catalogue at most): enough rows to fill the
        // persistent grid (8192 waves at 8 blocks per CU) many times over, so
        // that the timing follows throughput; a few thousand primaries leave
        // waves idle and rank the subdivisions by the latency of single rows
        // (2M D = 4 points: s = 3 chosen on 4096 primaries, 211 ms per launch
        // against 179 ms at s = 2)
        const auto quarter = spread(std::max<int64_t>(sample / 4, std::min<int64_t>(n / 16, 131072)));
        const int smax = p->D == 4 ? 4 : 6;
        for (int sdv = 1; sdv <= smax; sdv++) {
            st = npcf_set_tuning(p, sdv, 0, 0);
            if (st != NPCF_OK) return st;
            st = measure(quarter, h, c);
            if (st != NPCF_OK) return st;
            if (h < best_h) {
                best_h = h;
                best_s = sdv;
            }
        }
        st = npcf_set_tuning(p, best_s, 0, 0);
        if (st != NPCF_OK) return st;
        int best_g = 8;
        for (int g : {2, 3, 4, 6, 8}) {
            p->harm_bpc = g;
            st = measure(quarter, h, c);
            if (st != NPCF_OK) return st;
            if (h < best_h * (g == 8 ? 1.0 : 0.98)) {   // a different grid must win by 2%
                best_h = h;
                best_g = g;
            }
        }
        p->harm_bpc = best_g;
    }
    // coupling block size and chunk rows on the whole catalogue: the
    // automatic block size and a fixed one give different block counts on a
    // part of it than on the full launches (2M D = 4 points: 512 rows per
    // block won on a quarter by more than 2% and lost on the whole, 59.3
    // against 57.0 ms)
    int best_b = 0;
    double best_c = 1e300, best_q = 1e300;
    for (int b : {0, 256, 512, 1024, 2048}) {
        batch_release(p);
        p->couple_rows = b;
        st = measure(whole, h, c);
        if (st != NPCF_OK) return st;
        if (c < best_c * (b == 0 ? 1.0 : 0.98)) {   // the automatic rule unless 2% slower
            best_c = c;
            best_b = b;
            best_q = h + c;
        }
    }
    p->couple_rows = best_b;
    const int64_t full_rows = p->rows_cap_max;
    int64_t best_r = full_rows;
    for (int64_t r : {full_rows, std::max<int64_t>(1024, n / 32)}) {
        if (r > full_rows || r == best_r) continue;
        st = npcf_set_tuning(p, 0, 0, r);
        if (st != NPCF_OK) return st;
        st = measure(whole, h, c);
        if (st != NPCF_OK) return st;
        if (h + c < 0.98 * best_q) {
            best_q = h + c;
            best_r = r;
        }
    }
    st = npcf_set_tuning(p, 0, 0, best_r);
    if (st != NPCF_OK) return st;
    st = npcf_reset(p);
    if (st != NPCF_OK) return st;
    if (cache && *cache) {
        npcf_tuning t{};
        (void)npcf_get_tuning(p, &t);
        tune_cache_store(cache, key, t, best_h + best_c);
    }
    if (cell_subdiv) *cell_subdiv = best_s;
    if (couple_block) *couple_block = best_b;
    if (best_ms) *best_ms = best_h + best_c;
    return NPCF_OK;
}

npcf_status npcf_accumulate_static(npcf_plan_t p, const double *pos, const double *w, int64_t n, int64_t prim_begin,
                                   int64_t prim_end, int role)
{
    npcf_status st = check_inputs(p, pos, w, n, prim_begin, prim_end);
    if (st != NPCF_OK) return st;
    if (role != NPCF_ROLE_DATA && role != NPCF_ROLE_RANDOMS) return NPCF_E_INVALID;
    if (p->t.sphere) {
        std::snprintf(g_last_error, sizeof(g_last_error), "npcf_accumulate_static: flat geometry only");
        return NPCF_E_UNSUPPORTED;
    }
    if (!p->static_ws) {
        std::snprintf(g_last_error, sizeof(g_last_error), "npcf_accumulate_static: no static workspace on this device");
        return NPCF_E_DEVICE;
    }
    Workspace W;
    size_t need = 0;
    if (!carve_static(p, static_cast<unsigned char *>(p->static_ws), n, prim_end - prim_begin, W, &need)) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "npcf_accumulate_static: %lld points need %zu bytes of workspace, the static limit is %zu",
                      (long long)n, need, kStaticBytes);
        return NPCF_E_INVALID;
    }
    st = accumulate_impl(p, W, pos, w, n, prim_begin, prim_end, p->acc[role], p->pairs + role);
    if (st != NPCF_OK) p->failed = true;
    return st;
}

// Stage times (ms) accumulated since the last reset: [0] harmonic, [1] coupling + reduce, [2] cell list.
npcf_status npcf_stage_ms(npcf_plan_t p, double *ms3)
{
    if (!p || !ms3) return NPCF_E_INVALID;
    for (int k = 0; k < 3; k++) {
        double s = 0.0;
        for (auto &t : p->timers[k]) s += elapsed(t);
        ms3[k] = s;
    }
    return NPCF_OK;
}

}  // extern "C"
