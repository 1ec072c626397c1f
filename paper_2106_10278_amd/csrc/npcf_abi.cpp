// C ABI of the NPCF library (include/npcf.h): plan lifecycle, device
// workspace, and the per-call orchestration of
//   quantise -> cell list -> primary list -> [harmonic -> coupling -> FP64 reduce] per chunk
// on the plan's stream.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
    int ncs[kMaxD] = {1, 1, 1, 1};
    int64_t ncell = 1;
    int64_t rows_cap = 0;
    int njobs = 0;
    int max_block_terms = 0;  // N = 4: coupling terms one coupling block copies to LDS
    bool failed = false;

    DevAlloc mem;
    DevAlloc cellmem;  // cell arrays (re-allocated when the cell grid changes)
    // catalogue workspace
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
    // stage buffers
    float *A = nullptr, *wrow = nullptr;
    double *partial = nullptr;
    int64_t partial_len = 0;
    double *acc[2] = {nullptr, nullptr};
    double *out_dev = nullptr;
    unsigned long long *pairs = nullptr;  // [2]
    unsigned int *work = nullptr;
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
    // stage timing (harmonic, coupling, prep) in ms, accumulated since reset
    std::vector<StageTimer> timers[3];
    // batch state
    std::vector<double *> batch_acc;
    std::vector<hipEvent_t> batch_done;
    hipEvent_t batch_start = nullptr;
};

namespace {

npcf_status dev_err(hipError_t e) { return e == hipSuccess ? NPCF_OK : (e == hipErrorOutOfMemory ? NPCF_E_NOMEM : NPCF_E_DEVICE); }

#define NPCF_TRY(expr)                                  \
    do {                                                \
        hipError_t e__ = (expr);                        \
        if (e__ != hipSuccess) return dev_err(e__);     \
    } while (0)

template <class T>
hipError_t upload(T *dst, const std::vector<T> &src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

void compute_grid(npcf_plan_s *p)
{
    const double rmax = p->edges[p->nb];
    int64_t total = 1;
    for (int k = 0; k < kMaxD; k++) p->ncs[k] = 1;
    int s = p->cell_subdiv;
    for (;;) {
        total = 1;
        for (int k = 0; k < p->D; k++) {
            double c = std::floor(p->cfg.box[k] / (rmax / s));
            if (c < 1) c = 1;
            if (c > 4096) c = 4096;
            p->ncs[k] = (int)c;
            total *= p->ncs[k];
        }
        if (total <= (1LL << 24) || s == 1) break;
        s--;
    }
    p->ncell = total;
}

npcf_status alloc_cells(npcf_plan_s *p)
{
    p->cellmem.release();
    p->cellmem.ok = true;
    p->count = p->cellmem.get<uint32_t>(p->ncell + 1);
    p->cell_start = p->cellmem.get<uint32_t>(p->ncell + 1);
    p->cursor = p->cellmem.get<uint32_t>(p->ncell + 1);
    int64_t m = std::max<int64_t>(p->ncell + 1, p->max_points);
    p->scan_scratch_len = (m + 1023) / 1024 + 1;
    p->scan_scratch = p->cellmem.get<uint32_t>(p->scan_scratch_len);
    return p->cellmem.ok ? NPCF_OK : NPCF_E_NOMEM;
}

int couple_rows_per_block(const npcf_plan_s *p, int64_t nrows)
{
    if (p->couple_rows > 0) return ((p->couple_rows + 15) / 16) * 16;
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
npcf_status build_cells(npcf_plan_s *p, const double *pos, const double *w, int64_t n)
{
    hipStream_t s = p->stream;
    NPCF_TRY(launch_fill_u32(p->count, 0u, p->ncell + 1, s));
    NPCF_TRY(launch_quantize(p->D, p->cfg.periodic, pos, w, n, p->cfg.box, p->ncs, p->qtmp, p->cell, p->count, p->bad, s));
    NPCF_TRY(launch_exclusive_scan(p->count, p->cell_start, p->ncell + 1, p->scan_scratch, p->scan_scratch_len, s));
    NPCF_TRY(hipMemcpyAsync(p->cursor, p->cell_start, (p->ncell + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    NPCF_TRY(launch_scatter_perm(n, p->cell, p->cursor, p->perm, s));
    NPCF_TRY(launch_cellsort(n, p->cell, p->cell_start, p->perm, p->perm_sorted, s));
    NPCF_TRY(launch_gather(p->D, n, p->perm_sorted, p->qtmp, w, p->rec, p->ws, p->w64s, p->orig, s));
    return NPCF_OK;
}

HarmArgs harm_args(const npcf_plan_s *p, int rows, const int32_t *prim, unsigned long long *pairs)
{
    HarmArgs a{};
    a.rec = p->rec;
    for (int k = 0; k < kMaxD; k++) {
        a.ncs[k] = p->ncs[k];
        a.cell_len[k] = 4294967296.0 / p->ncs[k];
        a.inv_cell_len[k] = p->ncs[k] / 4294967296.0;
        double sc = (k < p->D) ? p->cfg.box[k] / 4294967296.0 : 1.0;
        a.scale64[k] = sc;
        a.scale[k] = (float)sc;
        a.rmax_lat[k] = p->edges[p->nb] / sc;
    }
    a.w = p->ws;
    a.cell_start = p->cell_start;
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
    a.A = p->A;
    a.wrow = p->wrow;
    a.pairs = pairs;
    a.work = p->work;
    a.periodic = p->cfg.periodic;
    return a;
}

npcf_status run_harmonic(npcf_plan_s *p, int rows, const int32_t *prim, unsigned long long *pairs)
{
    hipStream_t s = p->stream;
    NPCF_TRY(launch_fill_u32(p->work, 0u, 1, s));
    HarmArgs a = harm_args(p, rows, prim, pairs);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) ncu = prop.multiProcessorCount;
    }
    // persistent grid: a few workgroups per CU, rows handed out dynamically
    int grid = ncu * 8;
    int64_t need = ((int64_t)rows + 3) / 4;
    if (grid > need) grid = (int)std::max<int64_t>(1, need);
    StageTimer t;
    npcf_status st = timer_begin(p, 0, t);
    if (st != NPCF_OK) return st;
    hipError_t e;
    switch (p->D) {
    case 2: e = launch_harmonic_d2(p->L, a, grid, s); break;
    case 3: e = launch_harmonic_d3(p->L, a, grid, s); break;
    default: e = launch_harmonic_d4(p->L, a, grid, s); break;
    }
    NPCF_TRY(e);
    NPCF_TRY(hipEventRecord(t.b, s));
    p->timers[0].push_back(t);
    return NPCF_OK;
}

npcf_status run_couple(npcf_plan_s *p, int rows, double *acc)
{
    hipStream_t s = p->stream;
    const Tables &t = p->t;
    CoupleArgs a{};
    a.A = p->A;
    a.wrow = p->wrow;
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
    const int64_t len = (int64_t)p->njobs * 256;
    if ((int64_t)a.n_rowblocks * len > p->partial_len) {
        // grow the partial buffer (rare: only with small custom block sizes)
        void *np = nullptr;
        NPCF_TRY(hipStreamSynchronize(s));
        NPCF_TRY(hipMalloc(&np, (size_t)a.n_rowblocks * len * sizeof(double)));
        p->mem.ptrs.push_back(np);
        p->partial = (double *)np;
        p->partial_len = (int64_t)a.n_rowblocks * len;
    }
    a.partial = p->partial;
    StageTimer tm;
    npcf_status st = timer_begin(p, 1, tm);
    if (st != NPCF_OK) return st;
    NPCF_TRY(launch_couple_kernel(p->N, p->cfg.precision, a, p->njobs, t.nparts, p->d_sfac, s));
    NPCF_TRY(launch_reduce_partials(p->partial, a.n_rowblocks, len, acc, s));
    NPCF_TRY(hipEventRecord(tm.b, s));
    p->timers[1].push_back(tm);
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

npcf_status prepare(npcf_plan_s *p, const double *pos, const double *w, int64_t n, int64_t p0, int64_t p1)
{
    StageTimer t;
    npcf_status st = timer_begin(p, 2, t);
    if (st != NPCF_OK) return st;
    st = build_cells(p, pos, w, n);
    if (st != NPCF_OK) return st;
    NPCF_TRY(launch_primlist(n, p->orig, p0, p1, p->flag, p->flagpos, p->prim, p->scan_scratch, p->scan_scratch_len,
                             p->stream));
    NPCF_TRY(hipEventRecord(t.b, p->stream));
    p->timers[2].push_back(t);
    return NPCF_OK;
}

npcf_status accumulate_impl(npcf_plan_s *p, const double *pos, const double *w, int64_t n, int64_t p0, int64_t p1,
                            double *acc, unsigned long long *pairs)
{
    npcf_status st = prepare(p, pos, w, n, p0, p1);
    if (st != NPCF_OK) return st;
    const int64_t nprim = p1 - p0;
    for (int64_t c0 = 0; c0 < nprim; c0 += p->rows_cap) {
        const int rows = (int)std::min<int64_t>(p->rows_cap, nprim - c0);
        st = run_harmonic(p, rows, p->prim + c0, pairs);
        if (st != NPCF_OK) return st;
        st = run_couple(p, rows, acc);
        if (st != NPCF_OK) return st;
    }
    return NPCF_OK;
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

const char *npcf_version(void) { return "npcf-mi355x 0.1 (gfx950)"; }

npcf_status npcf_plan(const npcf_config *cfg, void *stream, int64_t max_points, npcf_plan_t *out)
{
    if (!out) return NPCF_E_INVALID;
    *out = nullptr;
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
    p->njobs = couple_njobs(p->N, t.nlam, t.nparts, t.mtiles);
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
    }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete p;
        return NPCF_E_DEVICE;
    }
    compute_grid(p);
    {
        const int L = p->L;
        const int lds = p->D == 2 ? harmonic_lds_bytes_d2(L) : (p->D == 3 ? harmonic_lds_bytes_d3(L) : harmonic_lds_bytes_d4(L));
        if (lds <= 0 || lds > 160 * 1024) {
            delete p;
            return NPCF_E_UNSUPPORTED;
        }
    }
    DevAlloc &m = p->mem;
    for (int k = 0; k < p->D; k++) p->qtmp[k] = m.get<uint32_t>(max_points);
    p->rec = m.get<uint4>(max_points);
    p->cell = m.get<uint32_t>(max_points);
    p->perm = m.get<int32_t>(max_points);
    p->perm_sorted = m.get<int32_t>(max_points);
    p->orig = m.get<int32_t>(max_points);
    p->prim = m.get<int32_t>(max_points);
    p->ws = m.get<float>(max_points);
    p->w64s = m.get<double>(max_points);
    p->flag = m.get<uint32_t>(max_points);
    p->flagpos = m.get<uint32_t>(max_points);
    const int64_t rowbytes = (int64_t)p->nb * 2 * t.nstate * sizeof(float);
    p->rows_cap = std::min<int64_t>(max_points, std::max<int64_t>(1024, kADefaultBudget / rowbytes));
    p->A = m.get<float>((size_t)p->rows_cap * p->nb * 2 * t.nstate);
    p->wrow = m.get<float>(p->rows_cap);
    // partials for the automatic coupling block size
    {
        int rpb = couple_rows_per_block(p, p->rows_cap);
        int64_t nrb = (p->rows_cap + rpb - 1) / rpb;
        p->partial_len = nrb * (int64_t)p->njobs * 256;
        p->partial = m.get<double>(p->partial_len);
    }
    p->acc[0] = m.get<double>((size_t)p->njobs * 256);
    p->acc[1] = m.get<double>((size_t)p->njobs * 256);
    p->out_dev = m.get<double>((size_t)t.nlam * t.nparts * t.nbt);
    p->pairs = m.get<unsigned long long>(2);
    p->work = m.get<unsigned int>(1);
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
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        p->mem.release();
        p->cellmem.release();
        delete p;
        return dev_err(e);
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
    for (auto e : p->batch_done) (void)hipEventDestroy(e);
    if (p->batch_start) (void)hipEventDestroy(p->batch_start);
    for (auto a : p->batch_acc) (void)hipFree(a);
    p->mem.release();
    p->cellmem.release();
    delete p;
    return NPCF_OK;
}

npcf_status npcf_set_tuning(npcf_plan_t p, int cell_subdiv, int couple_block)
{
    if (!p) return NPCF_E_INVALID;
    if (cell_subdiv < 0 || cell_subdiv > 4 || couple_block < 0) return NPCF_E_INVALID;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return NPCF_E_DEVICE;
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
    st = accumulate_impl(p, pos, w, n, prim_begin, prim_end, p->acc[role], p->pairs + role);
    if (st != NPCF_OK) p->failed = true;
    return st;
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
    NPCF_TRY(launch_finalize2(acc, acc_rand, t.nlam, t.nparts, t.mtiles, p->d_bt_row, p->d_bt_col, p->d_bt_scale, t.nbt,
                              p->cfg.norm == NPCF_NORM_BY_RANDOMS, t.lam0, p->out_dev, p->bad, s));
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
    st = prepare(p, pos, w, n, prim_begin, prim_end);
    if (st != NPCF_OK) {
        p->failed = true;
        return st;
    }
    std::vector<int32_t> prim(nprim), orig(n);
    NPCF_TRY(hipMemcpyAsync(prim.data(), p->prim, nprim * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    NPCF_TRY(hipMemcpyAsync(orig.data(), p->orig, n * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    std::vector<float> Ah;
    unsigned long long *scratch_pairs = p->pairs;  // counted as data pairs
    for (int64_t c0 = 0; c0 < nprim; c0 += p->rows_cap) {
        const int rows = (int)std::min<int64_t>(p->rows_cap, nprim - c0);
        st = run_harmonic(p, rows, p->prim + c0, scratch_pairs);
        if (st != NPCF_OK) {
            p->failed = true;
            return st;
        }
        Ah.resize((size_t)rows * per);
        NPCF_TRY(hipMemcpyAsync(Ah.data(), p->A, (size_t)rows * per * sizeof(float), hipMemcpyDeviceToHost, p->stream));
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
    (void)pos;
    (void)w;
    (void)n;
    if (!p || ncat < 1) return NPCF_E_INVALID;
    return NPCF_E_UNSUPPORTED;
}

npcf_status npcf_finalize_batch(npcf_plan_t p, int cat, double *out, size_t out_len, double *done_ms)
{
    (void)cat;
    (void)out;
    (void)out_len;
    (void)done_ms;
    if (!p) return NPCF_E_INVALID;
    return NPCF_E_UNSUPPORTED;
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
