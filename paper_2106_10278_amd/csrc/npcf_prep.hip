// Ingest and cell list of the NPCF harmonic stage.
//
//  - quantise: positions (FP64) onto the box * q / 2^32 lattice, cell id per
//    point, histogram of cell occupancy;
//  - exclusive scan of the histogram -> cell_start;
//  - scatter: every point takes a slot of its cell (atomic cursor);
//  - in-cell order: each cell's slots are re-ranked by original index so the
//    sorted order (and every floating-point sum downstream) is deterministic;
//  - gather: coalesced SoA arrays of lattice coordinates and weights in
//    sorted order.
//
// All kernels are HBM/latency bound and cheap next to the harmonic stage.
#include "npcf_internal.h"

namespace npcf {

namespace {

constexpr int kBlk = 256;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

struct QuantArgs {
    const double *pos;
    const double *w;
    int64_t n;
    double box[kMaxD];
    int ncs[kMaxD];
    int periodic;
    uint32_t *q[kMaxD];
    uint32_t *cell;
    uint32_t *count;
    int *bad;
};

template <int D>
__global__ void k_quantize(QuantArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    bool ok = isfinite(a.w[i]);
    uint64_t lin = 0;
    uint64_t mul = 1;
#pragma unroll
    for (int k = 0; k < D; k++) {
        double x = a.pos[(int64_t)k * a.n + i];
        ok = ok && isfinite(x);
        if (!a.periodic) ok = ok && x >= 0.0 && x < a.box[k];
        double t = x / a.box[k];
        t = t - floor(t);                       // periodic wrap into [0, 1)
        double qd = rint(t * 4294967296.0);     // nearest lattice point
        uint64_t qq = (uint64_t)(int64_t)qd;
        if (!a.periodic && qq > 0xffffffffull) qq = 0xffffffffull;
        uint32_t q = (uint32_t)(qq & 0xffffffffull);
        if (!ok) q = 0;
        a.q[k][i] = q;
        uint64_t c = ((uint64_t)q * (uint64_t)a.ncs[k]) >> 32;
        lin += c * mul;
        mul *= (uint64_t)a.ncs[k];
    }
    if (!ok) atomicOr(a.bad, 1);
    a.cell[i] = (uint32_t)lin;
    atomicAdd(&a.count[lin], 1u);
}

struct QuantBatchArgs {
    const double *const *pos;   // [ncat] device pointers, SoA [D][n_c]
    const double *const *w;     // [ncat]
    const int64_t *off;         // [ncat + 1] first global index of each catalogue
    int ncat;
    int64_t ntot;
    double box[kMaxD];
    int ncs[kMaxD];
    int64_t ncell_cat;
    int periodic;
    uint32_t *q[kMaxD];
    double *wall;
    uint32_t *cell;
    uint32_t *count;
    int *bad;
};

template <int D>
__global__ void k_quantize_batch(QuantBatchArgs a)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.ntot) return;
    int lo = 0, hi = a.ncat;  // catalogue c with off[c] <= g < off[c + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.off[mid] <= g) lo = mid;
        else hi = mid;
    }
    const int64_t i = g - a.off[lo];
    const int64_t n = a.off[lo + 1] - a.off[lo];
    const double *pos = a.pos[lo];
    const double wi = a.w[lo][i];
    bool ok = isfinite(wi);
    uint64_t lin = 0, mul = 1;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const double x = pos[(int64_t)k * n + i];
        ok = ok && isfinite(x);
        if (!a.periodic) ok = ok && x >= 0.0 && x < a.box[k];
        double t = x / a.box[k];
        t = t - floor(t);
        const double qd = rint(t * 4294967296.0);
        uint64_t qq = (uint64_t)(int64_t)qd;
        if (!a.periodic && qq > 0xffffffffull) qq = 0xffffffffull;
        uint32_t q = (uint32_t)(qq & 0xffffffffull);
        if (!ok) q = 0;
        a.q[k][g] = q;
        lin += (((uint64_t)q * (uint64_t)a.ncs[k]) >> 32) * mul;
        mul *= (uint64_t)a.ncs[k];
    }
    if (!ok) atomicOr(a.bad, 1);
    const uint64_t key = (uint64_t)lo * (uint64_t)a.ncell_cat + lin;
    a.wall[g] = wi;
    a.cell[g] = (uint32_t)key;
    atomicAdd(&a.count[key], 1u);
}

__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void k_timestamp(unsigned long long *ts)
{
    if (threadIdx.x == 0) *ts = (unsigned long long)wall_clock64();
}

// ---- exclusive scan (1024 elements per block, 256 threads x 4) -------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlk * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // Hillis-Steele over 256 threads in LDS.
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlk; off <<= 1) {
        uint32_t add = (t >= off) ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[kBlk - 1];
    uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void k_tile_sums(const uint32_t *in, int64_t n, uint32_t *sums)
{
    __shared__ uint32_t sh[kBlk];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++)
        if (base + j < n) s += in[base + j];
    uint32_t tot;
    block_exclusive_scan(s, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(uint32_t *sums, int64_t m)
{
    __shared__ uint32_t sh[kBlk];
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += kBlk) {
        int64_t i = base + threadIdx.x;
        uint32_t v = (i < m) ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, sh, tot);
        if (i < m) sums[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
}

__global__ void k_tile_scan(const uint32_t *in, uint32_t *out, int64_t n, const uint32_t *sums)
{
    __shared__ uint32_t sh[kBlk];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = (base + j < n) ? in[base + j] : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, sh, tot) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
}

__global__ void k_scatter_perm(int64_t n, const uint32_t *cell, uint32_t *cursor, int32_t *perm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t slot = atomicAdd(&cursor[cell[i]], 1u);
    perm[slot] = (int32_t)i;
}

// Rank each slot inside its cell by original index.  Cells above kMaxRank
// keep the (non-deterministic) atomic order.
constexpr uint32_t kMaxRank = 8192;

__global__ void k_cellsort(int64_t n, const uint32_t *cell, const uint32_t *cell_start, const int32_t *perm,
                           int32_t *perm_sorted)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t i = perm[j];
    uint32_t c = cell[i];
    uint32_t b = cell_start[c], e = cell_start[c + 1];
    if (e - b > kMaxRank) {
        perm_sorted[j] = i;
        return;
    }
    uint32_t rank = 0;
    for (uint32_t t = b; t < e; t++) rank += (perm[t] < i) ? 1u : 0u;
    perm_sorted[b + rank] = i;
}

struct GatherArgs {
    int64_t n;
    const int32_t *perm;
    const uint32_t *qtmp[kMaxD];
    const double *w;
    uint4 *rec;
    float *ws;
    double *w64s;
    int32_t *orig;
};

// Sorted catalogue as 16-byte records (one load per candidate in the
// harmonic stage): D = 2 (q0, q1, w, 0), D = 3 (q0, q1, q2, w), D = 4 (q0..q3)
// with w the FP32 weight bits; FP32 and FP64 weights also as arrays.
template <int D>
__global__ void k_gather(GatherArgs a)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    int32_t i = a.perm[j];
    double wi = a.w[i];
    if (!isfinite(wi)) wi = 0.0;
    const float wf = (float)wi;
    uint4 r;
    r.x = a.qtmp[0][i];
    r.y = a.qtmp[1][i];
    if (D == 2) {
        r.z = __float_as_uint(wf);
        r.w = 0u;
    } else if (D == 3) {
        r.z = a.qtmp[2][i];
        r.w = __float_as_uint(wf);
    } else {
        r.z = a.qtmp[2][i];
        r.w = a.qtmp[3][i];
    }
    a.rec[j] = r;
    a.ws[j] = wf;
    a.w64s[j] = wi;
    a.orig[j] = i;
}

__global__ void k_prim_flag(int64_t n, const int32_t *orig, int64_t p0, int64_t p1, uint32_t *flag)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t o = orig[j];
    flag[j] = (o >= p0 && o < p1) ? 1u : 0u;
}

__global__ void k_prim_compact(int64_t n, const uint32_t *flag, const uint32_t *pos, int32_t *prim)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (flag[j]) prim[pos[j]] = (int32_t)j;
}

inline unsigned grid_for(int64_t n, int blk = kBlk)
{
    int64_t g = (n + blk - 1) / blk;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t g = (n + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlk), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t g = (n + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)g), dim3(kBlk), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_quantize(int D, int periodic, const double *pos, const double *w, int64_t n, const double *box,
                            const int *ncs, uint32_t *const qtmp[kMaxD], uint32_t *cell, uint32_t *count, int *bad,
                            hipStream_t s)
{
    QuantArgs a{};
    a.pos = pos;
    a.w = w;
    a.n = n;
    for (int k = 0; k < kMaxD; k++) {
        a.box[k] = box[k];
        a.ncs[k] = ncs[k];
        a.q[k] = qtmp[k];
    }
    a.periodic = periodic;
    a.cell = cell;
    a.count = count;
    a.bad = bad;
    switch (D) {
    case 2: hipLaunchKernelGGL(k_quantize<2>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_quantize<3>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_quantize<4>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_quantize_batch(int D, int periodic, int ncat, const double *const *pos, const double *const *w,
                                 const int64_t *off, int64_t ntot, const double *box, const int *ncs,
                                 int64_t ncell_cat, uint32_t *const qtmp[kMaxD], double *wall, uint32_t *cell,
                                 uint32_t *count, int *bad, hipStream_t s)
{
    QuantBatchArgs a{};
    a.pos = pos;
    a.w = w;
    a.off = off;
    a.ncat = ncat;
    a.ntot = ntot;
    for (int k = 0; k < kMaxD; k++) {
        a.box[k] = box[k];
        a.ncs[k] = ncs[k];
        a.q[k] = qtmp[k];
    }
    a.ncell_cat = ncell_cat;
    a.periodic = periodic;
    a.wall = wall;
    a.cell = cell;
    a.count = count;
    a.bad = bad;
    switch (D) {
    case 2: hipLaunchKernelGGL(k_quantize_batch<2>, dim3(grid_for(ntot)), dim3(kBlk), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_quantize_batch<3>, dim3(grid_for(ntot)), dim3(kBlk), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_quantize_batch<4>, dim3(grid_for(ntot)), dim3(kBlk), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t g = (n + kBlk - 1) / kBlk;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_copy_u32, dim3((unsigned)g), dim3(kBlk), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_timestamp(unsigned long long *ts, hipStream_t s)
{
    hipLaunchKernelGGL(k_timestamp, dim3(1), dim3(64), 0, s, ts);
    return hipGetLastError();
}

// scratch must hold ceil(n / 1024) entries.
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *scratch,
                                 int64_t scratch_len, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles > scratch_len) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)tiles), dim3(kBlk), 0, s, in, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlk), 0, s, scratch, tiles);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)tiles), dim3(kBlk), 0, s, in, out, n, scratch);
    return hipGetLastError();
}

hipError_t launch_scatter_perm(int64_t n, const uint32_t *cell, uint32_t *cursor, int32_t *perm, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_perm, dim3(grid_for(n)), dim3(kBlk), 0, s, n, cell, cursor, perm);
    return hipGetLastError();
}

hipError_t launch_cellsort(int64_t n, const uint32_t *cell, const uint32_t *cell_start, const int32_t *perm,
                           int32_t *perm_sorted, hipStream_t s)
{
    hipLaunchKernelGGL(k_cellsort, dim3(grid_for(n)), dim3(kBlk), 0, s, n, cell, cell_start, perm, perm_sorted);
    return hipGetLastError();
}

hipError_t launch_gather(int D, int64_t n, const int32_t *perm_sorted, uint32_t *const qtmp[kMaxD],
                         const double *w, uint4 *rec, float *ws, double *w64s, int32_t *orig, hipStream_t s)
{
    GatherArgs a{};
    a.n = n;
    a.perm = perm_sorted;
    for (int k = 0; k < kMaxD; k++) a.qtmp[k] = qtmp[k] ? qtmp[k] : qtmp[0];
    a.w = w;
    a.rec = rec;
    a.ws = ws;
    a.w64s = w64s;
    a.orig = orig;
    switch (D) {
    case 2: hipLaunchKernelGGL(k_gather<2>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_gather<3>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_gather<4>, dim3(grid_for(n)), dim3(kBlk), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_primlist(int64_t n, const int32_t *orig, int64_t p0, int64_t p1, uint32_t *flag,
                           uint32_t *pos_out, int32_t *prim, uint32_t *scratch, int64_t scratch_len, hipStream_t s)
{
    hipLaunchKernelGGL(k_prim_flag, dim3(grid_for(n)), dim3(kBlk), 0, s, n, orig, p0, p1, flag);
    hipError_t e = launch_exclusive_scan(flag, pos_out, n, scratch, scratch_len, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prim_compact, dim3(grid_for(n)), dim3(kBlk), 0, s, n, flag, pos_out, prim);
    return hipGetLastError();
}

}  // namespace npcf
