// Gridded-data estimator (section "Application to Gridded Data"): for a field
// X on a periodic grid the harmonic coefficients of every node come from one
// correlation per (bin, state),
//   a^b_s(x) = sum_r w(x + r) conj(Y_s(rhat)) Theta^b(|r|),   w = X dV
// (the 1/v_b of eq. alm-bin-def is applied at finalize, as on the pair path),
// evaluated as the convolution w * K' with K'(r) = conj(Y_s(-rhat)) Theta^b(|r|):
//   a^b_s = FFT^-1[ FFT(w) FFT(K') ]
// (the kernel with its sign flip stands for the (-1)^l of the paper's form).
// The node rows of a then go through the same coupling kernels as the pair
// path.  FFTs: complex FP64, power-of-two sizes, one axis per pass, T lines
// per block in LDS (bit-reversed load, radix-2 passes, natural-order store).
#include "npcf_internal.h"
#include "npcf_harmonics.h"

namespace npcf {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int bitrev(int e, int log2n) { return (int)(__brev((unsigned)e) >> (32 - log2n)); }

// One axis of a batched FFT: lines of length n (element stride s) over
// `lines` lines (line L: outer L / s, inner L % s, first element
// (L / s) n s + L % s).  src may equal dst.  With premul, element addr of src
// is multiplied by premul[addr % ng] on load.
__global__ __launch_bounds__(256) void k_fft_axis(const double2 *src, double2 *dst, const double2 *tw, int n, int log2n,
                                                  int64_t s, int64_t lines, int T, int inverse, const double2 *premul,
                                                  int64_t ng)
{
    extern __shared__ __align__(16) char smem[];
    double2 *sh = reinterpret_cast<double2 *>(smem);   // [T][n]
    double2 *twl = sh + (size_t)T * n;                 // [n / 2]
    for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
        double2 w = tw[j];
        if (inverse) w.y = -w.y;
        twl[j] = w;
    }
    const int64_t L0 = (int64_t)blockIdx.x * T;
    const bool t_fast = s >= T;   // consecutive lines are adjacent in memory
    for (int q = threadIdx.x; q < T * n; q += blockDim.x) {
        int t, e;
        if (t_fast) {
            e = q / T;
            t = q - e * T;
        } else {
            t = q / n;
            e = q - t * n;
        }
        const int64_t L = L0 + t;
        if (L >= lines) continue;
        const int64_t addr = (L / s) * n * s + (L % s) + (int64_t)e * s;
        double2 v = src[addr];
        if (premul) v = cmul(v, premul[addr % ng]);
        sh[t * n + bitrev(e, log2n)] = v;
    }
    __syncthreads();
    const int nh = n / 2;
    for (int len = 2, ls = 1; len <= n; len <<= 1, ls++) {
        const int half = len >> 1;
        for (int k = threadIdx.x; k < T * nh; k += blockDim.x) {
            const int t = k / nh, j = k - t * nh;
            const int grp = j / half, pos = j - grp * half;
            const int i0 = t * n + grp * len + pos, i1 = i0 + half;
            const double2 w = twl[pos << (log2n - ls)];
            const double2 a = sh[i0], b = cmul(sh[i1], w);
            sh[i0] = make_double2(a.x + b.x, a.y + b.y);
            sh[i1] = make_double2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < T * n; q += blockDim.x) {
        int t, e;
        if (t_fast) {
            e = q / T;
            t = q - e * T;
        } else {
            t = q / n;
            e = q - t * n;
        }
        const int64_t L = L0 + t;
        if (L >= lines) continue;
        dst[(L / s) * n * s + (L % s) + (int64_t)e * s] = sh[t * n + e];
    }
}

// K'_{b,s} at every grid offset: node index -> minimum-image integer offset m,
// r = m h, bin of r^2 (FP64, the definition's arithmetic), and for an
// in-range r the harmonics of u = -rhat times 1 / ng (the inverse FFT is
// unnormalised).  kern is zero-filled before; states l1 = 0 get no
// imaginary part.
template <int D, int L>
__global__ __launch_bounds__(256) void k_grid_kernel(GridArgs g, double2 *kern)
{
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.ng) return;
    int64_t rem = node;
    double d[3] = {0.0, 0.0, 0.0};
    double r2 = 0.0;
    for (int k = D - 1; k >= 0; k--) {
        const int i = (int)(rem % g.dims[k]);
        rem /= g.dims[k];
        const int m = (i <= g.dims[k] / 2) ? i : i - g.dims[k];
        d[k] = (double)m * g.h[k];
    }
    for (int k = 0; k < D; k++) r2 += d[k] * d[k];
    if (!(r2 >= g.e2[0] && r2 < g.e2[g.nb])) return;
    int b = 0;
    while (b + 1 < g.nb && r2 >= g.e2[b + 1]) b++;
    const double inv = 1.0 / sqrt(r2);
    float u[D];
    for (int k = 0; k < D; k++) u[k] = (float)(-d[k] * inv);
    constexpr int nst = stored_states(D, L);
    double2 *out = kern + (int64_t)b * nst * g.ng + node;
    const float wk = (float)(1.0 / (double)g.ng);
    harm::harmonics<D, L>(u, wk, [&](int slot, float v) {
        double2 *p = out + (int64_t)(slot >> 1) * g.ng;
        if (slot & 1)
            p->y = (double)v;
        else
            p->x = (double)v;
    });
}

// w = X dV (FP64 and FP32), the forward-FFT input (w, 0), and a flag for
// non-finite field values.
__global__ void k_grid_weights(const double *field, int64_t ng, double dV, double *w64, float *w32, double2 *xin,
                               int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double x = field[i];
    if (!isfinite(x)) atomicOr(bad, 1);
    const double w = x * dV;
    w64[i] = w;
    w32[i] = (float)w;
    xin[i] = make_double2(w, 0.0);
}

// Rows of a for nodes [r0, r0 + rows): A[row][b][2 s + c] from the batch
// layout a[(b nst + s)][node] (tiled through LDS so that both sides are
// coalesced), and the rows' FP32 weights.
constexpr int kRowTile = 32;
__global__ __launch_bounds__(256) void k_grid_rows(const double2 *a, int64_t ng, int nbs, int nst, const uint8_t *sreal,
                                                   const float *w32, int64_t r0, int rows, float *A, float *wrow)
{
    __shared__ float2 tile[kRowTile][kRowTile + 1];
    const int64_t node0 = r0 + (int64_t)blockIdx.x * kRowTile;
    const int bs0 = blockIdx.y * kRowTile;
    const int tx = threadIdx.x & (kRowTile - 1), ty = threadIdx.x / kRowTile;   // 32 x 8
    for (int j = ty; j < kRowTile; j += 8) {
        const int bs = bs0 + j;
        const int64_t node = node0 + tx;
        float2 v = make_float2(0.f, 0.f);
        if (bs < nbs && node < r0 + rows) {
            const double2 x = a[(int64_t)bs * ng + node];
            v = make_float2((float)x.x, sreal[bs % nst] ? 0.f : (float)x.y);
        }
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < kRowTile; j += 8) {
        const int64_t node = node0 + j;
        const int bs = bs0 + tx;
        if (bs < nbs && node < r0 + rows)
            reinterpret_cast<float2 *>(A)[(node - r0) * nbs + bs] = tile[tx][j];
    }
    if (blockIdx.y == 0)
        for (int j = threadIdx.x; j < kRowTile; j += blockDim.x) {
            const int64_t node = node0 + j;
            if (node < r0 + rows) wrow[node - r0] = w32[node];
        }
}

__global__ void k_add_u64(unsigned long long *p, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(p, v);
}

__global__ void k_fill_c64(double2 *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

template <int D, int L>
hipError_t launch_kernel_dl(const GridArgs &g, double2 *kern, hipStream_t s)
{
    hipLaunchKernelGGL((k_grid_kernel<D, L>), dim3((unsigned)((g.ng + 255) / 256)), dim3(256), 0, s, g, kern);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_kernel(int D, int L, const GridArgs &g, double2 *kern, int64_t nkern, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_c64, dim3((unsigned)((nkern + 255) / 256)), dim3(256), 0, s, kern, nkern);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define NPCF_GK(DD, LL) \
    case LL: return launch_kernel_dl<DD, LL>(g, kern, s);
    if (D == 2) {
        switch (L) {
            NPCF_GK(2, 0) NPCF_GK(2, 1) NPCF_GK(2, 2) NPCF_GK(2, 3) NPCF_GK(2, 4) NPCF_GK(2, 5) NPCF_GK(2, 6)
            NPCF_GK(2, 7) NPCF_GK(2, 8) NPCF_GK(2, 9) NPCF_GK(2, 10) NPCF_GK(2, 11) NPCF_GK(2, 12) NPCF_GK(2, 13)
            NPCF_GK(2, 14) NPCF_GK(2, 15) NPCF_GK(2, 16)
        default: return hipErrorInvalidValue;
        }
    }
    if (D == 3) {
        switch (L) {
            NPCF_GK(3, 0) NPCF_GK(3, 1) NPCF_GK(3, 2) NPCF_GK(3, 3) NPCF_GK(3, 4) NPCF_GK(3, 5) NPCF_GK(3, 6)
            NPCF_GK(3, 7) NPCF_GK(3, 8) NPCF_GK(3, 9) NPCF_GK(3, 10)
        default: return hipErrorInvalidValue;
        }
    }
#undef NPCF_GK
    return hipErrorInvalidValue;
}

int fft_lines_per_block(int n) { return std::max(1, 2048 / n); }

int fft_lds_bytes(int n) { return (fft_lines_per_block(n) * n + n / 2) * (int)sizeof(double2); }

hipError_t launch_fft(const double2 *src, double2 *dst, const double2 *tw, int n, int64_t s, int64_t total, int inverse,
                      const double2 *premul, int64_t ng, hipStream_t st)
{
    int log2n = 0;
    while ((1 << log2n) < n) log2n++;
    const int T = fft_lines_per_block(n);
    const int64_t lines = total / n;
    const int64_t blocks = (lines + T - 1) / T;
    const int lds = fft_lds_bytes(n);
    hipError_t e = hipFuncSetAttribute((const void *)k_fft_axis, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_axis, dim3((unsigned)blocks), dim3(256), lds, st, src, dst, tw, n, log2n, s, lines, T,
                       inverse, premul, ng);
    return hipGetLastError();
}

hipError_t launch_grid_weights(const double *field, int64_t ng, double dV, double *w64, float *w32, double2 *xin,
                               int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_weights, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, field, ng, dV, w64, w32,
                       xin, bad);
    return hipGetLastError();
}

hipError_t launch_grid_rows(const double2 *a, int64_t ng, int nbs, int nst, const uint8_t *sreal, const float *w32,
                            int64_t r0, int rows, float *A, float *wrow, hipStream_t s)
{
    const dim3 grid((unsigned)((rows + kRowTile - 1) / kRowTile), (unsigned)((nbs + kRowTile - 1) / kRowTile));
    hipLaunchKernelGGL(k_grid_rows, grid, dim3(256), 0, s, a, ng, nbs, nst, sreal, w32, r0, rows, A, wrow);
    return hipGetLastError();
}

hipError_t launch_add_u64(unsigned long long *p, unsigned long long v, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace npcf
