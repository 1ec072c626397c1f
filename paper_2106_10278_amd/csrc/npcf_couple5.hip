// Coupling stage of the isotropic 5PCF (D = 3, N = 5; section "Hydrodynamic
// Turbulence"): the kernel that contracts S~_M (first two legs, coupled to
// l12) with T~_M (last two legs) over primaries and M on MFMA.  Tables and
// the job layout: C5Job / build_c5.
#include "npcf_couple_common.h"

namespace npcf {

namespace {

// FP16 hi + lo slice with a power-of-two scale per A row and per B column
// (lanes n, n+16, n+32, n+48 hold one row / column): used where a tile mixes
// rows of very different size, which one scale per tile would push into
// FP16's subnormal range.  c[v] (row 4 kq + v, column n) is returned unscaled
// in FP64 in out[v].
__device__ __forceinline__ float pow2_scale(float m)
{
    if (!(m > 0.f) || !isfinite(m)) return 1.f;
    int e;
    frexpf(m, &e);
    return ldexpf(1.f, -e);
}

__device__ __forceinline__ void mfma_k32_f16_rowscaled(const float (&Av)[8], const float (&Bv)[8], int kq, double (&out)[4])
{
    float ma = 0.f, mb = 0.f;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        ma = fmaxf(ma, fabsf(Av[i]));
        mb = fmaxf(mb, fabsf(Bv[i]));
    }
    ma = max_over_lane_bits45(ma);
    mb = max_over_lane_bits45(mb);
    const float sa = pow2_scale(ma), sb = pow2_scale(mb);
    v8h ah, al, bh, bl;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const float x = Av[i] * sa, y = Bv[i] * sb;
        ah[i] = (_Float16)x;
        al[i] = (_Float16)(x - (float)ah[i]);
        bh[i] = (_Float16)y;
        bl[i] = (_Float16)(y - (float)bh[i]);
    }
    v4f c = v4f{0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, c, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const float sr = __shfl(sa, 4 * kq + v);   // lane 4 kq + v holds row 4 kq + v's scale
        out[v] = (double)c[v] / ((double)sr * (double)sb);
    }
}

// ---------------------------------------------------------------------------
// N = 5, D = 3 (isotropic 5PCF): job = (l12, beta = b2, S-label group, column
// group).  Per staged step of 16 primaries and per M = 0..l12 the block forms
//   S~_M for its rows (S label, b1) with b2 = beta   (VALU, into LDS)
//   T~_M for its columns (T label, (b3, b4))          (VALU, into LDS)
// and each wave runs its 16-column tile against every row tile on MFMA with
// K = 16 primaries x {re, im}: A = (S~r, -S~i), B = (T~r, T~i), so the tile
// accumulates Re(S~ T~).  Every computed entry is an output of the b-tuple
// order (b1 < b2 = beta < b3 < b4, or every tuple in the full-tensor mode).
// ---------------------------------------------------------------------------
// one packed term (see C5Label): a_{s1} a_{s2} with conjugation flags, times coef
__device__ __forceinline__ void c5_term(uint2 v, int &s1, int &s2, bool &c1, bool &c2, float &coef)
{
    s1 = (int)(v.x & 0xff);
    s2 = (int)((v.x >> 8) & 0xff);
    c1 = (v.x >> 16) & 1;
    c2 = (v.x >> 17) & 1;
    coef = __uint_as_float(v.y);
}

template <int PREC>
__global__ __launch_bounds__(256) void k_couple5(CoupleArgs a, int ntiles)
{
    extern __shared__ __align__(16) char smem[];
    const int rowlen = a.nb * 2 * a.nstate;
    const int st2 = 2 * a.nstate;
    float *Ast = reinterpret_cast<float *>(smem);
    float *wst = Ast + kRowsStep * rowlen;
    float *Sst = wst + kRowsStep;               // [kC5Rows][kC5Stride]
    float *Tst = Sst + kC5Rows * kC5Stride;     // [kC5Cols][kC5Stride]
    int *tab = reinterpret_cast<int *>(Tst + kC5Cols * kC5Stride);
    int rb, jb;
    if (!block_work(a.n_rowblocks, a.nc5jobs, rb, jb)) return;
    const auto jobs = as_const(a.c5jobs);
    const int l12 = uni(jobs[jb].l12), beta = uni(jobs[jb].beta), nb1 = uni(jobs[jb].nb1);
    const int s_begin = uni(jobs[jb].s_begin), ns = uni(jobs[jb].ns), t_begin = uni(jobs[jb].t_begin);
    const int col_begin = uni(jobs[jb].col_begin), ncol = uni(jobs[jb].ncol);
    const int pair_begin = uni(jobs[jb].pair_begin), npair = uni(jobs[jb].npair);
    const int nrt = uni(jobs[jb].nrt), tile_begin = uni(jobs[jb].tile_begin);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int n = lane & 15;   // A row / B column within a tile
    const int kq = lane >> 4;  // K quarter: primaries 4 kq .. 4 kq + 3
    const bool has_cols = wave * 16 < ncol;

    // the job's term tables, copied to LDS once: per label its l12 + 2 range
    // entries (relative to its side's first term) and phase flag, then the terms
    const int nmt = l12 + 2;
    const int t0 = col_begin / npair, ntl = (col_begin + ncol - 1) / npair - t0 + 1;
    const auto labels = as_const(a.c5labels);
    const int smt0 = uni(labels[s_begin].mt), tmt0 = uni(labels[t_begin + t0].mt);
    const int sbase = uni(a.c5mterm[smt0]), tbase = uni(a.c5mterm[tmt0]);
    const int sterms = uni(a.c5mterm[smt0 + ns * nmt - 1]) - sbase;
    const int tterms = uni(a.c5mterm[tmt0 + ntl * nmt - 1]) - tbase;
    int *Smt = tab;                      // [ns * nmt]
    int *Tmt = Smt + ns * nmt;           // [ntl * nmt]
    int *Srot = Tmt + ntl * nmt;         // [ns]
    int *Trot = Srot + ns;               // [ntl]
    int *Srow = Trot + ntl;              // [kC5Rows]: S label | b1 << 16 of GEMM row r
    uint2 *Sterm = reinterpret_cast<uint2 *>(tab + (((ns + ntl) * (nmt + 1) + kC5Rows + 1) & ~1));   // 8-byte aligned
    uint2 *Tterm = Sterm + sterms;
    for (int i = threadIdx.x; i < ns * nmt; i += blockDim.x) Smt[i] = a.c5mterm[smt0 + i] - sbase;
    for (int i = threadIdx.x; i < ntl * nmt; i += blockDim.x) Tmt[i] = a.c5mterm[tmt0 + i] - tbase;
    for (int i = threadIdx.x; i < ns; i += blockDim.x) Srot[i] = a.c5labels[s_begin + i].rot;
    for (int i = threadIdx.x; i < ntl; i += blockDim.x) Trot[i] = a.c5labels[t_begin + t0 + i].rot;
    for (int i = threadIdx.x; i < kC5Rows; i += blockDim.x) Srow[i] = (i / nb1) | ((i % nb1) << 16);
    const int nrows_s = ns * nb1;
    for (int i = threadIdx.x; i < sterms; i += blockDim.x) Sterm[i] = a.c5terms[sbase + i];
    for (int i = threadIdx.x; i < tterms; i += blockDim.x) Tterm[i] = a.c5terms[tbase + i];

    // this thread's column items (column cl = threadIdx / 16 + 16 k, primary p = threadIdx % 16)
    const int p_item = threadIdx.x & 15;
    int tl_item[4];
    int2 bb_item[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int cl = (threadIdx.x >> 4) + 16 * k;
        tl_item[k] = 0;
        bb_item[k] = make_int2(0, 0);
        if (cl < ncol) {
            const int col = col_begin + cl;
            const int tl = col / npair;
            tl_item[k] = tl - t0;
            bb_item[k] = a.c5pairs[pair_begin + (col - tl * npair)];
        }
    }

    // rows and columns no item writes stay zero
    for (int t = threadIdx.x; t < (kC5Rows + kC5Cols) * kC5Stride; t += blockDim.x) Sst[t] = 0.f;

    double acc[8][4];
#pragma unroll
    for (int r = 0; r < 8; r++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[r][v] = 0.0;

    int r_begin = rb * a.rows_per_block;
    int r_end = r_begin + a.rows_per_block;
    if (a.rb_begin) {
        r_begin = a.rb_begin[rb];
        r_end = a.rb_end[rb];
    }
    if (r_end > a.nrows) r_end = a.nrows;

    for (int r0 = r_begin; r0 < r_end; r0 += kRowsStep) {
        __syncthreads();
        stage_rows(a, r0, r_end, Ast, wst);
        for (int M = 0; M <= l12; M++) {
            __syncthreads();
            // S~ rows: this thread's items (row = threadIdx / 16 + 16 k, primary p_item)
            {
                const float *Ap = Ast + p_item * rowlen;
                const float wp = wst[p_item];
                for (int row = threadIdx.x >> 4; row < nrows_s; row += 16) {
                    const int info = Srow[row];
                    const int sl = info & 0xffff, b1 = info >> 16;
                    const int tb = Smt[sl * nmt + M], te = Smt[sl * nmt + M + 1];
                    float sr = 0.f, si = 0.f;
                    for (int t = tb; t < te; t++) {
                        int s1, s2;
                        bool c1, c2;
                        float coef;
                        c5_term(Sterm[t], s1, s2, c1, c2, coef);
                        const float2 x = *reinterpret_cast<const float2 *>(Ap + b1 * st2 + 2 * s1);
                        const float2 y = *reinterpret_cast<const float2 *>(Ap + beta * st2 + 2 * s2);
                        const float xi = c1 ? -x.y : x.y;
                        const float yi = c2 ? -y.y : y.y;
                        sr += coef * (x.x * y.x - xi * yi);
                        si += coef * (x.x * yi + xi * y.x);
                    }
                    float re = sr * wp, im = si * wp;
                    if (Srot[sl]) {  // times -i
                        const float t1 = re;
                        re = im;
                        im = -t1;
                    }
                    float *dst = Sst + row * kC5Stride + 2 * p_item;
                    dst[0] = re;
                    dst[1] = -im;
                }
            }
            // T~ columns: this thread's items
            {
                const float *Ap = Ast + p_item * rowlen;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int cl = (threadIdx.x >> 4) + 16 * k;
                    if (cl < ncol) {
                        const int tl = tl_item[k];
                        const int2 bb = bb_item[k];
                        const int tb = Tmt[tl * nmt + M], te = Tmt[tl * nmt + M + 1];
                        float tr = 0.f, ti = 0.f;
                        for (int t = tb; t < te; t++) {
                            int s1, s2;
                            bool c1, c2;
                            float coef;
                            c5_term(Tterm[t], s1, s2, c1, c2, coef);
                            const float2 x = *reinterpret_cast<const float2 *>(Ap + bb.x * st2 + 2 * s1);
                            const float2 y = *reinterpret_cast<const float2 *>(Ap + bb.y * st2 + 2 * s2);
                            const float xi = c1 ? -x.y : x.y;
                            const float yi = c2 ? -y.y : y.y;
                            tr += coef * (x.x * y.x - xi * yi);
                            ti += coef * (x.x * yi + xi * y.x);
                        }
                        if (Trot[tl]) {
                            const float t1 = tr;
                            tr = ti;
                            ti = -t1;
                        }
                        float *dst = Tst + cl * kC5Stride + 2 * p_item;
                        dst[0] = tr;
                        dst[1] = ti;
                    }
                }
            }
            __syncthreads();
            if (has_cols) {
                float Bv[8];
                const float *bp = Tst + (wave * 16 + n) * kC5Stride + 8 * kq;
#pragma unroll
                for (int i = 0; i < 8; i++) Bv[i] = bp[i];
#pragma unroll
                for (int rt = 0; rt < 8; rt++) {
                    if (rt < nrt) {
                        float Av[8];
                        const float *ap = Sst + (rt * 16 + n) * kC5Stride + 8 * kq;
#pragma unroll
                        for (int i = 0; i < 8; i++) Av[i] = ap[i];
                        if constexpr (PREC == 2) {
                            // rows of one tile belong to different S labels
                            double o[4];
                            mfma_k32_f16_rowscaled(Av, Bv, kq, o);
#pragma unroll
                            for (int v = 0; v < 4; v++) acc[rt][v] += o[v];
                        } else {
                            v4f cc = v4f{0.f, 0.f, 0.f, 0.f};
                            double unscale;
                            mfma_k32<PREC>(Av, Bv, cc, unscale);
#pragma unroll
                            for (int v = 0; v < 4; v++) acc[rt][v] += (double)cc[v] * unscale;
                        }
                    }
                }
            }
        }
    }
    // per-block partials: partial[rb][tile][16][16]; lane holds rows 4 kq + v of column n
    if (has_cols) {
#pragma unroll
        for (int rt = 0; rt < 8; rt++) {
            if (rt < nrt) {
                double *dst = a.partial + ((size_t)rb * ntiles + tile_begin + rt * 4 + wave) * 256;
#pragma unroll
                for (int v = 0; v < 4; v++) dst[(4 * kq + v) * 16 + n] = acc[rt][v];
            }
        }
    }
}

}  // namespace

int couple5_lds_bytes(int nb, int nstate, int extra)
{
    return (kRowsStep * nb * 2 * nstate + kRowsStep + (kC5Rows + kC5Cols) * kC5Stride) * 4 + extra;
}

hipError_t launch_couple5(int precision, const CoupleArgs &a, int ntiles, hipStream_t s)
{
    const int nblk = ((a.n_rowblocks + kXcd - 1) / kXcd) * kXcd * a.nc5jobs;
    const int lds = couple5_lds_bytes(a.nb, a.nstate, a.c5_lds_extra);
    switch (precision) {
    case 0: return launch_with_lds(k_couple5<0>, nblk, lds, s, a, ntiles);
    case 1: return launch_with_lds(k_couple5<1>, nblk, lds, s, a, ntiles);
    case 2: return launch_with_lds(k_couple5<2>, nblk, lds, s, a, ntiles);
    case 3: return launch_with_lds(k_couple5<3>, nblk, lds, s, a, ntiles);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace npcf
