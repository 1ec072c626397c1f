// Coupling stage of the separable NPCF estimator (eq. NPCF-estimator-discrete,
// the per-primary sum over [l] weighted by C^{Lambda;0} of eq. Coupling-C),
// recast as small GEMMs that contract over the primary index on MFMA.
//
// N = 4 (D = 3 and D = 2).  For a job (Lambda, part, tile of radial pairs):
//   S_g[i, (b1,b2)] = w_i sum_terms c * op(a_i[b1][s1]) * op(a_i[b2][s2])      (VALU)
//   Z[(b1,b2), b3] += sum_g sum_i  part( S_g[i,(b1,b2)] * op(a_i[b3][s3_g]) )  (MFMA, K = primaries x {re,im})
// where g runs over m3 >= 0 for D = 3 (the -m3 half is folded into c by the
// symmetry a_{l,-m} = (-1)^m conj(a_{l,m}) of a real field) and over the single
// term for D = 2.
//
// N = 3: per Lambda = l, a Hermitian rank-K update
//   Z[b1, b2] += sum_i sum_{s in l} f_s w_i (a_i[b1][s] conj(a_i[b2][s]))   (MFMA, K = primaries x states x {re,im})
//
// Every MFMA chain covers one K = 32 slice and is folded into FP64 at once,
// so FP32 rounding never accumulates over more than 32 products; per-block
// FP64 partials are summed over blocks in a fixed order (deterministic).
// Precision variants of the slice:
//   0 plain  FP32 operands, 8 x v_mfma_f32_16x16x4_f32
//   1 BF16   hi + lo split, 3 x v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi)
//   2 FP16   hi + lo split after a power-of-two scaling of each operand tile,
//            3 x v_mfma_f32_16x16x32_f16
//   3 BF16   hi + mid + lo split, 6 products (all pairs of total order <= 2)
#include "npcf_couple_common.h"

namespace npcf {

namespace {

constexpr int kJobsPerWave = 4;
constexpr int kC3StageBytes = 48 * 1024;   // rows of a staged per step by the isotropic N = 3 kernel, at most

// ---------------------------------------------------------------------------
// N = 4
// ---------------------------------------------------------------------------
struct Job4 {
    int lam, part_kind, tile;
};

__device__ __forceinline__ Job4 decode_job4(const CoupleArgs &a, int job, int nparts)
{
    Job4 j;
    j.tile = job % a.mtiles;
    const int lp = job / a.mtiles;
    j.lam = lp / nparts;
    const int part = lp % nparts;
    j.part_kind = (nparts == 2) ? part : a.lam_part[j.lam];
    return j;
}

// complex S of a group for radial pair bb of primary p (already times w_p);
// the group's terms are read from the block's LDS copy `tl` (offset tbase)
__device__ __forceinline__ float2 form_s(const CoupleArgs &a, const CoupleGroup &g, const CoupleTerm *tl, int tbase,
                                         const float *Ast, int rowlen, int p, int2 bb, bool rowok, float wp)
{
    float sr = 0.f, si = 0.f;
    if (rowok) {
        const float *Ap = Ast + p * rowlen;
        const float *A1 = Ap + bb.x * 2 * a.nstate;
        const float *A2 = Ap + bb.y * 2 * a.nstate;
        for (int t = g.term_begin; t < g.term_end; t++) {
            const CoupleTerm tm = tl[t - tbase];
            const float2 x = *reinterpret_cast<const float2 *>(A1 + 2 * tm.s1);
            const float2 y = *reinterpret_cast<const float2 *>(A2 + 2 * tm.s2);
            const float xi = tm.conj1 ? -x.y : x.y;
            const float yi = tm.conj2 ? -y.y : y.y;
            sr += tm.coef * (x.x * y.x - xi * yi);
            si += tm.coef * (x.x * yi + xi * y.x);
        }
    }
    return make_float2(sr * wp, si * wp);
}

// The two K-components of part(S * a3): Re -> Sr a3r + (-Si) a3i; Im -> Sr a3i + Si a3r.
__device__ __forceinline__ void part_operands(int part_kind, float2 s, float a3r, float a3i, float &A0, float &B0,
                                              float &A1, float &B1)
{
    if (part_kind == 0) {
        A0 = s.x; B0 = a3r;
        A1 = -s.y; B1 = a3i;
    } else {
        A0 = s.x; B0 = a3i;
        A1 = s.y; B1 = a3r;
    }
}

// four waves per SIMD (FP16 took 134 VGPRs at three; at four it spills six
// values): c3 coupling FP16 24.2 -> 20.2 ms, the others unchanged
template <int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_couple4(CoupleArgs a, int njobs, int nparts)
{
    extern __shared__ __align__(16) char smem[];
    const int rowlen = a.nb * 2 * a.nstate;
    float *Ast = reinterpret_cast<float *>(smem);
    float *wst = Ast + kRowsStep * rowlen;
    const int njg = (njobs + 4 * kJobsPerWave - 1) / (4 * kJobsPerWave);
    int rb, jg;
    if (!block_work(a.n_rowblocks, njg, rb, jg)) return;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int job0 = jg * 4 * kJobsPerWave + wave * kJobsPerWave;

    // the coupling terms of this block's jobs, copied to LDS once
    CoupleTerm *tl = reinterpret_cast<CoupleTerm *>(wst + kRowsStep);
    int tbase, tend;
    {
        const int jfirst = jg * 4 * kJobsPerWave;
        int jlast = jfirst + 4 * kJobsPerWave - 1;
        if (jlast > njobs - 1) jlast = njobs - 1;
        const int lam0 = decode_job4(a, jfirst, nparts).lam, lam1 = decode_job4(a, jlast, nparts).lam;
        const int gb = a.lam_group_begin[lam0], ge = a.lam_group_begin[lam1 + 1];
        tbase = gb < ge ? a.groups[gb].term_begin : 0;
        tend = gb < ge ? a.groups[ge - 1].term_end : 0;
        for (int t = threadIdx.x; t < tend - tbase; t += blockDim.x) tl[t] = a.terms[tbase + t];
    }

    double acc64[kJobsPerWave][4];
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc64[j][v] = 0.0;

    int r_begin = rb * a.rows_per_block;
    int r_end = r_begin + a.rows_per_block;
    if (a.rb_begin) {
        r_begin = a.rb_begin[rb];
        r_end = a.rb_end[rb];
    }
    if (r_end > a.nrows) r_end = a.nrows;
    const int n = lane & 15;   // A row within the tile / output column b3
    const int kq = lane >> 4;  // K quarter

    for (int r0 = r_begin; r0 < r_end; r0 += kRowsStep) {
        __syncthreads();
        stage_rows(a, r0, r_end, Ast, wst);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kJobsPerWave; j++) {
            const int job = job0 + j;
            if (job >= njobs) break;
            const Job4 jb = decode_job4(a, job, nparts);
            const int m = jb.tile * 16 + n;
            const bool rowok = m < a.mrows;
            const int2 bb = rowok ? a.row_pairs[m] : make_int2(0, 0);
            const bool colok = n < a.nb;
            for (int gi = a.lam_group_begin[jb.lam]; gi < a.lam_group_begin[jb.lam + 1]; gi++) {
                const CoupleGroup g = a.groups[gi];
                float Av[8], Bv[8];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int p = 4 * kq + q;
                    const float2 sv = form_s(a, g, tl, tbase, Ast, rowlen, p, bb, rowok, wst[p]);
                    float a3r = 0.f, a3i = 0.f;
                    if (colok) {
                        const float2 v = *reinterpret_cast<const float2 *>(Ast + p * rowlen + n * 2 * a.nstate + 2 * g.s3);
                        a3r = v.x;
                        a3i = g.conj3 ? -v.y : v.y;
                    }
                    part_operands(jb.part_kind, sv, a3r, a3i, Av[2 * q], Bv[2 * q], Av[2 * q + 1], Bv[2 * q + 1]);
                }
                v4f c = v4f{0.f, 0.f, 0.f, 0.f};
                double unscale;
                mfma_k32<PREC>(Av, Bv, c, unscale);
#pragma unroll
                for (int v = 0; v < 4; v++) acc64[j][v] += (double)c[v] * unscale;
            }
        }
    }
    // per-block partials: partial[rb][job][16][16]; lane holds rows 4 kq + v of column n
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++) {
        const int job = job0 + j;
        if (job >= njobs) break;
        double *dst = a.partial + ((size_t)rb * njobs + job) * 256;
#pragma unroll
        for (int v = 0; v < 4; v++) dst[(4 * kq + v) * 16 + n] = acc64[j][v];
    }
}

// ---------------------------------------------------------------------------
// N = 4, D = 3, factorised: a job is (pair (l1, l2), tile of radial pairs)
// and produces every Lambda = (l1, l2, l3) of the pair.  Per group (pair, m3)
// each product P_{m1} = op(a_{l1}[b1]) op(a_{l2}[b2]) is formed once and added,
// with its coefficient for each l3, into that slot's S; each slot then takes
// its MFMA slice against a_{l3 m3}[b3].  Two jobs per wave (paired by cost).
// ---------------------------------------------------------------------------
// One group (pair, m3) of a job, slots [K0, K0 + NA) of its active ones:
// S of every such slot for this lane's 16-row tile row and its four
// primaries of the step, then one MFMA slice per slot, folded into the FP64
// accumulators.  A group with more active slots than its precision's cap
// takes several calls, forming its products again each time, so that the
// kernel fits four waves per SIMD (Couple4fShape).  Each slot's sum sees
// the same operations either way.
template <int PREC, int NA, int K0>
__device__ __forceinline__ void couple4f_group(const CoupleArgs &a, int pp, int g, const float *Ast, const float *wst,
                                               int rowlen, int st2, int kq, int n, int2 bb, bool rowok, bool colok,
                                               double (&acc)[kMaxSlots][4])
{
    const auto pairs = as_const(a.fpairs);
    const auto groups = as_const(a.fgroups);
    const auto prods = as_const(a.fprods);
    const auto coef = as_const(a.fcoef);
    const int pb = uni(groups[g].prod_begin), np = uni(groups[g].prod_end) - pb;
    const int cb = uni(groups[g].coef_begin);
    float sr[NA][4], si[NA][4];
#pragma unroll
    for (int k = 0; k < NA; k++)
#pragma unroll
        for (int q = 0; q < 4; q++) sr[k][q] = si[k][q] = 0.f;
    // the 8-byte product descriptors as one 64-bit word each: a wave-uniform
    // address, so a scalar load (the 16- and 8-bit fields alone became
    // vector loads, one memory round trip per product)
    const auto pd2 = (const __attribute__((address_space(4))) unsigned long long *)(prods + pb);
    for (int t = 0; t < np; t++) {
        const unsigned long long d = pd2[t];
        const uint32_t dx = (uint32_t)d, dy = (uint32_t)(d >> 32);
        const int s1 = uni((int)(int16_t)(dx & 0xFFFFu)), s2 = uni((int)(int16_t)(dx >> 16));
        const bool conj1 = (dy & 0xFFu) != 0, conj2 = (dy & 0xFF00u) != 0;
        float c[NA];
#pragma unroll
        for (int k = 0; k < NA; k++) c[k] = uni(coef[cb + t * kFCoefStride + K0 + k]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float *Ap = Ast + (4 * kq + q) * rowlen;
            const float2 x = *reinterpret_cast<const float2 *>(Ap + bb.x * st2 + 2 * s1);
            const float2 y = *reinterpret_cast<const float2 *>(Ap + bb.y * st2 + 2 * s2);
            const float xi = conj1 ? -x.y : x.y;
            const float yi = conj2 ? -y.y : y.y;
            const float pr = x.x * y.x - xi * yi;
            const float pi = x.x * yi + xi * y.x;
#pragma unroll
            for (int k = 0; k < NA; k++) {
                sr[k][q] += c[k] * pr;
                si[k][q] += c[k] * pi;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NA; k++) {
        // s3[] read as dwords (scalar loads), as the product descriptors
        const int ks = K0 + k;
        const uint32_t s3w = ((const __attribute__((address_space(4))) uint32_t *)&groups[g].s3[0])[ks >> 1];
        const int s3 = uni((int)(int16_t)(s3w >> (16 * (ks & 1))));
        const int part = uni(pairs[pp].part[ks]);
        float Av[8], Bv[8];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int p = 4 * kq + q;
            const float wp = wst[p];
            const float2 sv = rowok ? make_float2(sr[k][q] * wp, si[k][q] * wp) : make_float2(0.f, 0.f);
            float a3r = 0.f, a3i = 0.f;
            if (colok) {
                const float2 v = *reinterpret_cast<const float2 *>(Ast + p * rowlen + n * st2 + 2 * s3);
                a3r = v.x;
                a3i = v.y;
            }
            part_operands(part, sv, a3r, a3i, Av[2 * q], Bv[2 * q], Av[2 * q + 1], Bv[2 * q + 1]);
        }
        v4f cc = v4f{0.f, 0.f, 0.f, 0.f};
        double unscale;
        mfma_k32<PREC>(Av, Bv, cc, unscale);
#pragma unroll
        for (int v = 0; v < 4; v++) acc[K0 + k][v] += (double)cc[v] * unscale;
    }
}

// Active slots per pass and waves per SIMD of k_couple4f, per precision.
// kCap 6: every group in one pass; kCap 4: groups of five or six active
// slots in two passes (three, then the rest).  c2 coupling, ms per pass:
//   plain      35.5 at 3 waves; 29.9 at 4 in one pass (a 28-byte spill); 31.2 in two passes
//   BF16 x6    35.3 at 3 waves; 33.8 at 4 in one pass (80-byte spill); 33.3 in two (64 bytes);
//              34.1 with passes of at most three
//   BF16 hi+lo 33.7 at 3 waves; 31.2 at 4 in two passes
//   FP16       43.0 at 3 waves; 48.4 at 4 in two passes (its per-tile scales need more
//              registers: a 100-byte spill)
template <int PREC>
struct Couple4fShape {
    static constexpr int kCap = (PREC == 0 || PREC == 2) ? kMaxSlots : 4;
    static constexpr int kWaves = PREC == 2 ? 3 : 4;
};

template <int PREC>
__device__ __forceinline__ void couple4f_body(const CoupleArgs &a, int njobs)
{
    extern __shared__ __align__(16) char smem[];
    const int rowlen = a.nb * 2 * a.nstate;
    float *Ast = reinterpret_cast<float *>(smem);
    float *wst = Ast + kRowsStep * rowlen;
    const int ntg = (a.nftasks + 3) / 4;
    int rb, tg;
    if (!block_work(a.n_rowblocks, ntg, rb, tg)) return;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int task = tg * 4 + wave;
    const auto tasks = as_const(a.ftasks);
    const auto pairs = as_const(a.fpairs);
    const auto groups = as_const(a.fgroups);
    int jobs[2] = {-1, -1};
    if (task < a.nftasks) {
        jobs[0] = uni(tasks[task].x);
        jobs[1] = uni(tasks[task].y);
    }

    double acc0[kMaxSlots][4], acc1[kMaxSlots][4];
#pragma unroll
    for (int k = 0; k < kMaxSlots; k++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc0[k][v] = acc1[k][v] = 0.0;

    int r_begin = rb * a.rows_per_block;
    int r_end = r_begin + a.rows_per_block;
    if (a.rb_begin) {
        r_begin = a.rb_begin[rb];
        r_end = a.rb_end[rb];
    }
    if (r_end > a.nrows) r_end = a.nrows;
    const int n = lane & 15;   // GEMM row within the tile / output column b3
    const int kq = lane >> 4;  // K quarter: primaries 4 kq .. 4 kq + 3 of the step
    const int st2 = 2 * a.nstate;

    for (int r0 = r_begin; r0 < r_end; r0 += kRowsStep) {
        __syncthreads();
        stage_rows(a, r0, r_end, Ast, wst);
        __syncthreads();
        // the wave's two jobs, each into its own accumulators
        auto run_job = [&](int job, double (&acc)[kMaxSlots][4]) {
            if (job < 0) return;
            const int pp = uni(job / a.mtiles);
            const int tile = uni(job - pp * a.mtiles);
            const int m = tile * 16 + n;
            const bool rowok = m < a.mrows;
            const int2 bb = rowok ? a.row_pairs[m] : make_int2(0, 0);
            const bool colok = n < a.nb;
            const int gb = uni(pairs[pp].grp_begin), ge = uni(pairs[pp].grp_end);
            for (int g = gb; g < ge; g++) {
                const int nact = uni(groups[g].nact);
                if constexpr (Couple4fShape<PREC>::kCap == kMaxSlots) {
                    switch (nact) {
                    case 1: couple4f_group<PREC, 1, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 2: couple4f_group<PREC, 2, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 3: couple4f_group<PREC, 3, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 4: couple4f_group<PREC, 4, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 5: couple4f_group<PREC, 5, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    default: couple4f_group<PREC, kMaxSlots, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    }
                } else {
                    static_assert(Couple4fShape<PREC>::kCap == 4 && kMaxSlots == 6, "five or six slots in two passes");
                    switch (nact) {
                    case 1: couple4f_group<PREC, 1, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 2: couple4f_group<PREC, 2, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 3: couple4f_group<PREC, 3, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 4: couple4f_group<PREC, 4, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc); break;
                    case 5:
                        couple4f_group<PREC, 3, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc);
                        couple4f_group<PREC, 2, 3>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc);
                        break;
                    default:
                        couple4f_group<PREC, 3, 0>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc);
                        couple4f_group<PREC, 3, 3>(a, pp, g, Ast, wst, rowlen, st2, kq, n, bb, rowok, colok, acc);
                        break;
                    }
                }
            }
        };
        run_job(jobs[0], acc0);
        if (kFJobsPerWave > 1) run_job(jobs[1], acc1);
    }
    // per-block partials in the term-by-term layout: partial[rb][lam * mtiles + tile][16][16]
    auto write_job = [&](int job, const double (&acc)[kMaxSlots][4]) {
        if (job < 0) return;
        const int pp = uni(job / a.mtiles);
        const int tile = uni(job - pp * a.mtiles);
        const int nslot = uni(pairs[pp].nslot);
#pragma unroll
        for (int k = 0; k < kMaxSlots; k++) {
            if (k >= nslot) break;
            const int ojob = uni(pairs[pp].lam[k]) * a.mtiles + tile;
            double *dst = a.partial + ((size_t)rb * njobs + ojob) * 256;
#pragma unroll
            for (int v = 0; v < 4; v++) dst[(4 * kq + v) * 16 + n] = acc[k][v];
        }
    };
    write_job(jobs[0], acc0);
    if (kFJobsPerWave > 1) write_job(jobs[1], acc1);
}

// the factorised kernel per precision, each with its waves per SIMD
template <int PREC>
__global__ void k_couple4f(CoupleArgs a, int njobs);
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Couple4fShape<0>::kWaves))) void k_couple4f<0>(CoupleArgs a, int njobs)
{
    couple4f_body<0>(a, njobs);
}
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Couple4fShape<1>::kWaves))) void k_couple4f<1>(CoupleArgs a, int njobs)
{
    couple4f_body<1>(a, njobs);
}
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Couple4fShape<2>::kWaves))) void k_couple4f<2>(CoupleArgs a, int njobs)
{
    couple4f_body<2>(a, njobs);
}
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Couple4fShape<3>::kWaves))) void k_couple4f<3>(CoupleArgs a, int njobs)
{
    couple4f_body<3>(a, njobs);
}

// ---------------------------------------------------------------------------
// N = 3: job = (Lambda, part); part 0: Re, 1: Im (D = 2 only).  rs rows of a
// per step (at most kRowsStep; fewer where rows are long, so that several
// blocks share a CU's LDS) and jpw jobs per wave (at most kJobsPerWave; fewer
// where there are few jobs, so that every wave of a block has work).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_couple3(CoupleArgs a, int njobs, int nparts, const float *sfac,
                                                                                    int rs, int jpw)
{
    extern __shared__ __align__(16) char smem[];
    const int rowlen = a.nb * 2 * a.nstate;
    float *Ast = reinterpret_cast<float *>(smem);
    float *wst = Ast + rs * rowlen;
    float *sfs = wst + rs;   // per-state factors, copied once (read per operand element)
    const int njg = (njobs + 4 * jpw - 1) / (4 * jpw);
    int rb, jg;
    if (!block_work(a.n_rowblocks, njg, rb, jg)) return;
    for (int t = threadIdx.x; t < a.nstate; t += blockDim.x) sfs[t] = sfac[t];   // the row loop's first barrier orders it
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int job0 = jg * 4 * jpw + wave * jpw;

    double acc64[kJobsPerWave][4];
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc64[j][v] = 0.0;
    int r_begin = rb * a.rows_per_block;
    int r_end = r_begin + a.rows_per_block;
    if (a.rb_begin) {
        r_begin = a.rb_begin[rb];
        r_end = a.rb_end[rb];
    }
    if (r_end > a.nrows) r_end = a.nrows;
    const int n = lane & 15;   // b1 (A row) and b2 (B column) of this lane
    const int kq = lane >> 4;
    const bool bok = n < a.nb;

    for (int r0 = r_begin; r0 < r_end; r0 += rs) {
        __syncthreads();
        stage_rows_n(a, r0, r_end, rs, Ast, wst);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kJobsPerWave; j++) {
            const int job = job0 + j;
            if (j >= jpw || job >= njobs) break;
            const int lam = job / nparts;
            const int part_kind = (nparts == 2) ? (job % nparts) : 0;
            const CoupleGroup g = a.groups[a.lam_group_begin[lam]];
            const int kper = 2 * g.nst;   // K entries per primary: states x {re, im}
            const int ktot = rs * kper;
            for (int k0 = 0; k0 < ktot; k0 += 32) {
                float Av[8], Bv[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const int k = k0 + 8 * kq + i;
                    Av[i] = 0.f;
                    Bv[i] = 0.f;
                    if (k < ktot && bok) {
                        const int p = k / kper;
                        const int rr = k - p * kper;
                        const int s = g.s3 + (rr >> 1);
                        const int c = rr & 1;
                        const float2 x = *reinterpret_cast<const float2 *>(Ast + p * rowlen + n * 2 * a.nstate + 2 * s);
                        Bv[i] = c ? x.y : x.x;
                        const float wf = wst[p] * g.scale3 * sfs[s];
                        // Re(a[b1] conj(a[b2])) = ar ar' + ai ai';  Im = ai ar' - ar ai'
                        Av[i] = (part_kind == 0) ? wf * (c ? x.y : x.x) : wf * (c ? -x.x : x.y);
                    }
                }
                v4f cc = v4f{0.f, 0.f, 0.f, 0.f};
                double unscale;
                mfma_k32<PREC>(Av, Bv, cc, unscale);
#pragma unroll
                for (int v = 0; v < 4; v++) acc64[j][v] += (double)cc[v] * unscale;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++) {
        const int job = job0 + j;
        if (j >= jpw || job >= njobs) break;   // the next wave's jobs are not this wave's to write
        double *dst = a.partial + ((size_t)rb * njobs + job) * 256;
#pragma unroll
        for (int v = 0; v < 4; v++) dst[(4 * kq + v) * 16 + n] = acc64[j][v];
    }
}

// N = 3 from a term list (line-of-sight basis): job = Lambda,
//   Z[b1, b2] += sum_i w_i sum_t c_t part(a_i[b1][s1_t] conj(a_i[b2][s2_t]))
// with part = Re (lam_part 0) or Im (1), the +-m terms of the basis folded
// into c_t on the host, on MFMA with K = primaries x terms x {two real
// products}.
// four waves per SIMD (the BF16 x6 and FP16 forms took 130 and 128 VGPRs at
// three): c6 coupling, fixed block size, BF16 x6 21.0 -> 17.9 ms
template <int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_couple3t(CoupleArgs a, int njobs)
{
    extern __shared__ __align__(16) char smem[];
    const int rowlen = a.nb * 2 * a.nstate;
    float *Ast = reinterpret_cast<float *>(smem);
    float *wst = Ast + kRowsStep * rowlen;
    const int njg = (njobs + 4 * kJobsPerWave - 1) / (4 * kJobsPerWave);
    int rb, jg;
    if (!block_work(a.n_rowblocks, njg, rb, jg)) return;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int job0 = jg * 4 * kJobsPerWave + wave * kJobsPerWave;

    // the span of term ranges of this block's Lambdas (one group each),
    // copied to LDS once: each lane reads its operand's term per element
    // (at most max_block_terms, the host's bound over all blocks)
    CoupleTerm *tl = reinterpret_cast<CoupleTerm *>(wst + kRowsStep);
    int tbase = 0;
    {
        int tb = 0x7fffffff, te = 0;
        for (int lam = jg * 4 * kJobsPerWave; lam < njobs && lam < (jg + 1) * 4 * kJobsPerWave; lam++) {
            const CoupleGroup gg = a.groups[a.lam_group_begin[lam]];
            tb = min(tb, gg.term_begin);
            te = max(te, gg.term_end);
        }
        if (te > tb) {
            tbase = tb;
            for (int t = threadIdx.x; t < te - tb; t += blockDim.x) tl[t] = a.terms[tb + t];   // ordered by the row loop's first barrier
        }
    }

    double acc64[kJobsPerWave][4];
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc64[j][v] = 0.0;
    int r_begin = rb * a.rows_per_block;
    int r_end = r_begin + a.rows_per_block;
    if (a.rb_begin) {
        r_begin = a.rb_begin[rb];
        r_end = a.rb_end[rb];
    }
    if (r_end > a.nrows) r_end = a.nrows;
    const int n = lane & 15;   // b1 (A row) and b2 (B column) of this lane
    const int kq = lane >> 4;
    const bool bok = n < a.nb;

    for (int r0 = r_begin; r0 < r_end; r0 += kRowsStep) {
        __syncthreads();
        stage_rows(a, r0, r_end, Ast, wst);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kJobsPerWave; j++) {
            const int lam = job0 + j;
            if (lam >= njobs) break;
            const int im = a.lam_part[lam];
            const CoupleGroup g = a.groups[a.lam_group_begin[lam]];
            const int nt = g.term_end - g.term_begin;
            const int kper = 2 * nt;   // K entries per primary: terms x {two real products}
            const int ktot = kRowsStep * kper;
            for (int k0 = 0; k0 < ktot; k0 += 32) {
                float Av[8], Bv[8];
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    const int k = k0 + 8 * kq + i;
                    Av[i] = 0.f;
                    Bv[i] = 0.f;
                    if (k < ktot && bok) {
                        const int p = k / kper;
                        const int rr = k - p * kper;
                        const CoupleTerm tm = tl[g.term_begin - tbase + (rr >> 1)];
                        const int c = rr & 1;
                        const float *Ap = Ast + p * rowlen + n * 2 * a.nstate;
                        const float2 x = *reinterpret_cast<const float2 *>(Ap + 2 * tm.s1);
                        const float2 y = *reinterpret_cast<const float2 *>(Ap + 2 * tm.s2);
                        const float wf = wst[p] * tm.coef;
                        // Re(x conj(y)) = xr yr + xi yi;  Im(x conj(y)) = xi yr + (-xr) yi
                        if (!im) {
                            Av[i] = c ? wf * x.y : wf * x.x;
                            Bv[i] = c ? y.y : y.x;
                        } else {
                            Av[i] = c ? -wf * x.x : wf * x.y;
                            Bv[i] = c ? y.y : y.x;
                        }
                    }
                }
                v4f cc = v4f{0.f, 0.f, 0.f, 0.f};
                double unscale;
                mfma_k32<PREC>(Av, Bv, cc, unscale);
#pragma unroll
                for (int v = 0; v < 4; v++) acc64[j][v] += (double)cc[v] * unscale;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kJobsPerWave; j++) {
        const int job = job0 + j;
        if (job >= njobs) break;
        double *dst = a.partial + ((size_t)rb * njobs + job) * 256;
#pragma unroll
        for (int v = 0; v < 4; v++) dst[(4 * kq + v) * 16 + n] = acc64[j][v];
    }
}

__global__ void k_reduce_partials(const double *partial, int nrb, int64_t len, double *acc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int r = 0; r < nrb; r++) s += partial[(size_t)r * len + i];
    acc[i] += s;
}

struct FinArgs {
    const double *acc;
    const double *acc_rand;
    int nlam;
    int nparts;              // 2 for D = 2, else 1
    int mtiles;
    const int *bt_row;       // GEMM row of each radial tuple
    const int *bt_col;       // GEMM column
    const double *bt_scale;  // 1 / (V_D prod v_b)
    int nbt;
    int norm_by_randoms;
    int lam0;                // index of Lambda = 0 (randoms normalisation)
    double *out;
    int *bad;
};

__global__ void k_finalize_idx(const double *acc, const double *acc_rand, const int *idx, const double *sign,
                               const double *bt_scale, int nlam, int nbt, int norm_by_randoms, int lam0, double *out,
                               int *bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nlam * nbt) return;
    const int lam = (int)(i / nbt), t = (int)(i % nbt);
    double v = acc[idx[i]] * sign[lam] * bt_scale[t];
    if (norm_by_randoms) {
        const double r = acc_rand[idx[(int64_t)lam0 * nbt + t]] * sign[lam0] * bt_scale[t];
        if (r == 0.0 || !isfinite(r)) atomicOr(bad, 2);
        v = v / r;
    }
    out[i] = v;
}

__global__ void k_finalize(FinArgs f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)f.nlam * f.nparts * f.nbt;
    if (i >= total) return;
    const int part = (int)(i % f.nparts);
    const int64_t lt = i / f.nparts;
    const int t = (int)(lt % f.nbt);
    const int lam = (int)(lt / f.nbt);
    const int m = f.bt_row[t], c = f.bt_col[t];
    const int tile = m / 16;
    const size_t job = ((size_t)lam * f.nparts + part) * f.mtiles + tile;
    double v = f.acc[job * 256 + (m % 16) * 16 + c] * f.bt_scale[t];
    if (f.norm_by_randoms) {
        const size_t job0 = ((size_t)f.lam0 * f.nparts + 0) * f.mtiles + tile;
        const double r = f.acc_rand[job0 * 256 + (m % 16) * 16 + c] * f.bt_scale[t];
        if (r == 0.0 || !isfinite(r)) atomicOr(f.bad, 2);
        v = v / r;
    }
    f.out[i] = v;  // [lambda][t][part]
}

inline int couple_lds(const CoupleArgs &a)
{
    // rows of a, weights, then the term list (N = 4, line of sight) or the
    // per-state factors (isotropic N = 3)
    const int tail = a.max_block_terms * (int)sizeof(CoupleTerm) > a.nstate * 4 ? a.max_block_terms * (int)sizeof(CoupleTerm)
                                                                                : a.nstate * 4;
    return (kRowsStep * a.nb * 2 * a.nstate + kRowsStep) * 4 + tail;
}

}  // namespace

int couple_njobs(int N, int nlam, int nparts, int mtiles) { return N == 4 ? nlam * nparts * mtiles : nlam * nparts; }

int couple_jobs_per_block() { return 4 * kJobsPerWave; }

int couple_ftask_groups(int nftasks) { return (nftasks + 3) / 4; }

int couple_nblocks(int njobs, int nrb)
{
    const int njg = (njobs + 4 * kJobsPerWave - 1) / (4 * kJobsPerWave);
    const int per_xcd = njg * ((nrb + kXcd - 1) / kXcd);
    return per_xcd * kXcd;
}

hipError_t launch_couple_kernel(int N, int precision, const CoupleArgs &a, int njobs, int nparts, const float *sfac,
                                hipStream_t s)
{
    if (N == 5) return launch_couple5(precision, a, njobs, s);  // njobs: output tiles
    const int lds = couple_lds(a);
    int nblk = couple_nblocks(njobs, a.n_rowblocks);
    if (N == 4 && a.fpairs) {
        const int ntg = couple_ftask_groups(a.nftasks);
        nblk = ntg * ((a.n_rowblocks + kXcd - 1) / kXcd) * kXcd;
        const int lds_f = (kRowsStep * a.nb * 2 * a.nstate + kRowsStep) * 4;
        switch (precision) {
        case 0: return launch_with_lds(k_couple4f<0>, nblk, lds_f, s, a, njobs);
        case 1: return launch_with_lds(k_couple4f<1>, nblk, lds_f, s, a, njobs);
        case 2: return launch_with_lds(k_couple4f<2>, nblk, lds_f, s, a, njobs);
        case 3: return launch_with_lds(k_couple4f<3>, nblk, lds_f, s, a, njobs);
        default: return hipErrorInvalidValue;
        }
    }
    if (N == 4) {
        switch (precision) {
        case 0: return launch_with_lds(k_couple4<0>, nblk, lds, s, a, njobs, nparts);
        case 1: return launch_with_lds(k_couple4<1>, nblk, lds, s, a, njobs, nparts);
        case 2: return launch_with_lds(k_couple4<2>, nblk, lds, s, a, njobs, nparts);
        case 3: return launch_with_lds(k_couple4<3>, nblk, lds, s, a, njobs, nparts);
        default: return hipErrorInvalidValue;
        }
    }
    if (a.n3_terms) {
        switch (precision) {
        case 0: return launch_with_lds(k_couple3t<0>, nblk, lds, s, a, njobs);
        case 1: return launch_with_lds(k_couple3t<1>, nblk, lds, s, a, njobs);
        case 2: return launch_with_lds(k_couple3t<2>, nblk, lds, s, a, njobs);
        case 3: return launch_with_lds(k_couple3t<3>, nblk, lds, s, a, njobs);
        default: return hipErrorInvalidValue;
        }
    }
    // isotropic N = 3: long rows (D = 4 at lmax 6: 6.7 KB per primary) stage
    // fewer per step, so that three blocks (the kernel's three waves per SIMD)
    // fit in a CU's LDS; few jobs (one per Lambda and part) spread over the
    // block's four waves instead of filling the first ones
    int rs = kRowsStep;
    const int rowbytes = a.nb * 2 * a.nstate * 4;
    while (rs > 1 && rs * rowbytes > kC3StageBytes) rs /= 2;
    const int jpw = njobs <= 4 ? 1 : (njobs <= 8 ? 2 : kJobsPerWave);
    const int njg3 = (njobs + 4 * jpw - 1) / (4 * jpw);
    const int nblk3 = njg3 * ((a.n_rowblocks + kXcd - 1) / kXcd) * kXcd;
    const int lds3 = lds - (kRowsStep - rs) * (rowbytes + 4);
    switch (precision) {
    case 0: return launch_with_lds(k_couple3<0>, nblk3, lds3, s, a, njobs, nparts, sfac, rs, jpw);
    case 1: return launch_with_lds(k_couple3<1>, nblk3, lds3, s, a, njobs, nparts, sfac, rs, jpw);
    case 2: return launch_with_lds(k_couple3<2>, nblk3, lds3, s, a, njobs, nparts, sfac, rs, jpw);
    case 3: return launch_with_lds(k_couple3<3>, nblk3, lds3, s, a, njobs, nparts, sfac, rs, jpw);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce_partials(const double *partial, int nrb, int64_t len, double *acc, hipStream_t s)
{
    const int64_t g = (len + 255) / 256;
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)g), dim3(256), 0, s, partial, nrb, len, acc);
    return hipGetLastError();
}

hipError_t launch_finalize_idx(const double *acc, const double *acc_rand, const int *idx, const double *sign,
                               const double *bt_scale, int nlam, int nbt, int norm_by_randoms, int lam0, double *out,
                               int *bad, hipStream_t s)
{
    const int64_t total = (int64_t)nlam * nbt;
    hipLaunchKernelGGL(k_finalize_idx, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, acc, acc_rand, idx, sign,
                       bt_scale, nlam, nbt, norm_by_randoms, lam0, out, bad);
    return hipGetLastError();
}

hipError_t launch_finalize2(const double *acc, const double *acc_rand, int nlam, int nparts, int mtiles,
                            const int *bt_row, const int *bt_col, const double *bt_scale, int nbt, int norm_by_randoms,
                            int lam0, double *out, int *bad, hipStream_t s)
{
    FinArgs f{acc, acc_rand, nlam, nparts, mtiles, bt_row, bt_col, bt_scale, nbt, norm_by_randoms, lam0, out, bad};
    const int64_t total = (int64_t)nlam * nparts * nbt;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f);
    return hipGetLastError();
}

}  // namespace npcf
