// Harmonic stage of the separable NPCF estimator (eq. NPCF-estimator-discrete,
// the sum defining a^b_[l](y_j); bin integral of eq. alm-bin-def):
//
//   a^b_[l](y_j) = sum_k w_k conj(Y_[l](unit(y_k - y_j))) Theta^b(|y_k - y_j|)
//
// (the 1/v_b factor is applied when the estimator is finalised).
//
// Mapping to gfx950
//  - one wavefront per primary; rows are handed out by an atomic counter so
//    clustered catalogues balance; primaries are visited in cell order;
//  - stencil rows of cells are trimmed to the primary's own sphere, lane
//    parallel, into a list of contiguous candidate segments of the
//    counting-sorted catalogue (16-byte packed lattice records, one load per
//    candidate, next batch prefetched);
//  - phase A (lanes over candidates): exact int32 periodic separation,
//    conservative FP32 range test, ballot compaction into an LDS pair queue;
//  - phase B (lanes over 64 queued pairs): FP64 r^2 with the definition's
//    arithmetic (exact bins on lattice inputs), unit vector normalised in
//    FP64 and rounded to FP32, harmonics by Gegenbauer recurrences in FP32
//    registers;
//  - scatter without atomics or collisions: each lane takes its position in
//    the batch sorted by bin (bit-plane ballots; per-bin masks and counts on
//    the scalar unit) and writes every harmonic it emits into column
//    `position` of an LDS staging array whose rows follow the emission order
//    (row stride 65 floats: the writes of one row and the transposed reads
//    below both touch distinct banks);
//  - reduction: every E emitted rows (E <= 64) the lanes switch to rows, sum
//    each bin's contiguous run of columns in FP32 and add it to FP64
//    accumulators held in registers; the primary's row of a is written once.
//    The cost per batch is fixed whatever the mix of bins (clustered data put
//    bursts of one bin into a batch), and the summation order is fixed.
#pragma once
#include "npcf_harmonic_scan.h"
#include "npcf_harmonic_pass.h"

namespace npcf {
namespace harm {

// Emission order of the harmonics functions (npcf_harmonics.h): the slot of
// every emitted value, in the order emit() is called.  Only emitted slots
// appear (the imaginary slot of a state with l1 = 0 is never written).
template <int D, int L>
struct EmitTable {
    static constexpr int SLOTS = 2 * stored_states(D, L);
    static constexpr int NE = D == 2 ? 2 * L + 1
                              : (D == 3 ? SLOTS - (L + 1) : SLOTS - (L + 1) * (L + 2) / 2);
    int slot[NE];
    constexpr EmitTable() : slot{}
    {
        int e = 0;
        if (D == 2) {
            slot[e++] = 0;
            for (int l = 1; l <= L; l++) {
                slot[e++] = 2 * l;
                slot[e++] = 2 * l + 1;
            }
        } else if (D == 3) {
            for (int m = 0; m <= L; m++)
                for (int l = m; l <= L; l++) {
                    const int st = l * (l + 1) / 2 + m;
                    slot[e++] = 2 * st;
                    if (m > 0) slot[e++] = 2 * st + 1;
                }
        } else {
            for (int l1 = 0; l1 <= L; l1++)
                for (int l2 = l1; l2 <= L; l2++)
                    for (int l3 = l2; l3 <= L; l3++) {
                        const int st = l3 * (l3 + 1) * (l3 + 2) / 6 + l2 * (l2 + 1) / 2 + l1;
                        slot[e++] = 2 * st;
                        if (l1 > 0) slot[e++] = 2 * st + 1;
                    }
        }
    }
};

template <int D, int L>
struct Cfg {
    static constexpr int NST = stored_states(D, L);
    static constexpr int SLOTS = 2 * NST;
    static constexpr int NE = EmitTable<D, L>::NE;             // emitted values per pair
    static constexpr int NCH = (NE + 63) / 64;                 // staging chunks per pair
    static constexpr int E = (NE + NCH - 1) / NCH;             // staging rows per chunk
    static constexpr int SSTR = 65;                            // staging row stride (floats)
    static constexpr int NK = NCH * kMaxBins;                  // FP64 accumulators per lane
    static constexpr int QWORDS = (D == 4) ? 5 : 4;            // queue words per pair
    static constexpr int STAGE_BYTES = (E * SSTR * 4 + 15) / 16 * 16;  // per wave
    static constexpr int WAVE_BYTES = (kQCap * QWORDS * 4 + kSegCap * 8 + 15) / 16 * 16;  // queue, segments
    // LDS: the four waves' staging rows first (small immediate offsets for the
    // reduction's reads), then the bin tables, then each wave's queue and segments
    static constexpr int LDS_BYTES = 4 * STAGE_BYTES + kTableBytes + 4 * WAVE_BYTES;
};

// true if stored state st (index in the library's state order) has l1 > 0,
// i.e. an imaginary part that the harmonics emit
template <int D, int L>
__device__ __forceinline__ bool emitted_im(int st)
{
    if (D == 2) return st != 0;
    if (D == 3) {
        int l = 0;
        while ((l + 1) * (l + 2) / 2 <= st) l++;
        return st - l * (l + 1) / 2 != 0;
    }
    int l3 = 0;
    while ((l3 + 1) * (l3 + 2) * (l3 + 3) / 6 <= st) l3++;
    int r = st - l3 * (l3 + 1) * (l3 + 2) / 6;
    int l2 = 0;
    while ((l2 + 1) * (l2 + 2) / 2 <= r) l2++;
    return r - l2 * (l2 + 1) / 2 != 0;
}

template <int D, int L, bool PER>
__global__ __launch_bounds__(256) void k_harmonic(HarmArgs a)
{
    using C = Cfg<D, L>;
    constexpr int SLOTS = C::SLOTS;
    constexpr int E = C::E;
    constexpr int NE = C::NE;
    // candidate batches in flight in phase A: D = 4 rows of cells hold fewer
    // candidates per segment, so the loads of one batch alone do not cover
    // the latency (measured: 2M clustered D = 4 points 179 -> 177 ms with two; 800k
    // clustered D = 3 points 165 -> 166 ms)
    constexpr int kPrefetch = D == 4 ? 2 : 1;
    extern __shared__ __align__(16) char smem[];
    const int nb = a.nb;
    const int lane = (int)lane_id();
    const int wave = threadIdx.x >> 6;

    char *tabs = smem + 4 * C::STAGE_BYTES;
    double *e2 = reinterpret_cast<double *>(tabs);
    uint8_t *btab = reinterpret_cast<uint8_t *>(tabs + (kMaxBins + 1) * 8);
    for (int t = threadIdx.x; t <= nb; t += blockDim.x) e2[t] = a.e2[t];
    for (int t = threadIdx.x; t < a.nbucket; t += blockDim.x) btab[t] = a.bucket_bin[t];

    char *wb = tabs + kTableBytes + wave * C::WAVE_BYTES;
    int4 *q4 = reinterpret_cast<int4 *>(wb);                                     // [kQCap]
    float *qwx = reinterpret_cast<float *>(wb + kQCap * 16);                     // [kQCap] (D = 4 weight)
    uint2 *segs = reinterpret_cast<uint2 *>(wb + kQCap * C::QWORDS * 4);         // [kSegCap]
    float *stage = reinterpret_cast<float *>(smem + wave * C::STAGE_BYTES);  // [E][SSTR]
    __syncthreads();

    // this lane reduces staging row `lane` of every chunk k, i.e. emitted value
    // k E + lane; fslot[k] is its slot in the row of a (-1: none)
    constexpr EmitTable<D, L> ET{};
    int fslot[C::NCH];
#pragma unroll
    for (int k = 0; k < C::NCH; k++) {
        const int e = k * E + lane;
        fslot[k] = (lane < E && e < NE) ? ET.slot[e] : -1;
    }

    const int nacc = nb * SLOTS;
    double acc[C::NK];  // acc[k kMaxBins + b]: chunk k's row `lane`, bin b
#pragma unroll
    for (int k = 0; k < C::NK; k++) acc[k] = 0.0;

    const double e2lo = e2[0], e2hi = e2[nb];
    const double rmax2 = e2hi * (1.0 + 1e-9);

    for (;;) {
        const int row = next_row(a.work, lane);
        if (row >= a.nrows) break;
        const int ip = a.prim[row];
        const uint4 ri = a.rec[ip];
        // the primary's catalogue (batches) and that catalogue's cell table
        int cat = 0;
        if (a.cat_begin) {
            int lo = 0, hi = a.ncat;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.cat_begin[mid] <= ip) lo = mid;
                else hi = mid;
            }
            cat = lo;
        }
        const uint32_t *cs = a.cell_start + (size_t)cat * (size_t)a.ncell_cat;
        unsigned long long row_pairs = 0;
        uint32_t qi[D];
#pragma unroll
        for (int k = 0; k < D; k++) qi[k] = rec_coord<D>(ri, k);
        const float wi = (D == 4) ? a.w[ip] : (D == 3 ? __int_as_float((int)ri.w) : __int_as_float((int)ri.z));

        int qn = 0;      // queued pairs (wave-uniform)

        // ---- phase B: queued pairs [0, cnt) ---------------------------------
        auto process = [&](int cnt) __attribute__((always_inline)) {
            NPCF_WAVE_SYNC();
            const bool live = lane < cnt;
            int dq[D];
            float wk = 0.f;
            {
                const int4 e = live ? q4[lane] : make_int4(0, 0, 0, 0);
                dq[0] = e.x;
                dq[1] = e.y;
                if (D >= 3) dq[2] = e.z;
                if (D == 4) {
                    dq[3] = e.w;
                    wk = live ? qwx[lane] : 0.f;
                } else {
                    wk = __int_as_float(D == 3 ? e.w : e.z);
                }
            }
            // separation in FP64 from the exact integer offsets: r^2 summed axis
            // by axis without contraction (the definition's arithmetic, so the
            // bin is decided exactly as there), the unit vector normalised in
            // FP64 and rounded once to FP32 (its error enters Y_l about l times)
            double v[D];
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
                v[k] = mul_rn((double)dq[k], a.scale64[k]);
                r2 = add_rn(r2, mul_rn(v[k], v[k]));
            }
            int bin;
            {
                // guess from the bucket table, accepted when the two edges
                // around it (read together) bracket r^2; otherwise a walk
                int bk = (int)(((float)r2 - a.bucket_lo) * a.bucket_inv);
                bk = bk < 0 ? 0 : (bk >= a.nbucket ? a.nbucket - 1 : bk);
                bin = btab[bk];
                const double elo = e2[bin], ehi = e2[bin + 1];
                if ((r2 < elo) | (r2 >= ehi)) {   // both edges needed: one LDS round trip
                    while (bin + 1 < nb && r2 >= e2[bin + 1]) bin++;
                    while (bin > 0 && r2 < e2[bin]) bin--;
                }
            }
            const bool valid = live && r2 >= e2lo && r2 < e2hi;
            if (!valid) bin = 0;
            const unsigned long long vm = ballot(valid);
            row_pairs += (unsigned long long)__popcll(vm);
            // 1/r: hardware FP64 estimate plus one Newton step
            const double rs = valid ? r2 : 1.0;
            double rinv = __builtin_amdgcn_rsq(rs);
            rinv = rinv * (1.5 - 0.5 * rs * rinv * rinv);
            if (!valid) wk = 0.f;  // lanes without a pair evaluate harmonics of weight zero
            float u[D];
#pragma unroll
            for (int k = 0; k < D; k++) u[k] = valid ? (float)(v[k] * rinv) : 0.f;

            // position of this pair in the batch sorted by bin.  Per bin b the
            // lanes holding it, M_b, follow from four bit-plane ballots with
            // scalar operations; the bin's run of columns starts at the number
            // of valid lanes of smaller bins, and a lane of bin b takes
            // start_b + (lanes of M_b below it).  Lanes without a pair take the
            // columns after the last valid one (they stage zeros).  The scalar
            // side keeps each bin's count for the reduction.
            unsigned long long Bk[4];
#pragma unroll
            for (int k = 0; k < 4; k++) Bk[k] = ballot(((bin >> k) & 1) != 0);  // invalid lanes hold bin 0
            const int nvalid = __popcll(vm);
            int pos = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(~vm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)~vm, (unsigned)nvalid));
            int bcnt[kMaxBins];
            {
                int run = 0;
#pragma unroll
                for (int b = 0; b < kMaxBins; b++) {
                    bcnt[b] = 0;
                    if (b < nb) {
                        unsigned long long mb = vm;
#pragma unroll
                        for (int t = 0; t < 4; t++) mb &= ((b >> t) & 1) ? Bk[t] : ~Bk[t];
                        const int cnt = __popcll(mb);
                        if (cnt) {
                            const int cand = (int)__builtin_amdgcn_mbcnt_hi(
                                (unsigned)(mb >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mb, (unsigned)run));
                            if (__builtin_amdgcn_inverse_ballot_w64(mb)) pos = cand;
                            run += cnt;
                            bcnt[b] = cnt;
                        }
                    }
                }
            }

            // staged rows [0, rows) of chunk k: lanes over rows; each bin's run of
            // sorted columns summed in FP32 (four interleaved partial sums) and
            // added to the FP64 accumulator
            auto reduce = [&](int k, int rows) __attribute__((always_inline)) {
                NPCF_WAVE_SYNC();
                const float *srow = stage + (lane < rows ? lane : rows - 1) * C::SSTR;
                int j0 = 0;
#pragma unroll
                for (int b = 0; b < kMaxBins; b++) {
                    const int cnt = bcnt[b];
                    if (cnt) {
                        // sixteen, then eight columns in flight per step (the
                        // loads, not the adds, set the pace), four partial sums
                        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                        int t = j0;
                        const int te = j0 + cnt;
                        for (; t + 15 < te; t += 16) {
                            float x[16];
#pragma unroll
                            for (int q = 0; q < 16; q++) x[q] = srow[t + q];
                            s0 += (x[0] + x[4]) + (x[8] + x[12]);
                            s1 += (x[1] + x[5]) + (x[9] + x[13]);
                            s2 += (x[2] + x[6]) + (x[10] + x[14]);
                            s3 += (x[3] + x[7]) + (x[11] + x[15]);
                        }
                        if (t + 7 < te) {
                            float x[8];
#pragma unroll
                            for (int q = 0; q < 8; q++) x[q] = srow[t + q];
                            s0 += x[0] + x[4];
                            s1 += x[1] + x[5];
                            s2 += x[2] + x[6];
                            s3 += x[3] + x[7];
                            t += 8;
                        }
                        // the rest (< 8 columns) by its bits: at most three
                        // blocks of 4, 2 and 1 reads
                        const int rem = te - t;
                        if (rem & 4) {
                            const float x0 = srow[t], x1 = srow[t + 1], x2 = srow[t + 2], x3 = srow[t + 3];
                            s0 += x0;
                            s1 += x1;
                            s2 += x2;
                            s3 += x3;
                            t += 4;
                        }
                        if (rem & 2) {
                            s0 += srow[t];
                            s1 += srow[t + 1];
                            t += 2;
                        }
                        if (rem & 1) s2 += srow[t];
                        acc[k * kMaxBins + b] += (double)((s0 + s1) + (s2 + s3));
                        j0 = te;
                    }
                }
                NPCF_WAVE_SYNC();  // the next chunk overwrites the staging rows
            };

            int e = 0;  // emission counter (a constant at every call once unrolled)
            harmonics<D, L>(u, wk, [&](int, float v) {
                stage[(e % E) * C::SSTR + pos] = v;
                if (e % E == E - 1 || e == NE - 1) reduce(e / E, e % E + 1);
                e++;
            });
        };

        // ---- phase A: candidates into the pair queue -------------------------
        scan_candidates<D, PER, kPrefetch>(a, cs, qi, segs, lane, rmax2,
                                           [&](bool inr, const int (&dq)[D], const uint4 &cur, float curw) __attribute__((always_inline)) {
            queue_append<D>(inr, dq, cur, curw, q4, qwx, qn);
            if (qn >= 64) {
                process(64);
                const int rest = qn - 64;
                if (lane < rest) {
                    q4[lane] = q4[64 + lane];
                    if (D == 4) qwx[lane] = qwx[64 + lane];
                }
                qn = rest;
                NPCF_WAVE_SYNC();
            }
        });
        if (qn > 0) process(qn);
        // the primary's row of a (FP32): emitted slots from the accumulators,
        // zeros in the others; clear the accumulators
        float *Arow = a.A + (size_t)row * nacc;
#pragma unroll
        for (int k = 0; k < C::NCH; k++) {
#pragma unroll
            for (int b = 0; b < kMaxBins; b++) {
                if (b < nb && fslot[k] >= 0) Arow[b * SLOTS + fslot[k]] = (float)acc[k * kMaxBins + b];
                acc[k * kMaxBins + b] = 0.0;
            }
        }
        for (int t0 = 0; t0 < nacc; t0 += 64) {
            const int t = t0 + lane;
            const int sl = t % SLOTS;
            if (t < nacc && sl % 2 == 1 && !emitted_im<D, L>(sl / 2)) Arow[t] = 0.f;
        }
        finish_row(a.wrow, row, wi, a.pairs + cat, row_pairs, lane);
    }
}

template <int D, int L>
int lds_bytes() { return Cfg<D, L>::LDS_BYTES; }

template <int D, int L>
hipError_t launch_dl(const HarmArgs &a, int grid, hipStream_t s)
{
    if constexpr (pass_supported<D, L>()) {
        if (a.per_bin) {
            const int lds = pass_lds_bytes<D, L>();
            // periodic cubes have their own instance (CUBE); open boxes take
            // the general test whatever their shape
            if (a.periodic && a.cube) {
                hipError_t e = hipFuncSetAttribute((const void *)k_harmonic_pass<D, L, true, true>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_harmonic_pass<D, L, true, true>), dim3(grid), dim3(256), lds, s, a);
            } else if (a.periodic) {
                hipError_t e = hipFuncSetAttribute((const void *)k_harmonic_pass<D, L, true, false>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_harmonic_pass<D, L, true, false>), dim3(grid), dim3(256), lds, s, a);
            } else {
                hipError_t e = hipFuncSetAttribute((const void *)k_harmonic_pass<D, L, false, false>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL((k_harmonic_pass<D, L, false, false>), dim3(grid), dim3(256), lds, s, a);
            }
            return hipGetLastError();
        }
    }
    const int lds = lds_bytes<D, L>();
    if (a.periodic) {
        hipError_t e = hipFuncSetAttribute((const void *)k_harmonic<D, L, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_harmonic<D, L, true>), dim3(grid), dim3(256), lds, s, a);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)k_harmonic<D, L, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_harmonic<D, L, false>), dim3(grid), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace harm
}  // namespace npcf
