// Harmonic stage, bin-queue variant: the same sums as k_harmonic
// (eq. NPCF-estimator-discrete, a^b_[l] of eq. alm-bin-def), with batches
// that hold one bin only.
//
//  - phase A (lanes over candidates of the trimmed stencil segments): exact
//    int32 separation and a conservative FP32 range pre-test; the sorted
//    indices of the candidates that pass go to a first-level LDS queue;
//  - bin step, per 64 queued candidates: the records are read again, FP64 r^2
//    with the definition's arithmetic gives the exact bin, and each pair's
//    sorted index is appended to its bin's LDS queue (64 entries; the lane of
//    a bin's last member publishes the new count, lanes past a full queue
//    wait for it to be emptied);
//  - a full queue (or, at the end of a primary, any non-empty one) is one
//    batch of pairs of a single bin: its records are gathered again, the unit
//    vector normalised in FP64, the harmonics written to column `lane` of the
//    staging rows (rows in emission order, stride 65), and every row summed
//    over all 64 columns in one run into the bin's FP64 accumulator.
// With one bin per batch the reduction has no per-bin bookkeeping, which is
// what mixed-bin batches spend most of their time on.
#pragma once
#include "npcf_harmonic_impl.h"

namespace npcf {
namespace harm {

constexpr int kBinQ = 64;   // entries per bin queue

template <int D, int L>
struct CfgQ {
    using B = Cfg<D, L>;
    static constexpr int E = B::E;
    static constexpr int NE = B::NE;
    static constexpr int NCH = B::NCH;
    static constexpr int SSTR = 65;
    // segments, first-level queue and bin queues (sorted indices), bin counts, staging
    static constexpr int WAVE_BYTES =
        (kSegCap * 8 + kQCap * 4 + kMaxBins * kBinQ * 4 + kMaxBins * 4 + E * SSTR * 4 + 15) / 16 * 16;
};

template <int D, int L, bool PER>
__global__ __launch_bounds__(128) void k_harmonic_bq(HarmArgs a)
{
    using C = CfgQ<D, L>;
    constexpr int SLOTS = Cfg<D, L>::SLOTS;
    constexpr int E = C::E;
    constexpr int NE = C::NE;
    extern __shared__ __align__(16) char smem[];
    const int nb = a.nb;
    const int lane = (int)lane_id();
    const int wave = threadIdx.x >> 6;

    double *e2 = reinterpret_cast<double *>(smem);
    uint8_t *btab = reinterpret_cast<uint8_t *>(smem + (kMaxBins + 1) * 8);
    for (int t = threadIdx.x; t <= nb; t += blockDim.x) e2[t] = a.e2[t];
    for (int t = threadIdx.x; t < a.nbucket; t += blockDim.x) btab[t] = a.bucket_bin[t];

    char *wb = smem + kTableBytes + wave * C::WAVE_BYTES;
    uint2 *segs = reinterpret_cast<uint2 *>(wb);                                              // [kSegCap]
    int *q1 = reinterpret_cast<int *>(wb + kSegCap * 8);                                      // [kQCap]
    int *bq = reinterpret_cast<int *>(wb + kSegCap * 8 + kQCap * 4);                          // [kMaxBins][kBinQ]
    int *bcnt = reinterpret_cast<int *>(wb + kSegCap * 8 + kQCap * 4 + kMaxBins * kBinQ * 4);  // [kMaxBins]
    float *stage = reinterpret_cast<float *>(wb + kSegCap * 8 + kQCap * 4 + kMaxBins * kBinQ * 4 + kMaxBins * 4);
    if (lane < kMaxBins) bcnt[lane] = 0;
    __syncthreads();

    constexpr EmitTable<D, L> ET{};
    int fslot[C::NCH];
#pragma unroll
    for (int k = 0; k < C::NCH; k++) {
        const int e = k * E + lane;
        fslot[k] = (lane < E && e < NE) ? ET.slot[e] : -1;
    }

    const int nacc = nb * SLOTS;
    double acc[Cfg<D, L>::NK];  // acc[k kMaxBins + b]: chunk k's row `lane`, bin b
#pragma unroll
    for (int k = 0; k < Cfg<D, L>::NK; k++) acc[k] = 0.0;

    const float e2lo_f = a.e2lo_f, e2hi_f = a.e2hi_f;
    const double e2lo = e2[0], e2hi = e2[nb];
    const double rmax2 = e2hi * (1.0 + 1e-9);

    for (;;) {
        int row = 0;
        if (lane == 0) row = (int)atomicAdd(a.work, 1u);
        row = __shfl(row, 0);
        if (row >= a.nrows) break;
        const int ip = a.prim[row];
        const uint4 ri = a.rec[ip];
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

        // ---- one batch of bin b: queue entries [0, cnt) ----------------------
        auto process_bin = [&](int b, int cnt) __attribute__((always_inline)) {
            NPCF_WAVE_SYNC();
            const bool live = lane < cnt;
            const int idx = live ? bq[b * kBinQ + lane] : (int)ip;
            const uint4 r = a.rec[idx];
            float wk = live ? ((D == 4) ? a.w[idx] : (D == 3 ? __int_as_float((int)r.w) : __int_as_float((int)r.z))) : 0.f;
            double v[D];
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const int d = (int)(rec_coord<D>(r, k) - qi[k]);  // exact (checked in phase A)
                v[k] = __dmul_rn((double)d, a.scale64[k]);
                r2 = __dadd_rn(r2, __dmul_rn(v[k], v[k]));
            }
            const double rs = live ? r2 : 1.0;
            double rinv = __builtin_amdgcn_rsq(rs);
            rinv = rinv * (1.5 - 0.5 * rs * rinv * rinv);
            float u[D];
#pragma unroll
            for (int k = 0; k < D; k++) u[k] = live ? (float)(v[k] * rinv) : 0.f;
            if (!live) wk = 0.f;

            // staged rows [0, rows) of chunk k hold one bin: lanes over rows sum
            // all 64 columns (lanes without a pair wrote zeros)
            auto reduce = [&](int k, int rows) __attribute__((always_inline)) {
                NPCF_WAVE_SYNC();
                const float *srow = stage + (lane < rows ? lane : rows - 1) * C::SSTR;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
                for (int t = 0; t < 64; t += 8) {
                    float x[8];
#pragma unroll
                    for (int q = 0; q < 8; q++) x[q] = srow[t + q];
                    s0 += x[0] + x[4];
                    s1 += x[1] + x[5];
                    s2 += x[2] + x[6];
                    s3 += x[3] + x[7];
                }
                const double s = (double)((s0 + s1) + (s2 + s3));
                // one uniform branch per bin on a bit of 1 << b (written as an
                // index b the accumulators would leave registers)
                const unsigned bbit = 1u << b;
#pragma unroll
                for (int bb = 0; bb < kMaxBins; bb++)
                    if ((bbit >> bb) & 1u) acc[k * kMaxBins + bb] += s;
                NPCF_WAVE_SYNC();  // the next chunk overwrites the staging rows
            };
            int e = 0;  // emission counter (a constant at every call once unrolled)
            harmonics<D, L>(u, wk, [&](int, float val) __attribute__((always_inline)) {
                stage[(e % E) * C::SSTR + lane] = val;
                if (e % E == E - 1 || e == NE - 1) reduce(e / E, e % E + 1);
                e++;
            });
        };

        // ---- bin step: first-level entries [0, cnt) -> bin queues ------------
        auto bin_step = [&](int cnt) __attribute__((always_inline)) {
            NPCF_WAVE_SYNC();
            const bool live = lane < cnt;
            const int sidx = live ? q1[lane] : (int)ip;
            const uint4 r = a.rec[sidx];
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const int d = (int)(rec_coord<D>(r, k) - qi[k]);
                const double vv = __dmul_rn((double)d, a.scale64[k]);
                r2 = __dadd_rn(r2, __dmul_rn(vv, vv));
            }
            int bin;
            {
                int bk = (int)(((float)r2 - a.bucket_lo) * a.bucket_inv);
                bk = bk < 0 ? 0 : (bk >= a.nbucket ? a.nbucket - 1 : bk);
                bin = btab[bk];
                while (bin + 1 < nb && r2 >= e2[bin + 1]) bin++;
                while (bin > 0 && r2 < e2[bin]) bin--;
            }
            const bool valid = live && r2 >= e2lo && r2 < e2hi;
            if (!valid) bin = 0;
            const unsigned long long vm = ballot(valid);
            row_pairs += (unsigned long long)__popcll(vm);
            // rank among this batch's lanes of the same bin (bins < 16)
            unsigned long long same = vm;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const unsigned long long Bk = ballot(valid && ((bin >> k) & 1));
                const unsigned long long mk = 0ull - (unsigned long long)((bin >> k) & 1);
                same &= Bk ^ ~mk;
            }
            const int rank = rank_in_mask(same);
            const int tot = __popcll(same);
            const int base = valid ? bcnt[bin] : 0;
            const int slot = base + rank;
            if (valid && slot < kBinQ) bq[bin * kBinQ + slot] = sidx;
            NPCF_WAVE_SYNC();
            if (valid && rank == tot - 1) bcnt[bin] = base + tot;  // may exceed the queue
            NPCF_WAVE_SYNC();
            const unsigned long long full = ballot(lane < nb && bcnt[lane] >= kBinQ);
            if (full) {
                for (unsigned long long fm = full; fm; fm &= fm - 1) process_bin(__builtin_ctzll(fm), kBinQ);
                NPCF_WAVE_SYNC();
                // the lanes that found their queue full go to its front
                if (valid && slot >= kBinQ) bq[bin * kBinQ + slot - kBinQ] = sidx;
                if (lane < nb && ((full >> lane) & 1)) bcnt[lane] -= kBinQ;
                NPCF_WAVE_SYNC();
            }
        };
        int qn = 0;  // first-level entries (wave-uniform)

        // ---- stencil: per-axis cell ranges around the primary ----------------
        int lo[D], span[D];
        bool full[D];
#pragma unroll
        for (int k = 0; k < D; k++) {
            const double qk = (double)qi[k];
            long long l0 = (long long)floor((qk - a.rmax_lat[k] - 4.0) * a.inv_cell_len[k]);
            long long h0 = (long long)floor((qk + a.rmax_lat[k] + 4.0) * a.inv_cell_len[k]);
            full[k] = false;
            if (PER) {
                if (h0 - l0 + 1 >= a.ncs[k]) {
                    l0 = 0;
                    h0 = a.ncs[k] - 1;
                    full[k] = true;
                }
            } else {
                if (l0 < 0) l0 = 0;
                if (h0 > a.ncs[k] - 1) h0 = a.ncs[k] - 1;
            }
            lo[k] = (int)l0;
            span[k] = (int)(h0 - l0 + 1);
        }
        int nrow = 1;
#pragma unroll
        for (int k = 1; k < D; k++) nrow *= span[k];

        for (int rbase = 0; rbase < nrow; rbase += 64) {
            // each lane trims one row of cells to the sphere: up to two segments
            uint32_t sa0 = 0, sb0 = 0, sa1 = 0, sb1 = 0;
            bool has0 = false, has1 = false;
            const int rix = rbase + lane;
            if (rix < nrow) {
                int t = rix;
                double d2 = 0.0;
                long long lin = 0, mul = a.ncs[0];
#pragma unroll
                for (int k = 1; k < D; k++) {
                    const int c = lo[k] + t % span[k];
                    t /= span[k];
                    double dist = 0.0;
                    if (!full[k]) {
                        const double slo = (double)c * a.cell_len[k];
                        const double qk = (double)qi[k];
                        if (qk < slo) dist = slo - qk;
                        else if (qk >= slo + a.cell_len[k]) dist = qk - (slo + a.cell_len[k]);
                        dist = dist > 4.0 ? dist - 4.0 : 0.0;
                    }
                    const double dp = dist * a.scale64[k];
                    d2 += dp * dp;
                    int cw = c % a.ncs[k];
                    if (cw < 0) cw += a.ncs[k];
                    lin += (long long)cw * mul;
                    mul *= a.ncs[k];
                }
                if (d2 < rmax2) {
                    int xa, xb;
                    if (full[0]) {
                        xa = 0;
                        xb = a.ncs[0] - 1;
                    } else {
                        const double h = sqrt(rmax2 - d2) / a.scale64[0] + 4.0;
                        const double qx = (double)qi[0];
                        long long x0 = (long long)floor((qx - h) * a.inv_cell_len[0]);
                        long long x1 = (long long)floor((qx + h) * a.inv_cell_len[0]);
                        if (PER) {
                            if (x1 - x0 + 1 >= a.ncs[0]) {
                                x0 = 0;
                                x1 = a.ncs[0] - 1;
                            }
                        } else {
                            if (x0 < 0) x0 = 0;
                            if (x1 > a.ncs[0] - 1) x1 = a.ncs[0] - 1;
                        }
                        xa = (int)x0;
                        xb = (int)x1;
                    }
                    int ra0 = xa, rb0 = xb, ra1 = 0, rb1 = -1;
                    if (xa < 0) {
                        ra0 = xa + a.ncs[0]; rb0 = a.ncs[0] - 1;
                        ra1 = 0; rb1 = xb;
                    } else if (xb >= a.ncs[0]) {
                        ra0 = xa; rb0 = a.ncs[0] - 1;
                        ra1 = 0; rb1 = xb - a.ncs[0];
                    }
                    if (rb0 >= ra0) {
                        sa0 = cs[lin + ra0];
                        sb0 = cs[lin + rb0 + 1];
                        has0 = sb0 > sa0;
                    }
                    if (rb1 >= ra1) {
                        sa1 = cs[lin + ra1];
                        sb1 = cs[lin + rb1 + 1];
                        has1 = sb1 > sa1;
                    }
                }
            }
            const unsigned long long m0 = ballot(has0), m1 = ballot(has1);
            const int n0 = __popcll(m0);
            if (has0) segs[rank_in_mask(m0)] = make_uint2(sa0, sb0);
            if (has1) segs[n0 + rank_in_mask(m1)] = make_uint2(sa1, sb1);
            const int nseg = n0 + __popcll(m1);
            NPCF_WAVE_SYNC();

            for (int si = 0; si < nseg; si++) {
                const uint2 sg = segs[si];
                const uint32_t s0 = sg.x, s1 = sg.y;
                uint4 cur = make_uint4(0, 0, 0, 0);
                if (s0 + (uint32_t)lane < s1) cur = a.rec[s0 + lane];
                for (uint32_t b0 = s0; b0 < s1; b0 += 64) {
                    // prefetch the next batch of this segment
                    const uint32_t kn = b0 + 64 + (uint32_t)lane;
                    uint4 nxt = make_uint4(0, 0, 0, 0);
                    if (kn < s1) nxt = a.rec[kn];
                    bool inr = false;
                    int dq[D];
                    if (b0 + (uint32_t)lane < s1) {
                        float r2f = 0.f;
                        bool fits = true;
#pragma unroll
                        for (int k = 0; k < D; k++) {
                            const uint32_t qk = rec_coord<D>(cur, k);
                            int d;
                            if (PER) {
                                d = (int)(qk - qi[k]);  // two's-complement wrap = minimum image
                            } else {
                                const long long dl = (long long)qk - (long long)qi[k];
                                d = (int)dl;
                                fits = fits && (long long)d == dl;
                            }
                            dq[k] = d;
                            const float fv = (float)d * a.scale[k];
                            r2f += fv * fv;
                        }
                        inr = fits && r2f >= e2lo_f && r2f < e2hi_f;
                    }
                    const unsigned long long m = ballot(inr);
                    if (inr) q1[qn + rank_in_mask(m)] = (int)(b0 + (uint32_t)lane);
                    qn += __popcll(m);
                    if (qn >= 64) {
                        bin_step(64);
                        const int rest = qn - 64;
                        NPCF_WAVE_SYNC();
                        if (lane < rest) q1[lane] = q1[64 + lane];
                        qn = rest;
                        NPCF_WAVE_SYNC();
                    }
                    cur = nxt;
                }
            }
        }
        // drain the first-level queue, then the partly filled bin queues
        if (qn > 0) bin_step(qn);
        {
            NPCF_WAVE_SYNC();
            const unsigned long long nz = ballot(lane < nb && bcnt[lane] > 0);
            for (unsigned long long fm = nz; fm; fm &= fm - 1) {
                const int b = __builtin_ctzll(fm);
                process_bin(b, __shfl(lane < kMaxBins ? bcnt[lane] : 0, b));
            }
            NPCF_WAVE_SYNC();
            if (lane < kMaxBins) bcnt[lane] = 0;
            NPCF_WAVE_SYNC();
        }
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
        for (int t = lane; t < nacc; t += 64) {
            const int sl = t % SLOTS;
            if (sl % 2 == 1 && !emitted_im<D, L>(sl / 2)) Arow[t] = 0.f;
        }
        if (lane == 0) {
            a.wrow[row] = wi;
            if (row_pairs) atomicAdd(a.pairs + cat, row_pairs);
        }
    }
}

template <int D, int L>
int lds_bytes_bq() { return kTableBytes + 2 * CfgQ<D, L>::WAVE_BYTES; }

template <int D, int L>
hipError_t launch_dl_bq(const HarmArgs &a, int grid, hipStream_t s)
{
    const int lds = lds_bytes_bq<D, L>();
    if (a.periodic) {
        hipError_t e = hipFuncSetAttribute((const void *)k_harmonic_bq<D, L, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_harmonic_bq<D, L, true>), dim3(grid), dim3(128), lds, s, a);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)k_harmonic_bq<D, L, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_harmonic_bq<D, L, false>), dim3(grid), dim3(128), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace harm
}  // namespace npcf
