// Candidate scan of the harmonic stage (the pair sum of eq. alm-bin-def in
// its discrete form, eq. NPCF-estimator-discrete): for one primary, every
// secondary within r_max is visited once through the counting-sorted cell
// list, with the exact lattice offset and a conservative FP32 range test.
//
//  - per-axis cell ranges of the stencil around the primary;
//  - stencil rows of cells trimmed to the primary's sphere, one row per lane,
//    into at most two contiguous segments of sorted records each (two when
//    the row wraps the periodic box);
//  - batches of 64 candidates over the segments, kPrefetch batches of
//    16-byte record loads in flight (across segment ends);
//  - per candidate: int32 wrap-around offset (the exact periodic minimum
//    image) or the open-box offset, and the FP32 test e_0^2 <= r^2 < e_nb^2
//    widened to be conservative (the exact FP64 bin is decided later).
// The caller's take(inr, dq, rec, w) runs on every lane of the wave for each
// batch (wave-uniform call): inr tells whether the lane holds an in-range
// candidate, dq its lattice offset, rec its record and w its FP32 weight (D = 4).
#pragma once
#include "npcf_harmonics.h"

namespace npcf {
namespace harm {

constexpr int kQCap = 128;          // pair queue entries per wave
constexpr int kSegCap = 128;        // candidate segments per row chunk
constexpr int kMaxBucket = 1024;
// LDS regions start on 16-byte boundaries: the pair queue is read and
// written as 16-byte records (misaligned, each access stalls)
constexpr int kTableBytes = ((kMaxBins + 1) * 8 + kMaxBucket + 15) / 16 * 16;

#define NPCF_WAVE_SYNC()                                       \
    do {                                                       \
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                       \
    } while (0)

__device__ __forceinline__ unsigned lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// wave-wide ballot of a boolean straight into a 64-bit lane mask
__device__ __forceinline__ unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ int rank_in_mask(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// The next row of a persistent launch, for the whole wave.  Every lane takes
// part in the atomic (lane 0 adds one, the others zero) and v_readlane hands
// lane 0's value to the wave as a scalar, so no branch on the lane surrounds
// the row hand-out and the loop over rows exits on a uniform branch.  With the
// atomic under `if (lane == 0)` and the row broadcast by a shuffle, the
// compiler merged that branch with the lane-0 tail of the previous row and
// sent lanes 1..63 back to the loop head without lane 0: they re-read a row
// that never advanced (a variant of this kernel never finished: its loop
// latch took the lane-0 mask out of exec and branched to the shuffle).
__device__ __forceinline__ int next_row(unsigned int *work, int lane)
{
    const unsigned int r = atomicAdd(work, lane == 0 ? 1u : 0u);
    return (int)__builtin_amdgcn_readlane((int)r, 0);
}

// End of a row for the whole wave, with no branch on the lane: every lane
// stores the primary's weight (one address, one value) and adds to the pair
// counter (lane 0 the row's count, the others zero).
__device__ __forceinline__ void finish_row(float *wrow, int row, float wi, unsigned long long *pairs,
                                           unsigned long long row_pairs, int lane)
{
    wrow[row] = wi;
    atomicAdd(pairs, lane == 0 ? row_pairs : 0ull);
}

template <int D>
__device__ __forceinline__ uint32_t rec_coord(const uint4 &r, int k)
{
    return k == 0 ? r.x : (k == 1 ? r.y : (k == 2 ? r.z : r.w));
}

// Append this batch's in-range candidates to the wave's pair queue (records
// of 16 bytes: the lattice offsets and the weight bits; D = 4 keeps the
// weight beside them) at [qn, qn + count) in lane order; qn advances.
template <int D>
__device__ __forceinline__ void queue_append(bool inr, const int (&dq)[D], const uint4 &cur, float curw, int4 *q4,
                                             float *qwx, int &qn)
{
    const unsigned long long m = ballot(inr);
    if (inr) {
        const int slot = qn + rank_in_mask(m);
        int4 e;
        e.x = dq[0];
        e.y = dq[1];
        if (D == 2) {
            e.z = (int)cur.z;  // weight bits
            e.w = 0;
        } else if (D == 3) {
            e.z = dq[2];
            e.w = (int)cur.w;  // weight bits
        } else {
            e.z = dq[2];
            e.w = dq[3];
            qwx[slot] = curw;
        }
        q4[slot] = e;
    }
    qn += __popcll(m);
}

template <int D, bool PER, int kPrefetch, class Take>
__device__ __forceinline__ void scan_candidates(const HarmArgs &a, const uint32_t *cs, const uint32_t (&qi)[D],
                                                uint2 *segs, int lane, double rmax2, Take &&take)
{
    const float e2lo_f = a.e2lo_f, e2hi_f = a.e2hi_f;
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

        // candidate batches of 64 over the chunk's segments, streamed
        // through kPrefetch loads in flight (across segment ends): batch p
        // holds records [pb[p], pe[p]) of one segment, pb == pe past the end
        // The segment bounds are the same for every lane (one LDS address):
        // readfirstlane keeps them and the batch loop in scalar registers.
        int ci = 0;
        uint32_t cb = 0, ce = 0;
        if (nseg > 0) {
            const uint2 sg = segs[0];
            cb = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.x);
            ce = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.y);
        }
        auto advance = [&]() __attribute__((always_inline)) {
            cb += 64;
            if (cb >= ce) {
                ci++;
                if (ci < nseg) {
                    const uint2 sg = segs[ci];
                    cb = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.x);
                    ce = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.y);
                } else {
                    cb = 0;
                    ce = 0;
                }
            }
        };
        // every lane loads: lanes past the batch's end read record 0 (there is
        // at least the primary) and are masked at the test
        auto load = [&](uint4 &r, float &w) __attribute__((always_inline)) {
            const uint32_t g = cb + (uint32_t)lane;
            const uint32_t idx = g < ce ? g : 0u;
            r = a.rec[idx];
            w = D == 4 ? a.w[idx] : 0.f;
        };
        uint4 pr[kPrefetch];
        float pw[kPrefetch];
        uint32_t pb[kPrefetch], pe[kPrefetch];
#pragma unroll
        for (int p = 0; p < kPrefetch; p++) {
            pb[p] = cb;
            pe[p] = ce;
            load(pr[p], pw[p]);
            advance();
        }
        while (pb[0] < pe[0]) {
            const uint4 cur = pr[0];
            const float curw = pw[0];
            const uint32_t b0 = pb[0], s1 = pe[0];
            // shift the pipeline and issue the next batch's loads
#pragma unroll
            for (int p = 0; p + 1 < kPrefetch; p++) {
                pr[p] = pr[p + 1];
                pw[p] = pw[p + 1];
                pb[p] = pb[p + 1];
                pe[p] = pe[p + 1];
            }
            pb[kPrefetch - 1] = cb;
            pe[kPrefetch - 1] = ce;
            load(pr[kPrefetch - 1], pw[kPrefetch - 1]);
            advance();
            {
                // every lane holds a record, so the test needs no branch
                int dq[D];
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
                const bool inr = b0 + (uint32_t)lane < s1 && fits && r2f >= e2lo_f && r2f < e2hi_f;
                take(inr, dq, cur, curw);
            }
        }
    }
}

}  // namespace harm
}  // namespace npcf
