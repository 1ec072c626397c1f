// Harmonic stage, one radial bin per pass (eq. NPCF-estimator-discrete, the
// sum defining a^b_[l](y_j), for one b at a time):
//
//   a^b_[l](y_j) = sum_{k : e_b <= |y_k - y_j| < e_{b+1}} w_k conj(Y_[l](unit(y_k - y_j)))
//
// For each primary the wave scans the candidates of the bin's shell once per
// bin: stencil rows of cells are trimmed to the shell's outer sphere and
// lose the cells that lie wholly inside its inner one, so a pass visits
// about the shell's volume widened by a cell.  Every queued pair of a pass
// is in the pass's bin or rejected by the FP64 test, so each lane adds the
// harmonics it emits straight into its own FP32 sums (one register per slot,
// no sorting by bin, no staging), and every few batches the wave folds its
// lanes into FP64 values held one or two per lane.  D = 4 keeps its weight
// beside the record (in the queue too).  The FP32 pre-test on
// r^2 is widened by 1e-5 relative at both edges of the pass, and the FP64
// r^2 with the definition's arithmetic decides, as in the staged kernel.
#pragma once
#include "npcf_harmonic_scan.h"
#include "npcf_lanefold.h"

namespace npcf {
namespace harm {

constexpr int kPassSegCap = 256;      // candidate segments per 64 stencil rows (up to four per row)
// queued batches between folds of the lanes' sums (each lane adds one pair
// per batch).  c2 (32 + 32 sampled primaries, plain strict / conditioned
// per-multipole error; harmonic ms): every 2 batches 5.7e-7 / 6.5e-8, 130.2
// ms; 4: 8.0e-7 / 6.7e-8, 112.6 ms; 8: 6.4e-7 / 1.2e-7, 104.6 ms.  With the
// later scan changes: 8: 7.1e-7 / 1.0e-7, 75.5 ms; 16: 6.9e-7 / 1.6e-7,
// 71.7 ms, but on the bench's sample of 1054 primaries (half of them in the
// clustered data, with more batches per bin) 16 gave 1.2e-6 strict against
// 6.8e-7 at 8, over the plain bar of 1e-6: 8 stays
constexpr int kPassFoldBatches = 8;

// Candidates of the shell rlo2 <= r^2 < rhi2 (physical units, FP64; rlo2 and
// rhi2 taken slightly wide by the caller) through the cell list, tested
// against the FP32 bounds [flo, fhi) and handed to take() 64 at a time, as
// scan_candidates does for the whole range.  CUBE (every axis the same lattice
// scale): the FP32 test sums the squared lattice differences and the bounds
// come in squared lattice units, three multiplies fewer per candidate.  Per stencil row the x range of
// cells is cut to the outer sphere, and the cells wholly inside the inner
// sphere are left out (when no axis of the stencil wraps the whole periodic
// box), so a row gives up to two intervals of cells, each split in two where
// it wraps the periodic box.
template <int D, bool PER, bool CUBE, class Take>
__device__ __forceinline__ void scan_shell(const HarmArgs &a, const uint32_t *cs, const uint32_t (&qi)[D],
                                           uint2 *segs, int lane, double rlo2, double rhi2, float flo, float fhi,
                                           Take &&take)
{
    int lo[D], span[D];
    bool full[D];
    bool anyfull = false;
#pragma unroll
    for (int k = 0; k < D; k++) {
        const double qk = (double)qi[k];
        const double rk = sqrt(rhi2) / a.scale64[k];   // outer radius, lattice units of axis k
        long long l0 = (long long)floor((qk - rk - 4.0) * a.inv_cell_len[k]);
        long long h0 = (long long)floor((qk + rk + 4.0) * a.inv_cell_len[k]);
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
        anyfull = anyfull || full[k];
    }
    int nrow = 1;
#pragma unroll
    for (int k = 1; k < D; k++) nrow *= span[k];

    for (int rbase = 0; rbase < nrow; rbase += 64) {
        uint32_t sa[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0};
        bool has[4] = {false, false, false, false};
        const int rix = rbase + lane;
        if (rix < nrow) {
            int t = rix;
            double d2 = 0.0, d2f = 0.0;   // nearest and farthest squared distance over axes 1..D-1
            long long lin = 0, mul = a.ncs[0];
#pragma unroll
            for (int k = 1; k < D; k++) {
                const int c = lo[k] + t % span[k];
                t /= span[k];
                double dist = 0.0, far = 0.0;
                if (!full[k]) {
                    const double slo = (double)c * a.cell_len[k];
                    const double shi = slo + a.cell_len[k];
                    const double qk = (double)qi[k];
                    if (qk < slo) dist = slo - qk;
                    else if (qk >= shi) dist = qk - shi;
                    dist = dist > 4.0 ? dist - 4.0 : 0.0;
                    far = fmax(fabs(qk - slo), fabs(shi - qk)) + 4.0;
                }
                const double dp = dist * a.scale64[k], fp = far * a.scale64[k];
                d2 += dp * dp;
                d2f += fp * fp;
                int cw = c % a.ncs[k];
                if (cw < 0) cw += a.ncs[k];
                lin += (long long)cw * mul;
                mul *= a.ncs[k];
            }
            if (d2 < rhi2) {
                long long xa, xb;
                if (full[0]) {
                    xa = 0;
                    xb = a.ncs[0] - 1;
                } else {
                    const double h = sqrt(rhi2 - d2) / a.scale64[0] + 4.0;
                    const double qx = (double)qi[0];
                    xa = (long long)floor((qx - h) * a.inv_cell_len[0]);
                    xb = (long long)floor((qx + h) * a.inv_cell_len[0]);
                    if (PER) {
                        if (xb - xa + 1 >= a.ncs[0]) {
                            xa = 0;
                            xb = a.ncs[0] - 1;
                        }
                    } else {
                        if (xa < 0) xa = 0;
                        if (xb > a.ncs[0] - 1) xb = a.ncs[0] - 1;
                    }
                }
                // cells [ca, cb] wholly inside the inner sphere (its x half-width
                // in this row, less the margin, over the cell's farthest corner)
                long long ca = 1, cb = 0;
                if (!anyfull && d2f < rlo2) {
                    const double hin = sqrt(rlo2 - d2f) / a.scale64[0] - 4.0;
                    if (hin > 0.0) {
                        const double qx = (double)qi[0];
                        ca = (long long)ceil((qx - hin) * a.inv_cell_len[0]);
                        cb = (long long)floor((qx + hin) * a.inv_cell_len[0]) - 1;
                    }
                }
                long long iv0[2] = {xa, 0}, iv1[2] = {xb, -1};
                if (ca <= cb && ca <= xb && cb >= xa) {
                    iv0[0] = xa;
                    iv1[0] = ca - 1;
                    iv0[1] = cb + 1;
                    iv1[1] = xb;
                }
#pragma unroll
                for (int v = 0; v < 2; v++) {
                    long long u0 = iv0[v], u1 = iv1[v];
                    if (u1 < u0) continue;
                    long long r0a = u0, r0b = u1, r1a = 0, r1b = -1;
                    if (u0 < 0) {
                        r0a = u0 + a.ncs[0];
                        r0b = a.ncs[0] - 1;
                        r1a = 0;
                        r1b = u1;
                    } else if (u1 >= a.ncs[0]) {
                        r0a = u0;
                        r0b = a.ncs[0] - 1;
                        r1a = 0;
                        r1b = u1 - a.ncs[0];
                    }
                    if (r0b >= r0a) {
                        sa[2 * v] = cs[lin + r0a];
                        sb[2 * v] = cs[lin + r0b + 1];
                        has[2 * v] = sb[2 * v] > sa[2 * v];
                    }
                    if (r1b >= r1a) {
                        sa[2 * v + 1] = cs[lin + r1a];
                        sb[2 * v + 1] = cs[lin + r1b + 1];
                        has[2 * v + 1] = sb[2 * v + 1] > sa[2 * v + 1];
                    }
                }
            }
        }
        int nseg = 0;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const unsigned long long m = ballot(has[v]);
            if (has[v]) segs[nseg + rank_in_mask(m)] = make_uint2(sa[v], sb[v]);
            nseg += __popcll(m);
        }
        NPCF_WAVE_SYNC();

        // candidate batches of 64 over the segments, one batch of loads in
        // flight.  The segment bounds are the same for every lane (one LDS
        // address); reading them through readfirstlane keeps them, the batch
        // loop and the queue count in scalar registers, so the loop branches
        // on scalars instead of masking lanes
        int ci = 0;
        uint32_t cb0 = 0, ce0 = 0;
        if (nseg > 0) {
            const uint2 sg = segs[0];
            cb0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.x);
            ce0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.y);
        }
        auto advance = [&]() __attribute__((always_inline)) {
            cb0 += 64;
            if (cb0 >= ce0) {
                ci++;
                if (ci < nseg) {
                    const uint2 sg = segs[ci];
                    cb0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.x);
                    ce0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sg.y);
                } else {
                    cb0 = 0;
                    ce0 = 0;
                }
            }
        };
        // every lane loads: lanes past the batch's end read record 0 (there is
        // at least the primary) and are masked at the test by ok, which
        // travels with the record as a lane mask
        auto load = [&](uint4 &r, float &w, bool &ok) __attribute__((always_inline)) {
            const uint32_t g = cb0 + (uint32_t)lane;
            ok = g < ce0;
            const uint32_t idx = ok ? g : 0u;
            r = a.rec[idx];
            if (D == 4) w = a.w[idx];
        };
        bool more = cb0 < ce0;   // the batch in flight holds records (wave-uniform)
        uint4 pr;
        float pw = 0.f;   // D = 4: the weight beside the record
        bool pok;
        load(pr, pw, pok);
        advance();
        while (more) {
            const uint4 cur = pr;
            const float curw = pw;
            const bool curok = pok;
            more = cb0 < ce0;
            load(pr, pw, pok);
            advance();
            // every lane holds a record, so the test needs no branch
            int dq[D];
            float r2f = 0.f;
            bool fits = true;
#pragma unroll
            for (int k = 0; k < D; k++) {
                const uint32_t qk = rec_coord<D>(cur, k);
                int d;
                if (PER) {
                    d = (int)(qk - qi[k]);   // two's-complement wrap = minimum image
                } else {
                    const long long dl = (long long)qk - (long long)qi[k];
                    d = (int)dl;
                    fits = fits && (long long)d == dl;
                }
                dq[k] = d;
                const float fv = CUBE ? (float)d : (float)d * a.scale[k];
                r2f += fv * fv;
            }
            const bool inr = curok && fits && r2f >= flo && r2f < fhi;
            take(inr, dq, cur, curw);
        }
    }
}

// Values per lane of the per-bin kernel: every slot of a bin (the imaginary
// slots of real states stay zero), at most 128 (two per lane after the fold).
// D = 4 at lmax 6 has 168: its 168 register sums next to the recurrences'
// registers would leave one wave per SIMD (256 VGPRs), and it keeps the
// staging kernel (two waves).
template <int D, int L>
constexpr bool pass_supported() { return 2 * stored_states(D, L) <= 128; }

// Waves per SIMD the compiler is held to.  D = 3 at lmax 4 and 5 would take
// 100 and 108 VGPRs, four waves per SIMD; at 96 they run five (at lmax 5 up
// to four values spill, stored once per launch and reloaded per bin and per
// 64 stencil rows, outside the pair loop): c2 harmonic 95.2 -> 87.1 ms.
// Elsewhere no bound beyond the block size's.
template <int D, int L>
constexpr int pass_waves() { return D == 3 && (L == 4 || L == 5) ? 5 : 1; }

template <int D, int L, bool PER, bool CUBE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(pass_waves<D, L>()))) void k_harmonic_pass(HarmArgs a)
{
    constexpr int SLOTS = 2 * stored_states(D, L);
    constexpr int WAVE_BYTES = kQCap * (D == 4 ? 20 : 16) + kPassSegCap * 8;
    extern __shared__ __align__(16) char smem[];
    const int nb = a.nb;
    const int lane = (int)lane_id();
    const int wave = threadIdx.x >> 6;
    double *e2 = reinterpret_cast<double *>(smem);
    for (int t = threadIdx.x; t <= nb; t += blockDim.x) e2[t] = a.e2[t];
    char *wb = smem + kTableBytes + wave * WAVE_BYTES;
    int4 *q4 = reinterpret_cast<int4 *>(wb);                                   // [kQCap]
    float *qwx = reinterpret_cast<float *>(wb + kQCap * 16);                   // [kQCap] (D = 4 weight)
    uint2 *segs = reinterpret_cast<uint2 *>(wb + kQCap * (D == 4 ? 20 : 16));  // [kPassSegCap]
    __syncthreads();
    const int nacc = nb * SLOTS;

    for (;;) {
        const int row = next_row(a.work, lane);
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
        const float wi = D == 4 ? a.w[ip] : (D == 3 ? __int_as_float((int)ri.w) : __int_as_float((int)ri.z));
        float *Arow = a.A + (size_t)row * nacc;

        for (int b = 0; b < nb; b++) {
            const double elo = e2[b], ehi = e2[b + 1];
            float fs[SLOTS];
#pragma unroll
            for (int v = 0; v < SLOTS; v++) fs[v] = 0.f;
            double acc0 = 0.0, acc1 = 0.0;
            int batches = 0;   // batches since the last fold (wave-uniform)
            int qn = 0;        // queued pairs (wave-uniform)
            auto fold = [&]() __attribute__((always_inline)) {
                double y0, y1;
                fold_lanes<SLOTS>(fs, lane, y0, y1);
                acc0 += y0;
                acc1 += y1;
#pragma unroll
                for (int v = 0; v < SLOTS; v++) fs[v] = 0.f;
                batches = 0;
            };
            // the queued pairs [0, cnt): FP64 r^2 decides the bin, the
            // harmonics of the pairs in it go into the lanes' sums
            auto process = [&](int cnt) __attribute__((always_inline)) {
                NPCF_WAVE_SYNC();
                // every lane reads its queue entry (stale past cnt, masked
                // out by valid below: the harmonics see only valid values)
                const bool live = lane < cnt;
                int dq[D];
                float wk;
                {
                    const int4 e = q4[lane];
                    dq[0] = e.x;
                    dq[1] = e.y;
                    if (D >= 3) dq[2] = e.z;
                    if (D == 4) {
                        dq[3] = e.w;
                        wk = qwx[lane];
                    } else {
                        wk = __int_as_float(D == 3 ? e.w : e.z);
                    }
                }
                // r^2 summed axis by axis without contraction (the definition's
                // arithmetic), the unit vector normalised in FP64 and rounded
                // once to FP32
                double v[D];
                double r2 = 0.0;
#pragma unroll
                for (int k = 0; k < D; k++) {
                    v[k] = mul_rn((double)dq[k], a.scale64[k]);
                    r2 = add_rn(r2, mul_rn(v[k], v[k]));
                }
                const bool valid = live && r2 >= elo && r2 < ehi;
                row_pairs += (unsigned long long)__popcll(ballot(valid));
                const double rs = valid ? r2 : 1.0;
                double rinv = __builtin_amdgcn_rsq(rs);
                rinv = rinv * (1.5 - 0.5 * rs * rinv * rinv);
                float u[D];
#pragma unroll
                for (int k = 0; k < D; k++) u[k] = valid ? (float)(v[k] * rinv) : 0.f;
                harmonics<D, L>(u, valid ? wk : 0.f, [&](int slot, float val) { fs[slot] += val; });
                if (++batches == kPassFoldBatches) fold();
            };
            // the FP32 bounds, in squared lattice units for a cube
            const double fu = CUBE ? 1.0 / (a.scale64[0] * a.scale64[0]) : 1.0;
            scan_shell<D, PER, CUBE>(a, cs, qi, segs, lane, elo * (1.0 - 1e-9), ehi * (1.0 + 1e-9),
                                     (float)(elo * (1.0 - 1e-5) * fu), (float)(ehi * (1.0 + 1e-5) * fu),
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
            fold();
            // this bin's slots of the primary's row of a (FP32)
            if (lane < SLOTS) Arow[b * SLOTS + lane] = (float)acc0;
            if (lane + 64 < SLOTS) Arow[b * SLOTS + lane + 64] = (float)acc1;
        }
        finish_row(a.wrow, row, wi, a.pairs + cat, row_pairs, lane);
    }
}

template <int D, int L>
constexpr int pass_lds_bytes() { return kTableBytes + 4 * (kQCap * (D == 4 ? 20 : 16) + kPassSegCap * 8); }

}  // namespace harm
}  // namespace npcf
