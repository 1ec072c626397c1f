// Harmonic stage of the separable NPCF estimator (eq. NPCF-estimator-discrete,
// the sum defining a^b_[l](y_j); bin integral of eq. alm-bin-def):
//
//   a^b_[l](y_j) = sum_k w_k conj(Y_[l](unit(y_k - y_j))) Theta^b(|y_k - y_j|)
//
// (the 1/v_b factor is applied when the estimator is finalised).
//
// Mapping to gfx950
//  - one wavefront per primary (rows handed out by an atomic counter, so
//    clustered catalogues balance); primaries are visited in cell order;
//  - candidates come from the counting-sorted SoA lattice arrays: for each
//    stencil row of cells the primary's own sphere trims the x-range, so the
//    candidate stream is a few contiguous, coalesced segments;
//  - phase A (lanes over candidates): exact int32 periodic separation,
//    conservative FP32 range test, ballot compaction into an LDS queue;
//  - phase B (lanes over 64 queued pairs): FP64 binning that reproduces the
//    FP64 definition bit for bit on lattice inputs, FP32 unit vector, the
//    harmonics by Gegenbauer recurrences in registers (normalisations folded
//    into the recurrence constants), scatter-add into per-wave FP32 LDS
//    accumulators (R lane-interleaved replicas to spread same-address
//    collisions);
//  - every few batches the FP32 replicas are folded into per-wave FP64 LDS
//    accumulators, which hold the primary's a until it is written out.
#pragma once
#include "npcf_internal.h"

namespace npcf {

namespace harm {

constexpr int kQCap = 128;       // pair queue entries per wave
constexpr int kFlushBatches = 4; // fold FP32 replicas into FP64 every this many batches
constexpr int kMaxBucket = 2048;
constexpr int kTableBytes = (kMaxBins + 1) * 8 + kMaxBucket;

#define NPCF_WAVE_SYNC()                                   \
    do {                                                   \
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                   \
    } while (0)

template <int D>
struct Repl {
    static constexpr int R = (D == 4) ? 2 : 4;
};

__host__ __device__ constexpr int slot_pad(int slots) { return slots | 1; }

template <int D, int L>
__host__ __device__ constexpr int per_wave_bytes_fixed()
{
    return (D + 1) * kQCap * 4;  // queue
}

__host__ __device__ inline int align8(int x) { return (x + 7) & ~7; }

template <int D, int L>
__host__ __device__ inline int per_wave_bytes(int nb)
{
    constexpr int NST = stored_states(D, L);
    constexpr int SP = slot_pad(2 * NST);
    int q = per_wave_bytes_fixed<D, L>();
    int r = Repl<D>::R * nb * SP * 4;
    int d = nb * 2 * NST * 8;
    return align8(q + r) + d;
}

__device__ __forceinline__ unsigned lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ int rank_in_mask(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// ---- harmonics -------------------------------------------------------------
// The emitted value for stored state s is w * conj(Y_s(u)) split into real
// (slot 2s) and imaginary (slot 2s+1) parts; m = 0 (l1 = 0) states have no
// imaginary part and emit only the real slot.

// D = 2: Y_l = e^{i l theta1} / sqrt(2 pi); conj -> (u1 - i u2)^l / sqrt(2 pi).
template <int L, class F>
__device__ __forceinline__ void harm_d2(const float *u, float w, const float *__restrict__ hc, F &&emit)
{
    float pr = w * hc[0], pi = 0.f;
    emit(0, pr);
#pragma unroll
    for (int l = 1; l <= L; l++) {
        float nr = pr * u[0] + pi * u[1];
        float ni = pi * u[0] - pr * u[1];
        pr = nr;
        pi = ni;
        emit(2 * l, pr);
        emit(2 * l + 1, pi);
    }
}

// D = 3: Y_{m,l} = K (u1 + i u2)^m C^{(m+1/2)}_{l-m}(u3).  The normalised
// Gegenbauer values obey c_n = alpha_n u3 c_{n-1} - beta_n c_{n-2}; hc holds,
// for m = 0..L, c_0 followed by (alpha_n, beta_n) for n = 1..L-m.
template <int L, class F>
__device__ __forceinline__ void harm_d3(const float *u, float w, const float *__restrict__ hc, F &&emit)
{
    float pr = w, pi = 0.f;
    int ci = 0;
#pragma unroll
    for (int m = 0; m <= L; m++) {
        if (m > 0) {
            float nr = pr * u[0] + pi * u[1];
            float ni = pi * u[0] - pr * u[1];
            pr = nr;
            pi = ni;
        }
        float c1 = hc[ci++];
        float c2 = 0.f;
        {
            const int s = m * (m + 1) / 2 + m;
            emit(2 * s, c1 * pr);
            if (m > 0) emit(2 * s + 1, c1 * pi);
        }
#pragma unroll
        for (int l = m + 1; l <= L; l++) {
            float al = hc[ci++], be = hc[ci++];
            float c = al * u[2] * c1 - be * c2;
            c2 = c1;
            c1 = c;
            const int s = l * (l + 1) / 2 + m;
            emit(2 * s, c * pr);
            if (m > 0) emit(2 * s + 1, c * pi);
        }
    }
}

// D = 4: Y_{l1 l2 l3} = (u1 + i u2)^{l1} g_{l1}(l2) c_{l2}(l3) with
//   c_{l2}(l3) = N3 C^{(l2+1)}_{l3-l2}(u4)
//   g_{l1}(l2) = (2 pi)^{-1/2} N2 rho^{l2-l1} C^{(l1+1/2)}_{l2-l1}(u3/rho), rho^2 = u1^2+u2^2+u3^2,
// both by three-term recurrences; hc holds the c tables (for l2 = 0..L: c_0,
// (alpha, beta) for n = 1..L-l2), then the g tables (for l1 = 0..L).
template <int L, class F>
__device__ __forceinline__ void harm_d4(const float *u, float w, const float *__restrict__ hc, F &&emit)
{
    constexpr int NT = (L + 1) * (L + 2) / 2;
    float ct[NT];  // ct[tri(l2) + (l3 - l2)]
    float gt[NT];  // gt[tri(l1) + (l2 - l1)]
    const float rho2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    int ci = 0;
    int ti = 0;
#pragma unroll
    for (int l2 = 0; l2 <= L; l2++) {
        float c1 = hc[ci++], c2 = 0.f;
        ct[ti++] = c1;
#pragma unroll
        for (int n = 1; n <= L - l2; n++) {
            float al = hc[ci++], be = hc[ci++];
            float c = al * u[3] * c1 - be * c2;
            c2 = c1;
            c1 = c;
            ct[ti++] = c;
        }
    }
    ti = 0;
#pragma unroll
    for (int l1 = 0; l1 <= L; l1++) {
        float g1 = hc[ci++], g2 = 0.f;
        gt[ti++] = g1;
#pragma unroll
        for (int n = 1; n <= L - l1; n++) {
            float al = hc[ci++], be = hc[ci++];
            float g = al * u[2] * g1 - be * rho2 * g2;
            g2 = g1;
            g1 = g;
            gt[ti++] = g;
        }
    }
    float pr = w, pi = 0.f;
#pragma unroll
    for (int l1 = 0; l1 <= L; l1++) {
        if (l1 > 0) {
            float nr = pr * u[0] + pi * u[1];
            float ni = pi * u[0] - pr * u[1];
            pr = nr;
            pi = ni;
        }
#pragma unroll
        for (int l2 = l1; l2 <= L; l2++) {
            const float g = gt[(l1 * (2 * L + 3 - l1)) / 2 + (l2 - l1)];
#pragma unroll
            for (int l3 = l2; l3 <= L; l3++) {
                const float v = g * ct[(l2 * (2 * L + 3 - l2)) / 2 + (l3 - l2)];
                const int s = l3 * (l3 + 1) * (l3 + 2) / 6 + l2 * (l2 + 1) / 2 + l1;
                emit(2 * s, v * pr);
                if (l1 > 0) emit(2 * s + 1, v * pi);
            }
        }
    }
}

template <int D, int L, class F>
__device__ __forceinline__ void harmonics(const float *u, float w, const float *__restrict__ hc, F &&emit)
{
    if constexpr (D == 2) harm_d2<L>(u, w, hc, emit);
    else if constexpr (D == 3) harm_d3<L>(u, w, hc, emit);
    else harm_d4<L>(u, w, hc, emit);
}

// ---- the kernel ------------------------------------------------------------
template <int D, int L, bool PER>
__global__ __launch_bounds__(256) void k_harmonic(HarmArgs a)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int NST = stored_states(D, L);
    constexpr int SLOTS = 2 * NST;
    constexpr int SP = slot_pad(SLOTS);
    constexpr int R = Repl<D>::R;
    const int nb = a.nb;
    const int lane = (int)lane_id();
    const int wave = threadIdx.x >> 6;

    double *e2 = reinterpret_cast<double *>(smem);
    uint8_t *btab = reinterpret_cast<uint8_t *>(smem + (kMaxBins + 1) * 8);
    for (int t = threadIdx.x; t <= nb; t += blockDim.x) e2[t] = a.e2[t];
    for (int t = threadIdx.x; t < a.nbucket; t += blockDim.x) btab[t] = a.bucket_bin[t];

    char *wb = smem + kTableBytes + wave * per_wave_bytes<D, L>(nb);
    int *qd = reinterpret_cast<int *>(wb);                     // [D][kQCap]
    float *qw = reinterpret_cast<float *>(qd + D * kQCap);     // [kQCap]
    float *accR = qw + kQCap;                                  // [R][nb][SP]
    double *acc64 = reinterpret_cast<double *>(wb + align8((D + 1) * kQCap * 4 + R * nb * SP * 4));  // [nb][SLOTS]
    const int nacc = nb * SLOTS;
    for (int t = lane; t < R * nb * SP; t += kWave) accR[t] = 0.f;
    for (int t = lane; t < nacc; t += kWave) acc64[t] = 0.0;
    __syncthreads();

    const int rep = lane & (R - 1);
    unsigned long long my_pairs = 0;
    const float e2lo_f = a.e2lo_f, e2hi_f = a.e2hi_f;
    const double e2lo = e2[0], e2hi = e2[nb];

    for (;;) {
        int row = 0;
        if (lane == 0) row = (int)atomicAdd(a.work, 1u);
        row = __shfl(row, 0);
        if (row >= a.nrows) break;
        const int ip = a.prim[row];
        uint32_t qi[D];
#pragma unroll
        for (int k = 0; k < D; k++) qi[k] = a.q[k][ip];
        const float wi = a.w[ip];

        int qn = 0;       // queued pairs (wave-uniform)
        int nbatch = 0;

        // --- phase B: harmonics of queued pairs [0, cnt) and scatter-add ----
        auto process = [&](int cnt) {
            NPCF_WAVE_SYNC();
            const bool live = lane < cnt;
            int dq[D];
#pragma unroll
            for (int k = 0; k < D; k++) dq[k] = live ? qd[k * kQCap + lane] : 0;
            const float wk = live ? qw[lane] : 0.f;
            // FP64 squared distance, summed axis by axis without contraction
            double r2 = 0.0;
            float f[D];
#pragma unroll
            for (int k = 0; k < D; k++) {
                double v = __dmul_rn((double)dq[k], a.scale64[k]);
                r2 = __dadd_rn(r2, __dmul_rn(v, v));
                f[k] = (float)dq[k] * a.scale[k];
            }
            bool valid = live && r2 >= e2lo && r2 < e2hi;
            int bin = 0;
            if (valid) {
                float r2f = (float)r2;
                int bk = (int)((r2f - a.bucket_lo) * a.bucket_inv);
                bk = bk < 0 ? 0 : (bk >= a.nbucket ? a.nbucket - 1 : bk);
                bin = btab[bk];
                while (bin + 1 < nb && r2 >= e2[bin + 1]) bin++;
                while (bin > 0 && r2 < e2[bin]) bin--;
            }
            const unsigned long long vm = __ballot(valid);
            my_pairs += (unsigned long long)__popcll(vm);
            float fr2 = 0.f;
#pragma unroll
            for (int k = 0; k < D; k++) fr2 += f[k] * f[k];
            const float rinv = valid ? rsqrtf(fr2) : 0.f;
            float u[D];
#pragma unroll
            for (int k = 0; k < D; k++) u[k] = f[k] * rinv;
            float *base = accR + (rep * nb + bin) * SP;
            if (valid) {
                harmonics<D, L>(u, wk, a.hconst, [&](int slot, float v) {
                    __hip_atomic_fetch_add(base + slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                });
            }
            NPCF_WAVE_SYNC();
        };

        auto flush = [&]() {
            NPCF_WAVE_SYNC();
            for (int t = lane; t < nacc; t += kWave) {
                const int b = t / SLOTS;
                const int s = t - b * SLOTS;
                double sum = 0.0;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    float *p = accR + (r * nb + b) * SP + s;
                    sum += (double)*p;
                    *p = 0.f;
                }
                acc64[t] += sum;
            }
            NPCF_WAVE_SYNC();
        };

        // --- stencil rows around the primary --------------------------------
        int lo[D], hi[D];
        bool full[D];
#pragma unroll
        for (int k = 0; k < D; k++) {
            const double qk = (double)qi[k];
            long long l0 = (long long)floor((qk - a.rmax_lat[k] - 4.0) / a.cell_len[k]);
            long long h0 = (long long)floor((qk + a.rmax_lat[k] + 4.0) / a.cell_len[k]);
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
            hi[k] = (int)h0;
        }
        // physical r_max^2 (for the row trimming)
        const double rmax2 = e2hi * (1.0 + 1e-9);
        int nrow = 1;
#pragma unroll
        for (int k = 1; k < D; k++) nrow *= (hi[k] - lo[k] + 1);

        for (int rix = 0; rix < nrow; rix++) {
            // decode the row's unwrapped cell coordinates on axes 1..D-1
            int cc[D];
            int t = rix;
            double d2 = 0.0;
            long long lin = 0, mul = a.ncs[0];
#pragma unroll
            for (int k = 1; k < D; k++) {
                const int span = hi[k] - lo[k] + 1;
                cc[k] = lo[k] + t % span;
                t /= span;
                double dist = 0.0;
                if (!full[k]) {
                    const double slo = (double)cc[k] * a.cell_len[k];
                    const double shi = slo + a.cell_len[k];
                    const double qk = (double)qi[k];
                    if (qk < slo) dist = slo - qk;
                    else if (qk >= shi) dist = qk - shi;
                    dist = dist > 4.0 ? dist - 4.0 : 0.0;
                }
                const double dp = dist * a.scale64[k];
                d2 += dp * dp;
                int cw = cc[k] % a.ncs[k];
                if (cw < 0) cw += a.ncs[k];
                lin += (long long)cw * mul;
                mul *= a.ncs[k];
            }
            if (d2 >= rmax2) continue;
            // x-extent of the sphere on this row
            int xa, xb;
            if (full[0]) {
                xa = 0;
                xb = a.ncs[0] - 1;
            } else {
                const double h = sqrt(rmax2 - d2) / a.scale64[0] + 4.0;
                const double qx = (double)qi[0];
                long long x0 = (long long)floor((qx - h) / a.cell_len[0]);
                long long x1 = (long long)floor((qx + h) / a.cell_len[0]);
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
            // at most two contiguous runs after periodic wrap
            int ra[2], rb[2], nrun = 0;
            if (xa < 0) {
                ra[0] = xa + a.ncs[0]; rb[0] = a.ncs[0] - 1;
                ra[1] = 0; rb[1] = xb;
                nrun = 2;
            } else if (xb >= a.ncs[0]) {
                ra[0] = xa; rb[0] = a.ncs[0] - 1;
                ra[1] = 0; rb[1] = xb - a.ncs[0];
                nrun = 2;
            } else {
                ra[0] = xa; rb[0] = xb;
                nrun = 1;
            }
            for (int run = 0; run < nrun; run++) {
                const uint32_t s0 = a.cell_start[lin + ra[run]];
                const uint32_t s1 = a.cell_start[lin + rb[run] + 1];
                for (uint32_t b0 = s0; b0 < s1; b0 += kWave) {
                    const uint32_t k = b0 + (uint32_t)lane;
                    bool inr = false;
                    int dq[D];
                    float wk = 0.f;
                    if (k < s1) {
                        float r2f = 0.f;
                        bool fits = true;
#pragma unroll
                        for (int kk = 0; kk < D; kk++) {
                            const uint32_t qk = a.q[kk][k];
                            int d;
                            if (PER) {
                                d = (int)(qk - qi[kk]);  // two's-complement wrap = minimum image
                            } else {
                                const long long dl = (long long)qk - (long long)qi[kk];
                                d = (int)dl;
                                fits = fits && (long long)d == dl;
                            }
                            dq[kk] = d;
                            const float fv = (float)d * a.scale[kk];
                            r2f += fv * fv;
                        }
                        wk = a.w[k];
                        inr = fits && r2f >= e2lo_f && r2f < e2hi_f;
                    }
                    const unsigned long long m = __ballot(inr);
                    if (inr) {
                        const int slot = qn + rank_in_mask(m);
#pragma unroll
                        for (int kk = 0; kk < D; kk++) qd[kk * kQCap + slot] = dq[kk];
                        qw[slot] = wk;
                    }
                    qn += __popcll(m);
                    if (qn >= kWave) {
                        process(kWave);
                        // move the overflow [64, qn) to the front
                        const int rest = qn - kWave;
                        if (lane < rest) {
                            int tmp[D];
#pragma unroll
                            for (int kk = 0; kk < D; kk++) tmp[kk] = qd[kk * kQCap + kWave + lane];
                            const float tw = qw[kWave + lane];
#pragma unroll
                            for (int kk = 0; kk < D; kk++) qd[kk * kQCap + lane] = tmp[kk];
                            qw[lane] = tw;
                        }
                        qn = rest;
                        if (++nbatch % kFlushBatches == 0) flush();
                        NPCF_WAVE_SYNC();
                    }
                }
            }
        }
        if (qn > 0) process(qn);
        flush();
        // write the primary's a (FP32) and weight; clear the FP64 accumulators
        float *Arow = a.A + (size_t)row * nacc;
        for (int t = lane; t < nacc; t += kWave) {
            Arow[t] = (float)acc64[t];
            acc64[t] = 0.0;
        }
        if (lane == 0) a.wrow[row] = wi;
        NPCF_WAVE_SYNC();
    }
    if (lane == 0 && my_pairs) atomicAdd(a.pairs, my_pairs);
}

template <int D, int L>
hipError_t launch_dl(const HarmArgs &a, int grid, hipStream_t s)
{
    const int lds = kTableBytes + 4 * per_wave_bytes<D, L>(a.nb);
    if (a.periodic) {
        hipFuncSetAttribute((const void *)k_harmonic<D, L, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        hipLaunchKernelGGL((k_harmonic<D, L, true>), dim3(grid), dim3(256), lds, s, a);
    } else {
        hipFuncSetAttribute((const void *)k_harmonic<D, L, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        hipLaunchKernelGGL((k_harmonic<D, L, false>), dim3(grid), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

template <int D, int L>
int lds_bytes(int nb) { return kTableBytes + 4 * per_wave_bytes<D, L>(nb); }

}  // namespace harm
}  // namespace npcf
