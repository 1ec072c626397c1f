// Harmonic stage for points on the unit 2-sphere (section "Cosmic Microwave
// Background"): D = 2 harmonics of the direction of each secondary in a
// tangent frame at the primary, binned in great-circle angle,
//   a^b_l(p) = sum_q w_q conj(Y_l(phi_pq)) Theta^b(theta_pq)
// (1/v_b at finalize, as on the flat path), for every secondary q: the bins of
// the paper's CMB test reach 120 degrees, so a cell list would prune little.
//  - theta: e_b <= theta < e_{b+1}  <=>  cos e_{b+1} < p.q <= cos e_b, on an
//    FP64 dot product evaluated without contraction (the comparison matches a
//    plain FP64 evaluation bit for bit);
//  - frame: e1 = unit(z x p) (unit(x x p) when |p_z| > 0.9), e2 = p x e1;
//    (cos phi, sin phi) = (q.e1, q.e2) / |(q.e1, q.e2)|.
// A block is 8 waves, one primary each; secondaries come through LDS in FP32
// tiles (the points are packed to FP32 once per launch).  The FP32 cosine
// decides the bin (through a bucket table where no edge is near, else against
// the edge cosines) unless it lies within 1e-6 of an edge (its error is below
// 4e-7), where the FP64 dot product decides, so the decisions equal the FP64
// ones.  In-range pairs are queued by catalogue index; the harmonics take the
// tangent components from the FP64 positions in an FP64 frame, normalised in
// FP64 and rounded once to FP32.  As many bins as fit about 50 registers
// are taken per pass (more passes rescan the points, but fewer registers let
// four waves share a SIMD and each queued pair feeds fewer masked sums); each
// lane sums harmonics in FP32 (a 0/1 mask per bin) and every few tiles the
// wave reduces its lanes into FP64 values held one or two per lane.
#include "npcf_internal.h"
#include "npcf_harmonics.h"

namespace npcf {

namespace {

constexpr int kSphTile = 512;
constexpr int kSphWaves = 8;
constexpr int kSphFold = 4;         // tiles between folds of the lanes' FP32 sums
constexpr float kSphGuard = 1e-6f;  // FP32 cosines this close to an edge are decided in FP64

// bins per pass: as many as keep the lanes' FP32 sums within kSphRegBudget registers
constexpr int kSphRegBudget = 50;
__host__ __device__ constexpr int sph_group(int L)
{
    return (kSphRegBudget / (2 * (L + 1))) < 16 ? (kSphRegBudget / (2 * (L + 1))) : 16;
}

__device__ __forceinline__ double dot3_rn(double ax, double ay, double az, double bx, double by, double bz)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(ax, bx), __dmul_rn(ay, by)), __dmul_rn(az, bz));
}

#define NPCF_SPH_WAVE_SYNC()                                   \
    do {                                                       \
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                       \
    } while (0)

// DPP-permuted copy of x added to x: each lane adds the value of its partner
// (row_ror:8 pairs lanes l, l ^ 8 within a row of 16; row_half_mirror pairs
// l, l ^ 7 within 8 lanes; the quad permutations pair l, l ^ 2 and l, l ^ 1)
template <int CTRL>
__device__ __forceinline__ float add_partner(float x)
{
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// One butterfly step below the swaps: values v[q] and v[q + H] (H = 2^k, q
// with bit k clear) pair up; the lane whose bit k is set keeps the sum of
// the second over itself and its partner, the other the sum of the first.
template <int N, int CTRL>
__device__ __forceinline__ void fold_step(const float *v, float *out, bool bit)
{
    constexpr int H = N / 4;   // index bit of this step: the values are (i6, bits below) with N/2 of them
#pragma unroll
    for (int q = 0; q < N / 2; q++) {
        const int lo = (q & (H - 1)) | ((q & ~(H - 1)) << 1);
        const float u0 = add_partner<CTRL>(v[lo]), u1 = add_partner<CTRL>(v[lo + H]);
        out[q] = bit ? u1 : u0;
    }
}

// Sum of each of the NG (<= 128) values x[j] over the 64 lanes of the wave,
// scattered: lane l receives the totals of values l (y0) and l + 64 (y1; zero
// past NG).  A butterfly that halves the values at each step: lane bit 5
// through v_permlane32_swap, bit 4 through v_permlane16_swap, bits 3 to 0
// through DPP.  At each step the lane keeps the values whose index bit
// matches its lane bit, so after six steps lane l holds value l and l + 64.
template <int NG>
__device__ __forceinline__ void fold_lanes(const float *x, int lane, float &y0, float &y1)
{
    static_assert(NG <= 128, "at most two values per lane");
    float z[64];
#pragma unroll
    for (int q = 0; q < 64; q++) {
        const int i = (q & 31) | ((q & 32) << 1);   // value index with bit 5 clear
        const float a = i < NG ? x[i] : 0.f, b = i + 32 < NG ? x[i + 32] : 0.f;
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
        z[q] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float w[32];
#pragma unroll
    for (int q = 0; q < 32; q++) {
        const int i = (q & 15) | ((q & 16) << 1);   // index in z with bit 4 clear
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(z[i]), __float_as_uint(z[i + 16]), false, false);
        w[q] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float x3[16], x2[8], x1[4], x0[2];
    fold_step<32, 0x128>(w, x3, (lane & 8) != 0);    // row_ror:8
    fold_step<16, 0x141>(x3, x2, (lane & 4) != 0);   // row_half_mirror
    fold_step<8, 0x4E>(x2, x1, (lane & 2) != 0);     // quad_perm [2,3,0,1]
    fold_step<4, 0xB1>(x1, x0, (lane & 1) != 0);     // quad_perm [1,0,3,2]
    y0 = x0[0];
    y1 = x0[1];
}

template <int L>
__global__ __launch_bounds__(kSphWaves * 64) void k_sphere(SphereArgs a)
{
    __shared__ float4 tile[kSphTile];
    // per wave: in-range pairs waiting for the harmonics (catalogue index,
    // weight, bin)
    __shared__ int qidx[kSphWaves][128];
    __shared__ float qw[kSphWaves][128];
    __shared__ int qbin[kSphWaves][128];
    // the pass's edge cosines (FP32) and a bucket table over its cosine range.
    // Entry k is the bin of every cosine in bucket k when no edge, widened by
    // twice the guard, lies in buckets k - 1 .. k + 1 (the FP32 bucket index
    // of a cosine is off by at most one); such a cosine is then more than the
    // guard from every edge and the entry decides.  Otherwise the entry is
    // 0x80 | the bin at the bucket's upper end, a guess that the search
    // against the edge cosines corrects, followed by the guard test.
    constexpr int kBuckets = 8192;
    __shared__ float sce[kMaxBins + 1];
    __shared__ unsigned char sbk[kBuckets];
    constexpr int NV = 2 * (L + 1);   // real slots per bin (slot 1, the l = 0 imaginary part, stays 0)
    constexpr int G = sph_group(L);
    constexpr int NG = G * NV;        // values per pass, <= 50 (L <= 5): lane j keeps value j in FP64
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * kSphWaves + wave;
    const bool active = row < a.rows;
    const int64_t pi = a.p0 + (active ? row : 0);
    const double px = a.pos[pi], py = a.pos[a.n + pi], pz = a.pos[2 * a.n + pi];
    // tangent frame at p
    double ax = 0.0, ay = 0.0, az = 1.0;
    if (fabs(pz) > 0.9) {
        ax = 1.0;
        az = 0.0;
    }
    double e1x = ay * pz - az * py, e1y = az * px - ax * pz, e1z = ax * py - ay * px;
    const double inn = 1.0 / sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x *= inn;
    e1y *= inn;
    e1z *= inn;
    const double e2x = py * e1z - pz * e1y, e2y = pz * e1x - px * e1z, e2z = px * e1y - py * e1x;
    const float pxf = (float)px, pyf = (float)py, pzf = (float)pz;

    unsigned long long cnt_pairs = 0;   // wave-uniform
    for (int b0 = 0; b0 < a.nb; b0 += G) {
        const int ng = min(G, a.nb - b0);
        const double chi = a.cedge[b0], clo = a.cedge[b0 + ng];
        const float chif = (float)chi, clof = (float)clo;
        double acc0 = 0.0, acc1 = 0.0;   // FP64 sums of values lane and lane + 64
        float fs[G][NV];
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
            for (int v = 0; v < NV; v++) fs[g][v] = 0.f;
        const float bw = (chif - clof) / kBuckets, ibw = bw > 0.f ? 1.f / bw : 0.f;
        __syncthreads();
        for (int g = threadIdx.x; g <= ng; g += blockDim.x) sce[g] = (float)a.cedge[b0 + g];
        for (int k = threadIdx.x; k < kBuckets; k += blockDim.x) {
            const double lo = (double)clof + (k - 1) * (double)bw - 2.0 * kSphGuard;
            const double hi = (double)clof + (k + 2) * (double)bw + 2.0 * kSphGuard;
            const double mid = (double)clof + (k + 0.5) * (double)bw;
            const float ck = clof + (k + 1) * bw;   // upper end of bucket k
            bool edge = false;
            int b = 0, bg = 0;
            for (int g = 0; g <= ng; g++) {
                const double e = a.cedge[b0 + g];
                edge = edge || (e >= lo && e <= hi);
                if (g >= 1 && g < ng) {
                    b += mid <= e;
                    bg += ck <= (float)e;
                }
            }
            sbk[k] = (unsigned char)(edge ? (0x80 | bg) : b);
        }
        __syncthreads();
        int tiles = 0;
        int qn = 0;   // queued pairs (wave-uniform)
        // harmonics of the first cnt queued pairs, one per lane, into the bin sums
        auto process = [&](int cnt) {
            const bool live = lane < cnt;
            const int k = live ? qidx[wave][lane] : 0;
            const float wq = live ? qw[wave][lane] : 0.f;
            const int bl = live ? qbin[wave][lane] : 0;
            // tangent components from the FP64 positions and frame, normalised
            // in FP64 and rounded once to FP32 (each rounding of the direction
            // enters the l-th harmonic about l times)
            double qx = 0.0, qy = 0.0, qz = 0.0;
            if (live) {
                qx = a.pos[k];
                qy = a.pos[a.n + k];
                qz = a.pos[2 * a.n + k];
            }
            const double t1 = qx * e1x + qy * e1y + qz * e1z;
            const double t2 = qx * e2x + qy * e2y + qz * e2z;
            const double tn2 = t1 * t1 + t2 * t2;
            const bool ok = live && tn2 > 0.0;
            const double ts = ok ? tn2 : 1.0;
            double itn = __builtin_amdgcn_rsq(ts);
            itn = itn * (1.5 - 0.5 * ts * itn * itn);
            const float u[2] = {ok ? (float)(t1 * itn) : 0.f, ok ? (float)(t2 * itn) : 0.f};
            cnt_pairs += __popcll(__builtin_amdgcn_ballot_w64(ok));
            float hv[NV];
            hv[1] = 0.f;   // l = 0 is real
            harm::harmonics<2, L>(u, ok ? wq : 0.f, [&](int slot, float v) { hv[slot] = v; });
#pragma unroll
            for (int g = 0; g < G; g++) {
                const float m = (ok && g == bl) ? 1.f : 0.f;
#pragma unroll
                for (int v = 0; v < NV; v++) fs[g][v] = fmaf(m, hv[v], fs[g][v]);
            }
        };
        for (int64_t t0 = 0; t0 < a.n; t0 += kSphTile) {
            const int cnt_t = (int)(a.n - t0 < kSphTile ? a.n - t0 : kSphTile);
            __syncthreads();
            for (int i = threadIdx.x; i < cnt_t; i += blockDim.x) tile[i] = a.pf[t0 + i];
            __syncthreads();
            if (active) {
                // scan: bin of every point; in-range pairs go to the wave's queue
                for (int i0 = 0; i0 < cnt_t; i0 += 64) {
                    const int i = i0 + lane;
                    bool valid = false;
                    int bl = 0;
                    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (i < cnt_t) {
                        q = tile[i];
                        const float c32 = pxf * q.x + pyf * q.y + pzf * q.z;
                        // range prefilter on the same FP32 differences as the guard
                        // test below, so that a cosine admitted beyond an outer edge
                        // is always within the guard of it and decided in FP64
                        // (chif + guard rounded in FP32 would admit cosines up to
                        // one rounding beyond the guard)
                        if (c32 - chif <= kSphGuard && clof - c32 < kSphGuard) {
                            // bin from the bucket table; near an edge, from the FP32
                            // cosine against the edges, and within the guard band of
                            // an edge from the FP64 dot product
                            int kb = (int)((c32 - clof) * ibw);
                            kb = kb < 0 ? 0 : (kb >= kBuckets ? kBuckets - 1 : kb);
                            const int ent = sbk[kb];
                            bl = ent & 0x7F;
                            valid = true;
                            bool near = false;
                            if (ent & 0x80) {
                                while (bl + 1 < ng && c32 <= sce[bl + 1]) bl++;
                                while (bl > 0 && c32 > sce[bl]) bl--;
                                near = fabsf(c32 - sce[bl]) <= kSphGuard || fabsf(c32 - sce[bl + 1]) <= kSphGuard;
                            }
                            if (near) {
                                const int64_t k = t0 + i;
                                const double c = dot3_rn(px, py, pz, a.pos[k], a.pos[a.n + k], a.pos[2 * a.n + k]);
                                valid = c <= chi && c > clo;
                                bl = 0;
                                while (bl + 1 < ng && c <= a.cedge[b0 + bl + 1]) bl++;
                            }
                        }
                    }
                    const unsigned long long vm = __builtin_amdgcn_ballot_w64(valid);
                    const int slot = qn + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(vm >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((unsigned)vm, 0u));
                    if (valid) {
                        qidx[wave][slot] = (int)(t0 + i);
                        qw[wave][slot] = q.w;
                        qbin[wave][slot] = bl;
                    }
                    qn += __popcll(vm);
                    if (qn >= 64) {
                        NPCF_SPH_WAVE_SYNC();
                        process(64);
                        // move the rest (< 64) to the front
                        const int rest = qn - 64;
                        int mi = 0, mb = 0;
                        float mw = 0.f;
                        if (lane < rest) {
                            mi = qidx[wave][64 + lane];
                            mw = qw[wave][64 + lane];
                            mb = qbin[wave][64 + lane];
                        }
                        NPCF_SPH_WAVE_SYNC();
                        if (lane < rest) {
                            qidx[wave][lane] = mi;
                            qw[wave][lane] = mw;
                            qbin[wave][lane] = mb;
                        }
                        qn = rest;
                    }
                }
            }
            // every kSphFold tiles and at the end: lanes' FP32 sums into the FP64 values
            const bool last = t0 + kSphTile >= a.n;
            if (last && active && qn > 0) {
                NPCF_SPH_WAVE_SYNC();
                process(qn);
                qn = 0;
            }
            if (++tiles == kSphFold || last) {
                tiles = 0;
                float y0, y1;
                fold_lanes<NG>(&fs[0][0], lane, y0, y1);
                acc0 += (double)y0;
                acc1 += (double)y1;
#pragma unroll
                for (int g = 0; g < G; g++)
#pragma unroll
                    for (int v = 0; v < NV; v++) fs[g][v] = 0.f;
            }
        }
        if (active) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int j = lane + 64 * h;
                if (j < NG) {
                    const int g = j / NV, v = j - g * NV;
                    if (g < ng) a.A[((int64_t)row * a.nb + b0 + g) * NV + v] = (float)(h ? acc1 : acc0);
                }
            }
        }
    }
    if (active && lane == 0) {
        atomicAdd(a.pairs, cnt_pairs);
        a.wrow[row] = (float)a.w[pi];
    }
}

// the points in FP32 (x, y, z, w), once per launch: every block streams
// them all in every pass
__global__ __launch_bounds__(256) void k_sphere_pack(const double *pos, const double *w, int64_t n, float4 *pf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pf[i] = make_float4((float)pos[i], (float)pos[n + i], (float)pos[2 * n + i], (float)w[i]);
}

template <int L>
hipError_t launch_l(const SphereArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_sphere_pack, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a.pos, a.w, a.n, a.pf);
    const int blocks = (a.rows + kSphWaves - 1) / kSphWaves;
    hipLaunchKernelGGL(k_sphere<L>, dim3((unsigned)blocks), dim3(kSphWaves * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sphere(int L, const SphereArgs &a, hipStream_t s)
{
    switch (L) {
    case 0: return launch_l<0>(a, s);
    case 1: return launch_l<1>(a, s);
    case 2: return launch_l<2>(a, s);
    case 3: return launch_l<3>(a, s);
    case 4: return launch_l<4>(a, s);
    case 5: return launch_l<5>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace npcf
