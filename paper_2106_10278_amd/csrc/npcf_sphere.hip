// Harmonic stage for points of a constant-curvature space (section
// "Constant-Curvature Metric", eq. metric): K = +1, the unit D-sphere
// (chi(r) = sin r; D = 2 is the sky of section "Cosmic Microwave Background",
// D = 3 the unit 3-sphere), and K = -1, hyperbolic space H^D (chi(r) =
// sinh r) on the hyperboloid x0^2 - x1^2 - .. - xD^2 = 1 of R^{D,1}.  The
// radial coordinate of a pair is the geodesic distance theta_pq, the
// direction that of q in an orthonormal tangent frame at p, and
//   a^b_[l](p) = sum_q w_q conj(Y_[l](u_pq)) Theta^b(theta_pq)
// (1/v_b at finalize, as on the flat path), for every secondary q: the bins of
// the paper's CMB test reach 120 degrees, so a cell list would prune little.
//  - theta: the kernel's "cosine" c is p.q on the sphere and -<p, q> =
//    -p0 q0 + p1 q1 + .. in H^D (both fall as theta grows), and
//    e_b <= theta < e_{b+1}  <=>  ce_{b+1} < c <= ce_b with ce_b = cos e_b
//    or -cosh e_b, on an FP64 product evaluated left to right without
//    contraction (negation is exact and rounding symmetric, so -<p, q>
//    rounds to minus the oracle's <p, q> and the comparison matches a plain
//    FP64 evaluation bit for bit);
//  - frame, D = 2: e1 = unit(z x p) (unit(x x p) when |p_z| > 0.9), e2 = p x e1;
//    D = 3, p = a + b i + c j + d k a unit quaternion: e1, e2, e3 = p i, p j,
//    p k, i.e. (-b, a, d, -c), (-c, -d, a, b), (-d, c, -b, a), orthonormal,
//    orthogonal to p and positively oriented everywhere;
//    u = (q.e1, .., q.eD) / |(q.e1, .., q.eD)|;
//  - frame in H^D: the Lorentz boost taking the origin to p applied to the
//    coordinate axes, e_j(p) = (p_j, unit_j + p_j (p1..pD) / (1 + p0)), and
//    u_j = -<q, e_j(p)>, i.e. the Euclidean product of q with e_j(p) whose
//    time component is negated; the self pair is excluded by index (<p, p>
//    rounds with an error that grows as cosh^2 r).
// A block is 8 waves, one primary each; secondaries come through LDS in FP32
// tiles (the points are packed to FP32 once per launch).  The FP32 cosine
// decides the bin (through a bucket table where no edge is near, else against
// the edge cosines) unless it lies within a guard band of an edge: 1e-6 on the
// sphere (the FP32 error is below (D + 3) 2^-24 < 4e-7 for unit vectors),
// 1.5 x 2 (D + 3) 2^-24 x0max^2 in H^D (the terms sum to at most 2 p0 q0),
// where the FP64 product decides, so the decisions
// equal the FP64 ones.  In-range pairs are queued by catalogue index; the
// harmonics take the tangent components from the FP64 positions in an FP64
// frame, normalised in FP64 and rounded once to FP32.  As many bins as fit a
// register budget are taken per pass (more passes rescan the points, but
// fewer registers let more waves share a SIMD and each queued pair feeds
// fewer masked sums); each lane sums harmonics in FP32 (a 0/1 mask per bin)
// and every few tiles the wave reduces its lanes into FP64 values held one or
// two per lane.
#include "npcf_internal.h"
#include "npcf_harmonics.h"

namespace npcf {

namespace {

constexpr int kSphTile = 512;
constexpr int kSphWaves = 8;
constexpr int kSphFold = 4;         // tiles between folds of the lanes' FP32 sums
constexpr float kSphGuard = 1e-6f;  // FP32 cosines this close to an edge are decided in FP64 (at least)

// real slots per bin: 2 per stored state (the imaginary slots of real states stay 0)
__host__ __device__ constexpr int sph_slots(int D, int L) { return D == 2 ? 2 * (L + 1) : (L + 1) * (L + 2); }

// bins per pass: as many as keep the lanes' FP32 sums within the register
// budget (50 on S^2; 128 on S^3, whose 42 slots per bin at lmax 5 would
// otherwise take one bin per pass: three bins per pass there ran faster at
// two waves per SIMD than one or two bins at three or four), at least 1, at
// most 16, and at most 128 values in all (two per lane after the fold)
__host__ __device__ constexpr int sph_group(int D, int L)
{
    const int budget = D == 2 ? 50 : 128;
    const int g = budget / sph_slots(D, L);
    const int g1 = g < 1 ? 1 : (g > 16 ? 16 : g);
    return g1 * sph_slots(D, L) <= 128 ? g1 : 128 / sph_slots(D, L);
}

// p.q in FP64, left to right with every product and sum rounded (no contraction)
template <int D>
__device__ __forceinline__ double dot_rn(const double (&p)[D + 1], const double *pos, int64_t n, int64_t k)
{
    double c = __dmul_rn(p[0], pos[k]);
#pragma unroll
    for (int x = 1; x <= D; x++) c = __dadd_rn(c, __dmul_rn(p[x], pos[x * n + k]));
    return c;
}

// Orthonormal tangent frame at p (rows e[0..D-1]), see the header; in H^D
// the rows carry their time component negated, so that a component of q is
// the Euclidean product q . e[j].
template <int D, int K>
__device__ __forceinline__ void tangent_frame(const double (&p)[D + 1], double (&e)[D][D + 1])
{
    if constexpr (K < 0) {
        const double s = 1.0 / (1.0 + p[0]);
#pragma unroll
        for (int j = 1; j <= D; j++) {
            e[j - 1][0] = -p[j];
#pragma unroll
            for (int x = 1; x <= D; x++) e[j - 1][x] = (x == j ? 1.0 : 0.0) + p[j] * p[x] * s;
        }
    } else if constexpr (D == 2) {
        double ax = 0.0, ay = 0.0, az = 1.0;
        if (fabs(p[2]) > 0.9) {
            ax = 1.0;
            az = 0.0;
        }
        double e1x = ay * p[2] - az * p[1], e1y = az * p[0] - ax * p[2], e1z = ax * p[1] - ay * p[0];
        const double inn = 1.0 / sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
        e1x *= inn;
        e1y *= inn;
        e1z *= inn;
        e[0][0] = e1x;
        e[0][1] = e1y;
        e[0][2] = e1z;
        e[1][0] = p[1] * e1z - p[2] * e1y;
        e[1][1] = p[2] * e1x - p[0] * e1z;
        e[1][2] = p[0] * e1y - p[1] * e1x;
    } else {
        // right products of p = (a, b, c, d) with the quaternion units i, j, k
        const double qa = p[0], qb = p[1], qc = p[2], qd = p[3];
        e[0][0] = -qb; e[0][1] = qa;  e[0][2] = qd;  e[0][3] = -qc;
        e[1][0] = -qc; e[1][1] = -qd; e[1][2] = qa;  e[1][3] = qb;
        e[2][0] = -qd; e[2][1] = qc;  e[2][2] = -qb; e[2][3] = qa;
    }
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

template <int D, int L, int K>
__global__ __launch_bounds__(kSphWaves * 64) void k_sphere(SphereArgs a)
{
    __shared__ float4 tile[kSphTile];
    // per wave: in-range pairs waiting for the harmonics (catalogue index,
    // weight (S^2; the FP64 weight is read at the harmonics on S^3), bin)
    __shared__ int qidx[kSphWaves][128];
    __shared__ float qw[kSphWaves][D == 2 ? 128 : 1];
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
    constexpr int NV = sph_slots(D, L);
    constexpr int G = sph_group(D, L);
    constexpr int NG = G * NV;        // values per pass, <= 128: lane j keeps values j and j + 64 in FP64
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * kSphWaves + wave;
    const bool active = row < a.rows;
    const int64_t pi = a.p0 + (active ? row : 0);
    double p[D + 1];
#pragma unroll
    for (int x = 0; x <= D; x++) p[x] = a.pos[x * a.n + pi];
    double e[D][D + 1];
    tangent_frame<D, K>(p, e);
    // the "cosine" c = pc . q: p itself on the sphere, (-p0, p1, .., pD) in H^D
    double pc[D + 1];
#pragma unroll
    for (int x = 0; x <= D; x++) pc[x] = (K < 0 && x == 0) ? -p[0] : p[x];
    float pf32[4] = {(float)pc[0], (float)pc[1], (float)pc[2], D == 3 ? (float)pc[D] : 0.f};
    // guard band of the FP32 cosine (see the header)
    float guard = kSphGuard;
    if constexpr (K < 0) {
        const float xm = __uint_as_float(*a.x0max);
        guard = fmaxf(kSphGuard, 1.5f * 2.f * (D + 3) * 5.9604645e-8f * xm * xm);
    }

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
            const double lo = (double)clof + (k - 1) * (double)bw - 2.0 * guard;
            const double hi = (double)clof + (k + 2) * (double)bw + 2.0 * guard;
            const double mid = (double)clof + (k + 0.5) * (double)bw;
            const float ck = clof + (k + 1) * bw;   // upper end of bucket k
            bool edge = false;
            int b = 0, bg = 0;
            for (int g = 0; g <= ng; g++) {
                const double ec = a.cedge[b0 + g];
                edge = edge || (ec >= lo && ec <= hi);
                if (g >= 1 && g < ng) {
                    b += mid <= ec;
                    bg += ck <= (float)ec;
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
            const int bl = live ? qbin[wave][lane] : 0;
            // tangent components from the FP64 positions and frame, normalised
            // in FP64 and rounded once to FP32 (each rounding of the direction
            // enters the l-th harmonic about l times)
            double q[D + 1];
#pragma unroll
            for (int x = 0; x <= D; x++) q[x] = live ? a.pos[x * a.n + k] : 0.0;
            float wq = 0.f;
            if constexpr (D == 2) wq = live ? qw[wave][lane] : 0.f;
            else wq = live ? (float)a.w[k] : 0.f;
            double t[D];
            double tn2 = 0.0;
#pragma unroll
            for (int c = 0; c < D; c++) {
                double tc = q[0] * e[c][0];
#pragma unroll
                for (int x = 1; x <= D; x++) tc += q[x] * e[c][x];
                t[c] = tc;
                tn2 += tc * tc;
            }
            const bool ok = live && tn2 > 0.0;
            const double ts = ok ? tn2 : 1.0;
            double itn = __builtin_amdgcn_rsq(ts);
            itn = itn * (1.5 - 0.5 * ts * itn * itn);
            float u[D];
#pragma unroll
            for (int c = 0; c < D; c++) u[c] = ok ? (float)(t[c] * itn) : 0.f;
            cnt_pairs += __popcll(__builtin_amdgcn_ballot_w64(ok));
            // every emitted value straight into the masked bin sums (slots never
            // emitted, the imaginary parts of real states, keep their zeros)
            float m[G];
#pragma unroll
            for (int g = 0; g < G; g++) m[g] = (ok && g == bl) ? 1.f : 0.f;
            harm::harmonics<D, L>(u, ok ? wq : 0.f, [&](int slot, float v) {
#pragma unroll
                for (int g = 0; g < G; g++) fs[g][slot] = fmaf(m[g], v, fs[g][slot]);
            });
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
                        float c32 = pf32[0] * q.x + pf32[1] * q.y + pf32[2] * q.z;
                        if constexpr (D == 3) c32 += pf32[3] * q.w;
                        // range prefilter on the same FP32 differences as the guard
                        // test below, so that a cosine admitted beyond an outer edge
                        // is always within the guard of it and decided in FP64
                        // (chif + guard rounded in FP32 would admit cosines up to
                        // one rounding beyond the guard)
                        if (c32 - chif <= guard && clof - c32 < guard) {
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
                                near = fabsf(c32 - sce[bl]) <= guard || fabsf(c32 - sce[bl + 1]) <= guard;
                            }
                            if (near) {
                                const double c = dot_rn<D>(pc, a.pos, a.n, t0 + i);
                                valid = c <= chi && c > clo;
                                bl = 0;
                                while (bl + 1 < ng && c <= a.cedge[b0 + bl + 1]) bl++;
                            }
                        }
                    }
                    if constexpr (K < 0) valid = valid && (t0 + i != pi);   // the self pair, by index
                    const unsigned long long vm = __builtin_amdgcn_ballot_w64(valid);
                    const int slot = qn + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(vm >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((unsigned)vm, 0u));
                    if (valid) {
                        qidx[wave][slot] = (int)(t0 + i);
                        if constexpr (D == 2) qw[wave][slot] = q.w;
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
                            if constexpr (D == 2) mw = qw[wave][64 + lane];
                            mb = qbin[wave][64 + lane];
                        }
                        NPCF_SPH_WAVE_SYNC();
                        if (lane < rest) {
                            qidx[wave][lane] = mi;
                            if constexpr (D == 2) qw[wave][lane] = mw;
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

// the points in FP32, once per launch: every block streams them all in every
// pass.  S^2 and H^2: (x0, x1, x2, w); S^3 and H^3: the four coordinates.  In
// H^D also the largest x0 of the catalogue (as bits of a positive float,
// whose order is the integers'), for the guard band.
template <int D, int K>
__global__ __launch_bounds__(256) void k_sphere_pack(const double *pos, const double *w, int64_t n, float4 *pf,
                                                     unsigned *x0max)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        pf[i] = make_float4((float)pos[i], (float)pos[n + i], (float)pos[2 * n + i],
                            D == 2 ? (float)w[i] : (float)pos[3 * n + i]);
        if constexpr (K < 0) {
            // rounded up, so that the guard is never below the true one
            const float x0 = __double2float_ru(pos[i]);
            atomicMax(x0max, __float_as_uint(x0));
        }
    }
}

template <int D, int L, int K>
hipError_t launch_l(const SphereArgs &a, hipStream_t s)
{
    if (K < 0) {
        hipError_t e = launch_fill_u32(a.x0max, 0u, 1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_sphere_pack<D, K>), dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a.pos, a.w, a.n,
                       a.pf, a.x0max);
    const int blocks = (a.rows + kSphWaves - 1) / kSphWaves;
    hipLaunchKernelGGL((k_sphere<D, L, K>), dim3((unsigned)blocks), dim3(kSphWaves * 64), 0, s, a);
    return hipGetLastError();
}

template <int D, int K>
hipError_t launch_d(int L, const SphereArgs &a, hipStream_t s)
{
    switch (L) {
    case 0: return launch_l<D, 0, K>(a, s);
    case 1: return launch_l<D, 1, K>(a, s);
    case 2: return launch_l<D, 2, K>(a, s);
    case 3: return launch_l<D, 3, K>(a, s);
    case 4: return launch_l<D, 4, K>(a, s);
    case 5: return launch_l<D, 5, K>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sphere(int D, int L, int K, const SphereArgs &a, hipStream_t s)
{
    if (a.n <= 0 || a.rows <= 0) return hipSuccess;
    if (K > 0) {
        if (D == 2) return launch_d<2, 1>(L, a, s);
        if (D == 3) return launch_d<3, 1>(L, a, s);
    } else {
        if (D == 2) return launch_d<2, -1>(L, a, s);
        if (D == 3) return launch_d<3, -1>(L, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace npcf
