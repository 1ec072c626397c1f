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
// A block is 4 waves, one primary each.  Once per launch the secondaries are
// put in spatial order (a counting sort by Hilbert cell of the embedding
// coordinates: all D + 1 on the sphere, the D spatial ones in H^D, ranked
// within a cell by catalogue index) and packed to FP32, and every chunk of 64
// sorted points gets a bounding cap (centre, largest distance r).  Per pass
// each wave tests 64 caps at a time, one per lane, and scans only the chunks
// whose distance range [d - r, d + r] from its primary meets the pass's bins
// widened by a margin that covers the FP32 errors of d and r; a chunk's
// points come straight from memory, one per lane (1.6 MB per 100k points,
// held in L2), the next chunk's in flight while one is scanned, so the waves
// of a block never wait for each other inside a pass.  The primaries of the
// launch take the same order (neighbouring waves then read the same chunks
// from L2).  The FP32 cosine
// decides the bin (through a bucket table where no edge is near, else against
// the edge cosines) unless it lies within a guard band of an edge: 1e-6 on the
// sphere (the FP32 error is below (D + 3) 2^-24 < 4e-7 for unit vectors),
// 1.5 x 2 (D + 3) 2^-24 x0max^2 in H^D (the terms sum to at most 2 p0 q0),
// where the FP64 product decides, so the decisions
// equal the FP64 ones.  In-range pairs are queued by sorted index; the
// harmonics take the tangent components from the FP64 positions in an FP64
// frame, normalised in FP64 and rounded once to FP32.  As many bins as fit a
// register budget are taken per pass (more passes rescan the points, but
// fewer registers let more waves share a SIMD and each queued pair feeds
// fewer masked sums); each lane sums harmonics in FP32 (a 0/1 mask per bin)
// and every few batches the wave reduces its lanes into FP64 values held one
// or two per lane.
#include "npcf_internal.h"
#include "npcf_harmonics.h"
#include "npcf_lanefold.h"

namespace npcf {

namespace {

// waves per block, one primary each.  Blocks of 4 (was 8): c9 25.9 -> 25.2,
// c10 57.6 -> 56.3, c11 22.9 -> 21.5 ms, and the 3-sphere kernel can then
// run five waves per SIMD (sph_waves)
constexpr int kSphWaves = 4;
// queued batches between folds of the lanes' FP32 sums into FP64.  In
// spatial order the pairs of a run of batches share bin and sign, so a
// rounding in the fold weighs on the whole run: the fold comes after a fixed
// number of batches, and its top steps add in FP64.  Measured on the
// full-size 2-sphere workload (32 primaries, strict per-multipole error),
// five bins per pass: every 4 batches 4.2e-7, 8 4.7e-7, 16 5.8e-7 (passes of
// 30.7, 27.4 and 25.8 ms); one bin per pass, whose runs of one bin are
// longer: every 8 batches 6.8e-7, every 4 4.8e-7 (25.8 and 27.2 ms).  Every
// 8 batches, and every 4 at one bin per pass (where a fold is cheap).
constexpr int kSphFoldBatches = 8;
template <int G>
constexpr int sph_fold_batches() { return G == 1 ? 4 : kSphFoldBatches; }
constexpr float kSphGuard = 1e-6f;  // FP32 cosines this close to an edge are decided in FP64 (at least)

// p.q in FP64, left to right with every product and sum rounded (no contraction)
template <int D>
__device__ __forceinline__ double dot_rn(const double (&p)[D + 1], const double *pos, int64_t n, int64_t k)
{
    double c = mul_rn(p[0], pos[k]);
#pragma unroll
    for (int x = 1; x <= D; x++) c = add_rn(c, mul_rn(p[x], pos[x * n + k]));
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

// ---- spatial order and tile caps -------------------------------------------

// the key axes: every coordinate on the sphere, the spatial ones in H^D
template <int D, int K>
__host__ __device__ constexpr int key_axes() { return K > 0 ? D + 1 : D; }

// float bits whose unsigned order is the order of the floats
__device__ __forceinline__ unsigned ord_bits(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_float(unsigned u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// H^D: per-axis minimum and maximum of the spatial coordinates (bbox[a],
// bbox[4 + a], as ordered bits), reduced over the block before the atomics
template <int D>
__global__ __launch_bounds__(256) void k_curved_bounds(const double *pos, int64_t n, unsigned *bbox)
{
    __shared__ unsigned smin[4][256], smax[4][256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int a = 0; a < D; a++) {
        const unsigned o = i < n ? ord_bits((float)pos[(a + 1) * n + i]) : 0u;
        smin[a][threadIdx.x] = i < n ? o : 0xFFFFFFFFu;
        smax[a][threadIdx.x] = o;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int a = 0; a < D; a++) {
                smin[a][threadIdx.x] = min(smin[a][threadIdx.x], smin[a][threadIdx.x + h]);
                smax[a][threadIdx.x] = max(smax[a][threadIdx.x], smax[a][threadIdx.x + h]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int a = 0; a < D; a++) {
            atomicMin(&bbox[a], smin[a][0]);
            atomicMax(&bbox[4 + a], smax[a][0]);
        }
}

// Position along the Hilbert curve of the grid cell x[0..A-1] (bits per
// axis): Skilling's transform of the coordinates into the transposed Hilbert
// index (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707,
// 2004), whose bits are then interleaved, most significant first.  Cells
// consecutive on the curve are face neighbours, so runs of sorted points are
// compact (a Morton order jumps between octants).
template <int A>
__device__ __forceinline__ uint32_t hilbert_index(uint32_t (&x)[A], int bits)
{
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t lowm = q - 1;
#pragma unroll
        for (int i = 0; i < A; i++) {
            if (x[i] & q) {
                x[0] ^= lowm;   // invert
            } else {
                const uint32_t t = (x[0] ^ x[i]) & lowm;   // exchange
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
#pragma unroll
    for (int i = 1; i < A; i++) x[i] ^= x[i - 1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (x[A - 1] & q) t ^= q - 1;
#pragma unroll
    for (int i = 0; i < A; i++) x[i] ^= t;
    uint32_t h = 0;
    for (int b = bits - 1; b >= 0; b--)
#pragma unroll
        for (int i = 0; i < A; i++) h = (h << 1) | ((x[i] >> b) & 1u);
    return h;
}

// Hilbert cell of every point (bits per axis over [-1, 1] on the sphere, over
// the bounding box in H^D) and the cells' histogram
template <int D, int K>
__global__ __launch_bounds__(256) void k_curved_keys(const double *pos, int64_t n, const unsigned *bbox, int bits,
                                                     uint32_t *key, uint32_t *count)
{
    constexpr int A = key_axes<D, K>();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = 1 << bits;
    uint32_t c[A];
#pragma unroll
    for (int a = 0; a < A; a++) {
        const float x = (float)pos[(K > 0 ? a : a + 1) * n + i];
        const float lo = K > 0 ? -1.f : ord_float(bbox[a]);
        const float hi = K > 0 ? 1.f : ord_float(bbox[4 + a]);
        const float span = hi > lo ? hi - lo : 1.f;
        int ca = (int)((x - lo) / span * (float)m);
        c[a] = (uint32_t)(ca < 0 ? 0 : (ca >= m ? m - 1 : ca));
    }
    const uint32_t k = hilbert_index<A>(c, bits);
    key[i] = k;
    atomicAdd(&count[k], 1u);
}

// the sorted copies: FP64 coordinates and weights, FP32 packed points (S^2 and H^2: (x0, x1, x2, w); D = 3: the four coordinates);
// in H^D also the largest x0 (rounded up, reduced over the block first)
template <int D, int K>
__global__ __launch_bounds__(256) void k_curved_gather(const double *pos, const double *w, int64_t n,
                                                       const int32_t *perm_sorted, double *spos, double *sw,
                                                       float4 *pf, unsigned *x0max)
{
    __shared__ unsigned smax[256];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned mx = 0;
    if (j < n) {
        const int64_t i = perm_sorted[j];
#pragma unroll
        for (int x = 0; x <= D; x++) spos[x * n + j] = pos[x * n + i];
        sw[j] = w[i];
        pf[j] = make_float4((float)pos[i], (float)pos[n + i], (float)pos[2 * n + i],
                            D == 2 ? (float)w[i] : (float)pos[3 * n + i]);
        if constexpr (K < 0) mx = __float_as_uint(__double2float_ru(pos[i]));
    }
    if constexpr (K < 0) {
        smax[threadIdx.x] = mx;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + h]);
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicMax(x0max, smax[0]);
    }
}

// one wave per chunk of kSphChunk sorted points: the cap's centre (the
// normalised sum, Euclidean on the sphere, Minkowski in H^D) and its largest
// geodesic distance from the centre
template <int D, int K>
__global__ __launch_bounds__(256) void k_curved_caps(const float4 *pf, int64_t n, float *caps)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t t0 = c * kSphChunk;
    if (t0 >= n) return;   // the whole wave
    const bool live = t0 + lane < n;
    const float4 q = live ? pf[t0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float q3 = D == 3 ? q.w : 0.f;
    float cv[4] = {q.x, q.y, q.z, q3};
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) cv[x] += __shfl_xor(cv[x], m, 64);
    float nn;
    if constexpr (K > 0) nn = cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2] + cv[3] * cv[3];
    else nn = cv[0] * cv[0] - cv[1] * cv[1] - cv[2] * cv[2] - cv[3] * cv[3];
    const float inv = nn > 0.f ? rsqrtf(nn) : 0.f;
#pragma unroll
    for (int x = 0; x < 4; x++) cv[x] *= inv;
    // the extreme "cosine": min c.q on the sphere, max <c, q> in H^D
    float ext = 1.f;
    if (live) {
        if constexpr (K > 0) ext = cv[0] * q.x + cv[1] * q.y + cv[2] * q.z + cv[3] * q3;
        else ext = cv[0] * q.x - cv[1] * q.y - cv[2] * q.z - cv[3] * q3;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const float o = __shfl_xor(ext, m, 64);
        ext = K > 0 ? fminf(ext, o) : fmaxf(ext, o);
    }
    if (lane == 0) {
        float *cp = caps + c * 8;
#pragma unroll
        for (int x = 0; x < 4; x++) cp[x] = cv[x];
        cp[4] = (inv > 0.f) ? (K > 0 ? acosf(fmaxf(-1.f, fminf(1.f, ext))) : acoshf(fmaxf(1.f, ext))) : 1e30f;
        cp[5] = cp[6] = cp[7] = 0.f;
    }
}

// Waves per SIMD the compiler is held to: five for the one-bin 3-sphere
// kernel (106 VGPRs become 96, eight values spill): c10 56.3 -> 51.0 ms;
// eight for the one-bin 2-sphere kernel (78 VGPRs become 64, ten values
// spill): c9 25.2 -> 23.4 ms (seven waves: 24.0 ms).  In H^3 five waves spill
// 29 values and gain nothing (21.5 -> 21.6); H^2 keeps its own count too.
template <int D, int K, int G>
constexpr int sph_waves() { return K > 0 && G == 1 ? (D == 3 ? 5 : 8) : 1; }

template <int D, int L, int K, int G>
__global__ __launch_bounds__(kSphWaves * 64) __attribute__((amdgpu_waves_per_eu(sph_waves<D, K, G>()))) void k_sphere(SphereArgs a)
{
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
    constexpr int NG = G * NV;        // values per pass, <= 128: lane j keeps values j and j + 64 in FP64
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * kSphWaves + wave;
    const bool active = row < a.rows;
    // the primary: its place in the spatial order, its catalogue index and
    // its output row
    const int64_t js = active ? a.prim[row] : 0;
    const int64_t pi = a.sorig[js];
    const int64_t orow = pi - a.p0;
    double p[D + 1];
#pragma unroll
    for (int x = 0; x <= D; x++) p[x] = a.spos[x * a.n + js];
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
    // margin of the tile test: the FP32 "cosines" of d and of the cap radius
    // err by at most the guard, and acos / acosh turn an error g near the
    // ends of their range into at most sqrt(2 g) in distance (plus the
    // functions' own few ulps)
    const float cull_margin = 2e-3f + 2.f * sqrtf(2.f * guard);

    unsigned long long cnt_pairs = 0;   // wave-uniform
    for (int b0 = 0; b0 < a.nb; b0 += G) {
        const int ng = min(G, a.nb - b0);
        const double chi = a.cedge[b0], clo = a.cedge[b0 + ng];
        const float chif = (float)chi, clof = (float)clo;
        const float dlo = a.erad[b0] - cull_margin, dhi = a.erad[b0 + ng] + cull_margin;
        double acc0 = 0.0, acc1 = 0.0;   // FP64 sums of values lane and lane + 64
        float fs[G][NV];
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
            for (int v = 0; v < NV; v++) fs[g][v] = 0.f;
        const float bw = (chif - clof) / kBuckets, ibw = bw > 0.f ? 1.f / bw : 0.f;
        __syncthreads();
        for (int g = threadIdx.x; g <= ng; g += blockDim.x) sce[g] = (float)a.cedge[b0 + g];
        for (int k = threadIdx.x; k < (G > 1 ? kBuckets : 0); k += blockDim.x) {
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
        int batches = 0;   // batches since the last fold (wave-uniform)
        int qn = 0;        // queued pairs (wave-uniform)
        // the lanes' FP32 sums into the FP64 values
        auto fold = [&]() {
            double y0, y1;
            fold_lanes<NG>(&fs[0][0], lane, y0, y1);
            acc0 += y0;
            acc1 += y1;
#pragma unroll
            for (int g = 0; g < G; g++)
#pragma unroll
                for (int v = 0; v < NV; v++) fs[g][v] = 0.f;
            batches = 0;
        };
        // harmonics of the first cnt queued pairs, one per lane, into the bin sums
        auto process = [&](int cnt) {
            const bool live = lane < cnt;
            const int k = live ? qidx[wave][lane] : 0;
            int bl = 0;
            if constexpr (G > 1) bl = live ? qbin[wave][lane] : 0;
            // tangent components from the FP64 positions and frame, normalised
            // in FP64 and rounded once to FP32 (each rounding of the direction
            // enters the l-th harmonic about l times)
            double q[D + 1];
#pragma unroll
            for (int x = 0; x <= D; x++) q[x] = live ? a.spos[x * a.n + k] : 0.0;
            float wq = 0.f;
            if constexpr (D == 2) wq = live ? qw[wave][lane] : 0.f;
            else wq = live ? (float)a.sw[k] : 0.f;
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
        // the chunks of kSphChunk sorted points whose cap reaches this pass's
        // bins, in order: each lane tests one chunk of a group of 64, and the
        // ballot's bits are taken one by one (wave-uniform)
        const int64_t nch = (a.n + kSphChunk - 1) / kSphChunk;
        int64_t g0 = -64;
        unsigned long long gm = 0;
        auto next_chunk = [&]() -> int64_t {
            while (gm == 0) {
                g0 += 64;
                if (g0 >= nch) return -1;
                const int64_t c = g0 + lane;
                bool reach = false;
                if (c < nch) {
                    const float4 cc = reinterpret_cast<const float4 *>(a.caps)[2 * c];
                    const float r = a.caps[8 * c + 4];
                    const float cd = pf32[0] * cc.x + pf32[1] * cc.y + pf32[2] * cc.z + pf32[3] * cc.w;
                    const float d = K > 0 ? acosf(fmaxf(-1.f, fminf(1.f, cd))) : acoshf(fmaxf(1.f, -cd));
                    reach = !(d - r > dhi || d + r < dlo);
                }
                gm = __builtin_amdgcn_ballot_w64(reach);
            }
            const int bit = __builtin_ctzll(gm);
            gm &= gm - 1;
            return g0 + bit;
        };
        if (active) {
            // one chunk's points in flight while the previous one is scanned
            int64_t cur = next_chunk();
            float4 qcur = make_float4(0.f, 0.f, 0.f, 0.f);
            if (cur >= 0 && cur * kSphChunk + lane < a.n) qcur = a.pf[cur * kSphChunk + lane];
            while (cur >= 0) {
                const int64_t nxt = next_chunk();
                float4 qnxt = make_float4(0.f, 0.f, 0.f, 0.f);
                if (nxt >= 0 && nxt * kSphChunk + lane < a.n) qnxt = a.pf[nxt * kSphChunk + lane];
                // scan: bin of every point; in-range pairs go to the wave's queue
                const int64_t t = cur * kSphChunk + lane;   // this lane's point (sorted index)
                bool valid = false;
                int bl = 0;
                if (t < a.n) {
                    const float4 q = qcur;
                    float c32 = pf32[0] * q.x + pf32[1] * q.y + pf32[2] * q.z;
                    if constexpr (D == 3) c32 += pf32[3] * q.w;
                    // range prefilter on the same FP32 differences as the guard
                    // test below, so that a cosine admitted beyond an outer edge
                    // is always within the guard of it and decided in FP64
                    // (chif + guard rounded in FP32 would admit cosines up to
                    // one rounding beyond the guard)
                    if (c32 - chif <= guard && clof - c32 < guard) {
                        valid = true;
                        if constexpr (G == 1) {
                            // one bin per pass: only its two edges, no table
                            if (fabsf(c32 - chif) <= guard || fabsf(c32 - clof) <= guard) {
                                const double c = dot_rn<D>(pc, a.spos, a.n, t);
                                valid = c <= chi && c > clo;
                            }
                        } else {
                            // bin from the bucket table; near an edge, from the FP32
                            // cosine against the edges, and within the guard band of
                            // an edge from the FP64 dot product
                            int kb = (int)((c32 - clof) * ibw);
                            kb = kb < 0 ? 0 : (kb >= kBuckets ? kBuckets - 1 : kb);
                            const int ent = sbk[kb];
                            bl = ent & 0x7F;
                            bool near = false;
                            if (ent & 0x80) {
                                while (bl + 1 < ng && c32 <= sce[bl + 1]) bl++;
                                while (bl > 0 && c32 > sce[bl]) bl--;
                                near = fabsf(c32 - sce[bl]) <= guard || fabsf(c32 - sce[bl + 1]) <= guard;
                            }
                            if (near) {
                                const double c = dot_rn<D>(pc, a.spos, a.n, t);
                                valid = c <= chi && c > clo;
                                bl = 0;
                                while (bl + 1 < ng && c <= a.cedge[b0 + bl + 1]) bl++;
                            }
                        }
                    }
                    if constexpr (K < 0) valid = valid && (t != js);   // the self pair, by index
                }
                const unsigned long long vm = __builtin_amdgcn_ballot_w64(valid);
                const int slot = qn + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(vm >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((unsigned)vm, 0u));
                if (valid) {
                    qidx[wave][slot] = (int)t;
                    if constexpr (D == 2) qw[wave][slot] = qcur.w;
                    if constexpr (G > 1) qbin[wave][slot] = bl;
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
                        if constexpr (G > 1) mb = qbin[wave][64 + lane];
                    }
                    NPCF_SPH_WAVE_SYNC();
                    if (lane < rest) {
                        qidx[wave][lane] = mi;
                        if constexpr (D == 2) qw[wave][lane] = mw;
                        if constexpr (G > 1) qbin[wave][lane] = mb;
                    }
                    qn = rest;
                    if (++batches == sph_fold_batches<G>()) fold();
                }
                cur = nxt;
                qcur = qnxt;
            }
            // at the end: the last queued pairs, and the last fold
            if (qn > 0) {
                NPCF_SPH_WAVE_SYNC();
                process(qn);
                qn = 0;
            }
            fold();
        }
        if (active) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int j = lane + 64 * h;
                if (j < NG) {
                    const int g = j / NV, v = j - g * NV;
                    if (g < ng) a.A[(orow * a.nb + b0 + g) * NV + v] = (float)(h ? acc1 : acc0);
                }
            }
        }
    }
    if (active && lane == 0) {
        atomicAdd(a.pairs, cnt_pairs);
        a.wrow[orow] = (float)a.w[pi];
    }
}

template <int D, int L, int K>
hipError_t launch_l(const SphereArgs &a, hipStream_t s)
{
    if (a.group != sph_group(D, L, false) && a.group != sph_group(D, L, true)) return hipErrorInvalidValue;
    constexpr int A = key_axes<D, K>();
    const int64_t ncell = (int64_t)1 << (a.ncell_bits * A);
    const unsigned g = (unsigned)((a.n + 255) / 256);
    hipError_t e = launch_fill_u32(a.count, 0u, ncell + 1, s);
    if (e == hipSuccess && K < 0) e = launch_fill_u32(a.x0max, 0u, 1, s);
    if (e == hipSuccess && K < 0) e = launch_fill_u32(a.bbox, 0xFFFFFFFFu, 4, s);
    if (e == hipSuccess && K < 0) e = launch_fill_u32(a.bbox + 4, 0u, 4, s);
    if (e != hipSuccess) return e;
    if (K < 0) hipLaunchKernelGGL((k_curved_bounds<D>), dim3(g), dim3(256), 0, s, a.pos, a.n, a.bbox);
    hipLaunchKernelGGL((k_curved_keys<D, K>), dim3(g), dim3(256), 0, s, a.pos, a.n, a.bbox, a.ncell_bits, a.key, a.count);
    e = launch_exclusive_scan(a.count, a.cell_start, ncell + 1, a.scan, a.scan_len, s);
    if (e == hipSuccess) e = launch_copy_u32(a.cursor, a.cell_start, ncell + 1, s);
    if (e == hipSuccess) e = launch_scatter_perm(a.n, a.key, a.cursor, a.perm, s);
    if (e == hipSuccess) e = launch_cellsort(a.n, a.key, a.cell_start, a.perm, a.sorig, s);   // sorig: sorted -> catalogue
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_curved_gather<D, K>), dim3(g), dim3(256), 0, s, a.pos, a.w, a.n, (const int32_t *)a.sorig,
                       a.spos, a.sw, a.pf, a.x0max);
    e = launch_primlist(a.n, a.sorig, a.p0, a.p0 + a.rows, a.pflag, a.ppos, a.prim, a.scan, a.scan_len, s);
    if (e != hipSuccess) return e;
    const int64_t nch = (a.n + kSphChunk - 1) / kSphChunk;
    hipLaunchKernelGGL((k_curved_caps<D, K>), dim3((unsigned)((nch + 3) / 4)), dim3(256), 0, s, a.pf, a.n, a.caps);
    const int blocks = (a.rows + kSphWaves - 1) / kSphWaves;
    constexpr int GW = sph_group(D, L, false), GN = sph_group(D, L, true);
    if (a.group == GW) hipLaunchKernelGGL((k_sphere<D, L, K, GW>), dim3((unsigned)blocks), dim3(kSphWaves * 64), 0, s, a);
    else hipLaunchKernelGGL((k_sphere<D, L, K, GN>), dim3((unsigned)blocks), dim3(kSphWaves * 64), 0, s, a);
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
