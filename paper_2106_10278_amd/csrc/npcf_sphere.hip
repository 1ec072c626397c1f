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
// A block is 8 waves, one primary each; secondaries come through LDS in
// tiles (FP64 x, y, z, w); bins are taken 4 per pass, each wave's lanes sum
// the harmonics of their tile points in FP32 and fold into FP64 after every
// tile, then the wave reduces its lanes.
#include "npcf_internal.h"
#include "npcf_harmonics.h"

namespace npcf {

namespace {

constexpr int kSphTile = 512;
constexpr int kSphWaves = 8;
constexpr int kSphGroup = 4;   // bins per pass

__device__ __forceinline__ double dot3_rn(double ax, double ay, double az, double bx, double by, double bz)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(ax, bx), __dmul_rn(ay, by)), __dmul_rn(az, bz));
}

template <int L>
__global__ __launch_bounds__(kSphWaves * 64) void k_sphere(SphereArgs a)
{
    __shared__ double4 tile[kSphTile];
    constexpr int NV = 2 * (L + 1);   // real slots per bin (slot 1, the l = 0 imaginary part, stays 0)
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

    unsigned long long cnt = 0;
    for (int b0 = 0; b0 < a.nb; b0 += kSphGroup) {
        const int ng = min(kSphGroup, a.nb - b0);
        const double chi = a.cedge[b0], clo = a.cedge[b0 + ng];
        double acc[kSphGroup][NV];
#pragma unroll
        for (int g = 0; g < kSphGroup; g++)
#pragma unroll
            for (int v = 0; v < NV; v++) acc[g][v] = 0.0;
        for (int64_t t0 = 0; t0 < a.n; t0 += kSphTile) {
            const int cnt_t = (int)(a.n - t0 < kSphTile ? a.n - t0 : kSphTile);
            __syncthreads();
            for (int i = threadIdx.x; i < cnt_t; i += blockDim.x) {
                const int64_t k = t0 + i;
                tile[i] = make_double4(a.pos[k], a.pos[a.n + k], a.pos[2 * a.n + k], a.w[k]);
            }
            __syncthreads();
            if (!active) continue;
            float fs[kSphGroup][NV];
#pragma unroll
            for (int g = 0; g < kSphGroup; g++)
#pragma unroll
                for (int v = 0; v < NV; v++) fs[g][v] = 0.f;
            for (int i = lane; i < cnt_t; i += 64) {
                const double4 q = tile[i];
                const double c = dot3_rn(px, py, pz, q.x, q.y, q.z);
                if (!(c <= chi && c > clo)) continue;
                int bl = 0;
                while (bl + 1 < ng && c <= a.cedge[b0 + bl + 1]) bl++;
                const double t1 = q.x * e1x + q.y * e1y + q.z * e1z;
                const double t2 = q.x * e2x + q.y * e2y + q.z * e2z;
                const double tn2 = t1 * t1 + t2 * t2;
                if (!(tn2 > 0.0)) continue;
                const double itn = 1.0 / sqrt(tn2);
                const float u[2] = {(float)(t1 * itn), (float)(t2 * itn)};
                cnt++;
                float hv[NV];
                hv[1] = 0.f;   // l = 0 is real
                harm::harmonics<2, L>(u, (float)q.w, [&](int slot, float v) { hv[slot] = v; });
#pragma unroll
                for (int g = 0; g < kSphGroup; g++) {
                    const bool on = g == bl;
#pragma unroll
                    for (int v = 0; v < NV; v++) fs[g][v] += on ? hv[v] : 0.f;
                }
            }
#pragma unroll
            for (int g = 0; g < kSphGroup; g++)
#pragma unroll
                for (int v = 0; v < NV; v++) acc[g][v] += (double)fs[g][v];
        }
        // the wave's sums, written by lane 0
#pragma unroll
        for (int g = 0; g < kSphGroup; g++)
#pragma unroll
            for (int v = 0; v < NV; v++) {
                double x = acc[g][v];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
                acc[g][v] = x;
            }
        if (active && lane == 0) {
#pragma unroll
            for (int g = 0; g < kSphGroup; g++)
                if (g < ng) {
#pragma unroll
                    for (int v = 0; v < NV; v++) a.A[((int64_t)row * a.nb + b0 + g) * NV + v] = (float)acc[g][v];
                }
        }
    }
    if (active) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0) {
            atomicAdd(a.pairs, cnt);
            a.wrow[row] = (float)a.w[pi];
        }
    }
}

template <int L>
hipError_t launch_l(const SphereArgs &a, hipStream_t s)
{
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
