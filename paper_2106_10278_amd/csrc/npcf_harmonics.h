// Hyperspherical harmonics of Appendix A (eq. hypersph-def) in Cartesian
// Gegenbauer form, evaluated per pair in FP32 registers.  Each function
// streams w * conj(Y_s(u)) for every stored state s (l1 >= 0 half) to
// emit(slot, value): slot 2s holds the real part, 2s+1 the imaginary part
// (never emitted for l1 = 0, which is real).
#pragma once
#include "npcf_internal.h"

namespace npcf {
namespace harm {

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

}  // namespace harm
}  // namespace npcf
