// Hyperspherical harmonics of Appendix A (eq. hypersph-def) in Cartesian
// Gegenbauer form, evaluated per pair in FP32 registers.  Each function
// streams w * conj(Y_s(u)) for every stored state s (l1 >= 0 half) to
// emit(slot, value): slot 2s holds the real part, 2s+1 the imaginary part
// (never emitted for l1 = 0, which is real).
#pragma once
#include "npcf_internal.h"
#include <type_traits>

namespace npcf {
namespace harm {

// ---- recurrence constants, evaluated at compile time ---------------------------------
// Normalised Gegenbauer values c_n = K_n C^{(lambda)}_n obey c_0 = K_0 and
//   c_n = alpha_n t c_{n-1} - beta_n s c_{n-2},
//   alpha_n = (K_n / K_{n-1}) 2 (n + lambda - 1) / n,  beta_n = (K_n / K_{n-2}) (n + 2 lambda - 2) / n,
// with K_n^2 / K_{n-1}^2 = n (n + lambda) / ((n - 1 + 2 lambda)(n - 1 + lambda)) and
// K_0^2 = lambda Gamma(lambda) / (sqrt(pi) Gamma(lambda + 1/2)) (the inverse norm of
// C^{(lambda)}_0 on [-1, 1] with weight (1 - t^2)^{lambda - 1/2}).
constexpr double kPi = 3.14159265358979323846;

constexpr double ct_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    double r = x > 1.0 ? x : 1.0;  // Newton from above: monotone decrease to sqrt(x)
    for (int i = 0; i < 200; i++) {
        const double n = 0.5 * (r + x / r);
        if (!(n < r)) break;
        r = n;
    }
    return r;
}

// Gamma(lambda) / Gamma(lambda + 1/2) for lambda in {1/2, 1, 3/2, 2, ...}
constexpr double gamma_ratio(double lambda)
{
    double lam = (lambda - (double)(int)lambda) != 0.0 ? 0.5 : 1.0;
    double g = lam == 0.5 ? ct_sqrt(kPi) : 2.0 / ct_sqrt(kPi);
    while (lam < lambda) {
        g *= lam / (lam + 0.5);
        lam += 1.0;
    }
    return g;
}

// c_0 followed by (alpha_n, beta_n) for n = 1..nmax, each times pref
constexpr int push_gegenbauer(float *out, int at, double lambda, int nmax, double pref)
{
    double k0 = pref * ct_sqrt(lambda * gamma_ratio(lambda) / ct_sqrt(kPi));
    out[at++] = (float)k0;
    double r1 = 1.0, r2 = 1.0;  // K_{n-1}/K_{n-2}, K_n/K_{n-1}
    for (int n = 1; n <= nmax; n++) {
        r1 = r2;
        r2 = ct_sqrt(n * (n + lambda) / ((n - 1 + 2.0 * lambda) * (n - 1 + lambda)));
        out[at++] = (float)(r2 * 2.0 * (n + lambda - 1.0) / n);
        out[at++] = (float)(n >= 2 ? r2 * r1 * (n + 2.0 * lambda - 2.0) / n : 0.0);
    }
    return at;
}

template <int D, int L>
struct HarmConst {
    static constexpr int N = D == 2 ? 1 : (D == 3 ? (L + 1) * (L + 1) : 2 * (L + 1) * (L + 1));
    float v[N];
    constexpr HarmConst() : v{}
    {
        const double inv_sqrt_2pi = 1.0 / ct_sqrt(2.0 * kPi);
        int at = 0;
        if (D == 2) {
            v[0] = (float)inv_sqrt_2pi;
        } else if (D == 3) {
            for (int m = 0; m <= L; m++) at = push_gegenbauer(v, at, m + 0.5, L - m, inv_sqrt_2pi);
        } else {
            for (int l2 = 0; l2 <= L; l2++) at = push_gegenbauer(v, at, l2 + 1.0, L - l2, 1.0);
            for (int l1 = 0; l1 <= L; l1++) at = push_gegenbauer(v, at, l1 + 0.5, L - l1, inv_sqrt_2pi);
        }
    }
};

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).  Every
// index below is a constant, so the emitted slots, table offsets and the
// caller's emission counter fold at compile time (triangular loops under
// #pragma unroll are not always unrolled fully).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Offset of (alpha_n, beta_n, ...) tables in HarmConst: c_0 then 2 per step.
constexpr int geg_table_offset(int first_nmax, int j)
{
    int off = 0;
    for (int t = 0; t < j; t++) off += 1 + 2 * (first_nmax - t);
    return off;
}

// The emitted value for stored state s is w * conj(Y_s(u)) split into real
// (slot 2s) and imaginary (slot 2s+1) parts; m = 0 (l1 = 0) states have no
// imaginary part and emit only the real slot.

// D = 2: Y_l = e^{i l theta1} / sqrt(2 pi); conj -> (u1 - i u2)^l / sqrt(2 pi).
template <int L, class F>
__device__ __forceinline__ void harm_d2(const float *u, float w, F &&emit)
{
    constexpr HarmConst<2, L> H{};
    float pr = w * H.v[0], pi = 0.f;
    emit(0, pr);
    static_for<1, L + 1>([&](auto lc) {
        constexpr int l = lc;
        const float nr = pr * u[0] + pi * u[1];
        const float ni = pi * u[0] - pr * u[1];
        pr = nr;
        pi = ni;
        emit(2 * l, pr);
        emit(2 * l + 1, pi);
    });
}

// D = 3: Y_{m,l} = K (u1 + i u2)^m C^{(m+1/2)}_{l-m}(u3).  The normalised
// Gegenbauer values obey c_n = alpha_n u3 c_{n-1} - beta_n c_{n-2}; the table
// holds, for m = 0..L, c_0 followed by (alpha_n, beta_n) for n = 1..L-m.
template <int L, class F>
__device__ __forceinline__ void harm_d3(const float *u, float w, F &&emit)
{
    constexpr HarmConst<3, L> H{};
    float pr = w, pi = 0.f;
    static_for<0, L + 1>([&](auto mc) {
        constexpr int m = mc;
        constexpr int base = geg_table_offset(L, m);
        if constexpr (m > 0) {
            const float nr = pr * u[0] + pi * u[1];
            const float ni = pi * u[0] - pr * u[1];
            pr = nr;
            pi = ni;
        }
        float c1 = H.v[base], c2 = 0.f;
        {
            constexpr int s = m * (m + 1) / 2 + m;
            emit(2 * s, c1 * pr);
            if constexpr (m > 0) emit(2 * s + 1, c1 * pi);
        }
        static_for<m + 1, L + 1>([&](auto lc) {
            constexpr int l = lc;
            constexpr int n = l - m;
            const float c = H.v[base + 2 * n - 1] * u[2] * c1 - H.v[base + 2 * n] * c2;
            c2 = c1;
            c1 = c;
            constexpr int s = l * (l + 1) / 2 + m;
            emit(2 * s, c * pr);
            if constexpr (m > 0) emit(2 * s + 1, c * pi);
        });
    });
}

// D = 4: Y_{l1 l2 l3} = (u1 + i u2)^{l1} g_{l1}(l2) c_{l2}(l3) with
//   c_{l2}(l3) = N3 C^{(l2+1)}_{l3-l2}(u4)
//   g_{l1}(l2) = (2 pi)^{-1/2} N2 rho^{l2-l1} C^{(l1+1/2)}_{l2-l1}(u3/rho), rho^2 = u1^2+u2^2+u3^2,
// both by three-term recurrences; the table holds the c tables (for
// l2 = 0..L: c_0, (alpha, beta) for n = 1..L-l2), then the g tables (l1 = 0..L).
template <int L, class F>
__device__ __forceinline__ void harm_d4(const float *u, float w, F &&emit)
{
    constexpr HarmConst<4, L> H{};
    constexpr int NT = (L + 1) * (L + 2) / 2;
    constexpr int GBASE = geg_table_offset(L, L + 1);
    float ct[NT];  // ct[tri(l2) + (l3 - l2)]
    float gt[NT];  // gt[tri(l1) + (l2 - l1)]
    const float rho2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    static_for<0, L + 1>([&](auto jc) {
        constexpr int j = jc;
        constexpr int cb = geg_table_offset(L, j);
        constexpr int gb = GBASE + geg_table_offset(L, j);
        constexpr int ti = (j * (2 * L + 3 - j)) / 2;
        float c1 = H.v[cb], c2 = 0.f, g1 = H.v[gb], g2 = 0.f;
        ct[ti] = c1;
        gt[ti] = g1;
        static_for<1, L - j + 1>([&](auto nc) {
            constexpr int n = nc;
            const float c = H.v[cb + 2 * n - 1] * u[3] * c1 - H.v[cb + 2 * n] * c2;
            c2 = c1;
            c1 = c;
            ct[ti + n] = c;
            const float g = H.v[gb + 2 * n - 1] * u[2] * g1 - H.v[gb + 2 * n] * rho2 * g2;
            g2 = g1;
            g1 = g;
            gt[ti + n] = g;
        });
    });
    float pr = w, pi = 0.f;
    static_for<0, L + 1>([&](auto l1c) {
        constexpr int l1 = l1c;
        if constexpr (l1 > 0) {
            const float nr = pr * u[0] + pi * u[1];
            const float ni = pi * u[0] - pr * u[1];
            pr = nr;
            pi = ni;
        }
        static_for<l1, L + 1>([&](auto l2c) {
            constexpr int l2 = l2c;
            const float g = gt[(l1 * (2 * L + 3 - l1)) / 2 + (l2 - l1)];
            const float gr = g * pr, gi = g * pi;
            static_for<l2, L + 1>([&](auto l3c) {
                constexpr int l3 = l3c;
                const float c = ct[(l2 * (2 * L + 3 - l2)) / 2 + (l3 - l2)];
                constexpr int s = l3 * (l3 + 1) * (l3 + 2) / 6 + l2 * (l2 + 1) / 2 + l1;
                emit(2 * s, c * gr);
                if constexpr (l1 > 0) emit(2 * s + 1, c * gi);
            });
        });
    });
}

template <int D, int L, class F>
__device__ __forceinline__ void harmonics(const float *u, float w, F &&emit)
{
    if constexpr (D == 2) harm_d2<L>(u, w, emit);
    else if constexpr (D == 3) harm_d3<L>(u, w, emit);
    else harm_d4<L>(u, w, emit);
}

}  // namespace harm
}  // namespace npcf
