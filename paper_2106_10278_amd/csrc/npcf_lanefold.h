// Wave-level reduction of per-lane FP32 sums (gfx950): every lane holds
// the same NG values (its own partial sums), and after the fold lane l holds
// the wave's totals of values l and l + 64, the last three steps added in
// FP64.  Shared by the curved-space kernel and the flat kernel's per-bin
// passes.
#pragma once
#include <hip/hip_runtime.h>

namespace npcf {

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

// The same step on FP64 values: the lane keeps one of each pair and adds the
// partner's copy of it, moved by DPP as two 32-bit halves
template <int N, int CTRL>
__device__ __forceinline__ void fold_step64(const double *v, double *out, bool bit)
{
    constexpr int H = N / 4;
#pragma unroll
    for (int q = 0; q < N / 2; q++) {
        const int lo = (q & (H - 1)) | ((q & ~(H - 1)) << 1);
        const double keep = bit ? v[lo + H] : v[lo], send = bit ? v[lo] : v[lo + H];
        const unsigned long long sb = (unsigned long long)__double_as_longlong(send);
        const unsigned plo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)sb, CTRL, 0xF, 0xF, false);
        const unsigned phi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(sb >> 32), CTRL, 0xF, 0xF, false);
        out[q] = keep + __longlong_as_double((long long)(((unsigned long long)phi << 32) | plo));
    }
}

// Sum of each of the NG (<= 128) values x[j] over the 64 lanes of the wave,
// scattered: lane l receives the totals of values l (y0) and l + 64 (y1; zero
// past NG).  A butterfly that halves the values at each step: lane bit 5
// through v_permlane32_swap, bit 4 through v_permlane16_swap, bits 3 to 0
// through DPP.  At each step the lane keeps the values whose index bit
// matches its lane bit, so after six steps lane l holds value l and l + 64.
// The last three steps add in FP64: in spatial order the lanes' sums of one
// bin share their sign, and a rounding in the top steps, where one or two
// partial sums carry the whole total, weighs most on it.
template <int NG>
__device__ __forceinline__ void fold_lanes(const float *x, int lane, double &y0, double &y1)
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
    float x3[16];
    fold_step<32, 0x128>(w, x3, (lane & 8) != 0);    // row_ror:8
    double d3[16], x2[8], x1[4], x0[2];
#pragma unroll
    for (int q = 0; q < 16; q++) d3[q] = (double)x3[q];
    fold_step64<16, 0x141>(d3, x2, (lane & 4) != 0);   // row_half_mirror
    fold_step64<8, 0x4E>(x2, x1, (lane & 2) != 0);     // quad_perm [2,3,0,1]
    fold_step64<4, 0xB1>(x1, x0, (lane & 1) != 0);     // quad_perm [1,0,3,2]
    y0 = x0[0];
    y1 = x0[1];
}

}  // namespace npcf
