// Device helpers shared by the coupling kernels (npcf_couple.hip: N = 3, 4;
// npcf_couple5.hip: N = 5): MFMA K = 32 slices in the four precisions, the
// XCD-aware block mapping, staging of rows of a, scalar-path helpers.
#pragma once

#include "npcf_internal.h"

namespace npcf {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kRowsStep = 16;   // primaries staged in LDS per step
constexpr int kXcd = 8;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// x of the partner lane under a DPP lane pattern (within rows of 16 lanes)
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Largest m over the lanes l, l ^ 16, l ^ 32, l ^ 48, in every lane: each
// permlane swap of a register with itself hands a lane the value of lane
// l ^ 16 (l ^ 32) in one of the two results.  No LDS traffic.
__device__ __forceinline__ float max_over_lane_bits45(float m)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(m), __float_as_uint(m), false, false);
    m = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
    r = __builtin_amdgcn_permlane32_swap(__float_as_uint(m), __float_as_uint(m), false, false);
    return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// Largest m over the wave, in every lane: DPP steps pair lanes l ^ 1, l ^ 2
// (quad permutations), l ^ 7 (mirror within 8) and l ^ 8 (rotation by 8
// within 16), then the permlane swaps cover lane bits 4 and 5.
__device__ __forceinline__ float wave_max(float m)
{
    m = fmaxf(m, dpp_f<0xB1>(m));
    m = fmaxf(m, dpp_f<0x4E>(m));
    m = fmaxf(m, dpp_f<0x141>(m));
    m = fmaxf(m, dpp_f<0x128>(m));
    return max_over_lane_bits45(m);
}

// Power-of-two scale that brings the wave's largest |x| into [0.5, 1) (1 when
// every x is zero).  FP16's exponent range is too narrow for products of
// coefficients spanning many octaves without it.
__device__ __forceinline__ float wave_pow2_scale(float m)
{
    m = wave_max(m);
    if (!(m > 0.f) || !isfinite(m)) return 1.f;
    int e;
    frexpf(m, &e);
    return ldexpf(1.f, -e);
}

typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// x = hi + mid + lo in BF16 (each rounded to nearest), two values per packed
// conversion; a BF16 value widens to FP32 exactly by placing its 16 bits on
// top of a zero half, so each residual is one subtraction.
__device__ __forceinline__ void split3_bf16(const float (&x)[8], v8bf &hi, v8bf &mid, v8bf &lo)
{
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        const v2f v = {x[i], x[i + 1]};
        const v2bf h = __builtin_convertvector(v, v2bf);
        const uint32_t hb = __builtin_bit_cast(uint32_t, h);
        const v2f r = {v[0] - __uint_as_float(hb << 16), v[1] - __uint_as_float(hb & 0xFFFF0000u)};
        const v2bf m = __builtin_convertvector(r, v2bf);
        const uint32_t mb = __builtin_bit_cast(uint32_t, m);
        const v2f t = {r[0] - __uint_as_float(mb << 16), r[1] - __uint_as_float(mb & 0xFFFF0000u)};
        const v2bf l = __builtin_convertvector(t, v2bf);
        hi[i] = h[0];
        hi[i + 1] = h[1];
        mid[i] = m[0];
        mid[i + 1] = m[1];
        lo[i] = l[0];
        lo[i + 1] = l[1];
    }
}

// One K = 32 slice: lane l holds 8 (A, B) operand pairs; A row = l % 16,
// B column = l % 16, and the 4 lane quarters together cover 32 K indices
// (the order of K is immaterial to the sum).  Accumulates into c (from zero)
// and returns the factor that undoes any operand scaling.
template <int PREC>
__device__ __forceinline__ void mfma_k32(const float (&Av)[8], const float (&Bv)[8], v4f &c, double &unscale)
{
    unscale = 1.0;
    if constexpr (PREC == 0) {
#pragma unroll
        for (int i = 0; i < 8; i++) c = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[i], Bv[i], c, 0, 0, 0);
    } else if constexpr (PREC == 1) {
        v8bf ah, al, bh, bl;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            ah[i] = (__bf16)Av[i];
            al[i] = (__bf16)(Av[i] - (float)ah[i]);
            bh[i] = (__bf16)Bv[i];
            bl[i] = (__bf16)(Bv[i] - (float)bh[i]);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    } else if constexpr (PREC == 2) {
        float ma = 0.f, mb = 0.f;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            ma = fmaxf(ma, fabsf(Av[i]));
            mb = fmaxf(mb, fabsf(Bv[i]));
        }
        const float sa = wave_pow2_scale(ma), sb = wave_pow2_scale(mb);
        v8h ah, al, bh, bl;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const float x = Av[i] * sa, y = Bv[i] * sb;
            ah[i] = (_Float16)x;
            al[i] = (_Float16)(x - (float)ah[i]);
            bh[i] = (_Float16)y;
            bl[i] = (_Float16)(y - (float)bh[i]);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, c, 0, 0, 0);
        unscale = 1.0 / ((double)sa * (double)sb);
    } else {
        v8bf ah, am, al, bh, bm, bl;
        split3_bf16(Av, ah, am, al);
        split3_bf16(Bv, bh, bm, bl);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    }
}

// XCD-aware block -> (rowblock, jobgroup): blocks are dispatched round-robin
// over the 8 XCDs, so the job groups of one rowblock are given consecutive
// slots on one XCD and its rows of a are served from that XCD's L2.
__device__ __forceinline__ bool block_work(int nrb, int njg, int &rb, int &jg)
{
    const int b = blockIdx.x;
    const int x = b % kXcd;
    const int s = b / kXcd;
    rb = (s / njg) * kXcd + x;
    jg = s % njg;
    return rb < nrb;
}

// Stage kRowsStep rows of a (and their weights) into LDS, zero-padding rows
// at and past r_end (the end of this block's rows).
__device__ __forceinline__ void stage_rows(const CoupleArgs &a, int r0, int r_end, float *Ast, float *wst)
{
    const int rowlen = a.nb * 2 * a.nstate;
    const int total = kRowsStep * rowlen;
    const int r_lim = r_end - r0;
    const float *src = a.A + (size_t)r0 * rowlen;
    for (int t = threadIdx.x; t < total; t += blockDim.x) Ast[t] = (t < r_lim * rowlen) ? src[t] : 0.f;
    for (int t = threadIdx.x; t < kRowsStep; t += blockDim.x) wst[t] = (t < r_lim) ? a.wrow[r0 + t] : 0.f;
}

// The same for rs <= kRowsStep rows (kernels whose rows are long stage fewer
// of them, so that more blocks fit in a CU's LDS).
__device__ __forceinline__ void stage_rows_n(const CoupleArgs &a, int r0, int r_end, int rs, float *Ast, float *wst)
{
    const int rowlen = a.nb * 2 * a.nstate;
    const int total = rs * rowlen;
    const int r_lim = r_end - r0;
    const float *src = a.A + (size_t)r0 * rowlen;
    for (int t = threadIdx.x; t < total; t += blockDim.x) Ast[t] = (t < r_lim * rowlen) ? src[t] : 0.f;
    for (int t = threadIdx.x; t < rs; t += blockDim.x) wst[t] = (t < r_lim) ? a.wrow[r0 + t] : 0.f;
}

template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p)
{
    // read-only tables: the constant address space lets uniform loads go
    // through the scalar unit
    return (const __attribute__((address_space(4))) T *)p;
}

// a wave-uniform value held in a scalar register (table indices and
// coefficients, so their loads and uses stay on the scalar path)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

template <class K, class... Args>
hipError_t launch_with_lds(K kernel, int nblk, int lds, hipStream_t s, Args... args)
{
    hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(nblk), dim3(256), lds, s, args...);
    return hipGetLastError();
}

}  // namespace

}  // namespace npcf
