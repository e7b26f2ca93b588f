// Cross-lane primitives of the gfx950 kernels of libffrt (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffrt {

// ------------------------------------------------------------------------------------------------
// Cross-lane exchanges that stay in the VALU (no LDS crossbar traffic): v_permlane32_swap and
// v_permlane16_swap exchange the two 32-lane halves / neighbouring 16-lane rows of two registers, and DPP
// reads the partner lane L ^ 15 (row_mirror), L ^ 7 (row_half_mirror), L ^ 2 and L ^ 1 (quad_perm).  The
// six masks 32, 16, 15, 7, 2, 1 span all six lane bits, so reducing over them covers the whole wave.
// ------------------------------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ uint32_t dpp_xor(uint32_t v) {
    static_assert(M == 15 || M == 7 || M == 2 || M == 1, "DPP partner mask");
    constexpr int ctrl = M == 15 ? 0x140 : (M == 7 ? 0x141 : (M == 2 ? 0x4E : 0xB1));
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, false);
}
template <int M>
__device__ __forceinline__ float dpp_xor(float v) {
    return __builtin_bit_cast(float, dpp_xor<M>(__builtin_bit_cast(uint32_t, v)));
}
template <int M>
__device__ __forceinline__ int dpp_xor(int v) {
    return (int)dpp_xor<M>((uint32_t)v);
}
// (a, b) -> halves / rows swapped: for lanes whose bit log2(OFF) is clear, first = a[L], second =
// a[L + OFF]; for the others, first = b[L - OFF], second = b[L].
template <int OFF, class T>
__device__ __forceinline__ void lane_swap(T a, T b, T& first, T& second) {
    static_assert(OFF == 32 || OFF == 16, "permlane swap distance");
    const uint32_t ua = __builtin_bit_cast(uint32_t, a), ub = __builtin_bit_cast(uint32_t, b);
    if constexpr (OFF == 32) {
        auto r = __builtin_amdgcn_permlane32_swap(ua, ub, false, false);
        first = __builtin_bit_cast(T, (uint32_t)r[0]);
        second = __builtin_bit_cast(T, (uint32_t)r[1]);
    } else {
        auto r = __builtin_amdgcn_permlane16_swap(ua, ub, false, false);
        first = __builtin_bit_cast(T, (uint32_t)r[0]);
        second = __builtin_bit_cast(T, (uint32_t)r[1]);
    }
}
// Whole-wave reduction; every lane receives the result.
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
    T x, y;
    lane_swap<32>(v, v, x, y);
    v = op(x, y);
    lane_swap<16>(v, v, x, y);
    v = op(x, y);
    v = op(v, dpp_xor<15>(v));
    v = op(v, dpp_xor<7>(v));
    v = op(v, dpp_xor<2>(v));
    v = op(v, dpp_xor<1>(v));
    return v;
}
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    return wave_reduce(v, [](T a, T b) { return a + b; });
}
__device__ __forceinline__ int wave_min(int v) {
    return wave_reduce(v, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ int wave_max(int v) {
    return wave_reduce(v, [](int a, int b) { return max(a, b); });
}

// One butterfly step of a wave reduce-scatter: lanes with bit OFF clear keep entries [0, HALF) and add the
// partner's copy of them, the others keep [HALF, 2 HALF).  The partner differs in bit OFF (and, for the
// DPP steps, in lower bits too, which the later steps pair up in turn).
template <int HALF, int OFF>
__device__ __forceinline__ void halve(float* v, int lane) {
    if constexpr (OFF == 32 || OFF == 16) {
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            float x, y;
            lane_swap<OFF>(v[j], v[j + HALF], x, y);
            v[j] = x + y;
        }
    } else {
        constexpr int M = OFF == 8 ? 15 : (OFF == 4 ? 7 : OFF);
        const bool upper = (lane & OFF) != 0;
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            float lo = v[j], hi = v[j + HALF];
            float send = upper ? lo : hi;
            float keep = upper ? hi : lo;
            v[j] = keep + dpp_xor<M>(send);
        }
    }
}

// Sum NV per-lane values over the wave; entry k of the total ends in the lanes with lane >> (6 - log2 NV)
// == k (for NV < 64 every such lane holds it; the lane with the low bits clear is used).
template <int NV>
__device__ __forceinline__ float wave_reduce_scatter(float* v, int lane) {
    static_assert(NV == 16 || NV == 32 || NV == 64, "NV");
    float s;
    if constexpr (NV == 16) {
        halve<8, 32>(v, lane); halve<4, 16>(v, lane); halve<2, 8>(v, lane); halve<1, 4>(v, lane);
        s = v[0];
        s += dpp_xor<2>(s);
        s += dpp_xor<1>(s);
    } else if constexpr (NV == 32) {
        halve<16, 32>(v, lane); halve<8, 16>(v, lane); halve<4, 8>(v, lane); halve<2, 4>(v, lane);
        halve<1, 2>(v, lane);
        s = v[0];
        s += dpp_xor<1>(s);
    } else {
        halve<32, 32>(v, lane); halve<16, 16>(v, lane); halve<8, 8>(v, lane); halve<4, 4>(v, lane);
        halve<2, 2>(v, lane); halve<1, 1>(v, lane);
        s = v[0];
    }
    return s;
}

}  // namespace ffrt
