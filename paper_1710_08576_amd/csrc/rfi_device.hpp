// rfi_device.hpp -- device helpers for the gfx950 kernels of librfimad.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfi {

// ------------------------------------------------------------------------
// Wave-level primitives (64-lane wavefronts).
// ------------------------------------------------------------------------

// Orders this wave's LDS accesses across lanes without a workgroup barrier:
// a wave's LDS instructions execute in issue order, so a compiler fence at
// wavefront scope is all that is needed.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Inclusive prefix sum within aligned groups of G lanes (G a power of two).
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v)
{
    const int l = lane_id() & (G - 1);
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, G);
        if (l >= d) v += t;
    }
    return v;
}

template <int G>
__device__ __forceinline__ int group_min(int v)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, G));
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t v)
{
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, G);
    return v;
}

// ------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies; the key is bumped by the two Weyl constants after
// every round.
// ------------------------------------------------------------------------
struct Philox4x64 {
    uint64_t w[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t ctr0, uint64_t key0, uint64_t key1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
    uint64_t a = ctr0, b = 0, c = 0, d = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa_lo = a * kMulA, pa_hi = __umul64hi(a, kMulA);
        const uint64_t pc_lo = c * kMulB, pc_hi = __umul64hi(c, kMulB);
        const uint64_t na = pc_hi ^ b ^ key0;
        const uint64_t nc = pa_hi ^ d ^ key1;
        a = na;
        b = pc_lo;
        c = nc;
        d = pa_lo;
        key0 += kWeylA;
        key1 += kWeylB;
    }
    Philox4x64 r;
    r.w[0] = a;
    r.w[1] = b;
    r.w[2] = c;
    r.w[3] = d;
    return r;
}

// ------------------------------------------------------------------------
// Packed-byte helpers for int8 samples held four to a dword.
// ------------------------------------------------------------------------
typedef short short2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_clamp_i16(uint32_t v, uint32_t lo, uint32_t hi)
{
    short2v a = __builtin_bit_cast(short2v, v);
    a = __builtin_elementwise_max(a, __builtin_bit_cast(short2v, lo));
    a = __builtin_elementwise_min(a, __builtin_bit_cast(short2v, hi));
    return __builtin_bit_cast(uint32_t, a);
}

// Byte-wise signed clamp of four int8 lanes to [lo, hi].  Each byte is
// moved to the high half of a 16-bit lane (value b * 256, sign kept), the
// two halves are clamped with packed i16 max/min, and the bytes are put back.
// lo256 / hi256: (lo * 256) and (hi * 256) replicated in both i16 halves.
__device__ __forceinline__ uint32_t clamp_i8x4(uint32_t x, uint32_t lo256, uint32_t hi256)
{
    const uint32_t odd = x & 0xFF00FF00u;           // bytes 1, 3
    const uint32_t even = (x << 8) & 0xFF00FF00u;   // bytes 0, 2
    const uint32_t oc = pk_clamp_i16(odd, lo256, hi256);
    const uint32_t ec = pk_clamp_i16(even, lo256, hi256);
    return oc | (ec >> 8);
}

// 0xFF in every byte of `diff` that is non-zero, 0x00 elsewhere.
__device__ __forceinline__ uint32_t nonzero_byte_mask(uint32_t diff)
{
    const uint32_t h = (((diff & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | diff) & 0x80808080u;
    return (h >> 7) * 0xFFu;
}

// 0xFFFF in every 16-bit half of `diff` that is non-zero.
__device__ __forceinline__ uint32_t nonzero_half_mask(uint32_t diff)
{
    const uint32_t h = (((diff & 0x7FFF7FFFu) + 0x7FFF7FFFu) | diff) & 0x80008000u;
    return (h >> 15) * 0xFFFFu;
}

__device__ __forceinline__ uint32_t rep_i16(int v)
{
    const uint32_t h = (uint32_t)v & 0xFFFFu;
    return h | (h << 16);
}

}  // namespace rfi
