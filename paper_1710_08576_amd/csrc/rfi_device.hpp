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

// DPP lane move with zero fill: lanes whose source is outside the row (or
// whose row is masked off) receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp0(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// Inclusive prefix sum within aligned groups of G lanes (G a power of two,
// G <= 64), on DPP row shifts and row broadcasts (no LDS round trip).
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v)
{
    if constexpr (G >= 2) {
        const int l = lane_id() & 15;
        uint32_t t = dpp0<0x111>(v);  // row_shr:1
        v += (G >= 16 || (l & (G - 1)) >= 1) ? t : 0u;
        if constexpr (G >= 4) {
            t = dpp0<0x112>(v);  // row_shr:2
            v += (G >= 16 || (l & (G - 1)) >= 2) ? t : 0u;
        }
        if constexpr (G >= 8) {
            t = dpp0<0x114>(v);  // row_shr:4
            v += (G >= 16 || (l & (G - 1)) >= 4) ? t : 0u;
        }
        if constexpr (G >= 16) v += dpp0<0x118>(v);        // row_shr:8
        if constexpr (G >= 32) v += dpp0<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
        if constexpr (G >= 64) v += dpp0<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    }
    return v;
}

// Bits of a where m is set, of b elsewhere (one v_bfi_b32).
__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b)
{
    return (a & m) | (b & ~m);
}

// Number of lanes of this lane's aligned group of G whose predicate holds.
template <int G>
__device__ __forceinline__ int group_count(bool pred)
{
    const uint64_t b = __ballot(pred);
    if constexpr (G == 64) {
        return (int)__popcll(b);
    } else {
        const int shift = lane_id() & ~(G - 1);
        return (int)__popc((uint32_t)(b >> shift) & (uint32_t)((1ull << G) - 1));
    }
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
// Global-memory access.  Stream addresses are rebuilt from integer offsets,
// so the compiler cannot see that they point to global memory; these casts
// keep the sample traffic on global_load/global_store instead of flat.
// ------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_cu32x4;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

__device__ __forceinline__ uint4 gload16(const void* p)
{
    const u32x4 t = *(g_cu32x4*)p;
    return make_uint4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ void gstore16(void* p, uint4 v)
{
    u32x4 t;
    t.x = v.x;
    t.y = v.y;
    t.z = v.z;
    t.w = v.w;
    *(g_u32x4*)p = t;
}

// Non-temporal variants for the sample stream (read once, written once).
__device__ __forceinline__ uint4 gload16_nt(const void* p)
{
    const u32x4 t = __builtin_nontemporal_load((g_cu32x4*)p);
    return make_uint4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ void gstore16_nt(void* p, uint4 v)
{
    u32x4 t;
    t.x = v.x;
    t.y = v.y;
    t.z = v.z;
    t.w = v.w;
    __builtin_nontemporal_store(t, (g_u32x4*)p);
}

template <typename T>
__device__ __forceinline__ T gload(const T* p)
{
    return *(__attribute__((address_space(1))) const T*)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// Keeps the scheduler from hoisting work across this point (limits the
// number of live registers in long unrolled sequences).
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Pins a wave-uniform running sum in a scalar register at this point of
// the program (an empty asm statement, no instruction): without it the
// compiler reassociates a chain of ballot popcounts and keeps every ballot
// mask alive until the end of the chain.
__device__ __forceinline__ void pin_sgpr(uint32_t& x) { asm volatile("" : "+s"(x)); }

// ------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies; the key is bumped by the two Weyl constants after
// every round.
// ------------------------------------------------------------------------
struct Philox4x64 {
    uint64_t w[4];
};

// Full 64 x 64 -> 128-bit product from four 32 x 32 -> 64 partial products,
// each a single v_mad_u64_u32 with the carry-in folded into the addend.
__device__ __forceinline__ void mul64_wide(uint64_t a, uint64_t k, uint64_t& lo, uint64_t& hi)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t k0 = (uint32_t)k, k1 = (uint32_t)(k >> 32);
    const uint64_t p00 = (uint64_t)a0 * k0;
    const uint64_t t = (uint64_t)a0 * k1 + (p00 >> 32);
    const uint64_t u = (uint64_t)a1 * k0 + (uint32_t)t;
    lo = (uint64_t)(uint32_t)p00 | (u << 32);
    hi = (uint64_t)a1 * k1 + (t >> 32) + (u >> 32);
}

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t ctr0, uint64_t key0, uint64_t key1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
    uint64_t a = ctr0, b = 0, c = 0, d = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t pa_lo, pa_hi, pc_lo, pc_hi;
        mul64_wide(a, kMulA, pa_lo, pa_hi);
        mul64_wide(c, kMulB, pc_lo, pc_hi);
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

typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_usubsat(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(ushort2v, a),
                                                                      __builtin_bit_cast(ushort2v, b)));
}

// min(a, 1) in both unsigned 16-bit halves, as one v_pk_min_u16 (the
// generic form is split by the compiler into per-half compares).  The
// constant 0x00010001 comes from a scalar register: an inline constant in a
// packed instruction would feed only the low half.
__device__ __forceinline__ uint32_t pk_umin1(uint32_t a)
{
    uint32_t r;
    asm volatile("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "s"(0x00010001u));
    return r;
}

// Byte-permute selector of the int8 samples of x outside [lo, hi]: byte k
// of the result is k for a kept sample and k + 4 for a flagged one, so
// v_perm_b32(other, x, sel) takes flagged bytes from `other` (0 for zeroing,
// noise bytes for noise).  lo_u / hi_u: (lo + 128) << 8 and (hi + 128) << 8
// in both 16-bit halves.  The bytes are biased to unsigned and moved to the
// high byte of 16-bit lanes; a saturating subtract is non-zero exactly when
// a bound is crossed.
__device__ __forceinline__ uint32_t flag_sel_i8x4(uint32_t x, uint32_t lo_u, uint32_t hi_u)
{
    const uint32_t xb = x ^ 0x80808080u;
    const uint32_t odd = xb & 0xFF00FF00u;          // bytes 1, 3
    const uint32_t even = (xb << 8) & 0xFF00FF00u;  // bytes 0, 2
    const uint32_t fo = pk_umin1(pk_usubsat(lo_u, odd) | pk_usubsat(odd, hi_u));
    const uint32_t fe = pk_umin1(pk_usubsat(lo_u, even) | pk_usubsat(even, hi_u));
    return 0x03020100u | (fo << 10) | (fe << 2);
}

__device__ __forceinline__ uint32_t byte_perm(uint32_t hi_src, uint32_t lo_src, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi_src, lo_src, sel);
}

// 0xFF in every byte of `diff` that is non-zero, 0x00 elsewhere.
__device__ __forceinline__ uint32_t nonzero_byte_mask(uint32_t diff)
{
    const uint32_t h = (((diff & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | diff) & 0x80808080u;
    // 0x80 -> 0xFF per byte: (0x80 << 1) - (0x80 >> 7) = 0xFF, modulo 2^32 at
    // the top byte (no full-width multiply).
    return (h << 1) - (h >> 7);
}

// 0xFFFF in every 16-bit half of `diff` that is non-zero.
__device__ __forceinline__ uint32_t nonzero_half_mask(uint32_t diff)
{
    const uint32_t h = (((diff & 0x7FFF7FFFu) + 0x7FFF7FFFu) | diff) & 0x80008000u;
    return (h << 1) - (h >> 15);
}

// |a - b| of the two int16 halves, as uint16 halves (0 .. 65535).
__device__ __forceinline__ uint32_t pk_absdiff_i16(uint32_t a, uint32_t b)
{
    const short2v x = __builtin_bit_cast(short2v, a), y = __builtin_bit_cast(short2v, b);
    const ushort2v hi = __builtin_bit_cast(ushort2v, __builtin_elementwise_max(x, y));
    const ushort2v lo = __builtin_bit_cast(ushort2v, __builtin_elementwise_min(x, y));
    return __builtin_bit_cast(uint32_t, (ushort2v)(hi - lo));
}

// Unsigned 16-bit lane arithmetic on two halves (v_pk_* instructions).
__device__ __forceinline__ uint32_t pk_sub_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, (ushort2v)(__builtin_bit_cast(ushort2v, a) - __builtin_bit_cast(ushort2v, b)));
}

__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(ushort2v, a),
                                                                  __builtin_bit_cast(ushort2v, b)));
}

__device__ __forceinline__ uint32_t pk_shl2_u16(uint32_t a)
{
    return __builtin_bit_cast(uint32_t, (ushort2v)(__builtin_bit_cast(ushort2v, a) << (ushort2v){2, 2}));
}

// 0xFFFF in every 16-bit half of `diff` that is non-zero: min(half, 1)
// subtracted from zero.
__device__ __forceinline__ uint32_t pk_mask_nonzero_u16(uint32_t diff)
{
    return pk_sub_u16(0u, pk_umin1(diff));
}

__device__ __forceinline__ uint32_t rep_i16(int v)
{
    const uint32_t h = (uint32_t)v & 0xFFFFu;
    return h | (h << 16);
}

}  // namespace rfi
