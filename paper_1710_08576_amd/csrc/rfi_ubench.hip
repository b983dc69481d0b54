// rfi_ubench.hip -- HBM copy microbenchmark (see rfi_ubench.h).
#include <hip/hip_runtime.h>

#include "rfi_device.hpp"
#include "rfi_ubench.h"

namespace rfi {

// LANE_MAJOR: each lane's 64 bytes are contiguous (loads 16 bytes apart);
// otherwise each load instruction of a wave covers 1 KiB contiguously.
template <bool NT, bool LANE_MAJOR = false>
__global__ __launch_bounds__(256) void k_copy_tile(const uint8_t* __restrict__ x, uint8_t* __restrict__ y)
{
    constexpr int kLaneStride = LANE_MAJOR ? 64 : 16;
    constexpr int kLoadStride = LANE_MAJOR ? 16 : 1024;
    const size_t base = (size_t)blockIdx.x * 16384 + (threadIdx.x >> 6) * 4096 + (threadIdx.x & 63) * kLaneStride;
    uint4 v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if constexpr (NT) {
            const u32x4 t = __builtin_nontemporal_load((const u32x4*)(x + base + i * kLoadStride));
            v[i] = make_uint4(t.x, t.y, t.z, t.w);
        } else {
            v[i] = gload16(x + base + i * kLoadStride);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if constexpr (NT) {
            u32x4 t;
            t.x = v[i].x;
            t.y = v[i].y;
            t.z = v[i].z;
            t.w = v[i].w;
            __builtin_nontemporal_store(t, (u32x4*)(y + base + i * kLoadStride));
        } else {
            gstore16(y + base + i * kLoadStride, v[i]);
        }
    }
}

// As k_copy_tile<true>, but lanes 8g .. 8g+7 (mod 32) take their four
// loads in the rotated order (t + g) mod 4: each load instruction then
// covers eight 128-byte segments of four 1 KiB blocks.
__global__ __launch_bounds__(256) void k_copy_tile_rot(const uint8_t* __restrict__ x, uint8_t* __restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int g = (lane >> 3) & 3;
    const size_t base = (size_t)blockIdx.x * 16384 + (threadIdx.x >> 6) * 4096 + lane * 16;
    u32x4 v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = __builtin_nontemporal_load((const u32x4*)(x + base + ((t + g) & 3) * 1024));
#pragma unroll
    for (int t = 0; t < 4; ++t) __builtin_nontemporal_store(v[t], (u32x4*)(y + base + ((t + g) & 3) * 1024));
}

__global__ __launch_bounds__(256) void k_copy_stride(const uint8_t* __restrict__ x, uint8_t* __restrict__ y,
                                                     size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
        gstore16(y + i * 16, gload16(x + i * 16));
}

// LDS histogram rate: each workgroup loads a 16 KiB tile in the filter's
// shape (64 B per lane, four 16-byte loads at a 1 KiB stride) and counts its
// bytes into per-wave LDS histograms of R replicas (replica = lane % R,
// 264-word stride, as the int8 tile kernels do), one LDS atomic per sample;
// the workgroup's totals are then added to row (workgroup % 256) of a
// 256 x 256 global array (spreading the global atomics over rows keeps
// their contention out of the measurement).
template <int R>
__global__ __launch_bounds__(256) void k_lds_hist(const uint8_t* __restrict__ x, uint32_t* __restrict__ out)
{
    constexpr int kStride = 264;
    __shared__ __align__(16) uint32_t h[4 * R * kStride];
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t* hw = h + wave * R * kStride;
    for (int j = lane * 4; j < R * kStride; j += 256) *reinterpret_cast<uint4*>(hw + j) = make_uint4(0, 0, 0, 0);
    const uint8_t* xt = x + (size_t)blockIdx.x * 16384 + wave * 4096 + lane * 16;
    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 t = gload16_nt(xt + i * 1024);
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
    }
    wave_sync();
    uint32_t* hl = hw + (lane % R) * kStride;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        atomicAdd(hl + (v[q] & 0xFFu), 1u);
        atomicAdd(hl + ((v[q] >> 8) & 0xFFu), 1u);
        atomicAdd(hl + ((v[q] >> 16) & 0xFFu), 1u);
        atomicAdd(hl + (v[q] >> 24), 1u);
        sched_fence();
    }
    __syncthreads();
    const int bin = (int)threadIdx.x;
    uint32_t t = 0;
    for (int w = 0; w < 4; ++w)
        for (int r = 0; r < R; ++r) t += h[(w * R + r) * kStride + bin];
    if (t) atomicAdd(out + (blockIdx.x & 255u) * 256u + bin, t);
}

}  // namespace rfi

extern "C" int rfi_ubench_lds_hist(const void* x, uint64_t bytes, int32_t replicas, uint32_t* hist_out,
                                   void* stream)
{
    if (!x || !hist_out || bytes == 0 || bytes % 16384 != 0) return -1;
    if (replicas != 1 && replicas != 2 && replicas != 4 && replicas != 8) return -1;
    if (((uintptr_t)x & 15u) || ((uintptr_t)hist_out & 3u)) return -2;
    const uint64_t tiles = bytes / 16384;
    if (tiles > (1u << 30)) return -1;
    const uint8_t* xs = static_cast<const uint8_t*>(x);
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((unsigned)tiles), b(256);
    if (replicas == 1) hipLaunchKernelGGL(rfi::k_lds_hist<1>, g, b, 0, s, xs, hist_out);
    else if (replicas == 2) hipLaunchKernelGGL(rfi::k_lds_hist<2>, g, b, 0, s, xs, hist_out);
    else if (replicas == 4) hipLaunchKernelGGL(rfi::k_lds_hist<4>, g, b, 0, s, xs, hist_out);
    else hipLaunchKernelGGL(rfi::k_lds_hist<8>, g, b, 0, s, xs, hist_out);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int rfi_ubench_copy(const void* x, void* y, uint64_t bytes, int32_t variant, void* stream)
{
    if (!x || !y || bytes == 0 || bytes % 16384 != 0 || variant < 0 || variant > 4) return -1;
    if (((uintptr_t)x | (uintptr_t)y) & 15u) return -2;
    const uint8_t* xs = static_cast<const uint8_t*>(x);
    uint8_t* ys = static_cast<uint8_t*>(y);
    if (xs < ys + bytes && ys < xs + bytes) return -1;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t tiles = bytes / 16384;
    if (tiles > (1u << 30)) return -1;
    if (variant == 0) hipLaunchKernelGGL(rfi::k_copy_tile<false>, dim3((unsigned)tiles), dim3(256), 0, s, xs, ys);
    else if (variant == 1) hipLaunchKernelGGL(rfi::k_copy_tile<true>, dim3((unsigned)tiles), dim3(256), 0, s, xs, ys);
    else if (variant == 4) hipLaunchKernelGGL(rfi::k_copy_tile_rot, dim3((unsigned)tiles), dim3(256), 0, s, xs, ys);
    else if (variant == 3) {
        auto k = rfi::k_copy_tile<true, true>;
        hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), 0, s, xs, ys);
    }
    else {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        hipLaunchKernelGGL(rfi::k_copy_stride, dim3((unsigned)(cus * 8)), dim3(256), 0, s, xs, ys, (size_t)(bytes / 16));
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}
