// rfi_power.hip -- the improvement metric of Sec. III-A on the device.
//
// The paper scores a filter in dB as ten times the base-10 logarithm of
// S_U / S_F, S relating the mean of the integrated power to its RMS, before
// (U) and after (F) filtering.  Here the power is integrated over blocks of
// consecutive time samples:
//
//   rfi_block_power   P[s][b] = sum of x^2 over block b of stream s (exact,
//                     int64), one read of the samples;
//   rfi_improvement   per stream, S = the average over segments of
//                     seg_blocks whole blocks of (RMS deviation about the
//                     segment mean) / (segment mean), for the unfiltered and
//                     the filtered powers, and I = 10 log10(S_U / S_F)
//                     (binary64; positive when filtering steadies the power).
//
// Block power is HBM-bound (1 or 2 B per sample read, 8 B per block
// written).  A workgroup sums one part of at most 64 KiB of one block with
// 16-B loads (int8: v_dot4 of each word with itself; int16: v_dot2 of the
// absolute values), so a large block is spread over many workgroups; the
// parts of a block are then added by a second small kernel.  Work tables
// are kept per (lengths, block) signature and stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rfi_device.hpp"
#include "rfi_mad.h"
#include "rfi_runtime.hpp"

namespace rfi {

namespace {

constexpr int kPowBlock = 256;
constexpr int64_t kPartBytes = 65536;

struct PowRow {
    int64_t x_off;        // first element of the stream in the packed batch
    int64_t length;       // samples
    int64_t part_begin;   // first part of the stream (global part index)
    int64_t block_begin;  // first block of the stream (global block index)
};

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

// Bytes of the 32-bit word at byte address a that lie in [lo, hi).
__device__ __forceinline__ uint32_t byte_range_mask(int64_t a, int64_t lo, int64_t hi)
{
    const int64_t j0 = min64(max64(lo - a, 0), 4);
    const int64_t j1 = min64(max64(hi - a, 0), 4);
    const uint32_t below_hi = j1 >= 4 ? 0xFFFFFFFFu : ((1u << (8 * j1)) - 1u);
    const uint32_t below_lo = j0 >= 4 ? 0xFFFFFFFFu : ((1u << (8 * j0)) - 1u);
    return below_hi & ~below_lo;
}

template <int ELEM>
__device__ __forceinline__ void accumulate_word(uint32_t w, int32_t& acc8, uint64_t& acc16)
{
    if constexpr (ELEM == 1) {
        acc8 = __builtin_amdgcn_sdot4((int)w, (int)w, acc8, false);
    } else {
        const int lo = (int)(int16_t)(w & 0xFFFFu), hi = (int)(int16_t)(w >> 16);
        us2 a;
        a.x = (unsigned short)(lo < 0 ? -lo : lo);  // 32768 for -32768
        a.y = (unsigned short)(hi < 0 ? -hi : hi);
        acc16 += __builtin_amdgcn_udot2(a, a, 0u, false);  // <= 2^31, no wrap
    }
}

__device__ __forceinline__ int find_row(const PowRow* rows, int n, int64_t idx, bool by_part)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = by_part ? rows[mid].part_begin : rows[mid].block_begin;
        if (b <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint64_t block_reduce_u64(uint64_t v, uint64_t* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int tid = (int)threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    uint64_t t = 0;
    if (tid == 0)
        for (int i = 0; i < kPowBlock / 64; ++i) t += red[i];
    return t;
}

// One workgroup per part.  ppb: parts per whole block; direct: ppb == 1,
// the part sum is the block's power.
template <int ELEM>
__global__ __launch_bounds__(kPowBlock) void k_block_power(const uint8_t* x, const PowRow* rows,
                                                           int n_rows, int64_t block, int64_t ppb,
                                                           int64_t* parts, int64_t* power, int direct)
{
    __shared__ uint64_t red[kPowBlock / 64];
    const int64_t part = (int64_t)blockIdx.x;
    const int s = find_row(rows, n_rows, part, true);
    const PowRow r = rows[s];
    const int64_t i = part - r.part_begin;
    const int64_t b = i / ppb, p = i % ppb;
    constexpr int64_t kPartElems = kPartBytes / ELEM;
    const int64_t blo = b * block + p * kPartElems;
    const int64_t bhi = min64(min64(blo + kPartElems, (b + 1) * block), r.length);
    // Byte range of the part, relative to the stream's first element.
    const int64_t lo = blo * ELEM, hi = bhi * ELEM;
    const uint8_t* base = x + r.x_off * ELEM;
    const int64_t c0 = lo >> 4, c1 = (hi + 15) >> 4;  // 16-B chunks touching the part
    int32_t acc8 = 0;
    uint64_t acc16 = 0;
    const int tid = (int)threadIdx.x;
    int64_t c = c0 + tid;
    // Four chunks in flight per thread; every chunk read ends inside the
    // stream's 64-element padded extent (c1 * 16 <= align16(L * ELEM)).
    for (; c + 3 * kPowBlock < c1; c += 4 * kPowBlock) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = gload16_nt(base + 16 * (c + u * kPowBlock));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t a = 16 * (c + u * kPowBlock);
            uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
            if (a < lo || a + 16 > hi) {
#pragma unroll
                for (int q = 0; q < 4; ++q) w[q] &= byte_range_mask(a + 4 * q, lo, hi);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) accumulate_word<ELEM>(w[q], acc8, acc16);
        }
    }
    for (; c < c1; c += kPowBlock) {
        const uint4 v = gload16_nt(base + 16 * c);
        const int64_t a = 16 * c;
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[q] &= byte_range_mask(a + 4 * q, lo, hi);
            accumulate_word<ELEM>(w[q], acc8, acc16);
        }
    }
    const uint64_t mine = ELEM == 1 ? (uint64_t)(int64_t)acc8 : acc16;
    const uint64_t total = block_reduce_u64(mine, red);
    if (tid == 0) {
        if (direct) gstore(power + r.block_begin + b, (int64_t)total);
        else gstore(parts + part, (int64_t)total);
    }
}

// One thread per block: the sum of its parts.
__global__ __launch_bounds__(kPowBlock) void k_block_power_sum(const PowRow* rows, int n_rows,
                                                               int64_t block, int64_t ppb, int64_t n_blocks,
                                                               const int64_t* parts, int64_t* power, int elem)
{
    const int64_t g = (int64_t)blockIdx.x * kPowBlock + threadIdx.x;
    if (g >= n_blocks) return;
    const int s = find_row(rows, n_rows, g, false);
    const PowRow r = rows[s];
    const int64_t b = g - r.block_begin;
    const int64_t part_elems = kPartBytes / elem;
    const int64_t len = min64(block, r.length - b * block);
    const int64_t np = (len + part_elems - 1) / part_elems;
    const int64_t* src = parts + r.part_begin + b * ppb;
    int64_t t = 0;
    for (int64_t i = 0; i < np; ++i) t += src[i];
    gstore(power + g, t);
}

// S of n_seg segments of seg consecutive values: per segment two passes
// (mean, then squared deviations) in binary64, the segment's RMS deviation
// over its mean, each thread a strided set of segments, then the average by
// a fixed-shape tree over threads.
__device__ double s_ratio_avg(const int64_t* p, int64_t n_seg, int32_t seg, double* red)
{
    const int tid = (int)threadIdx.x;
    double acc = 0.0;
    for (int64_t j = tid; j < n_seg; j += kPowBlock) {
        const int64_t* v = p + j * seg;
        double sum = 0.0;
        for (int32_t i = 0; i < seg; ++i) sum += (double)v[i];
        const double mu = sum / (double)seg;
        double dev = 0.0;
        for (int32_t i = 0; i < seg; ++i) {
            const double d = (double)v[i] - mu;
            dev += d * d;
        }
        acc += sqrt(dev / (double)seg) / mu;
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = kPowBlock / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0] / (double)n_seg;
    __syncthreads();
    return r;
}

// One workgroup per stream: out[3s..3s+2] = S_U, S_F, I (dB).
__global__ __launch_bounds__(kPowBlock) void k_improvement(const PowRow* rows, int64_t block, int32_t seg,
                                                           const int64_t* pu, const int64_t* pf, double* out)
{
    __shared__ double red[kPowBlock];
    const int s = (int)blockIdx.x;
    const PowRow r = rows[s];
    const int64_t n_seg = (r.length / block) / seg;
    double su, sf;
    if (n_seg == 0) {
        su = sf = __builtin_nan("");
    } else {
        su = s_ratio_avg(pu + r.block_begin, n_seg, seg, red);
        sf = s_ratio_avg(pf + r.block_begin, n_seg, seg, red);
    }
    if (threadIdx.x == 0) {
        gstore(out + 3 * s, su);
        gstore(out + 3 * s + 1, sf);
        gstore(out + 3 * s + 2, 10.0 * log10(su / sf));
    }
}

// ---------------------------------------------------------------------------
// Host side: per-signature tables.
// ---------------------------------------------------------------------------
struct PowKey {
    int device;
    uintptr_t stream;  // the parts buffer is per stream: calls on one stream are ordered
    int elem;          // 0: improvement only (no parts)
    int32_t block;
    std::vector<int64_t> L;
    bool operator<(const PowKey& o) const
    {
        if (device != o.device) return device < o.device;
        if (stream != o.stream) return stream < o.stream;
        if (elem != o.elem) return elem < o.elem;
        if (block != o.block) return block < o.block;
        return L < o.L;
    }
};

struct PowPlan {
    PowRow* d_rows = nullptr;
    int64_t* d_parts = nullptr;
    int32_t n_rows = 0;
    int64_t n_parts = 0, n_blocks = 0, ppb = 1;
    int device = 0;
};

std::mutex g_pow_mu;
std::map<PowKey, PowPlan*> g_pow;
std::vector<PowKey> g_pow_order;
constexpr size_t kPowCacheMax = 8;

void pow_free(PowPlan* p)
{
    if (!p) return;
    // the plan's kernels run on its own device, which need not be current
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_rows);
    (void)hipFree(p->d_parts);
    if (have && cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

// Rows, part and block counts of a batch; false if a count overflows.
bool pow_rows(int elem, int32_t n, const int64_t* L, int32_t block, std::vector<PowRow>& rows,
              int64_t& n_parts, int64_t& n_blocks, int64_t& ppb, int64_t& total_elems)
{
    const int64_t part_elems = kPartBytes / std::max(elem, 1);
    ppb = ((int64_t)block + part_elems - 1) / part_elems;
    rows.resize(n);
    int64_t off = 0, parts = 0, blocks = 0;
    for (int32_t s = 0; s < n; ++s) {
        const int64_t nb = (L[s] + block - 1) / block;
        const int64_t full = L[s] / block, last = L[s] - full * block;
        rows[s] = PowRow{off, L[s], parts, blocks};
        parts += full * ppb + (last + part_elems - 1) / part_elems;
        blocks += nb;
        off += (L[s] + 63) / 64 * 64;
        if (parts > ((int64_t)1 << 31) - 1) return false;
    }
    n_parts = parts;
    n_blocks = blocks;
    total_elems = off;
    return true;
}

int pow_plan(int elem, int32_t n, const int64_t* L, int32_t block, hipStream_t stream, PowPlan** out)
{
    PowKey key;
    if (hipGetDevice(&key.device) != hipSuccess) key.device = 0;
    key.stream = (uintptr_t)stream;
    key.elem = elem;
    key.block = block;
    key.L.assign(L, L + n);
    auto it = g_pow.find(key);
    if (it != g_pow.end()) {
        *out = it->second;
        return RFI_OK;
    }
    std::vector<PowRow> rows;
    PowPlan* p = new PowPlan;
    int64_t total = 0;
    if (!pow_rows(elem, n, L, block, rows, p->n_parts, p->n_blocks, p->ppb, total)) {
        delete p;
        return RFI_ERR_INVALID;
    }
    p->n_rows = n;
    p->device = key.device;
    hipError_t e = hipMalloc(&p->d_rows, sizeof(PowRow) * rows.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_rows, rows.data(), sizeof(PowRow) * rows.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && elem > 0 && p->ppb > 1 && p->n_parts > 0)
        e = hipMalloc(&p->d_parts, sizeof(int64_t) * p->n_parts);
    if (e != hipSuccess) {
        pow_free(p);
        return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
    }
    if (g_pow.size() >= kPowCacheMax) {
        auto old = g_pow.find(g_pow_order.front());
        pow_free(old->second);
        g_pow.erase(old);
        g_pow_order.erase(g_pow_order.begin());
    }
    g_pow[key] = p;
    g_pow_order.push_back(key);
    *out = p;
    return RFI_OK;
}

bool lengths_ok(int32_t n, const int64_t* L)
{
    if (n < 0 || (n > 0 && !L)) return false;
    for (int32_t s = 0; s < n; ++s)
        if (L[s] < 0 || L[s] > ((int64_t)1 << 61)) return false;
    return true;
}

}  // namespace

void power_shutdown()
{
    std::lock_guard<std::mutex> g(g_pow_mu);
    for (auto& kv : g_pow) pow_free(kv.second);
    g_pow.clear();
    g_pow_order.clear();
}

}  // namespace rfi

using namespace rfi;

extern "C" {

int rfi_block_power(const void* x, int32_t elem_bytes, int32_t n_streams, const int64_t* lengths,
                    int32_t block, int64_t* power_out, void* stream)
{
    if ((elem_bytes != 1 && elem_bytes != 2) || block < 1 || block > RFI_MAX_BLOCK) return RFI_ERR_INVALID;
    if (!lengths_ok(n_streams, lengths)) return RFI_ERR_INVALID;
    std::vector<PowRow> rows;
    int64_t n_parts = 0, n_blocks = 0, ppb = 1, total = 0;
    if (!pow_rows(elem_bytes, n_streams, lengths, block, rows, n_parts, n_blocks, ppb, total))
        return RFI_ERR_INVALID;
    if (n_blocks == 0) return RFI_OK;
    if (!x || !power_out) return RFI_ERR_INVALID;
    if (((uintptr_t)x & 15u) || ((uintptr_t)power_out & 7u)) return RFI_ERR_ALIGN;
    const uintptr_t xa = (uintptr_t)x, xb = (uintptr_t)(total * elem_bytes);
    const uintptr_t pa = (uintptr_t)power_out, pb = (uintptr_t)(n_blocks * 8);
    if (pa < xa + xb && xa < pa + pb) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(g_pow_mu);
    PowPlan* p = nullptr;
    int rc = pow_plan(elem_bytes, n_streams, lengths, block, (hipStream_t)stream, &p);
    if (rc != RFI_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int direct = p->ppb == 1 ? 1 : 0;
    const uint8_t* xb8 = static_cast<const uint8_t*>(x);
    if (elem_bytes == 1)
        hipLaunchKernelGGL(k_block_power<1>, dim3((unsigned)p->n_parts), dim3(kPowBlock), 0, s, xb8, p->d_rows,
                           p->n_rows, (int64_t)block, p->ppb, p->d_parts, power_out, direct);
    else
        hipLaunchKernelGGL(k_block_power<2>, dim3((unsigned)p->n_parts), dim3(kPowBlock), 0, s, xb8, p->d_rows,
                           p->n_rows, (int64_t)block, p->ppb, p->d_parts, power_out, direct);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && !direct) {
        const int64_t grid = (p->n_blocks + kPowBlock - 1) / kPowBlock;
        hipLaunchKernelGGL(k_block_power_sum, dim3((unsigned)grid), dim3(kPowBlock), 0, s, p->d_rows, p->n_rows,
                           (int64_t)block, p->ppb, p->n_blocks, p->d_parts, power_out, (int)elem_bytes);
        e = hipGetLastError();
    }
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

int rfi_improvement(const int64_t* power_u, const int64_t* power_f, int32_t n_streams, const int64_t* lengths,
                    int32_t block, int32_t seg_blocks, double* out, void* stream)
{
    if (block < 1 || block > RFI_MAX_BLOCK || seg_blocks < 1) return RFI_ERR_INVALID;
    if (!lengths_ok(n_streams, lengths)) return RFI_ERR_INVALID;
    if (n_streams == 0) return RFI_OK;
    if (!out) return RFI_ERR_INVALID;
    if ((uintptr_t)out & 7u) return RFI_ERR_ALIGN;
    int64_t n_blocks = 0;
    for (int32_t s = 0; s < n_streams; ++s) n_blocks += (lengths[s] + block - 1) / block;
    if (n_blocks > 0) {
        if (!power_u || !power_f) return RFI_ERR_INVALID;
        if (((uintptr_t)power_u | (uintptr_t)power_f) & 7u) return RFI_ERR_ALIGN;
        const uintptr_t oa = (uintptr_t)out, ob = (uintptr_t)(24 * (int64_t)n_streams);
        const uintptr_t pb = (uintptr_t)(8 * n_blocks);
        for (const int64_t* q : {power_u, power_f}) {
            const uintptr_t qa = (uintptr_t)q;
            if (oa < qa + pb && qa < oa + ob) return RFI_ERR_INVALID;
        }
    }
    std::lock_guard<std::mutex> g(g_pow_mu);
    PowPlan* p = nullptr;
    int rc = pow_plan(0, n_streams, lengths, block, (hipStream_t)stream, &p);
    if (rc != RFI_OK) return rc;
    hipLaunchKernelGGL(k_improvement, dim3((unsigned)n_streams), dim3(kPowBlock), 0, (hipStream_t)stream,
                       p->d_rows, (int64_t)block, seg_blocks, power_u, power_f, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

}  // extern "C"
