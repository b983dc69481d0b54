// rfi_noalloc.hip -- rfi_mad_filter_noalloc: the int8 batch filter for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight real-time loops).
//
// rfi_mad_filter keeps a plan per argument signature: per-stream
// descriptors and a work-item table in device memory it allocates.  This
// variant keeps the same two tables in one file-scope device array,
// `scratch`, of fixed size, and writes them on the device: the per-stream
// parameters travel in kernel arguments (k_noalloc_tables, at most
// kNaChunk streams per launch), so the call makes no host-to-device copy
// and allocates nothing, on the device or on the host.  The filter launches
// that follow are those of rfi_mad_filter's untuned split schedule (one
// launch for the windows of irregular size or position, one per window
// class and mode), reading the tables from the scratch array, so the bytes
// written are identical.
//
// Each GPU holds its own copy of `scratch` at its own address, found once
// per device with hipGetSymbolAddress and used from then on; every call on
// one GPU rewrites the tables of the previous call, so calls that overlap on
// one GPU (two host threads, or two HIP streams not ordered by the caller)
// race on them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "rfi_internal.hpp"
#include "rfi_runtime.hpp"

namespace rfi {

constexpr int kNaMaxStreams = RFI_NOALLOC_MAX_STREAMS;
constexpr int64_t kNaScratchBytes = (int64_t)4 << 20;
constexpr int64_t kNaDescBytes = (int64_t)kNaMaxStreams * (int64_t)sizeof(StreamDesc);
constexpr int64_t kNaMaxItems = (kNaScratchBytes - kNaDescBytes) / (int64_t)sizeof(Item);
static_assert(kNaDescBytes % 256 == 0 && sizeof(Item) == 16, "items stay 16-byte aligned");
static_assert(kNaMaxItems == RFI_NOALLOC_MAX_ITEMS, "header limit");

// Descriptors at byte 0 (kNaMaxStreams entries), work items after them.
// Host code never names this array except in hipGetSymbolAddress: its
// host-side name is not a device address.
static __device__ __align__(256) uint8_t scratch[kNaScratchBytes];

namespace {

// Streams whose tables one k_noalloc_tables launch writes.
constexpr int kNaChunk = 32;

struct NaStream {
    int64_t length;
    int64_t x_off;          // first element (packed layout)
    int64_t stats_off;      // first window (packed statistics)
    int64_t tile_pos;       // index of its first tile item
    int64_t n_tiles;
    int64_t gen_pos;        // index of its first generic item
    int64_t first_generic;  // window index of its first generic item
    int64_t n_generic;
    int32_t window;
    float k;
    int32_t mode;
    int32_t pad;
};

struct NaArgs {
    StreamDesc* desc;
    Item* items;
    int32_t s0;  // stream index of st[0]
    int32_t n;   // streams in st
    int64_t tile_samples;
    NaStream st[kNaChunk];
};
static_assert(sizeof(NaArgs) <= 4096, "kernel arguments");

// blockIdx.y: stream of the chunk; the x dimension strides over its items.
// The host has checked that every index written lies inside the array.
__global__ __launch_bounds__(256) void k_noalloc_tables(NaArgs a)
{
    const int j = (int)blockIdx.y;
    if (j >= a.n) return;
    const NaStream& q = a.st[j];
    const int s = a.s0 + j;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        StreamDesc d;
        d.x_off = (uint64_t)q.x_off;
        d.y_off = (uint64_t)q.x_off;
        d.stats_off = (uint64_t)(q.stats_off * (int64_t)sizeof(rfi_window_stats));
        d.head_off = 0;
        d.length = q.length;
        d.abs_base = 0;
        d.window = q.window;
        d.k = q.k;
        d.mode = q.mode;
        d.key = (uint32_t)s;
        d.head_len = 0;
        d.flags = kPadded;
        a.desc[s] = d;
    }
    for (int64_t t = tid; t < q.n_tiles; t += stride)
        a.items[q.tile_pos + t] = Item{s, kItemTile, t * a.tile_samples};
    for (int64_t g = tid; g < q.n_generic; g += stride)
        a.items[q.gen_pos + g] = Item{s, kItemGeneric, q.first_generic + g};
}

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
uint8_t* g_na_ptr[kNaMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
int na_scratch(uint8_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kNaMaxDevices) return RFI_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p) return hip_fail(hipErrorInvalidSymbol);
        g_na_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_na_ptr[dev];
    return RFI_OK;
}

// Item groups in the order of the split schedule: generic items, then the
// tiles of window class c and mode m at 1 + 3 c + m.
constexpr int kNaGroups = 1 + kI8Classes * 3;
constexpr int64_t kNaTileSamples = kTileBytes;  // int8

// Per stream: tiles, first generic window and generic items (as plan_build).
void na_counts(int64_t L, int32_t W, int64_t& nt, int64_t& first_generic, int64_t& ngen, int& grp)
{
    const int64_t nw = (L + W - 1) / W;
    const int cls = i8_tile_class(W);
    nt = 0;
    first_generic = 0;
    if (cls >= 0) {
        nt = L / kNaTileSamples;
        first_generic = nt * (kNaTileSamples / W);
    }
    ngen = nw - first_generic;
    grp = cls;
}

// Occupancy cap of the untuned split schedule (as rfi_mad_filter's plans).
constexpr int kNaWgPerCu = 8;

}  // namespace
}  // namespace rfi

using namespace rfi;

extern "C" int rfi_mad_filter_noalloc(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                                      const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                                      rfi_window_stats* stats_out, void* stream)
{
    int rc = rfi_validate(1, x, y, n_streams, lengths, windows, k, mode, stats_out);
    if (rc != RFI_OK) return rc;
    int64_t total = 0;
    rfi_layout(n_streams, lengths, windows, nullptr, nullptr, &total);
    if (n_streams == 0 || total == 0) return RFI_OK;
    if (n_streams > kNaMaxStreams) return RFI_ERR_UNSUPPORTED;

    // Pass 1: items per group, the modes of the generic items and the
    // longest generic window (which picks the generic kernel's workgroup).
    int64_t count[kNaGroups] = {};
    int gen_modes = 0;
    int64_t gen_nmax = 0;
    for (int32_t s = 0; s < n_streams; ++s) {
        int64_t nt, fg, ng;
        int cls;
        na_counts(lengths[s], windows[s], nt, fg, ng, cls);
        if (nt > 0) count[1 + 3 * cls + mode[s]] += nt;
        if (ng > 0) {
            count[0] += ng;
            gen_modes |= 1 << mode[s];
            gen_nmax = std::max<int64_t>(gen_nmax, std::min<int64_t>(windows[s], lengths[s] - fg * windows[s]));
        }
    }
    int64_t begin[kNaGroups], n_items = 0;
    for (int g = 0; g < kNaGroups; ++g) {
        begin[g] = n_items;
        n_items += count[g];
        if (n_items > kNaMaxItems) return RFI_ERR_UNSUPPORTED;
    }

    uint8_t* base = nullptr;
    rc = na_scratch(&base);
    if (rc != RFI_OK) return rc;
    StreamDesc* desc = reinterpret_cast<StreamDesc*>(base);
    Item* items = reinterpret_cast<Item*>(base + kNaDescBytes);
    hipStream_t hs = (hipStream_t)stream;

    // Pass 2: the tables, kNaChunk streams per launch.
    int64_t cursor[kNaGroups];
    for (int g = 0; g < kNaGroups; ++g) cursor[g] = begin[g];
    int64_t soff = 0, woff = 0;
    NaArgs a;
    a.desc = desc;
    a.items = items;
    a.tile_samples = kNaTileSamples;
    for (int32_t s0 = 0; s0 < n_streams; s0 += kNaChunk) {
        a.s0 = s0;
        a.n = std::min<int32_t>(kNaChunk, n_streams - s0);
        int64_t most = 1;
        for (int j = 0; j < a.n; ++j) {
            const int32_t s = s0 + j;
            NaStream& q = a.st[j];
            int cls;
            na_counts(lengths[s], windows[s], q.n_tiles, q.first_generic, q.n_generic, cls);
            q.length = lengths[s];
            q.x_off = soff;
            q.stats_off = woff;
            q.window = windows[s];
            q.k = k[s];
            q.mode = mode[s];
            q.pad = 0;
            q.tile_pos = 0;
            if (q.n_tiles > 0) {
                int64_t& c = cursor[1 + 3 * cls + mode[s]];
                q.tile_pos = c;
                c += q.n_tiles;
            }
            q.gen_pos = cursor[0];
            cursor[0] += q.n_generic;
            most = std::max(most, std::max(q.n_tiles, q.n_generic));
            soff += (lengths[s] + 63) / 64 * 64;
            woff += (lengths[s] + windows[s] - 1) / windows[s];
        }
        const unsigned gx = (unsigned)std::min<int64_t>((most + 255) / 256, 256);
        hipLaunchKernelGGL(k_noalloc_tables, dim3(gx, (unsigned)a.n), dim3(256), 0, hs, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }

    // The filter launches of the split schedule.
    LaunchArgs la = {};
    la.streams = desc;
    la.seed = seed;
    la.x_base = (uint64_t)(uintptr_t)x;
    la.y_base = (uint64_t)(uintptr_t)y;
    la.stats_base = (uint64_t)(uintptr_t)stats_out;
    la.no_stats = stats_out ? 0 : 1;
    set_wg_per_cu(kNaWgPerCu);
    for (int g = 0; g < kNaGroups; ++g) {
        if (count[g] == 0) continue;
        la.items = items + begin[g];
        la.n_items = count[g];
        const int grid = (int)std::min<int64_t>(count[g], (int64_t)1 << 30);
        hipError_t e;
        if (g == 0) {
            const int small = gen_nmax <= 4066 ? 64 : gen_nmax <= 8162 ? 128 : 0;
            e = launch_i8_generic(la, gen_modes, grid, hs, small);
        } else {
            const int cls = (g - 1) / 3, m = (g - 1) % 3;
            e = launch_i8_tiles(cls, 1 << m, 1, la, grid, hs);
        }
        if (e != hipSuccess) return hip_fail(e);
    }
    return RFI_OK;
}
