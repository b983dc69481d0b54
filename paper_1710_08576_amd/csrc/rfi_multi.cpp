// rfi_multi.cpp -- several outputs from one read of an int8 batch.
//
// Each output o has its own threshold multiple and replacement mode per
// stream; output o is bit-identical to rfi_mad_filter with that output's k
// and mode.  Outputs with no noise stream share one read: tiles of whole
// windows (W a tile class) are read once and written once per output by
// k_i8_multi; the remaining windows (stream tails, irregular W) go through
// the generic kernel once per output.  An output with noise streams is a
// single-output call of its own (a noise output in the shared kernel keeps
// a second copy of the tile and the pooled draws in registers, which cost
// more occupancy than a second read saves).  Work tables are kept per
// argument signature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rfi_runtime.hpp"

using namespace rfi;

namespace {

int64_t align64(int64_t n) { return (n + 63) / 64 * 64; }

struct MultiKey {
    int device;
    uint64_t seed;
    int32_t n_out;
    std::vector<int64_t> L;
    std::vector<int32_t> W;
    std::vector<uint32_t> K;
    std::vector<int32_t> M;
    bool operator<(const MultiKey& o) const
    {
        if (device != o.device) return device < o.device;
        if (seed != o.seed) return seed < o.seed;
        if (n_out != o.n_out) return n_out < o.n_out;
        if (L != o.L) return L < o.L;
        if (W != o.W) return W < o.W;
        if (K != o.K) return K < o.K;
        return M < o.M;
    }
};

struct MultiPlan {
    int32_t n_out = 0;
    uint64_t seed = 0;
    StreamDesc* d_desc[3] = {nullptr, nullptr, nullptr};
    Item* d_items = nullptr;
    std::vector<int64_t> cls_begin, cls_count;  // tile items per class, then generic
    int64_t gen_begin = 0, gen_count = 0;
    int device = 0;  // the plan's buffers and kernels live here
};

void multi_free(MultiPlan* p)
{
    if (!p) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (auto* d : p->d_desc) (void)hipFree(d);
    (void)hipFree(p->d_items);
    if (have && cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

int multi_build(int32_t n_out, int32_t n, const int64_t* L, const int32_t* W, const float* K,
                const int32_t* M, uint64_t seed, MultiPlan** out)
{
    MultiPlan* p = new MultiPlan;
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    p->n_out = n_out;
    p->seed = seed;
    std::vector<std::vector<Item>> groups(kI8Classes + 1);
    std::vector<std::vector<StreamDesc>> desc(n_out, std::vector<StreamDesc>(n));
    int64_t soff = 0, woff = 0;
    for (int s = 0; s < n; ++s) {
        for (int o = 0; o < n_out; ++o) {
            StreamDesc& d = desc[o][s];
            std::memset(&d, 0, sizeof(d));
            d.x_off = (uint64_t)soff;
            d.y_off = (uint64_t)soff;
            d.stats_off = (uint64_t)(woff * (int64_t)sizeof(rfi_window_stats));
            d.length = L[s];
            d.window = W[s];
            d.k = K[(int64_t)o * n + s];
            d.mode = M[(int64_t)o * n + s];
            d.key = (uint32_t)s;
            d.flags = kPadded;
        }
        const int64_t nw = (L[s] + W[s] - 1) / W[s];
        const int cls = i8_tile_class(W[s]);
        int64_t first_generic = 0;
        if (cls >= 0) {
            const int64_t nt = L[s] / kTileBytes;
            for (int64_t t = 0; t < nt; ++t) groups[cls + 1].push_back(Item{s, kItemTile, t * kTileBytes});
            first_generic = nt * (kTileBytes / W[s]);
        }
        for (int64_t w = first_generic; w < nw; ++w) groups[0].push_back(Item{s, kItemGeneric, w});
        soff += align64(L[s]);
        woff += nw;
    }
    std::vector<Item> items;
    p->cls_begin.assign(kI8Classes, 0);
    p->cls_count.assign(kI8Classes, 0);
    for (int c = 0; c < kI8Classes; ++c) {
        p->cls_begin[c] = (int64_t)items.size();
        p->cls_count[c] = (int64_t)groups[c + 1].size();
        items.insert(items.end(), groups[c + 1].begin(), groups[c + 1].end());
    }
    p->gen_begin = (int64_t)items.size();
    p->gen_count = (int64_t)groups[0].size();
    items.insert(items.end(), groups[0].begin(), groups[0].end());
    hipError_t e = hipSuccess;
    for (int o = 0; o < n_out && e == hipSuccess; ++o) {
        e = hipMalloc(&p->d_desc[o], sizeof(StreamDesc) * n);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_desc[o], desc[o].data(), sizeof(StreamDesc) * n, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !items.empty()) {
        e = hipMalloc(&p->d_items, sizeof(Item) * items.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        multi_free(p);
        return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
    }
    *out = p;
    return RFI_OK;
}

int multi_execute(MultiPlan* p, const void* x, int8_t* const* y, rfi_window_stats* const* st, hipStream_t s)
{
    MultiArgs ma;
    std::memset(&ma, 0, sizeof(ma));
    ma.a.streams = p->d_desc[0];
    ma.a.seed = p->seed;
    ma.a.x_base = (uint64_t)(uintptr_t)x;
    ma.a.no_stats = 1;  // the selection pass writes no statistics
    ma.n_out = p->n_out;
    for (int o = 0; o < p->n_out; ++o) {
        ma.desc[o] = p->d_desc[o];
        ma.y_base[o] = (uint64_t)(uintptr_t)y[o];
        ma.stats_base[o] = (uint64_t)(uintptr_t)(st ? st[o] : nullptr);
    }
    set_wg_per_cu(0);
    for (int c = 0; c < kI8Classes; ++c) {
        if (p->cls_count[c] == 0) continue;
        MultiArgs mc = ma;
        mc.a.items = p->d_items + p->cls_begin[c];
        mc.a.n_items = p->cls_count[c];
        if (mc.a.n_items > (1 << 30)) return RFI_ERR_INVALID;
        hipError_t e = launch_i8_multi(c, mc, (int)mc.a.n_items, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    for (int o = 0; o < p->n_out && p->gen_count > 0; ++o) {
        LaunchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.streams = p->d_desc[o];
        a.items = p->d_items + p->gen_begin;
        a.n_items = p->gen_count;
        a.seed = p->seed;
        a.x_base = (uint64_t)(uintptr_t)x;
        a.y_base = (uint64_t)(uintptr_t)y[o];
        a.stats_base = ma.stats_base[o];
        a.no_stats = ma.stats_base[o] == 0 ? 1 : 0;
        if (a.n_items > (1 << 30)) return RFI_ERR_INVALID;
        // outputs with noise streams are single-output calls of their own
        hipError_t e = launch_i8_generic(a, 3, (int)a.n_items, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    return RFI_OK;
}

std::mutex g_multi_mu;
std::map<MultiKey, MultiPlan*> g_multi;
std::vector<MultiKey> g_multi_order;
constexpr size_t kMultiCacheMax = 8;

}  // namespace

extern "C" {

int rfi_mad_filter_multi(const int8_t* x, int32_t n_out, int8_t* const* y, int32_t n_streams,
                         const int64_t* lengths, const int32_t* windows, const float* k,
                         const int32_t* mode, uint64_t seed, rfi_window_stats* const* stats_out,
                         void* stream)
{
    if (n_out < 1 || n_out > 3 || !y || !k || !mode) return RFI_ERR_INVALID;
    int64_t elems = 0;
    if (rfi_layout(n_streams, lengths, windows, nullptr, nullptr, &elems) < 0) return RFI_ERR_INVALID;
    for (int o = 0; o < n_out; ++o) {
        int rc = rfi_validate(1, x, y[o], n_streams, lengths, windows, k + (int64_t)o * n_streams,
                              mode + (int64_t)o * n_streams, stats_out ? stats_out[o] : nullptr);
        if (rc != RFI_OK) return rc;
        // outputs may not overlap the input or each other
        const uintptr_t yo = (uintptr_t)y[o], xo = (uintptr_t)x;
        if (elems > 0 && yo < xo + (uintptr_t)elems && xo < yo + (uintptr_t)elems) return RFI_ERR_INVALID;
        for (int q = 0; q < o; ++q) {
            const uintptr_t yq = (uintptr_t)y[q];
            if (elems > 0 && yo < yq + (uintptr_t)elems && yq < yo + (uintptr_t)elems) return RFI_ERR_INVALID;
        }
    }
    if (n_streams == 0 || elems == 0) return RFI_OK;
    // Outputs with a noise stream run alone; the others share one read.
    std::vector<int> shared;
    for (int o = 0; o < n_out; ++o) {
        const int32_t* mo = mode + (int64_t)o * n_streams;
        if (std::find(mo, mo + n_streams, (int32_t)RFI_MODE_NOISE) != mo + n_streams) {
            int rc = rfi_mad_filter(x, y[o], n_streams, lengths, windows, k + (int64_t)o * n_streams, mo,
                                    seed, stats_out ? stats_out[o] : nullptr, stream);
            if (rc != RFI_OK) return rc;
        } else {
            shared.push_back(o);
        }
    }
    if (shared.empty()) return RFI_OK;
    if (shared.size() == 1) {
        const int o = shared[0];
        return rfi_mad_filter(x, y[o], n_streams, lengths, windows, k + (int64_t)o * n_streams,
                              mode + (int64_t)o * n_streams, seed, stats_out ? stats_out[o] : nullptr, stream);
    }
    const int32_t ns = (int32_t)shared.size();
    std::vector<float> ks((size_t)ns * n_streams);
    std::vector<int32_t> ms((size_t)ns * n_streams);
    std::vector<int8_t*> ys(ns);
    std::vector<rfi_window_stats*> sts(ns);
    for (int i = 0; i < ns; ++i) {
        const int o = shared[i];
        std::memcpy(&ks[(size_t)i * n_streams], k + (int64_t)o * n_streams, sizeof(float) * n_streams);
        std::memcpy(&ms[(size_t)i * n_streams], mode + (int64_t)o * n_streams, sizeof(int32_t) * n_streams);
        ys[i] = y[o];
        sts[i] = stats_out ? stats_out[o] : nullptr;
    }
    MultiKey key;
    if (hipGetDevice(&key.device) != hipSuccess) key.device = 0;
    key.seed = seed;
    key.n_out = ns;
    key.L.assign(lengths, lengths + n_streams);
    key.W.assign(windows, windows + n_streams);
    key.K.resize(ks.size());
    std::memcpy(key.K.data(), ks.data(), sizeof(float) * ks.size());
    key.M = ms;
    std::lock_guard<std::mutex> g(g_multi_mu);
    MultiPlan* p = nullptr;
    auto it = g_multi.find(key);
    if (it != g_multi.end()) {
        p = it->second;
    } else {
        if (g_multi.size() >= kMultiCacheMax) {
            auto old = g_multi.find(g_multi_order.front());
            multi_free(old->second);
            g_multi.erase(old);
            g_multi_order.erase(g_multi_order.begin());
        }
        int rc = multi_build(ns, n_streams, lengths, windows, ks.data(), ms.data(), seed, &p);
        if (rc != RFI_OK) return rc;
        g_multi[key] = p;
        g_multi_order.push_back(key);
    }
    return multi_execute(p, x, ys.data(), sts.data(), (hipStream_t)stream);
}

}  // extern "C"

namespace rfi {

void multi_shutdown()
{
    std::lock_guard<std::mutex> g(g_multi_mu);
    for (auto& kv : g_multi) multi_free(kv.second);
    g_multi.clear();
    g_multi_order.clear();
}

}  // namespace rfi
