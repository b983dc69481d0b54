// rfi_mom.cpp -- median-of-MAD filtering (Eq. (3)) of int8 batches.
//
// Three passes per call, all on the caller's stream:
//   1. window statistics (median, own MAD) by the tile/generic kernels in
//      their statistics-only mode (a plan whose streams all use it);
//   2. per stream, the lower median of the MADs of each window's K-window
//      history (block counts + binary search over the 256 MAD values);
//   3. Eqs. (1)-(2) with that value, which also rewrites each window's flag
//      count and threshold.
// Work tables and temporaries are kept per argument signature and stream
// (calls on one stream are ordered; calls on different streams use
// different temporaries).
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

struct MomKey {
    int device;
    uintptr_t stream;  // temporaries are per stream: calls on one stream are ordered
    int64_t pre;       // history slots per stream (0, or K - 1 with a carried history)
    uint64_t seed;
    std::vector<int64_t> L;
    std::vector<int32_t> W;
    std::vector<uint32_t> K;
    std::vector<int32_t> M;
    bool operator<(const MomKey& o) const
    {
        if (device != o.device) return device < o.device;
        if (stream != o.stream) return stream < o.stream;
        if (pre != o.pre) return pre < o.pre;
        if (seed != o.seed) return seed < o.seed;
        if (L != o.L) return L < o.L;
        if (W != o.W) return W < o.W;
        if (K != o.K) return K < o.K;
        return M < o.M;
    }
};

struct MomPlan {
    rfi_plan* stats_plan = nullptr;
    StreamDesc* d_desc = nullptr;
    MomStream* d_streams = nullptr;
    MomItem* d_items = nullptr;
    int64_t* d_woff = nullptr;
    uint8_t* d_mad = nullptr;
    uint8_t* d_emad = nullptr;  // history slots + MADs (pre > 0)
    int32_t* d_dm = nullptr;
    uint32_t* d_hcnt = nullptr;
    rfi_window_stats* d_stats = nullptr;  // used when the caller passes none
    int32_t n_streams = 0;
    int64_t pre = 0, total_ext = 0;
    int64_t n_items = 0, total_windows = 0, max_blocks = 0;
    uint64_t seed = 0;
    int device = 0;  // the plan's buffers and kernels live here
};

void mom_free(MomPlan* p)
{
    if (!p) return;
    if (p->stats_plan) plan_free(p->stats_plan);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_desc);
    (void)hipFree(p->d_streams);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_woff);
    (void)hipFree(p->d_mad);
    (void)hipFree(p->d_emad);
    (void)hipFree(p->d_dm);
    (void)hipFree(p->d_hcnt);
    (void)hipFree(p->d_stats);
    if (have && cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

template <class T>
int upload(T** dst, const std::vector<T>& src)
{
    if (src.empty()) return RFI_OK;
    hipError_t e = hipMalloc(dst, sizeof(T) * src.size());
    if (e == hipSuccess) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    if (e == hipErrorOutOfMemory) return RFI_ERR_NOMEM;
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

template <class T>
int alloc(T** dst, int64_t n)
{
    if (n <= 0) return RFI_OK;
    hipError_t e = hipMalloc(dst, sizeof(T) * (size_t)n);
    if (e == hipErrorOutOfMemory) return RFI_ERR_NOMEM;
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

int mom_build(int32_t n, const int64_t* L, const int32_t* W, const float* K, const int32_t* M,
              uint64_t seed, int64_t pre, MomPlan** out)
{
    MomPlan* p = new MomPlan;
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    p->n_streams = n;
    p->seed = seed;
    p->pre = pre;
    std::vector<int32_t> mstats(n, kModeStats);
    int rc = plan_build(1, n, L, W, K, mstats.data(), seed, &p->stats_plan);
    if (rc == RFI_OK) rc = rfi_plan_set_schedule(p->stats_plan, RFI_SCHED_SPLIT);
    std::vector<StreamDesc> desc(n);
    std::vector<MomStream> ms(n);
    std::vector<MomItem> items;
    std::vector<int64_t> woff(n);
    int64_t soff = 0, wo = 0, eo = 0, rows = 0;
    for (int s = 0; s < n && rc == RFI_OK; ++s) {
        StreamDesc& d = desc[s];
        std::memset(&d, 0, sizeof(d));
        d.x_off = (uint64_t)soff;
        d.y_off = (uint64_t)soff;
        d.stats_off = (uint64_t)(wo * (int64_t)sizeof(rfi_window_stats));
        d.length = L[s];
        d.window = W[s];
        d.k = K[s];
        d.mode = M[s];
        d.key = (uint32_t)s;
        d.flags = kPadded;
        const int64_t nw = (L[s] + W[s] - 1) / W[s];
        const int64_t ne = pre + nw;  // the stream's MAD sequence: history slots, then windows
        ms[s].woff = wo;
        ms[s].nw = nw;
        ms[s].eoff = pre > 0 ? eo : wo;
        ms[s].pre = pre;
        ms[s].hoff = rows;
        p->max_blocks = std::max<int64_t>(p->max_blocks, (ne + kMomBlock - 1) / kMomBlock);
        rows += ne / kMomBlock + 1 + (ne % kMomBlock ? 1 : 0);
        eo += ne;
        woff[s] = wo;
        const int64_t per = std::max<int64_t>(1, std::min<int64_t>(256, 16384 / W[s]));
        for (int64_t w = 0; w < nw; w += per)
            items.push_back(MomItem{s, (int32_t)std::min<int64_t>(per, nw - w), w});
        soff += align64(L[s]);
        wo += nw;
    }
    p->total_windows = wo;
    p->total_ext = pre > 0 ? eo : 0;
    p->n_items = (int64_t)items.size();
    if (rc == RFI_OK) rc = upload(&p->d_desc, desc);
    if (rc == RFI_OK) rc = upload(&p->d_streams, ms);
    if (rc == RFI_OK) rc = upload(&p->d_items, items);
    if (rc == RFI_OK) rc = upload(&p->d_woff, woff);
    // The selection reads a stream's MAD sequence in whole aligned dwords:
    // 4 bytes past the end keep the last one inside the allocation.
    if (rc == RFI_OK) rc = alloc(&p->d_mad, wo + 4);
    if (rc == RFI_OK && p->total_ext > 0) rc = alloc(&p->d_emad, p->total_ext + 4);
    if (rc == RFI_OK) rc = alloc(&p->d_dm, wo);
    if (rc == RFI_OK) rc = alloc(&p->d_hcnt, rows * 256);
    if (rc != RFI_OK) {
        mom_free(p);
        return rc;
    }
    *out = p;
    return RFI_OK;
}

int mom_execute(MomPlan* p, const void* x, void* y, rfi_window_stats* st, int32_t mom_k, const int64_t* abs_add,
                uint8_t* hist, int32_t* hist_len, hipStream_t s)
{
    if (!st) {
        if (!p->d_stats) {
            int rc = alloc(&p->d_stats, p->total_windows);
            if (rc != RFI_OK) return rc;
        }
        st = p->d_stats;
    }
    int rc = plan_execute(p->stats_plan, x, y, st, s, RFI_SCHED_SPLIT);
    if (rc != RFI_OK) return rc;
    hipError_t e = launch_mom_gather(st, p->total_windows, p->d_mad, s);
    const uint8_t* emad = p->d_mad;
    if (e == hipSuccess && p->pre > 0) {
        e = launch_mom_extend(p->d_streams, p->n_streams, p->total_ext, p->d_mad, hist, p->d_emad, s);
        emad = p->d_emad;
    }
    if (e == hipSuccess)
        e = launch_mom_counts(p->d_streams, p->n_streams, p->max_blocks, emad, p->d_hcnt, s);
    if (e == hipSuccess)
        e = launch_mom_select(p->d_streams, p->n_streams, p->total_windows, mom_k, emad, p->d_hcnt,
                              p->pre > 0 ? hist_len : nullptr, p->d_dm, s);
    if (e == hipSuccess && p->pre > 0) e = launch_mom_history(p->d_streams, p->n_streams, emad, hist, hist_len, s);
    if (e == hipSuccess) {
        LaunchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.streams = p->d_desc;
        a.n_items = p->n_items;
        a.seed = p->seed;
        a.x_base = (uint64_t)(uintptr_t)x;
        a.y_base = (uint64_t)(uintptr_t)y;
        e = launch_mom_apply(a, p->d_items, p->n_items, p->d_dm, p->d_woff, abs_add, st, s);
    }
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

std::mutex g_mom_mu;
std::map<MomKey, MomPlan*> g_mom;
std::vector<MomKey> g_mom_order;
constexpr size_t kMomCacheMax = 8;

int mom_call(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths, const int32_t* windows,
             const float* k, const int32_t* mode, int32_t mom_k, uint64_t seed, const int64_t* abs_base,
             uint8_t* hist, int32_t* hist_len, bool carry, rfi_window_stats* stats_out, void* stream)
{
    if (mom_k < 1) return RFI_ERR_INVALID;
    int rc = rfi_validate(1, x, y, n_streams, lengths, windows, k, mode, stats_out);
    if (rc != RFI_OK) return rc;
    if (carry && mom_k > 1 && n_streams > 0) {
        if (!hist || !hist_len) return RFI_ERR_INVALID;
        if ((uintptr_t)hist_len & 3u) return RFI_ERR_ALIGN;
    }
    if (abs_base && ((uintptr_t)abs_base & 7u)) return RFI_ERR_ALIGN;
    int64_t total = 0;
    rfi_layout(n_streams, lengths, windows, nullptr, nullptr, &total);
    if (n_streams == 0 || total == 0) return RFI_OK;
    MomKey key;
    if (hipGetDevice(&key.device) != hipSuccess) key.device = 0;
    key.stream = (uintptr_t)stream;
    key.pre = carry ? (int64_t)mom_k - 1 : 0;
    key.seed = seed;
    key.L.assign(lengths, lengths + n_streams);
    key.W.assign(windows, windows + n_streams);
    key.K.resize(n_streams);
    std::memcpy(key.K.data(), k, sizeof(float) * n_streams);
    key.M.assign(mode, mode + n_streams);
    std::lock_guard<std::mutex> g(g_mom_mu);
    MomPlan* p = nullptr;
    auto it = g_mom.find(key);
    if (it != g_mom.end()) {
        p = it->second;
    } else {
        if (g_mom.size() >= kMomCacheMax) {
            auto old = g_mom.find(g_mom_order.front());
            mom_free(old->second);
            g_mom.erase(old);
            g_mom_order.erase(g_mom_order.begin());
        }
        rc = mom_build(n_streams, lengths, windows, k, mode, seed, key.pre, &p);
        if (rc != RFI_OK) return rc;
        g_mom[key] = p;
        g_mom_order.push_back(key);
    }
    return mom_execute(p, x, y, stats_out, mom_k, abs_base, hist, hist_len, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int rfi_mom_filter(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                   uint64_t seed, rfi_window_stats* stats_out, void* stream)
{
    return mom_call(x, y, n_streams, lengths, windows, k, mode, mom_k, seed, nullptr, nullptr, nullptr, false,
                    stats_out, stream);
}

int rfi_mom_filter_carry(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                         const int32_t* windows, const float* k, const int32_t* mode, int32_t mom_k,
                         uint64_t seed, const int64_t* abs_base, uint8_t* mad_history, int32_t* history_len,
                         rfi_window_stats* stats_out, void* stream)
{
    return mom_call(x, y, n_streams, lengths, windows, k, mode, mom_k, seed, abs_base, mad_history, history_len,
                    mom_k > 1, stats_out, stream);
}

}  // extern "C"

namespace rfi {

void mom_shutdown()
{
    std::lock_guard<std::mutex> g(g_mom_mu);
    for (auto& kv : g_mom) mom_free(kv.second);
    g_mom.clear();
    g_mom_order.clear();
}

}  // namespace rfi
