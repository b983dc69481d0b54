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
//
// A large batch is cut into chunks of whole streams.  Pass 1 of a chunk is
// bound by the selection's LDS atomics and pass 3 by HBM, so pass 3 of
// chunk c runs on an auxiliary stream beside passes 1-2 of chunk c + 1 on
// the caller's stream; the auxiliary stream is forked from and joined back
// to the caller's with events (graph edges under capture).
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

// The tables of one chunk: streams s0 .. s0 + n_streams - 1 of the call,
// whose samples start byte0 bytes and whose windows start win0 records
// into the call's buffers.
struct MomChunk {
    rfi_plan* stats_plan = nullptr;
    StreamDesc* d_desc = nullptr;
    MomStream* d_streams = nullptr;
    MomItem* d_items = nullptr;
    int64_t* d_woff = nullptr;
    uint8_t* d_mad = nullptr;
    uint8_t* d_emad = nullptr;  // history slots + MADs (pre > 0)
    int32_t* d_dm = nullptr;
    uint32_t* d_hcnt = nullptr;
    int32_t s0 = 0, n_streams = 0;
    int64_t byte0 = 0, win0 = 0;
    int64_t total_ext = 0, n_items = 0, total_windows = 0, max_blocks = 0;
};

struct MomPlan {
    std::vector<MomChunk> chunks;
    rfi_window_stats* d_stats = nullptr;  // used when the caller passes none
    hipStream_t aux = nullptr;            // pass 3 of all but the last chunk
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<hipEvent_t> ready;        // chunk c's pass 2 done
    int64_t pre = 0, total_windows = 0;
    uint64_t seed = 0;
    int device = 0;  // the plan's buffers and kernels live here
};

void mom_free(MomPlan* p)
{
    if (!p) return;
    for (auto& c : p->chunks)
        if (c.stats_plan) plan_free(c.stats_plan);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (auto& c : p->chunks) {
        (void)hipFree(c.d_desc);
        (void)hipFree(c.d_streams);
        (void)hipFree(c.d_items);
        (void)hipFree(c.d_woff);
        (void)hipFree(c.d_mad);
        (void)hipFree(c.d_emad);
        (void)hipFree(c.d_dm);
        (void)hipFree(c.d_hcnt);
    }
    (void)hipFree(p->d_stats);
    for (hipEvent_t e : p->ready) (void)hipEventDestroy(e);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    if (p->aux) (void)hipStreamDestroy(p->aux);
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

// Tables of streams s0 .. s0 + n - 1 (L, W, K, M point at stream s0).
int chunk_build(MomChunk& c, int32_t s0, int32_t n, const int64_t* L, const int32_t* W, const float* K,
                const int32_t* M, uint64_t seed, int64_t pre)
{
    c.s0 = s0;
    c.n_streams = n;
    std::vector<int32_t> mstats(n, kModeStats);
    int rc = plan_build(1, n, L, W, K, mstats.data(), seed, &c.stats_plan);
    if (rc == RFI_OK) rc = rfi_plan_set_schedule(c.stats_plan, RFI_SCHED_SPLIT);
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
        d.key = (uint32_t)(s0 + s);  // the stream's index in the call: the noise key
        d.flags = kPadded;
        const int64_t nw = (L[s] + W[s] - 1) / W[s];
        const int64_t ne = pre + nw;  // the stream's MAD sequence: history slots, then windows
        ms[s].woff = wo;
        ms[s].nw = nw;
        ms[s].eoff = pre > 0 ? eo : wo;
        ms[s].pre = pre;
        ms[s].hoff = rows;
        c.max_blocks = std::max<int64_t>(c.max_blocks, (ne + kMomBlock - 1) / kMomBlock);
        rows += ne / kMomBlock + 1 + (ne % kMomBlock ? 1 : 0);
        eo += ne;
        woff[s] = wo;
        const int64_t per = std::max<int64_t>(1, std::min<int64_t>(256, 16384 / W[s]));
        for (int64_t w = 0; w < nw; w += per)
            items.push_back(MomItem{s, (int32_t)std::min<int64_t>(per, nw - w), w});
        soff += align64(L[s]);
        wo += nw;
    }
    c.total_windows = wo;
    c.total_ext = pre > 0 ? eo : 0;
    c.n_items = (int64_t)items.size();
    if (rc == RFI_OK) rc = upload(&c.d_desc, desc);
    if (rc == RFI_OK) rc = upload(&c.d_streams, ms);
    if (rc == RFI_OK) rc = upload(&c.d_items, items);
    if (rc == RFI_OK) rc = upload(&c.d_woff, woff);
    // The selection reads a stream's MAD sequence in whole aligned dwords:
    // 4 bytes past the end keep the last one inside the allocation.
    if (rc == RFI_OK) rc = alloc(&c.d_mad, wo + 4);
    if (rc == RFI_OK && c.total_ext > 0) rc = alloc(&c.d_emad, c.total_ext + 4);
    if (rc == RFI_OK) rc = alloc(&c.d_dm, wo);
    if (rc == RFI_OK) rc = alloc(&c.d_hcnt, rows * 256);
    return rc;
}

// Batches of at least this many samples are cut into up to kMomChunks
// chunks of about equal size (whole streams).
constexpr int64_t kMomChunkMinSamples = int64_t(1) << 26;
constexpr int kMomChunks = 4;

int mom_build(int32_t n, const int64_t* L, const int32_t* W, const float* K, const int32_t* M,
              uint64_t seed, int64_t pre, MomPlan** out)
{
    MomPlan* p = new MomPlan;
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    p->seed = seed;
    p->pre = pre;
    int64_t total = 0;
    for (int s = 0; s < n; ++s) total += L[s];
    const int nc = total >= kMomChunkMinSamples ? std::min<int>(kMomChunks, n) : 1;
    // chunk boundaries: whole streams, each chunk about total / nc samples
    std::vector<int32_t> first{0};
    int64_t acc = 0;
    for (int s = 0; s < n; ++s) {
        acc += L[s];
        const int left = n - (s + 1);
        if ((int)first.size() < nc && left > 0 && acc * nc >= total * (int64_t)first.size()) first.push_back(s + 1);
    }
    first.push_back(n);
    int rc = RFI_OK;
    int64_t byte0 = 0, win0 = 0;
    p->chunks.resize(first.size() - 1);
    for (size_t ci = 0; ci + 1 < first.size() && rc == RFI_OK; ++ci) {
        MomChunk& c = p->chunks[ci];
        const int32_t s0 = first[ci], cn = first[ci + 1] - first[ci];
        rc = chunk_build(c, s0, cn, L + s0, W + s0, K + s0, M + s0, seed, pre);
        c.byte0 = byte0;
        c.win0 = win0;
        for (int s = s0; s < s0 + cn; ++s) {
            byte0 += align64(L[s]);
            win0 += (L[s] + W[s] - 1) / W[s];
        }
    }
    p->total_windows = win0;
    if (rc == RFI_OK && p->chunks.size() > 1) {
        hipError_t e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
        p->ready.assign(p->chunks.size(), nullptr);
        for (auto& ev : p->ready)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    if (rc != RFI_OK) {
        mom_free(p);
        return rc;
    }
    *out = p;
    return RFI_OK;
}

// Passes 1 and 2 of a chunk on s.
int chunk_select(MomChunk& c, int64_t pre, const uint8_t* x, uint8_t* y, rfi_window_stats* st, int32_t mom_k,
                 uint8_t* hist, int32_t* hist_len, hipStream_t s)
{
    rfi_window_stats* cst = st + c.win0;
    int rc = plan_execute(c.stats_plan, x + c.byte0, y + c.byte0, cst, s, RFI_SCHED_SPLIT);
    if (rc != RFI_OK) return rc;
    hipError_t e = launch_mom_gather(cst, c.total_windows, c.d_mad, s);
    const uint8_t* emad = c.d_mad;
    uint8_t* ch = hist ? hist + (int64_t)c.s0 * pre : nullptr;
    int32_t* chl = hist_len ? hist_len + c.s0 : nullptr;
    if (e == hipSuccess && pre > 0) {
        e = launch_mom_extend(c.d_streams, c.n_streams, c.total_ext, c.d_mad, ch, c.d_emad, s);
        emad = c.d_emad;
    }
    if (e == hipSuccess) e = launch_mom_counts(c.d_streams, c.n_streams, c.max_blocks, emad, c.d_hcnt, s);
    if (e == hipSuccess)
        e = launch_mom_select(c.d_streams, c.n_streams, c.total_windows, mom_k, emad, c.d_hcnt,
                              pre > 0 ? chl : nullptr, c.d_dm, s);
    if (e == hipSuccess && pre > 0) e = launch_mom_history(c.d_streams, c.n_streams, emad, ch, chl, s);
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

// Pass 3 of a chunk on s.
hipError_t chunk_apply(MomChunk& c, uint64_t seed, const uint8_t* x, uint8_t* y, rfi_window_stats* st,
                       const int64_t* abs_add, hipStream_t s)
{
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.streams = c.d_desc;
    a.n_items = c.n_items;
    a.seed = seed;
    a.x_base = (uint64_t)(uintptr_t)(x + c.byte0);
    a.y_base = (uint64_t)(uintptr_t)(y + c.byte0);
    return launch_mom_apply(a, c.d_items, c.n_items, c.d_dm, c.d_woff, abs_add ? abs_add + c.s0 : nullptr,
                            st + c.win0, s);
}

int mom_execute(MomPlan* p, const void* xv, void* yv, rfi_window_stats* st, int32_t mom_k, const int64_t* abs_add,
                uint8_t* hist, int32_t* hist_len, hipStream_t s)
{
    if (!st) {
        if (!p->d_stats) {
            int rc = alloc(&p->d_stats, p->total_windows);
            if (rc != RFI_OK) return rc;
        }
        st = p->d_stats;
    }
    const uint8_t* x = static_cast<const uint8_t*>(xv);
    uint8_t* y = static_cast<uint8_t*>(yv);
    const size_t nc = p->chunks.size();
    if (nc == 1) {
        int rc = chunk_select(p->chunks[0], p->pre, x, y, st, mom_k, hist, hist_len, s);
        if (rc != RFI_OK) return rc;
        hipError_t e = chunk_apply(p->chunks[0], p->seed, x, y, st, abs_add, s);
        return e == hipSuccess ? RFI_OK : hip_fail(e);
    }
    // Pass 3 of chunk c on aux beside passes 1-2 of chunk c + 1 on s.
    int rc = RFI_OK;
    hipError_t e = hipEventRecord(p->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->aux, p->fork, 0);
    for (size_t c = 0; c < nc && e == hipSuccess && rc == RFI_OK; ++c) {
        rc = chunk_select(p->chunks[c], p->pre, x, y, st, mom_k, hist, hist_len, s);
        if (rc != RFI_OK) break;
        e = hipEventRecord(p->ready[c], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->aux, p->ready[c], 0);
        if (e == hipSuccess) e = chunk_apply(p->chunks[c], p->seed, x, y, st, abs_add, p->aux);
    }
    // join the auxiliary stream, also after an error, so it never stays forked
    hipError_t j = hipEventRecord(p->join, p->aux);
    if (j == hipSuccess) j = hipStreamWaitEvent(s, p->join, 0);
    if (e == hipSuccess) e = j;
    if (rc != RFI_OK) return rc;
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
