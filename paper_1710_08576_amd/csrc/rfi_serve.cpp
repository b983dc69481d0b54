// rfi_serve.cpp -- serving runtime of librfimad: blocks of many streams
// arrive over time and are filtered with continuous batching.
//
// Per stream the device holds the carry (the samples of the unfinished
// window, double-buffered) and the host tracks its length and the absolute
// index of its first sample, so a block is filtered exactly as if the whole
// stream had been one batch (same windows, same noise keys).
//
// Each stream is bound to one "lane" (a HIP stream).  A lane dispatches
// batches: admitted blocks of its streams, taken round-robin in each
// stream's order, up to max_batch blocks, as one fused kernel launch over a
// work table plus one carry-update launch.  Within a batch, the head window
// of a stream's next block reads its carry straight from the previous
// block's buffer; the carry left at the end of the batch is copied to the
// stream's device carry buffer by the carry-update launch, so the carry
// chain across batches follows HIP stream order.  A lane keeps
// up to kSlotsPerLane batches in flight; blocks that arrive meanwhile wait
// for the next batch of their lane (continuous batching), so the work of
// different lanes, and of queued batches, overlaps on the device.  Blocks
// are admitted against an HBM budget (input + output + statistics bytes of
// unfinished blocks) and an in-flight limit.
//
// Ticket records live in a map keyed by ticket id and are retired: a
// completed record once it has been polled done (at the next admission), a
// completed record never polled once kTicketHistory later tickets have
// completed, and a replay's records as soon as their results are taken.
// Memory thus stays bounded over an unbounded run.
//
// A batch is built on the host before anything reaches the device; if its
// tables cannot be staged or copied, the stream state it changed (carry
// position and length, absolute index, pending queue, ticket states) is
// restored and its blocks wait for the next dispatch.  A failed kernel
// launch or completion query leaves device state unknown: the server is
// then faulted and every later call returns RFI_ERR_HIP.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "rfi_runtime.hpp"

using namespace rfi;

namespace {

constexpr int kSlotsPerLane = 2;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t align64(int64_t n) { return (n + 63) / 64 * 64; }

struct SrvStream {
    bool active = false;
    int32_t W = 0;
    float k = 0.f;
    int32_t mode = 0;
    int lane = 0;
    void* carry[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t carry_len = 0;
    int64_t next_abs = 0;
    std::deque<uint64_t> pending;  // admitted, not yet dispatched, in order
};

enum TicketState { kAdmitted = 0, kDispatched = 1, kDone = 2 };

// Completed, never-polled records kept before the oldest is retired.
constexpr size_t kTicketHistory = 65536;

struct TicketRec {
    bool polled = false;
    uint32_t stream = 0;
    const void* block = nullptr;
    void* out = nullptr;
    int64_t n = 0;
    rfi_window_stats* stats = nullptr;
    int64_t emitted_samples = 0, emitted_windows = 0;
    int state = kAdmitted;
    uint64_t bytes = 0;
    int64_t t_submit = 0, t_done = 0;
};

struct Slot {
    char* d_buf = nullptr;    // descriptors | items | carry items (device)
    char* h_stage = nullptr;  // the same tables staged in pinned host memory
    size_t cap = 0;
    bool busy = false;
    hipEvent_t ev = nullptr;
    std::vector<uint64_t> tickets;
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Where the carry of a stream lies while a batch is being built: in the
// stream's device carry buffer (at batch start) or at the end of a block
// already in the batch.  `open` turns false once a block leaves a carry
// that spans the old carry and that whole block; that carry goes through
// the carry-update launch, so later blocks of the stream wait for the next
// batch.
struct Chain {
    uint64_t src = 0;
    int32_t len = 0;
    bool in_buffer = true;
    bool open = true;
};

constexpr size_t kSlotPrealloc = 1 << 20;  // table bytes per slot at creation

struct SavedState {
    int cur;
    int32_t carry_len;
    int64_t next_abs;
};

struct Lane {
    hipStream_t s = nullptr;
    Slot slots[kSlotsPerLane];
    std::deque<int> inflight;  // slot indices in launch order
    int rr = 0;                // round-robin start among the lane's streams
    std::vector<uint32_t> members;
    // Work tables of the batch being built (kept to reuse their storage).
    std::vector<StreamDesc> descs;
    std::vector<Item> items;
    std::vector<CarryItem> carries;
    std::vector<uint64_t> batch;
    std::vector<Chain> chains;
    std::vector<SavedState> saved;  // members' state before the batch
};

}  // namespace

struct rfi_server {
    rfi_server_config cfg;
    int device = 0;
    std::vector<SrvStream> streams;
    std::unordered_map<uint64_t, TicketRec> recs;  // live ticket records by id
    uint64_t next_id = 1;                          // ids 1 .. next_id - 1 issued
    std::deque<uint64_t> completed;                // completion order (history bound)
    std::vector<uint64_t> polled;                  // polled done, retired at the next admission
    uint64_t live_peak = 0;
    // Replay in progress: results of its tickets [first, first + n) are
    // written here at completion and the records retired at once.
    uint64_t sink_first = 0;
    int64_t sink_n = 0;
    int64_t* sink_done = nullptr;
    int64_t* sink_emitted = nullptr;
    std::vector<Lane> lanes;
    uint64_t bytes_inflight = 0;
    int64_t inflight = 0;
    uint64_t n_admitted = 0, n_refused = 0, n_completed = 0, n_launches = 0;
    int persist_grid = 0;
    hipError_t fault = hipSuccess;  // first failed launch or completion query
    // Testing aid: uploads number fail_from .. fail_from + fail_count - 1
    // (counted from 1 per server) fail as if staging memory were exhausted
    // (environment RFI_SERVE_FAIL_UPLOAD=first[:count], read at creation).
    uint64_t uploads = 0, fail_from = 0, fail_count = 0;
    std::mutex mu;
};

namespace {

uint64_t block_bytes(const rfi_server* srv, const SrvStream& st, int64_t n)
{
    const int64_t e = srv->cfg.elem_size;
    const int64_t out = n + st.W - 1;
    return (uint64_t)(n * e + out * e + ((out + st.W - 1) / st.W) * (int64_t)sizeof(rfi_window_stats));
}

// Makes room for the tables of one batch; both copies have the same size.
int ensure_slot(Slot& sl, size_t bytes)
{
    if (bytes <= sl.cap) return RFI_OK;
    const size_t c = std::max<size_t>(bytes, sl.cap * 2 + 4096);
    if (sl.d_buf) (void)hipFree(sl.d_buf);
    if (sl.h_stage) (void)hipHostFree(sl.h_stage);
    sl.d_buf = nullptr;
    sl.h_stage = nullptr;
    sl.cap = 0;
    hipError_t e = hipMalloc((void**)&sl.d_buf, c);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_stage, c, hipHostMallocDefault);
    if (e == hipErrorOutOfMemory) return RFI_ERR_NOMEM;
    if (e != hipSuccess) return hip_fail(e);
    sl.cap = c;
    return RFI_OK;
}

// Stages the tables in the slot and copies them to the device on stream s
// (one copy); returns the device addresses of the three tables.
int upload(Slot& sl, const std::vector<StreamDesc>& descs, const std::vector<Item>& items,
           const std::vector<CarryItem>& carries, hipStream_t s, StreamDesc** dd, Item** di,
           CarryItem** dc)
{
    const size_t bd = descs.size() * sizeof(StreamDesc), bi = items.size() * sizeof(Item),
                 bc = carries.size() * sizeof(CarryItem);
    const size_t oi = align256(bd), oc = oi + align256(bi), total = oc + bc;
    int rc = ensure_slot(sl, total);
    if (rc != RFI_OK) return rc;
    if (bd) std::memcpy(sl.h_stage, descs.data(), bd);
    if (bi) std::memcpy(sl.h_stage + oi, items.data(), bi);
    if (bc) std::memcpy(sl.h_stage + oc, carries.data(), bc);
    if (total) {
        hipError_t e = hipMemcpyAsync(sl.d_buf, sl.h_stage, total, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    *dd = reinterpret_cast<StreamDesc*>(sl.d_buf);
    *di = reinterpret_cast<Item*>(sl.d_buf + oi);
    *dc = reinterpret_cast<CarryItem*>(sl.d_buf + oc);
    return RFI_OK;
}

// Work of one block appended to the batch tables (host side); updates the
// stream's carry bookkeeping.
void plan_block(rfi_server* srv, SrvStream& st, uint32_t sid, TicketRec& t, Chain& ch, Lane& L)
{
    const int elem = srv->cfg.elem_size;
    const int64_t c = st.carry_len, n = t.n, W = st.W;
    const int64_t total = c + n;
    const int64_t nw = total / W;
    const int64_t emitted = nw * W;
    const int64_t newc = total - emitted;
    auto base_desc = [&]() {
        StreamDesc d;
        std::memset(&d, 0, sizeof(d));
        d.window = st.W;
        d.k = st.k;
        d.mode = st.mode;
        d.key = sid;
        d.flags = t.stats ? 0 : kNoStats;
        return d;
    };
    if (nw > 0) {
        const int64_t h = c > 0 ? 1 : 0;
        if (h) {
            StreamDesc d = base_desc();
            d.x_off = (uint64_t)(uintptr_t)t.block;
            d.head_off = ch.src;
            d.head_len = (int32_t)c;
            d.length = W;
            d.y_off = (uint64_t)(uintptr_t)t.out;
            d.stats_off = (uint64_t)(uintptr_t)t.stats;
            d.abs_base = st.next_abs;
            L.items.push_back(Item{(int32_t)L.descs.size(), kItemGeneric, 0});
            L.descs.push_back(d);
        }
        const int64_t nb = nw - h;
        if (nb > 0) {
            StreamDesc d = base_desc();
            const uint64_t x = (uint64_t)(uintptr_t)t.block + (uint64_t)((h ? W - c : 0) * elem);
            const uint64_t y = (uint64_t)(uintptr_t)t.out + (uint64_t)(h * W * elem);
            d.x_off = x;
            d.y_off = y;
            d.stats_off = (uint64_t)(uintptr_t)(t.stats ? t.stats + h : nullptr);
            d.length = nb * W;
            d.abs_base = st.next_abs + h * W;
            const int ds = (int32_t)L.descs.size();
            L.descs.push_back(d);
            const int cls = elem == 1 ? i8_tile_class(st.W) : i16_tile_class(st.W);
            const int64_t tile_samples = kTileBytes / elem;
            int64_t first_generic = 0;
            // Tiles draw noise four samples (one Philox block) at a time from
            // the tile's first sample on, so that sample must start a block.
            if (cls >= 0 && (x % 16) == 0 && (y % 16) == 0 && (d.abs_base % 4) == 0) {
                const int64_t nt = (nb * W) / tile_samples;
                for (int64_t i = 0; i < nt; ++i) L.items.push_back(Item{ds, kItemTile, i * tile_samples});
                first_generic = nt * (tile_samples / W);
            }
            for (int64_t w = first_generic; w < nb; ++w) L.items.push_back(Item{ds, kItemGeneric, w});
        }
    }
    if (newc > 0 && nw == 0 && c > 0) {
        // The new carry is the old one followed by the whole block.
        CarryItem ci;
        ci.head = ch.src;
        ci.head_len = (int32_t)c;
        ci.body = (uint64_t)(uintptr_t)t.block;
        ci.dst = (uint64_t)(uintptr_t)st.carry[st.cur ^ 1];
        ci.from = 0;
        ci.count = (int32_t)newc;
        ci.elem = elem;
        L.carries.push_back(ci);
        st.cur ^= 1;
        ch.src = ci.dst;
        ch.in_buffer = true;
        ch.open = false;
    } else if (newc > 0) {
        // The new carry is the tail of this block (or, for an empty block,
        // still the old carry).
        if (n > 0) {
            ch.src = (uint64_t)(uintptr_t)t.block + (uint64_t)((n - newc) * elem);
            ch.in_buffer = false;
        }
    } else {
        ch.src = (uint64_t)(uintptr_t)st.carry[st.cur];
        ch.in_buffer = true;
    }
    ch.len = (int32_t)newc;
    st.carry_len = (int32_t)newc;
    st.next_abs += emitted;
    t.emitted_samples = emitted;
    t.emitted_windows = nw;
}

// End of a stream's part of a batch: a carry left inside a block is copied
// to the stream's other carry buffer (after the batch's filter launch).
void close_chain(rfi_server* srv, SrvStream& st, Chain& ch, Lane& L)
{
    if (ch.len > 0 && !ch.in_buffer) {
        CarryItem ci;
        ci.head = ch.src;
        ci.head_len = ch.len;
        ci.body = 0;
        ci.dst = (uint64_t)(uintptr_t)st.carry[st.cur ^ 1];
        ci.from = 0;
        ci.count = ch.len;
        ci.elem = srv->cfg.elem_size;
        L.carries.push_back(ci);
        st.cur ^= 1;
    }
}

// Launches one batch on a lane if it has pending blocks and a free slot.
int dispatch_lane(rfi_server* srv, int li)
{
    Lane& L = srv->lanes[li];
    int si = -1;
    for (int s = 0; s < kSlotsPerLane; ++s)
        if (!L.slots[s].busy) {
            si = s;
            break;
        }
    if (si < 0 || L.members.empty()) return RFI_OK;
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    L.descs.clear();
    L.items.clear();
    L.carries.clear();
    L.batch.clear();
    const int nm = (int)L.members.size();
    L.chains.assign(nm, Chain());
    L.saved.resize(nm);
    for (int j = 0; j < nm; ++j) {
        const SrvStream& st = srv->streams[L.members[j]];
        L.chains[j].src = (uint64_t)(uintptr_t)st.carry[st.cur];
        L.chains[j].len = st.carry_len;
        L.saved[j] = SavedState{st.cur, st.carry_len, st.next_abs};
    }
    // Round-robin passes: each pass takes the next block of every stream
    // whose chain is still open.
    bool progress = true;
    while (progress && (int)L.batch.size() < srv->cfg.max_batch) {
        progress = false;
        for (int jj = 0; jj < nm && (int)L.batch.size() < srv->cfg.max_batch; ++jj) {
            const int j = (L.rr + jj) % nm;
            const uint32_t sid = L.members[j];
            SrvStream& st = srv->streams[sid];
            if (st.pending.empty() || !L.chains[j].open) continue;
            const uint64_t tk = st.pending.front();
            st.pending.pop_front();
            TicketRec& t = srv->recs.at(tk);
            plan_block(srv, st, sid, t, L.chains[j], L);
            t.state = kDispatched;
            L.batch.push_back(tk);
            progress = true;
        }
    }
    if (L.batch.empty()) return RFI_OK;
    for (int j = 0; j < nm; ++j) close_chain(srv, srv->streams[L.members[j]], L.chains[j], L);
    L.rr = (L.rr + 1) % nm;
    Slot& sl = L.slots[si];
    StreamDesc* dd = nullptr;
    Item* di = nullptr;
    CarryItem* dc = nullptr;
    int rc = RFI_OK;
    if (++srv->uploads >= srv->fail_from && srv->uploads < srv->fail_from + srv->fail_count) rc = RFI_ERR_NOMEM;
    if (rc == RFI_OK) rc = upload(sl, L.descs, L.items, L.carries, L.s, &dd, &di, &dc);
    if (rc != RFI_OK) {
        // Nothing of this batch reached the device: undo it.
        for (int j = 0; j < nm; ++j) {
            SrvStream& st = srv->streams[L.members[j]];
            st.cur = L.saved[j].cur;
            st.carry_len = L.saved[j].carry_len;
            st.next_abs = L.saved[j].next_abs;
        }
        for (auto it = L.batch.rbegin(); it != L.batch.rend(); ++it) {
            TicketRec& t = srv->recs.at(*it);
            t.state = kAdmitted;
            t.emitted_samples = t.emitted_windows = 0;
            srv->streams[t.stream].pending.push_front(*it);
        }
        L.rr = (L.rr + nm - 1) % nm;
        return rc;
    }
    hipError_t e = hipSuccess;
    const std::vector<Item>& items = L.items;
    const std::vector<CarryItem>& carries = L.carries;
    if (!items.empty()) {
        LaunchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.streams = dd;
        a.items = di;
        a.n_items = (int64_t)items.size();
        a.seed = srv->cfg.seed;
        set_wg_per_cu(0);
        int64_t grid = a.n_items;
        if (srv->cfg.schedule == RFI_SCHED_FUSED_PERSIST) grid = std::min<int64_t>(grid, srv->persist_grid);
        e = srv->cfg.elem_size == 1 ? launch_i8_fused(7, a, (int)grid, L.s)
                                    : launch_i16_fused(a, (int)grid, L.s);
        ++srv->n_launches;
    }
    if (e == hipSuccess && !carries.empty()) {
        e = launch_carry(dc, (int)carries.size(), L.s);
        ++srv->n_launches;
    }
    if (e == hipSuccess) e = hipEventRecord(sl.ev, L.s);
    if (e != hipSuccess) {
        // Part of the batch may be on the device: the server cannot tell
        // what its streams' carries hold any more.
        srv->fault = e;
        return hip_fail(e);
    }
    sl.busy = true;
    sl.tickets.assign(L.batch.begin(), L.batch.end());
    L.inflight.push_back(si);
    return RFI_OK;
}

// Marks completed batches; returns the number of tickets completed and,
// if min_id > 0, counts in *ours those with id >= min_id.
int64_t reap(rfi_server* srv, uint64_t min_id = 0, int64_t* ours = nullptr)
{
    int64_t done = 0;
    for (auto& L : srv->lanes) {
        while (!L.inflight.empty()) {
            Slot& sl = L.slots[L.inflight.front()];
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                srv->fault = q;
                return done;
            }
            const int64_t t = now_ns();
            for (uint64_t tk : sl.tickets) {
                auto it = srv->recs.find(tk);
                TicketRec& r = it->second;
                r.state = kDone;
                r.t_done = t;
                srv->bytes_inflight -= r.bytes;
                --srv->inflight;
                ++srv->n_completed;
                ++done;
                if (ours && tk >= min_id) ++*ours;
                if (srv->sink_n > 0 && tk >= srv->sink_first && tk < srv->sink_first + (uint64_t)srv->sink_n) {
                    srv->sink_done[tk - srv->sink_first] = t;
                    srv->sink_emitted[tk - srv->sink_first] = r.emitted_samples;
                    srv->recs.erase(it);
                    continue;
                }
                srv->completed.push_back(tk);
                if (srv->completed.size() > kTicketHistory) {
                    srv->recs.erase(srv->completed.front());
                    srv->completed.pop_front();
                }
            }
            sl.tickets.clear();
            sl.busy = false;
            L.inflight.pop_front();
        }
    }
    return done;
}

int submit_locked(rfi_server* srv, uint32_t sid, const void* block, void* out, int64_t n,
                  rfi_window_stats* stats, uint64_t* ticket)
{
    if (sid >= (uint32_t)srv->streams.size() || !srv->streams[sid].active || n < 0) return RFI_ERR_INVALID;
    if (n > 0 && (!block || !out)) return RFI_ERR_INVALID;
    if (((uintptr_t)block | (uintptr_t)out | (uintptr_t)stats) & 15u) return RFI_ERR_ALIGN;
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    SrvStream& st = srv->streams[sid];
    const uint64_t bytes = block_bytes(srv, st, n);
    for (uint64_t id : srv->polled) srv->recs.erase(id);
    srv->polled.clear();
    if (srv->inflight >= srv->cfg.max_inflight ||
        (srv->bytes_inflight + bytes > srv->cfg.hbm_budget_bytes && srv->inflight > 0)) {
        ++srv->n_refused;
        return RFI_ERR_BUSY;
    }
    TicketRec t;
    t.stream = sid;
    t.block = block;
    t.out = out;
    t.n = n;
    t.stats = stats;
    t.bytes = bytes;
    t.t_submit = now_ns();
    const uint64_t id = srv->next_id++;
    srv->recs.emplace(id, t);
    srv->live_peak = std::max<uint64_t>(srv->live_peak, srv->recs.size());
    st.pending.push_back(id);
    srv->bytes_inflight += bytes;
    ++srv->inflight;
    ++srv->n_admitted;
    if (ticket) *ticket = id;
    return RFI_OK;
}

int dispatch_all(rfi_server* srv)
{
    for (int li = 0; li < (int)srv->lanes.size(); ++li) {
        int rc = dispatch_lane(srv, li);
        if (rc != RFI_OK) return rc;
    }
    return RFI_OK;
}


int sync_all(rfi_server* srv)
{
    for (;;) {
        if (srv->fault != hipSuccess) return hip_fail(srv->fault);
        reap(srv);
        if (srv->fault != hipSuccess) return hip_fail(srv->fault);
        int rc = dispatch_all(srv);
        if (rc != RFI_OK) return rc;
        if (srv->inflight == 0) return RFI_OK;
        for (auto& L : srv->lanes) {
            hipError_t e = hipStreamSynchronize(L.s);
            if (e != hipSuccess) return hip_fail(e);
        }
    }
}

}  // namespace

extern "C" {

int rfi_server_create(const rfi_server_config* cfg, rfi_server** out)
{
    if (!out) return RFI_ERR_INVALID;
    *out = nullptr;
    if (!cfg || (cfg->elem_size != 1 && cfg->elem_size != 2) || cfg->max_streams < 1 || cfg->max_streams > (1 << 20) ||
        cfg->max_inflight < 1 || cfg->max_batch < 1 || cfg->n_lanes < 1 || cfg->n_lanes > 64 ||
        (cfg->schedule != RFI_SCHED_AUTO && cfg->schedule != RFI_SCHED_FUSED &&
         cfg->schedule != RFI_SCHED_FUSED_PERSIST))
        return RFI_ERR_INVALID;
    rfi_server* srv = new rfi_server;
    srv->cfg = *cfg;
    if (hipGetDevice(&srv->device) != hipSuccess) srv->device = 0;
    srv->persist_grid = persistent_grid(cfg->elem_size, -1, 7, true);
    if (const char* f = std::getenv("RFI_SERVE_FAIL_UPLOAD")) {
        char* end = nullptr;
        const unsigned long long first = std::strtoull(f, &end, 10);
        unsigned long long count = 1;
        if (end && *end == ':') count = std::strtoull(end + 1, nullptr, 10);
        if (first > 0) {
            srv->fail_from = first;
            srv->fail_count = count;
        }
    }
    srv->streams.resize(cfg->max_streams);
    srv->lanes.resize(cfg->n_lanes);
    for (auto& L : srv->lanes) {
        hipError_t e = hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking);
        int rc = RFI_OK;
        for (int s = 0; s < kSlotsPerLane && e == hipSuccess && rc == RFI_OK; ++s) {
            e = hipEventCreateWithFlags(&L.slots[s].ev, hipEventDisableTiming);
            // Growing a slot later synchronises the device; start large.
            if (e == hipSuccess) rc = ensure_slot(L.slots[s], kSlotPrealloc);
        }
        // The batch kernels this lane will launch, once, with no items.
        if (e == hipSuccess && rc == RFI_OK) e = warm_fused(cfg->elem_size, false, L.s);
        if (e == hipSuccess && rc == RFI_OK && cfg->schedule == RFI_SCHED_FUSED_PERSIST)
            e = warm_fused(cfg->elem_size, true, L.s);
        if (e == hipSuccess && rc == RFI_OK) e = hipStreamSynchronize(L.s);
        if (e != hipSuccess || rc != RFI_OK) {
            rfi_server_destroy(srv);
            return e != hipSuccess ? hip_fail(e) : rc;
        }
    }
    *out = srv;
    return RFI_OK;
}

int rfi_server_add_stream(rfi_server* srv, uint32_t stream_id, int32_t window, float k, int32_t mode)
{
    if (!srv || stream_id >= (uint32_t)srv->streams.size()) return RFI_ERR_INVALID;
    const int64_t L1 = 1;
    if (validate_values(srv->cfg.elem_size, 1, &L1, &window, &k, &mode) != RFI_OK) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    SrvStream& st = srv->streams[stream_id];
    if (st.active) return RFI_ERR_INVALID;
    const size_t bytes = (size_t)align64(window) * srv->cfg.elem_size;
    for (int b = 0; b < 2; ++b) {
        hipError_t e = hipMalloc(&st.carry[b], bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
    }
    st.active = true;
    st.W = window;
    st.k = k;
    st.mode = mode;
    st.lane = (int)(stream_id % srv->lanes.size());
    st.cur = 0;
    st.carry_len = 0;
    st.next_abs = 0;
    srv->lanes[st.lane].members.push_back(stream_id);
    return RFI_OK;
}

int rfi_server_submit(rfi_server* srv, uint32_t stream_id, const void* block_dev, void* out_dev,
                      int64_t n, rfi_window_stats* stats_dev, uint64_t* ticket)
{
    if (!srv) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    int rc = submit_locked(srv, stream_id, block_dev, out_dev, n, stats_dev, ticket);
    if (rc != RFI_OK) return rc;
    // The block is admitted: a batch that could not be staged stays queued
    // for the next dispatch; only a fault is reported here.
    rc = dispatch_lane(srv, srv->streams[stream_id].lane);
    return srv->fault != hipSuccess ? rc : RFI_OK;
}

int rfi_server_dispatch(rfi_server* srv)
{
    if (!srv) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    reap(srv);
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    return dispatch_all(srv);
}

int rfi_server_poll(rfi_server* srv, uint64_t ticket, int32_t* done, int64_t* samples_emitted,
                    int64_t* windows_emitted)
{
    if (!srv || ticket == 0) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    if (ticket >= srv->next_id) return RFI_ERR_INVALID;
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    reap(srv);
    int rc = srv->fault != hipSuccess ? hip_fail(srv->fault) : dispatch_all(srv);
    auto it = srv->recs.find(ticket);
    if (it == srv->recs.end()) {  // retired: it completed earlier
        if (done) *done = 1;
        if (samples_emitted) *samples_emitted = -1;
        if (windows_emitted) *windows_emitted = -1;
        return rc;
    }
    TicketRec& t = it->second;
    if (done) *done = t.state == kDone ? 1 : 0;
    if (samples_emitted) *samples_emitted = t.state >= kDispatched ? t.emitted_samples : 0;
    if (windows_emitted) *windows_emitted = t.state >= kDispatched ? t.emitted_windows : 0;
    if (t.state == kDone && !t.polled) {
        t.polled = true;
        srv->polled.push_back(ticket);
    }
    return rc;
}

int rfi_server_sync(rfi_server* srv)
{
    if (!srv) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    return sync_all(srv);
}

int rfi_server_flush(rfi_server* srv, uint32_t stream_id, void* out_dev, rfi_window_stats* stats_dev,
                     int64_t* n_out)
{
    if (!srv || stream_id >= (uint32_t)srv->streams.size()) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    SrvStream& st = srv->streams[stream_id];
    if (!st.active) return RFI_ERR_INVALID;
    if (((uintptr_t)out_dev | (uintptr_t)stats_dev) & 15u) return RFI_ERR_ALIGN;
    int rc = sync_all(srv);
    if (rc != RFI_OK) return rc;
    const int64_t c = st.carry_len;
    if (n_out) *n_out = c;
    if (c == 0) return RFI_OK;
    if (!out_dev) return RFI_ERR_INVALID;
    StreamDesc d;
    std::memset(&d, 0, sizeof(d));
    d.head_off = (uint64_t)(uintptr_t)st.carry[st.cur];
    d.head_len = (int32_t)c;
    d.x_off = d.head_off;  // no body samples
    d.length = c;
    d.y_off = (uint64_t)(uintptr_t)out_dev;
    d.stats_off = (uint64_t)(uintptr_t)stats_dev;
    d.flags = stats_dev ? 0 : kNoStats;
    d.abs_base = st.next_abs;
    d.window = st.W;
    d.k = st.k;
    d.mode = st.mode;
    d.key = stream_id;
    Lane& L = srv->lanes[st.lane];
    StreamDesc* dd = nullptr;
    Item* di = nullptr;
    CarryItem* dc = nullptr;
    rc = upload(L.slots[0], std::vector<StreamDesc>{d}, std::vector<Item>{Item{0, kItemGeneric, 0}},
                std::vector<CarryItem>{}, L.s, &dd, &di, &dc);
    if (rc != RFI_OK) return rc;
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.streams = dd;
    a.items = di;
    a.n_items = 1;
    a.seed = srv->cfg.seed;
    set_wg_per_cu(0);
    hipError_t e = srv->cfg.elem_size == 1 ? launch_i8_generic(a, 1 << st.mode, 1, L.s) : launch_i16_generic(a, 1, L.s);
    ++srv->n_launches;
    if (e == hipSuccess) e = hipStreamSynchronize(L.s);
    if (e != hipSuccess) return hip_fail(e);
    st.next_abs += c;
    st.carry_len = 0;
    return RFI_OK;
}

int rfi_server_snapshot(rfi_server* srv, uint32_t stream_id, int64_t* next_index, int32_t* carry_len,
                        void* carry_host)
{
    if (!srv || stream_id >= (uint32_t)srv->streams.size()) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    SrvStream& st = srv->streams[stream_id];
    if (!st.active) return RFI_ERR_INVALID;
    int rc = sync_all(srv);
    if (rc != RFI_OK) return rc;
    if (next_index) *next_index = st.next_abs;
    if (carry_len) *carry_len = st.carry_len;
    if (st.carry_len > 0) {
        if (!carry_host) return RFI_ERR_INVALID;
        hipError_t e = hipMemcpy(carry_host, st.carry[st.cur], (size_t)st.carry_len * srv->cfg.elem_size,
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
    }
    return RFI_OK;
}

int rfi_server_restore(rfi_server* srv, uint32_t stream_id, int64_t next_index, int32_t carry_len,
                       const void* carry_host)
{
    if (!srv || stream_id >= (uint32_t)srv->streams.size()) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    SrvStream& st = srv->streams[stream_id];
    if (!st.active || next_index < 0 || carry_len < 0 || carry_len >= st.W) return RFI_ERR_INVALID;
    if (carry_len > 0 && !carry_host) return RFI_ERR_INVALID;
    int rc = sync_all(srv);
    if (rc != RFI_OK) return rc;
    if (carry_len > 0) {
        hipError_t e = hipMemcpy(st.carry[st.cur], carry_host, (size_t)carry_len * srv->cfg.elem_size,
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
    }
    st.carry_len = carry_len;
    st.next_abs = next_index;
    return RFI_OK;
}

int rfi_server_counters(rfi_server* srv, uint64_t* admitted, uint64_t* refused, uint64_t* completed,
                        uint64_t* launches, uint64_t* live_records, uint64_t* live_peak)
{
    if (!srv) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    if (admitted) *admitted = srv->n_admitted;
    if (refused) *refused = srv->n_refused;
    if (completed) *completed = srv->n_completed;
    if (launches) *launches = srv->n_launches;
    if (live_records) *live_records = srv->recs.size();
    if (live_peak) *live_peak = srv->live_peak;
    return RFI_OK;
}

int rfi_server_ticket_times(rfi_server* srv, uint64_t ticket, int64_t* t_submit_ns, int64_t* t_done_ns)
{
    if (!srv || ticket == 0) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    if (ticket >= srv->next_id) return RFI_ERR_INVALID;
    auto it = srv->recs.find(ticket);
    if (it == srv->recs.end()) {  // retired
        if (t_submit_ns) *t_submit_ns = -1;
        if (t_done_ns) *t_done_ns = -1;
        return RFI_OK;
    }
    const TicketRec& t = it->second;
    if (t_submit_ns) *t_submit_ns = t.t_submit;
    if (t_done_ns) *t_done_ns = t.state == kDone ? t.t_done : 0;
    return RFI_OK;
}

int rfi_server_replay(rfi_server* srv, int64_t n_blocks, const uint32_t* stream_ids,
                      const int64_t* arrival_ns, const void* const* blocks, void* const* outs,
                      const int64_t* lengths, rfi_window_stats* const* stats, int64_t* latency_ns,
                      int64_t* samples_emitted)
{
    if (!srv || n_blocks < 0 || (n_blocks > 0 && (!stream_ids || !arrival_ns || !blocks || !outs ||
                                                  !lengths || !latency_ns)))
        return RFI_ERR_INVALID;
    for (int64_t i = 1; i < n_blocks; ++i)
        if (arrival_ns[i] < arrival_ns[i - 1]) return RFI_ERR_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->fault != hipSuccess) return hip_fail(srv->fault);
    std::vector<int64_t> done_at(n_blocks, 0), emitted(n_blocks, 0);
    std::deque<int64_t> waiting;  // arrived, not yet admitted (arrival order)
    // The lock is held throughout, so this call's tickets are numbered
    // consecutively from first_id in arrival order; their results are taken
    // at completion (sink) and their records retired at once.
    const uint64_t first_id = srv->next_id;
    srv->sink_first = first_id;
    srv->sink_n = n_blocks;
    srv->sink_done = done_at.data();
    srv->sink_emitted = emitted.data();
    int64_t next = 0, finished = 0;
    int rc = RFI_OK;
    const int64_t t0 = now_ns();
    while (finished < n_blocks) {
        const int64_t now = now_ns() - t0;
        while (next < n_blocks && arrival_ns[next] <= now) waiting.push_back(next++);
        while (!waiting.empty()) {
            const int64_t i = waiting.front();
            uint64_t id = 0;
            rc = submit_locked(srv, stream_ids[i], blocks[i], outs[i], lengths[i], stats ? stats[i] : nullptr, &id);
            if (rc == RFI_ERR_BUSY) {
                rc = RFI_OK;
                break;
            }
            if (rc != RFI_OK) break;
            waiting.pop_front();
        }
        if (rc != RFI_OK) {
            (void)sync_all(srv);
            break;
        }
        rc = dispatch_all(srv);
        if (rc != RFI_OK) break;
        reap(srv, first_id, &finished);
        if (srv->fault != hipSuccess) {
            rc = hip_fail(srv->fault);
            break;
        }
    }
    srv->sink_n = 0;
    srv->sink_done = srv->sink_emitted = nullptr;
    if (rc != RFI_OK) return rc;
    for (int64_t i = 0; i < n_blocks; ++i) {
        latency_ns[i] = done_at[i] - (t0 + arrival_ns[i]);
        if (samples_emitted) samples_emitted[i] = emitted[i];
    }
    return RFI_OK;
}

int rfi_server_destroy(rfi_server* srv)
{
    if (!srv) return RFI_OK;
    for (auto& L : srv->lanes) {
        if (L.s) (void)hipStreamSynchronize(L.s);
    }
    for (auto& L : srv->lanes) {
        for (auto& sl : L.slots) {
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.d_buf) (void)hipFree(sl.d_buf);
            if (sl.h_stage) (void)hipHostFree(sl.h_stage);
        }
        if (L.s) (void)hipStreamDestroy(L.s);
    }
    for (auto& st : srv->streams)
        for (auto* p : st.carry)
            if (p) (void)hipFree(p);
    delete srv;
    return RFI_OK;
}

}  // extern "C"
