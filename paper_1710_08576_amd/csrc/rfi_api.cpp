// rfi_api.cpp -- C ABI of librfimad: argument checks, packed layout, plans
// (work tables + launch schedules + HIP-graph replay), the autotuner and the
// cached batch entry points.  Kernels live in rfi_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rfi_internal.hpp"
#include "rfi_runtime.hpp"

using namespace rfi;

namespace rfi {

static thread_local hipError_t t_last_hip = hipSuccess;

int hip_fail(hipError_t e)
{
    t_last_hip = e;
    return RFI_ERR_HIP;
}

static int64_t align64(int64_t n) { return (n + 63) / 64 * 64; }

int validate_values(int elem, int32_t n, const int64_t* L, const int32_t* W, const float* K,
                    const int32_t* M)
{
    if (elem != 1 && elem != 2) return RFI_ERR_INVALID;
    if (n < 0) return RFI_ERR_INVALID;
    if (n == 0) return RFI_OK;
    if (!L || !W || !K || !M) return RFI_ERR_INVALID;
    for (int32_t s = 0; s < n; ++s) {
        if (!std::isfinite(K[s]) || K[s] < 0.0f || K[s] > RFI_MAX_K) return RFI_ERR_INVALID;
        if (M[s] < RFI_MODE_ZERO || M[s] > RFI_MODE_NOISE) return RFI_ERR_INVALID;
    }
    if (rfi_layout(n, L, W, nullptr, nullptr, nullptr) < 0) return RFI_ERR_INVALID;
    return RFI_OK;
}

// ---------------------------------------------------------------------------
// Autotune table: launch choice per (GPU architecture, coarse plan
// signature), filled by rfi_plan_autotune, saved to and loaded from JSON.
// ---------------------------------------------------------------------------
struct TuneEntry {
    int sched;
    int tpw;
    int cap;
    float ms;
};

// Occupancy cap (workgroups per CU).  Without tuning: 8, which measured at
// or above the uncapped rate for every int8 window class and mode (fewer
// resident workgroups contend less for LDS banks and the L2).
constexpr int kDefaultWgPerCu = 8;
constexpr TuneEntry kUntuned = {RFI_SCHED_SPLIT, 1, kDefaultWgPerCu, 0.0f};

static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;  // key: "<arch>/<signature hex>"

static const char* const kSchedNames[RFI_SCHED_COUNT] = {
    "auto", "split", "split_persist", "fused", "per_stream", "fused_persist", "split_concurrent",
    "fused_concurrent", "one_launch", "one_launch_persist"};

static TuneEntry tuned(const std::string& key)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    return it == g_tune.end() ? kUntuned : it->second;
}

static void record_tuned(const std::string& key, const TuneEntry& e)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = e;
}

// Architecture name of device `dev` up to the first ':' ("gfx950"), cached.
static std::string device_arch(int dev)
{
    static std::mutex mu;
    static std::map<int, std::string> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch.resize(c);
    }
    cache[dev] = arch;
    return arch;
}

static std::string tune_key(const std::string& arch, uint64_t sig)
{
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)sig);
    return arch + "/" + buf;
}

// Tiny reader for the file rfi_tune_save writes: the objects of the
// "entries" array, each a flat object of string and number values.
static bool json_string(const std::string& obj, const char* key, std::string& out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    p = obj.find('"', p);
    if (p == std::string::npos) return false;
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos) return false;
    out = obj.substr(p + 1, q - p - 1);
    return true;
}

static bool json_number(const std::string& obj, const char* key, double& out)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    out = std::strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
}

int tune_load_file(const char* path)
{
    if (!path) return RFI_ERR_INVALID;
    FILE* f = std::fopen(path, "rb");
    if (!f) return RFI_ERR_INVALID;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    const size_t e = text.find("\"entries\"");
    if (e == std::string::npos) return RFI_ERR_INVALID;
    size_t p = text.find('[', e);
    if (p == std::string::npos) return RFI_ERR_INVALID;
    std::vector<std::pair<std::string, TuneEntry>> got;
    for (;;) {
        const size_t o = text.find_first_of("{]", p + 1);
        if (o == std::string::npos) return RFI_ERR_INVALID;
        if (text[o] == ']') break;
        const size_t c = text.find('}', o);
        if (c == std::string::npos) return RFI_ERR_INVALID;
        const std::string obj = text.substr(o, c - o + 1);
        std::string arch, sig, sched;
        double tpw = 0, cap = -1, ms = 0;
        if (!json_string(obj, "arch", arch) || !json_string(obj, "signature", sig) ||
            !json_string(obj, "schedule", sched) || !json_number(obj, "tiles_per_wg", tpw) ||
            !json_number(obj, "wg_per_cu", cap))
            return RFI_ERR_INVALID;
        (void)json_number(obj, "ms", ms);
        int si = -1;
        for (int i = 1; i < RFI_SCHED_COUNT; ++i)
            if (sched == kSchedNames[i]) si = i;
        char* end = nullptr;
        const unsigned long long sv = std::strtoull(sig.c_str(), &end, 16);
        if (si < 0 || sig.empty() || *end != '\0' || (tpw != 1 && tpw != 2) || cap < 0 || cap > 32)
            return RFI_ERR_INVALID;
        got.push_back({tune_key(arch, sv), TuneEntry{si, (int)tpw, (int)cap, (float)ms}});
        p = c;
    }
    for (const auto& kv : got) record_tuned(kv.first, kv.second);
    return RFI_OK;
}

int tune_save_file(const char* path)
{
    if (!path) return RFI_ERR_INVALID;
    std::map<std::string, TuneEntry> snap;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        snap = g_tune;
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return RFI_ERR_INVALID;
    std::fprintf(f, "{\n \"format\": \"rfimad autotune 1\",\n \"entries\": [");
    bool first = true;
    for (const auto& kv : snap) {
        const size_t slash = kv.first.find('/');
        const std::string arch = kv.first.substr(0, slash), sig = kv.first.substr(slash + 1);
        const uint64_t sv = std::strtoull(sig.c_str(), nullptr, 16);
        // readable form of the signature: dtype, window classes, irregular
        // windows, noise streams, generic work items
        std::string classes;
        const int elem = (int)(sv & 0xFF);
        for (int c = 0; c < 15; ++c)
            if (sv & (1ull << (8 + c))) {
                const int w = elem == 1 ? (512 << c) : 8192;
                classes += (classes.empty() ? "" : ", ") + std::to_string(w);
            }
        std::fprintf(f,
                     "%s\n  {\"arch\": \"%s\", \"signature\": \"%s\", \"elem_size\": %d, \"window_classes\": [%s], "
                     "\"irregular_windows\": %s, \"noise\": %s, \"generic_items\": %s, \"schedule\": \"%s\", "
                     "\"tiles_per_wg\": %d, \"wg_per_cu\": %d, \"ms\": %.6g}",
                     first ? "" : ",", arch.c_str(), sig.c_str(), elem, classes.c_str(),
                     (sv >> 23) & 1 ? "true" : "false", (sv >> 32) & 1 ? "true" : "false",
                     (sv >> 33) & 1 ? "true" : "false", kSchedNames[kv.second.sched], kv.second.tpw, kv.second.cap,
                     (double)kv.second.ms);
        first = false;
    }
    std::fprintf(f, "\n ]\n}\n");
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return RFI_ERR_INVALID;
    }
    return RFI_OK;
}

// RFI_TUNE_FILE: loaded at the first plan built in the process (a missing
// file is no error), written again after every autotune.
static const char* tune_env_file() { return std::getenv("RFI_TUNE_FILE"); }

static void tune_env_load_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const char* f = tune_env_file();
        if (f && *f) (void)tune_load_file(f);
    });
}

}  // namespace rfi

// ---------------------------------------------------------------------------
// Plans.
// ---------------------------------------------------------------------------
struct PlanLaunch {
    int kind;   // 0 tiles of one class, 1 generic, 2 fused (mode-major items)
    int queue;  // SPLIT_CONCURRENT: 0 = the caller's stream, 1.. = auxiliary streams
    int cls;    // tile class for kind 0
    int modes;  // bit m: some stream of the launch uses mode m
    int64_t first, count;
    int grid;
    int small = 0;  // generic: 64 / 128 if every window spans at most 256 / 512 chunks
};

struct GraphEntry {
    uint64_t x, y, st;
    hipStream_t s;
    int sched;
    int tpw;  // effective tiles per workgroup and occupancy cap at capture
    int cap;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct rfi_plan {
    int elem = 1;
    int n = 0;
    int device = 0;
    uint64_t seed = 0;
    std::vector<int64_t> L;
    std::vector<int32_t> W;
    std::vector<float> K;
    std::vector<int32_t> M;
    std::vector<StreamDesc> hdesc;
    std::vector<Item> hitems;
    // the same items twice: mode-major (fused launches), then from
    // one_first in the single-launch order
    std::vector<Item> hitems_fused;
    int64_t one_first = 0;
    StreamDesc* ddesc = nullptr;
    Item* ditems = nullptr;
    Item* ditems_fused = nullptr;
    int64_t n_windows = 0, n_tiles = 0, n_generic = 0;
    int schedule = RFI_SCHED_AUTO;
    int use_graph = 0;
    int tpw = 0;  // int8 tiles per workgroup in loop-free launches (0: tuned)
    int wg_per_cu = -1;  // occupancy cap (0: none, -1: tuned)
    std::string tune_key;  // "<arch>/<signature>" of the autotune table
    std::vector<PlanLaunch> launches[RFI_SCHED_COUNT];
    std::vector<GraphEntry> graphs;
    // SPLIT_CONCURRENT: auxiliary streams and fork/join events (created on
    // first use, default priority).
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
};

namespace rfi {

uint64_t plan_signature(const rfi_plan* p)
{
    // dtype, window classes present, noise present, generic present
    uint64_t sig = (uint64_t)p->elem;
    for (int s = 0; s < p->n; ++s) {
        const int cls = p->elem == 1 ? i8_tile_class(p->W[s]) : i16_tile_class(p->W[s]);
        sig |= 1ull << (8 + (cls < 0 ? 15 : cls));
        if (p->M[s] == RFI_MODE_NOISE) sig |= 1ull << 32;
    }
    if (p->n_generic) sig |= 1ull << 33;
    return sig;
}

static int tile_class(int elem, int32_t w) { return elem == 1 ? i8_tile_class(w) : i16_tile_class(w); }

static hipError_t run_launch(const rfi_plan* p, const PlanLaunch& l, const LaunchArgs& base,
                             hipStream_t s)
{
    const TuneEntry te = tuned(p->tune_key);
    set_wg_per_cu(p->wg_per_cu >= 0 ? p->wg_per_cu : te.cap);
    LaunchArgs a = base;
    a.items = (l.kind == 2 ? p->ditems_fused : p->ditems) + l.first;
    a.n_items = l.count;
    if (p->elem == 1) {
        if (l.kind == 0) return launch_i8_tiles(l.cls, l.modes, p->tpw > 0 ? p->tpw : te.tpw, a, l.grid, s);
        if (l.kind == 1) return launch_i8_generic(a, l.modes, l.grid, s, l.small);
        return launch_i8_fused(l.modes, a, l.grid, s);
    }
    if (l.kind == 0) return launch_i16_tiles(l.cls, l.modes, a, l.grid, s);
    if (l.kind == 1) return launch_i16_generic(a, l.grid, s);
    return launch_i16_fused(a, l.grid, s);
}

static void build_launches(rfi_plan* p)
{
    const int elem = p->elem;
    const int ncls = elem == 1 ? kI8Classes : kI16Classes;
    // Items are ordered: generic items, then tiles of class 0, 1, ...; in
    // each group by stream, then position.  Ranges per group:
    std::vector<int64_t> gbegin(ncls + 1, 0), gend(ncls + 1, 0);
    std::vector<int> gmodes(ncls + 1, 0);
    {
        int64_t pos = 0;
        for (int g = 0; g <= ncls; ++g) {
            gbegin[g] = pos;
            while (pos < (int64_t)p->hitems.size()) {
                const Item& it = p->hitems[pos];
                const int cls = it.kind == kItemGeneric ? -1 : tile_class(elem, p->W[it.stream]);
                const int grp = cls < 0 ? 0 : cls + 1;
                if (grp != g) break;
                gmodes[g] |= 1 << p->M[it.stream];
                ++pos;
            }
            gend[g] = pos;
        }
    }
    auto clamp_grid = [](int64_t c) { return (int)std::min<int64_t>(std::max<int64_t>(c, 1), 1 << 30); };
    for (int sched = 0; sched < RFI_SCHED_COUNT; ++sched) p->launches[sched].clear();
    // Split schedules: one launch for the generic items, and one per (tile
    // class, mode) pair present, so every tile launch runs a kernel compiled
    // for a single mode (leaner than one that branches over all three).
    for (int g = 0; g <= ncls; ++g) {
        const int64_t c = gend[g] - gbegin[g];
        if (c == 0) continue;
        const int cls = g - 1;
        int64_t b = gbegin[g];
        while (b < gend[g]) {
            int64_t e = gend[g];
            int modes = gmodes[g];
            if (g > 0) {
                const int m = p->M[p->hitems[b].stream];
                e = b;
                while (e < gend[g] && p->M[p->hitems[e].stream] == m) ++e;
                modes = 1 << m;
            }
            PlanLaunch l{g == 0 ? 1 : 0, 0, cls, modes, b, e - b, clamp_grid(e - b)};
            if (g == 0 && elem == 1) {
                // longest window of the launch; n + 30 <= 16 * 4 * NT keeps
                // it within 4 * NT chunks at any alignment
                int64_t nmax = 0;
                for (int64_t i = b; i < e; ++i) {
                    const Item& it = p->hitems[i];
                    const int64_t w = p->W[it.stream];
                    nmax = std::max<int64_t>(nmax, std::min<int64_t>(w, p->L[it.stream] - it.first * w));
                }
                l.small = nmax <= 4066 ? 64 : nmax <= 8162 ? 128 : 0;
            }
            p->launches[RFI_SCHED_SPLIT].push_back(l);
            l.grid = (int)std::min<int64_t>(e - b, persistent_grid(elem, cls, l.modes, false));
            p->launches[RFI_SCHED_SPLIT_PERSIST].push_back(l);
            b = e;
        }
    }
    // Fused schedules: one launch per mode present (int8; its kernel is
    // compiled for that mode), each over every class and the generic items
    // of that mode; int16 runs them all in one launch.
    {
        int64_t b = 0;
        const int64_t nf = p->one_first;
        while (b < nf) {
            int64_t e = nf;
            int modes = 7;
            if (elem == 1) {
                const int m = p->M[p->hitems_fused[b].stream];
                e = b;
                while (e < nf && p->M[p->hitems_fused[e].stream] == m) ++e;
                modes = 1 << m;
            }
            PlanLaunch f{2, 0, -1, modes, b, e - b, clamp_grid(e - b)};
            p->launches[RFI_SCHED_FUSED].push_back(f);
            f.grid = (int)std::min<int64_t>(e - b, persistent_grid(elem, -1, modes, true));
            p->launches[RFI_SCHED_FUSED_PERSIST].push_back(f);
            b = e;
        }
    }
    // One launch over every item of every class and mode (in the
    // heaviest-first order), one workgroup per item or a persistent grid:
    // the whole batch as a single kernel, compiled for the modes present.
    {
        const int64_t nf = (int64_t)p->hitems_fused.size() - p->one_first;
        if (nf > 0) {
            int modes = 0;
            for (int64_t i = p->one_first; i < p->one_first + nf; ++i)
                modes |= 1 << p->M[p->hitems_fused[i].stream];
            PlanLaunch f{2, 0, -1, modes, p->one_first, nf, clamp_grid(nf)};
            p->launches[RFI_SCHED_ONE_LAUNCH].push_back(f);
            f.grid = (int)std::min<int64_t>(nf, persistent_grid(elem, -1, modes, true));
            p->launches[RFI_SCHED_ONE_LAUNCH_PERSIST].push_back(f);
        }
    }
    // One ordinary launch per stream and kind (the plain baseline).
    for (int s = 0; s < p->n; ++s) {
        for (int g = 0; g <= ncls; ++g) {
            int64_t b = -1, e = -1;
            for (int64_t i = gbegin[g]; i < gend[g]; ++i) {
                if (p->hitems[i].stream == s) {
                    if (b < 0) b = i;
                    e = i + 1;
                } else if (b >= 0) {
                    break;
                }
            }
            if (b < 0) continue;
            PlanLaunch l{g == 0 ? 1 : 0, 0, g - 1, 1 << p->M[s], b, e - b, clamp_grid(e - b)};
            p->launches[RFI_SCHED_PER_STREAM].push_back(l);
        }
    }
    // Concurrent split: SPLIT's launches over four queues, largest first to
    // the least loaded queue (by items).
    {
        std::vector<PlanLaunch> ls = p->launches[RFI_SCHED_SPLIT];
        std::stable_sort(ls.begin(), ls.end(),
                         [](const PlanLaunch& a, const PlanLaunch& b) { return a.count > b.count; });
        int64_t load[4] = {0, 0, 0, 0};
        for (auto& l : ls) {
            int q = 0;
            for (int i = 1; i < 4; ++i)
                if (load[i] < load[q]) q = i;
            l.queue = q;
            load[q] += l.count;
        }
        p->launches[RFI_SCHED_SPLIT_CONCURRENT] = ls;
        std::vector<PlanLaunch> fs = p->launches[RFI_SCHED_FUSED];
        for (size_t i = 0; i < fs.size(); ++i) fs[i].queue = (int)(i % 4);
        p->launches[RFI_SCHED_FUSED_CONCURRENT] = fs;
    }
    p->launches[RFI_SCHED_AUTO] = p->launches[RFI_SCHED_SPLIT];
}

int plan_build(int elem, int32_t n, const int64_t* L, const int32_t* W, const float* K,
               const int32_t* M, uint64_t seed, rfi_plan** out)
{
    std::unique_ptr<rfi_plan> p(new rfi_plan);
    p->elem = elem;
    p->n = n;
    p->seed = seed;
    p->L.assign(L, L + n);
    p->W.assign(W, W + n);
    p->K.assign(K, K + n);
    p->M.assign(M, M + n);
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    const int64_t tile_samples = kTileBytes / elem;
    const int ncls = elem == 1 ? kI8Classes : kI16Classes;
    // Item order: generic items, then the tiles of class 0, 1, ...; within a
    // class by mode, then stream, then position.
    // (modes 0..2 and the internal statistics-only mode)
    constexpr int kModes = kModeStats + 1;
    std::vector<std::vector<Item>> groups((ncls + 1) * kModes);
    int64_t soff = 0, woff = 0;
    p->hdesc.resize(n);
    for (int s = 0; s < n; ++s) {
        StreamDesc& d = p->hdesc[s];
        std::memset(&d, 0, sizeof(d));
        d.x_off = (uint64_t)(soff * elem);
        d.y_off = (uint64_t)(soff * elem);
        d.stats_off = (uint64_t)(woff * (int64_t)sizeof(rfi_window_stats));
        d.head_off = 0;
        d.length = L[s];
        d.abs_base = 0;
        d.window = W[s];
        d.k = K[s];
        d.mode = M[s];
        d.key = (uint32_t)s;
        d.head_len = 0;
        d.flags = kPadded;
        const int64_t nw = (L[s] + W[s] - 1) / W[s];
        const int cls = tile_class(elem, W[s]);
        int64_t first_generic = 0;
        if (cls >= 0) {
            const int64_t nt = L[s] / tile_samples;
            auto& grp = groups[(cls + 1) * kModes + M[s]];
            for (int64_t t = 0; t < nt; ++t) grp.push_back(Item{s, kItemTile, t * tile_samples});
            first_generic = nt * (tile_samples / W[s]);
            p->n_tiles += nt;
        }
        for (int64_t w = first_generic; w < nw; ++w) groups[0].push_back(Item{s, kItemGeneric, w});
        p->n_generic += nw - first_generic;
        p->n_windows += nw;
        soff += align64(L[s]);
        woff += nw;
    }
    for (auto& g : groups) p->hitems.insert(p->hitems.end(), g.begin(), g.end());
    for (int m = 0; m < 3; ++m) {  // the statistics-only mode has no fused launch
        for (const Item& it : groups[0])
            if (M[it.stream] == m) p->hitems_fused.push_back(it);
        for (int c = 0; c < ncls; ++c) {
            const auto& g = groups[(c + 1) * kModes + m];
            p->hitems_fused.insert(p->hitems_fused.end(), g.begin(), g.end());
        }
    }
    // The single-launch schedules take the same items in a second order,
    // appended after the mode-major one: generic windows first, then the
    // noise tiles, then the others, narrow classes first in each, so that
    // a launch handing out items in order ends on its cheapest tiles.
    p->one_first = (int64_t)p->hitems_fused.size();
    for (int m : {RFI_MODE_NOISE, RFI_MODE_ZERO, RFI_MODE_CLIP})
        for (const Item& it : groups[0])
            if (M[it.stream] == m) p->hitems_fused.push_back(it);
    for (int c = 0; c < ncls; ++c) {
        const auto& g = groups[(c + 1) * kModes + RFI_MODE_NOISE];
        p->hitems_fused.insert(p->hitems_fused.end(), g.begin(), g.end());
    }
    for (int c = 0; c < ncls; ++c)
        for (int m : {RFI_MODE_ZERO, RFI_MODE_CLIP}) {
            const auto& g = groups[(c + 1) * kModes + m];
            p->hitems_fused.insert(p->hitems_fused.end(), g.begin(), g.end());
        }
    if (n > 0) {
        hipError_t e = hipMalloc(&p->ddesc, sizeof(StreamDesc) * n);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
        e = hipMemcpy(p->ddesc, p->hdesc.data(), sizeof(StreamDesc) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (!p->hitems.empty()) {
        hipError_t e = hipMalloc(&p->ditems, sizeof(Item) * p->hitems.size());
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
        e = hipMemcpy(p->ditems, p->hitems.data(), sizeof(Item) * p->hitems.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
        if (!p->hitems_fused.empty()) {
            e = hipMalloc(&p->ditems_fused, sizeof(Item) * p->hitems_fused.size());
            if (e != hipSuccess) return e == hipErrorOutOfMemory ? RFI_ERR_NOMEM : hip_fail(e);
            e = hipMemcpy(p->ditems_fused, p->hitems_fused.data(), sizeof(Item) * p->hitems_fused.size(),
                          hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e);
        }
    }
    build_launches(p.get());
    p->tune_key = tune_key(device_arch(p->device), plan_signature(p.get()));
    tune_env_load_once();
    *out = p.release();
    return RFI_OK;
}

static void drop_graphs(rfi_plan* p)
{
    for (auto& g : p->graphs) {
        (void)hipStreamSynchronize(g.s);
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
}

void plan_free(rfi_plan* p)
{
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    drop_graphs(p);
    for (int i = 0; i < 3; ++i) {
        if (p->aux[i]) (void)hipStreamDestroy(p->aux[i]);
        if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->ddesc || p->ditems) (void)hipDeviceSynchronize();
    if (p->ddesc) (void)hipFree(p->ddesc);
    if (p->ditems) (void)hipFree(p->ditems);
    if (p->ditems_fused) (void)hipFree(p->ditems_fused);
    (void)hipSetDevice(cur);
    delete p;
}

static int effective_schedule(const rfi_plan* p)
{
    if (p->schedule != RFI_SCHED_AUTO) return p->schedule;
    return tuned(p->tune_key).sched;
}

// Issues a schedule's launches on s; SPLIT_CONCURRENT forks them over the
// plan's auxiliary streams and joins them back on s (under capture the
// fork and join become graph edges).
static hipError_t run_schedule(rfi_plan* p, const std::vector<PlanLaunch>& ls, const LaunchArgs& base,
                               hipStream_t s, int sched)
{
    if (sched != RFI_SCHED_SPLIT_CONCURRENT && sched != RFI_SCHED_FUSED_CONCURRENT) {
        for (const auto& l : ls) {
            hipError_t e = run_launch(p, l, base, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!p->fork) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        if (!p->aux[i]) e = hipStreamCreateWithFlags(&p->aux[i], hipStreamNonBlocking);
        if (e == hipSuccess && !p->join[i]) e = hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(p->fork, s);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipStreamWaitEvent(p->aux[i], p->fork, 0);
    for (const auto& l : ls) {
        if (e != hipSuccess) break;
        e = run_launch(p, l, base, l.queue == 0 ? s : p->aux[l.queue - 1]);
    }
    for (int i = 0; i < 3; ++i) {
        // join every branch, also after an error, so no branch stays forked
        hipError_t j = hipEventRecord(p->join[i], p->aux[i]);
        if (j == hipSuccess) j = hipStreamWaitEvent(s, p->join[i], 0);
        if (e == hipSuccess) e = j;
    }
    return e;
}

int plan_execute(rfi_plan* p, const void* x, void* y, rfi_window_stats* st, hipStream_t s,
                 int sched_override)
{
    const int sched = sched_override >= 0 ? sched_override : effective_schedule(p);
    LaunchArgs base;
    std::memset(&base, 0, sizeof(base));
    base.streams = p->ddesc;
    base.seed = p->seed;
    base.x_base = (uint64_t)(uintptr_t)x;
    base.y_base = (uint64_t)(uintptr_t)y;
    base.stats_base = (uint64_t)(uintptr_t)st;
    base.no_stats = st ? 0 : 1;
    const auto& ls = p->launches[sched];
    if (p->use_graph && s != nullptr && !ls.empty()) {
        const TuneEntry te = tuned(p->tune_key);
        const int tpw = p->tpw > 0 ? p->tpw : te.tpw;
        const int cap = p->wg_per_cu >= 0 ? p->wg_per_cu : te.cap;
        for (auto& g : p->graphs) {
            if (g.x == base.x_base && g.y == base.y_base && g.st == base.stats_base && g.s == s &&
                g.sched == sched && g.tpw == tpw && g.cap == cap) {
                hipError_t e = hipGraphLaunch(g.exec, s);
                return e == hipSuccess ? RFI_OK : hip_fail(e);
            }
        }
        if (p->graphs.size() >= 8) {
            (void)hipStreamSynchronize(p->graphs.front().s);
            (void)hipGraphExecDestroy(p->graphs.front().exec);
            (void)hipGraphDestroy(p->graphs.front().graph);
            p->graphs.erase(p->graphs.begin());
        }
        GraphEntry g{base.x_base, base.y_base, base.stats_base, s, sched, tpw, cap, nullptr, nullptr};
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e);
        const hipError_t le = run_schedule(p, ls, base, s, sched);
        e = hipStreamEndCapture(s, &g.graph);
        if (le != hipSuccess) return hip_fail(le);
        if (e != hipSuccess) return hip_fail(e);
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return hip_fail(e);
        }
        p->graphs.push_back(g);
        e = hipGraphLaunch(g.exec, s);
        return e == hipSuccess ? RFI_OK : hip_fail(e);
    }
    const hipError_t e = run_schedule(p, ls, base, s, sched);
    return e == hipSuccess ? RFI_OK : hip_fail(e);
}

}  // namespace rfi

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
extern "C" {

const char* rfi_status_string(int status)
{
    switch (status) {
        case RFI_OK: return "ok";
        case RFI_ERR_INVALID: return "invalid argument";
        case RFI_ERR_ALIGN: return "pointer not 16-byte aligned";
        case RFI_ERR_UNSUPPORTED: return "unsupported request";
        case RFI_ERR_NOMEM: return "out of memory";
        case RFI_ERR_HIP: return hipGetErrorString(t_last_hip);
        case RFI_ERR_BUSY: return "admission refused: budget or in-flight limit reached";
        default: return "unknown status";
    }
}

const char* rfi_version(void) { return "rfimad 0.1 gfx950"; }

int64_t rfi_layout(int32_t n_streams, const int64_t* lengths, const int32_t* windows,
                   int64_t* sample_offsets, int64_t* window_offsets, int64_t* total_elems)
{
    if (n_streams < 0 || (n_streams > 0 && (!lengths || !windows))) return RFI_ERR_INVALID;
    int64_t samples = 0, wins = 0;
    const int64_t kLimit = (int64_t)1 << 61;
    for (int32_t s = 0; s < n_streams; ++s) {
        if (lengths[s] < 0 || lengths[s] > kLimit || windows[s] < 1 || windows[s] > RFI_MAX_WINDOW)
            return RFI_ERR_INVALID;
        if (sample_offsets) sample_offsets[s] = samples;
        if (window_offsets) window_offsets[s] = wins;
        samples += align64(lengths[s]);
        wins += (lengths[s] + windows[s] - 1) / windows[s];
        if (samples > kLimit) return RFI_ERR_INVALID;
    }
    if (total_elems) *total_elems = samples;
    return wins;
}

int rfi_validate(int32_t elem_size, const void* x, const void* y, int32_t n_streams,
                 const int64_t* lengths, const int32_t* windows, const float* k,
                 const int32_t* mode, const void* stats_out)
{
    int rc = rfi::validate_values(elem_size, n_streams, lengths, windows, k, mode);
    if (rc != RFI_OK || n_streams == 0) return rc;
    int64_t total = 0;
    const int64_t wins = rfi_layout(n_streams, lengths, windows, nullptr, nullptr, &total);
    if (total == 0) return RFI_OK;
    if (!x || !y) return RFI_ERR_INVALID;
    const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, sa = (uintptr_t)stats_out;
    if ((xa | ya | sa) & 15u) return RFI_ERR_ALIGN;
    const uintptr_t bytes = (uintptr_t)total * (uintptr_t)elem_size;
    auto overlap = [](uintptr_t a, uintptr_t an, uintptr_t b, uintptr_t bn) { return a < b + bn && b < a + an; };
    if (xa != ya && overlap(xa, bytes, ya, bytes)) return RFI_ERR_INVALID;
    if (stats_out && wins > 0) {
        const uintptr_t sb = (uintptr_t)wins * sizeof(rfi_window_stats);
        if (overlap(sa, sb, xa, bytes) || overlap(sa, sb, ya, bytes)) return RFI_ERR_INVALID;
    }
    return RFI_OK;
}

int rfi_plan_create(int32_t elem_size, int32_t n_streams, const int64_t* lengths,
                    const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                    rfi_plan** out)
{
    if (!out) return RFI_ERR_INVALID;
    *out = nullptr;
    // Argument values only: buffers are bound at execute.
    int rc = rfi::validate_values(elem_size, n_streams, lengths, windows, k, mode);
    if (rc != RFI_OK) return rc;
    return plan_build(elem_size, n_streams, lengths, windows, k, mode, seed, out);
}

int rfi_plan_set_schedule(rfi_plan* plan, int32_t schedule)
{
    if (!plan || schedule < 0 || schedule >= RFI_SCHED_COUNT) return RFI_ERR_INVALID;
    plan->schedule = schedule;
    return RFI_OK;
}

int rfi_plan_get_schedule(const rfi_plan* plan)
{
    if (!plan) return RFI_ERR_INVALID;
    return effective_schedule(plan);
}

int rfi_plan_set_graph(rfi_plan* plan, int32_t use_graph)
{
    if (!plan) return RFI_ERR_INVALID;
    plan->use_graph = use_graph ? 1 : 0;
    return RFI_OK;
}

int rfi_plan_set_option(rfi_plan* plan, int32_t option, int32_t value)
{
    if (!plan) return RFI_ERR_INVALID;
    if (option == RFI_OPT_TILES_PER_WG) {
        if (value < 0 || value > 2) return RFI_ERR_INVALID;
        plan->tpw = value;
        drop_graphs(plan);
        return RFI_OK;
    }
    if (option == RFI_OPT_WG_PER_CU) {
        if (value < -1 || value > 32) return RFI_ERR_INVALID;
        plan->wg_per_cu = value;
        drop_graphs(plan);
        return RFI_OK;
    }
    return RFI_ERR_INVALID;
}

int rfi_plan_execute(rfi_plan* plan, const void* x, void* y, rfi_window_stats* stats_out,
                     void* stream)
{
    if (!plan) return RFI_ERR_INVALID;
    int rc = rfi_validate(plan->elem, x, y, plan->n, plan->L.data(), plan->W.data(), plan->K.data(),
                          plan->M.data(), stats_out);
    if (rc != RFI_OK) return rc;
    return plan_execute(plan, x, y, stats_out, (hipStream_t)stream, -1);
}

int rfi_plan_info(const rfi_plan* plan, int32_t* n_launches, int64_t* n_windows, int64_t* n_tiles,
                  int64_t* n_generic)
{
    if (!plan) return RFI_ERR_INVALID;
    if (n_launches) *n_launches = (int32_t)plan->launches[effective_schedule(plan)].size();
    if (n_windows) *n_windows = plan->n_windows;
    if (n_tiles) *n_tiles = plan->n_tiles;
    if (n_generic) *n_generic = plan->n_generic;
    return RFI_OK;
}

int rfi_plan_autotune(rfi_plan* plan, const void* x, void* y, rfi_window_stats* stats_out,
                      void* stream, int32_t iters, int32_t* best_schedule, float* best_ms)
{
    if (!plan || iters < 1) return RFI_ERR_INVALID;
    int rc = rfi_validate(plan->elem, x, y, plan->n, plan->L.data(), plan->W.data(), plan->K.data(),
                          plan->M.data(), stats_out);
    if (rc != RFI_OK) return rc;
    // Every candidate runs several times on these buffers: in place, each
    // run would filter the output of the one before.
    if (x == y && plan->n_windows > 0) return RFI_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return hip_fail(hipGetLastError());
    int best = RFI_SCHED_SPLIT, best_tpw = 1, best_cap = kDefaultWgPerCu;
    float best_t = 1e30f;
    const int saved_tpw = plan->tpw, saved_cap = plan->wg_per_cu;
    struct Cand { int sched, tpw, cap; };
    const Cand cands[] = {{RFI_SCHED_SPLIT, 1, 8}, {RFI_SCHED_SPLIT, 1, 6}, {RFI_SCHED_SPLIT, 1, 0},
                          {RFI_SCHED_SPLIT, 2, 8}, {RFI_SCHED_SPLIT_PERSIST, 1, 8},
                          {RFI_SCHED_FUSED, 1, 8}, {RFI_SCHED_FUSED, 1, 0},
                          {RFI_SCHED_FUSED_PERSIST, 1, 0}, {RFI_SCHED_SPLIT_CONCURRENT, 1, 8},
                          {RFI_SCHED_SPLIT_CONCURRENT, 1, 0}, {RFI_SCHED_FUSED_CONCURRENT, 1, 8},
                          {RFI_SCHED_ONE_LAUNCH, 1, 8}, {RFI_SCHED_ONE_LAUNCH, 1, 0},
                          {RFI_SCHED_ONE_LAUNCH_PERSIST, 1, 0}};
    for (const Cand& cand : cands) {
        const int c = cand.sched;
        if (plan->launches[c].empty()) continue;
        plan->tpw = cand.tpw;
        plan->wg_per_cu = cand.cap;
        rc = plan_execute(plan, x, y, stats_out, s, c);  // warm-up (graph capture)
        if (rc != RFI_OK) break;
        std::vector<float> ts;
        for (int i = 0; i < iters; ++i) {
            (void)hipEventRecord(e0, s);
            rc = plan_execute(plan, x, y, stats_out, s, c);
            (void)hipEventRecord(e1, s);
            if (rc != RFI_OK) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ts.push_back(ms);
        }
        if (rc != RFI_OK) break;
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        if (med < best_t) {
            best_t = med;
            best = c;
            best_tpw = cand.tpw;
            best_cap = cand.cap;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->tpw = saved_tpw;
    plan->wg_per_cu = saved_cap;
    if (rc != RFI_OK) return rc;
    plan->schedule = best;
    plan->tpw = best_tpw;
    plan->wg_per_cu = best_cap;
    drop_graphs(plan);
    record_tuned(plan->tune_key, TuneEntry{best, best_tpw, best_cap, best_t});
    if (const char* f = tune_env_file())
        if (*f && tune_save_file(f) != RFI_OK) return RFI_ERR_INVALID;
    if (best_schedule) *best_schedule = best;
    if (best_ms) *best_ms = best_t;
    return RFI_OK;
}

int rfi_plan_destroy(rfi_plan* plan)
{
    plan_free(plan);
    return RFI_OK;
}

int rfi_tune_save(const char* path) { return rfi::tune_save_file(path); }

int rfi_tune_load(const char* path) { return rfi::tune_load_file(path); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Cached batch entry points.
// ---------------------------------------------------------------------------
namespace {

struct CacheKey {
    int elem;
    int device;
    uint64_t seed;
    std::vector<int64_t> L;
    std::vector<int32_t> W;
    std::vector<uint32_t> K;  // bit patterns
    std::vector<int32_t> M;
    bool operator<(const CacheKey& o) const
    {
        if (elem != o.elem) return elem < o.elem;
        if (device != o.device) return device < o.device;
        if (seed != o.seed) return seed < o.seed;
        if (L != o.L) return L < o.L;
        if (W != o.W) return W < o.W;
        if (K != o.K) return K < o.K;
        return M < o.M;
    }
};

std::mutex g_cache_mu;
std::map<CacheKey, rfi_plan*> g_cache;
std::vector<CacheKey> g_cache_order;
constexpr size_t kCacheMax = 32;

int cached_filter(int elem, const void* x, void* y, int32_t n, const int64_t* L, const int32_t* W,
                  const float* K, const int32_t* M, uint64_t seed, rfi_window_stats* st, void* stream)
{
    int rc = rfi_validate(elem, x, y, n, L, W, K, M, st);
    if (rc != RFI_OK) return rc;
    int64_t total = 0;
    rfi_layout(n, L, W, nullptr, nullptr, &total);
    if (n == 0 || total == 0) return RFI_OK;
    CacheKey key;
    key.elem = elem;
    if (hipGetDevice(&key.device) != hipSuccess) key.device = 0;
    key.seed = seed;
    key.L.assign(L, L + n);
    key.W.assign(W, W + n);
    key.K.resize(n);
    std::memcpy(key.K.data(), K, sizeof(float) * n);
    key.M.assign(M, M + n);
    std::lock_guard<std::mutex> g(g_cache_mu);
    rfi_plan* p = nullptr;
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        p = it->second;
    } else {
        if (g_cache.size() >= kCacheMax) {
            auto old = g_cache.find(g_cache_order.front());
            rfi::plan_free(old->second);
            g_cache.erase(old);
            g_cache_order.erase(g_cache_order.begin());
        }
        rc = rfi::plan_build(elem, n, L, W, K, M, seed, &p);
        if (rc != RFI_OK) return rc;
        g_cache[key] = p;
        g_cache_order.push_back(key);
    }
    return rfi::plan_execute(p, x, y, st, (hipStream_t)stream, -1);
}

}  // namespace

extern "C" {

int rfi_mad_filter(const int8_t* x, int8_t* y, int32_t n_streams, const int64_t* lengths,
                   const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                   rfi_window_stats* stats_out, void* stream)
{
    return cached_filter(1, x, y, n_streams, lengths, windows, k, mode, seed, stats_out, stream);
}

int rfi_mad_filter_i16(const int16_t* x, int16_t* y, int32_t n_streams, const int64_t* lengths,
                       const int32_t* windows, const float* k, const int32_t* mode, uint64_t seed,
                       rfi_window_stats* stats_out, void* stream)
{
    return cached_filter(2, x, y, n_streams, lengths, windows, k, mode, seed, stats_out, stream);
}

int rfi_shutdown(void)
{
    rfi::mom_shutdown();
    rfi::multi_shutdown();
    rfi::power_shutdown();
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (auto& kv : g_cache) rfi::plan_free(kv.second);
    g_cache.clear();
    g_cache_order.clear();
    return RFI_OK;
}

}  // extern "C"
