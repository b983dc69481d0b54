// rfi_internal.hpp -- structures shared by the host runtime and the kernels
// of librfimad (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfi_mad.h"

namespace rfi {

// Samples of one workgroup tile: 16 KiB (4 waves x 64 lanes x 64 bytes).
constexpr int kTileBytes = 16384;
constexpr int kBlock = 256;

// Per-stream parameters, resident in device memory for the life of a plan.
// Addresses are byte offsets added to the base addresses of LaunchArgs, so
// one table serves any buffers (plans) or holds absolute addresses with
// zero bases (serving).
struct StreamDesc {
    uint64_t x_off;      // first input element
    uint64_t y_off;      // first output element (logical index 0)
    uint64_t stats_off;  // stats entry of window 0
    uint64_t head_off;   // carry samples that precede x (serving)
    int64_t length;      // logical samples: head_len + body samples
    int64_t abs_base;    // absolute stream index of logical sample 0
    int32_t window;      // W
    float k;             // threshold multiple
    int32_t mode;        // rfi_mode
    uint32_t key;        // Philox key word 1 (stream index or stream id)
    int32_t head_len;    // carry samples at head_off
    int32_t flags;       // kNoStats, kPadded
};
constexpr int32_t kNoStats = 1;
// The stream lies in the packed batch layout, whose buffers extend to a
// multiple of 64 elements past its end (reads may round up to 16 bytes).
constexpr int32_t kPadded = 2;

// A stream as the kernels see it, with addresses resolved.
struct StreamView {
    const void* x;
    void* y;
    rfi_window_stats* stats;  // NULL: no statistics
    const void* x_head;
    int64_t length;
    int64_t abs_base;
    int32_t window;
    float k;
    int32_t mode;
    uint32_t key;
    int32_t head_len;
    int32_t padded;  // kPadded
};

// One unit of work for a workgroup.
//   kind == kItemTile:    a 16 KiB tile of whole, aligned windows of a stream
//                         whose W is a tile class; `first` = first sample.
//   kind == kItemGeneric: one window of any size/alignment; `first` = its
//                         window index.
struct Item {
    int32_t stream;
    int32_t kind;
    int64_t first;
};
constexpr int32_t kItemTile = 0;
constexpr int32_t kItemGeneric = 1;

// Window classes with a register-resident tile path.
//   int8:  512, 1024, 2048, 4096 (one wave per window or less),
//          8192, 16384 (2 or 4 waves per window);
//   int16: 8192 (four waves per window).
inline __host__ __device__ int i8_tile_class(int32_t w)
{
    switch (w) {
        case 512: return 0;
        case 1024: return 1;
        case 2048: return 2;
        case 4096: return 3;
        case 8192: return 4;
        case 16384: return 5;
        default: return -1;
    }
}
constexpr int kI8Classes = 6;
inline __host__ __device__ int i16_tile_class(int32_t w) { return w == 8192 ? 0 : -1; }
constexpr int kI16Classes = 1;

// Internal mode: compute window statistics only (median, MAD, and the flag
// count and threshold of the window's own MAD); write no samples.  Used by
// the median-of-MAD path's first pass.
constexpr int32_t kModeStats = 3;

// Kernel launch requests issued by the host runtime.
struct LaunchArgs {
    const StreamDesc* streams;
    const Item* items;
    int64_t n_items;
    uint64_t seed;
    uint64_t x_base;      // added to StreamDesc::x_off / head_off
    uint64_t y_base;      // added to StreamDesc::y_off
    uint64_t stats_base;  // added to StreamDesc::stats_off
    int32_t no_stats;     // 1: write no statistics at all
    int32_t pad;
};

__host__ __device__ inline StreamView resolve(const StreamDesc& d, const LaunchArgs& a)
{
    StreamView v;
    v.x = reinterpret_cast<const void*>(static_cast<uintptr_t>(a.x_base + d.x_off));
    v.y = reinterpret_cast<void*>(static_cast<uintptr_t>(a.y_base + d.y_off));
    v.stats = (a.no_stats || (d.flags & kNoStats))
                  ? nullptr
                  : reinterpret_cast<rfi_window_stats*>(static_cast<uintptr_t>(a.stats_base + d.stats_off));
    v.x_head = reinterpret_cast<const void*>(static_cast<uintptr_t>(a.x_base + d.head_off));
    v.length = d.length;
    v.abs_base = d.abs_base;
    v.window = d.window;
    v.k = d.k;
    v.mode = d.mode;
    v.key = d.key;
    v.head_len = d.head_len;
    v.padded = (d.flags & kPadded) != 0;
    return v;
}

// Host wrappers around the kernels (defined in rfi_kernels.hip).
// cls: tile class (-1 = generic items); modes: bit m set if mode m occurs;
// fused: one kernel for all kinds.
hipError_t launch_i8_tiles(int cls, int modes, int tpw, const LaunchArgs& a, int grid, hipStream_t s);
// modes: bit m set if some window of the launch uses mode m.
// small_nt: 64 or 128 if every window of the launch spans at most 4 x that
// many 16-byte chunks (workgroups of that many threads when the launch has
// one workgroup per item); 0: 256-thread workgroups.
hipError_t launch_i8_generic(const LaunchArgs& a, int modes, int grid, hipStream_t s, int small_nt = 0);
hipError_t launch_i8_fused(int modes, const LaunchArgs& a, int grid, hipStream_t s);
hipError_t launch_i16_tiles(int cls, int modes, const LaunchArgs& a, int grid, hipStream_t s);
hipError_t launch_i16_generic(const LaunchArgs& a, int grid, hipStream_t s);
hipError_t launch_i16_fused(const LaunchArgs& a, int grid, hipStream_t s);
// One workgroup of the all-modes fused kernel (int8) or of the int16 fused
// kernel with no items.  A kernel that needs private (scratch) memory has
// it set up by the runtime at its first dispatch on a hardware queue, which
// can hold that queue for milliseconds; a server runs this once per lane
// when it is created, so that no block's latency pays for it.
hipError_t warm_fused(int elem_size, bool persist, hipStream_t s);

// Several outputs from one read (int8 tile items): output o uses the
// descriptors desc[o] (its k and mode; offsets as a.streams) and the bases
// y_base[o], stats_base[o] (0: no statistics).  a.items: tiles of one class.
struct MultiArgs {
    LaunchArgs a;
    const StreamDesc* desc[3];
    uint64_t y_base[3];
    uint64_t stats_base[3];
    int32_t n_out;
    int32_t pad;
};
// Outputs in zero or clip mode only.
hipError_t launch_i8_multi(int cls, const MultiArgs& ma, int grid, hipStream_t s);

// Median of MAD (int8).  Windows of all streams are numbered globally in
// the packed stats order; mad[g] is window g's own MAD, dm[g] receives the
// lower median of the MADs of its stream's last K windows.  Each stream's
// MAD sequence (emad, from eoff) is `pre` history slots (the MADs of earlier
// calls, right-aligned, hist_len[s] of them valid) followed by its windows;
// pre = 0 when there is no history, and emad is mad itself.
struct MomStream {
    int64_t woff;   // first window of the stream in the stats order
    int64_t nw;     // windows of the stream in this call
    int64_t eoff;   // first entry of the stream's MAD sequence
    int64_t pre;    // history slots before its first window (0 or K - 1)
    int64_t hoff;   // first row of the stream's block-count table
};
constexpr int kMomBlock = 64;  // entries per row of the block-count table
// hcnt[(hoff + b) * 256 + v] = #{j < 64 b : emad_j <= v} over the stream's
// sequence (pre + nw entries).  max_blocks: the largest ceil((pre + nw) / 64).
hipError_t launch_mom_counts(const MomStream* streams, int n_streams, int64_t max_blocks,
                             const uint8_t* emad, uint32_t* hcnt, hipStream_t s);
// hist_len: NULL when no stream has history slots.
hipError_t launch_mom_select(const MomStream* streams, int n_streams, int64_t total_windows,
                             int32_t mom_k, const uint8_t* emad, const uint32_t* hcnt,
                             const int32_t* hist_len, int32_t* dm, hipStream_t s);
// emad of streams with history slots: hist[s * pre + i] for the slots, then
// mad[woff + w] (total_ext = sum of pre + nw).
hipError_t launch_mom_extend(const MomStream* streams, int n_streams, int64_t total_ext,
                             const uint8_t* mad, const uint8_t* hist, uint8_t* emad, hipStream_t s);
// New history: the last min(pre, hist_len + nw) entries of each stream's
// sequence, right-aligned in hist[s * pre ..], and hist_len updated.
hipError_t launch_mom_history(const MomStream* streams, int n_streams, const uint8_t* emad, uint8_t* hist,
                              int32_t* hist_len, hipStream_t s);
// Replacement pass: items of up to 256 windows (<= 16 KiB) of one stream;
// window params from stats (median) and dm; rewrites n_flagged and threshold.
struct MomItem {
    int32_t stream;
    int32_t n_windows;
    int64_t first_window;  // within the stream
};
// abs_add: NULL, or per stream an offset added to its absolute sample index.
hipError_t launch_mom_apply(const LaunchArgs& a, const MomItem* items, int64_t n_items,
                            const int32_t* dm, const int64_t* stream_woff, const int64_t* abs_add,
                            rfi_window_stats* stats, hipStream_t s);
// Copies the MAD of every window out of the stats array (int8 MADs fit a byte).
hipError_t launch_mom_gather(const rfi_window_stats* stats, int64_t total_windows, uint8_t* mad,
                             hipStream_t s);

// Serving carry update: copies logical elements [from, from + count) of the
// concatenation (head[0 .. head_len), body[...]) to dst.  Addresses are
// absolute device addresses.
struct CarryItem {
    uint64_t head;
    uint64_t body;
    uint64_t dst;
    int32_t head_len;
    int32_t from;
    int32_t count;
    int32_t elem;  // 1 or 2 bytes
};
hipError_t launch_carry(const CarryItem* items, int n_items, hipStream_t s);

// Occupancy cap for the launches issued by this thread (0: none).
void set_wg_per_cu(int n);

// Occupancy-derived persistent grid size for a kernel choice.
int persistent_grid(int elem_size, int cls, int modes, bool fused);

}  // namespace rfi
