// rfi_kernels.hip -- gfx950 kernels of librfimad.
//
// Method (Buch et al., Sec. II-D): per non-overlapping window, the median
// M(x), the MAD D, the thresholds M(x) +/- k * (1.4826 * D) of Eq. (1) and the
// replacement of Eq. (2).  The work is a pure stream: every sample is read
// once from HBM and written once, so the kernels are built around 128-bit
// coalesced loads into registers and keep all per-window work in LDS.
//
// int8 windows: one 256-bin LDS histogram of x + 128 per window; a
//   segmented wave scan turns it into cumulative counts C[v]; the median is
//   the first bin with C >= r + 1 (r = floor((N-1)/2)); the MAD is the first
//   d with C[m+d] - C[m-d-1] >= r + 1, i.e. the |x - m| histogram folded out
//   of the same counts, so the samples are histogrammed once.  The flag
//   count is N - (C[hi] - C[lo-1]) and needs no extra pass.
// int16 windows (W 8192 tiles): a 12-bit coarse histogram of x + 32768 and
//   a 4-bit fine digit give the median; the MAD is bracketed to 16 values
//   from the same cumulative coarse counts and resolved by one filtered pass
//   over |x - m|.  Other int16 windows: an 8+8-bit radix select over global
//   memory (generic path).
// Replacement: the per-sample test |x - m| > t equals x < m - floor(t) or
//   x > m + floor(t) because |x - m| is an integer, so after one binary32
//   threshold per window everything is integer; int8 samples are clamped
//   four to a dword with packed 16-bit max/min.
// Noise: the flagged 4-sample parts of a workgroup's tile are pooled into
//   one list, one thread draws one Philox4x64-10 block per entry, and the
//   owners merge the noise bytes back, so the cost follows the number of
//   flagged parts, not the worst lane.
// Also here: the several-outputs tile kernel, the median-of-MAD passes
//   (MAD gather, block counts, search, history, replacement) and the serving
//   carry copy.
#include "rfi_device.hpp"
#include "rfi_internal.hpp"

namespace rfi {

__constant__ int16_t c_q8[4096] = {
#include "q8_table.inc"
};

struct WinParams {
    int32_t lo;   // lowest unflagged value, m - floor(t) saturated
    int32_t hi;   // highest unflagged value, m + floor(t) saturated
    int32_t m;    // median
    int32_t sq8;  // (int)(1.4826f * D * 256), Q8 robust sigma for noise
};

__device__ __forceinline__ uint64_t pick4(const Philox4x64& r, int i)
{
    const uint64_t a = (i & 1) ? r.w[1] : r.w[0];
    const uint64_t b = (i & 1) ? r.w[3] : r.w[2];
    return (i & 2) ? b : a;
}

// Robust sigma, threshold and the integer bounds of one window (Eq. (1)).
__device__ __forceinline__ float threshold_of(int D, float k, float& sig)
{
    sig = __fmul_rn(1.4826f, (float)D);
    return __fmul_rn(k, sig);
}

// ---------------------------------------------------------------------------
// int8: selection from a 256-bin histogram owned by an aligned group of G
// lanes (G = 8..64, 256 / G bins per lane).  On return the bins hold
// inclusive cumulative counts and every lane of the group has mb (median
// + 128) and D.  Used when a wave holds several windows.
// ---------------------------------------------------------------------------
// Smallest d in [0, 256) with f(d) >= need, for f non-decreasing with
// f(255) >= need, i.e. the number of d with f(d) < need.  The G lanes of a
// group test G evenly spaced candidates per step (a G-ary search), so the
// answer takes log_G(256) steps instead of a test of every d.
template <int G, int SPAN, class F>
__device__ __forceinline__ int group_search(int lo, uint32_t need, const F& f)
{
    if constexpr (SPAN <= 1) {
        return lo;
    } else {
        constexpr int STEP = SPAN >= G ? SPAN / G : 1;
        constexpr int NC = SPAN >= G ? G : SPAN;  // candidates tested
        const int sl = lane_id() & (G - 1);
        const int d = min(lo + (sl + 1) * STEP - 1, 255);
        const bool below = (NC == G || sl < NC) && f(d) < need;
        return group_search<G, STEP>(lo + group_count<G>(below) * STEP, need, f);
    }
}

// Narrow histograms are scanned by groups of G lanes, each lane over 256 / G
// consecutive bins read as 16-byte chunks.  With G = 16 (16 bins, four
// chunks per lane) bin v lives in word nphys(v): the chunks inside a lane's
// run are permuted by XOR with bits 6-7 of v, so that the group's 16-byte
// reads of the same chunk fall in different banks (without it the 16 lanes
// of a group meet in four).  Measured 4-6 % faster at W 512 and 1024; at
// G = 32 (W 2048) it did not pay, and G = 64 has a single chunk: identity.
template <int G>
__device__ __forceinline__ int nphys(int v)
{
    return G == 16 ? (v ^ (((v >> 6) & 3) << 2)) : v;
}
// nphys of the four bytes of u at once.
template <int G>
__device__ __forceinline__ uint32_t nphys4(uint32_t u)
{
    return G == 16 ? (u ^ ((u >> 4) & 0x0C0C0C0Cu)) : u;
}

// Median bin and MAD of one window from its 256-bin histogram hw (bin v
// counts samples x = v - 128), by the G lanes of a group.  Leaves the
// cumulative counts C[v] = #{x <= v - 128} in hw.
template <int G>
__device__ __forceinline__ void select_i8(uint32_t* hw, uint32_t need, int& mb, int& D)
{
    constexpr int BPL = 256 / G;
    const int sl = lane_id() & (G - 1);
    uint32_t* my = hw + sl * BPL;
    const int key = G == 16 ? (((sl >> 2) & 3) << 2) : 0;  // chunk permutation of nphys
    uint32_t c[BPL];
#pragma unroll
    for (int j = 0; j < BPL; j += 4) {
        const uint4 t = *reinterpret_cast<const uint4*>(my + (j ^ key));
        c[j] = t.x;
        c[j + 1] = t.y;
        c[j + 2] = t.z;
        c[j + 3] = t.w;
    }
#pragma unroll
    for (int j = 1; j < BPL; ++j) c[j] += c[j - 1];
    const uint32_t incl = group_incl_scan<G>(c[BPL - 1]);
    const uint32_t excl = incl - c[BPL - 1];
#pragma unroll
    for (int j = 0; j < BPL; ++j) c[j] += excl;
#pragma unroll
    for (int j = 0; j < BPL; j += 4)
        *reinterpret_cast<uint4*>(my + (j ^ key)) = make_uint4(c[j], c[j + 1], c[j + 2], c[j + 3]);
    wave_sync();
    // The median bin is the first v with C[v] >= need.
    mb = group_search<G, 256>(0, need, [&](int v) { return hw[nphys<G>(v)]; });
    // #{|x - m| <= d} = C[min(mb + d, 255)] - C[mb - d - 1] is non-decreasing
    // in d and reaches the window size at d = 255; D is its first d >= need.
    const int m0 = mb;
    D = group_search<G, 256>(0, need, [&](int d) {
        const int dn = m0 - d - 1;
        return hw[nphys<G>(min(m0 + d, 255))] - (dn >= 0 ? hw[nphys<G>(max(dn, 0))] : 0u);
    });
}

// Window parameters and statistics from the cumulative histogram hw.
template <int G>
__device__ __forceinline__ void params_i8(const uint32_t* hw, int mb, int D, float k, int n,
                                          WinParams& p, rfi_window_stats& s)
{
    float sig;
    const float t = threshold_of(D, k, sig);
    const int T = (int)floorf(t);
    const int m = mb - 128;
    const int lo = max(m - T, -128), hi = min(m + T, 127);
    const int lob = lo + 128, hib = hi + 128;
    const uint32_t inside = hw[nphys<G>(hib)] - (lob > 0 ? hw[nphys<G>(max(lob - 1, 0))] : 0u);
    p.lo = lo;
    p.hi = hi;
    p.m = m;
    p.sq8 = (int)__fmul_rn(sig, 256.0f);
    s.median = m;
    s.mad = D;
    s.n_flagged = (uint32_t)n - inside;
    s.threshold = t;
}

// ---------------------------------------------------------------------------
// Wide windows (W >= 4096, whole waves per window).  Each wave keeps four
// replicas of a 256-bin histogram (lane & 3 picks one; replicas start eight
// banks apart, which spreads same-bin atomics of a wave), indexed by the raw
// byte so a sample costs one bit-field extract and one address add.
// ---------------------------------------------------------------------------
constexpr int kRepStride = 264;                // 256 bins + 8 words
constexpr int kWaveHistWords = 4 * kRepStride;  // per wave
// Padded cumulative array: pc[0..3] = 0 (C[-4..-1]), pc[4 + v] = C[v] for
// the biased value v = 0..255, pc[260..263] = N.
constexpr int kPadC = 264;

__device__ __forceinline__ void wide_hist_zero(uint32_t* h)
{
    const int lane = lane_id();
    uint4* p = reinterpret_cast<uint4*>(h);
#pragma unroll
    for (int i = 0; i < (kWaveHistWords / 4 + 63) / 64; ++i) {
        const int idx = i * 64 + lane;
        if (idx < kWaveHistWords / 4) p[idx] = make_uint4(0, 0, 0, 0);
    }
}

// hl: this lane's replica.
__device__ __forceinline__ void wide_hist_add(uint32_t* hl, uint32_t x)
{
    atomicAdd(hl + (x & 0xFFu), 1u);
    atomicAdd(hl + ((x >> 8) & 0xFFu), 1u);
    atomicAdd(hl + ((x >> 16) & 0xFFu), 1u);
    atomicAdd(hl + (x >> 24), 1u);
}

// Counts of the biased bins 4*lane .. 4*lane+3 (biased bin v holds the raw
// byte (v + 128) & 255), summed over the four replicas.
__device__ __forceinline__ void wide_hist_totals(const uint32_t* h, uint32_t (&c)[4])
{
    const int rb = (4 * lane_id() + 128) & 255;
    c[0] = c[1] = c[2] = c[3] = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint4 t = *reinterpret_cast<const uint4*>(h + r * kRepStride + rb);
        c[0] += t.x;
        c[1] += t.y;
        c[2] += t.z;
        c[3] += t.w;
    }
}

// Selection over a whole wave holding the counts of bins 4*lane.. in c:
// writes the padded cumulative array pc and returns the wave-uniform mb
// (median + 128) and D.  The padding lets every lane read four consecutive
// counts without clamping its indices.
__device__ __forceinline__ void wide_select(uint32_t (&c)[4], uint32_t* pc, uint32_t need, int& mb,
                                            int& D)
{
    const int lane = lane_id();
    c[1] += c[0];
    c[2] += c[1];
    c[3] += c[2];
    const uint32_t incl = group_incl_scan<64>(c[3]);
    const uint32_t excl = incl - c[3];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] += excl;
    *reinterpret_cast<uint4*>(pc + 4 + 4 * lane) = make_uint4(c[0], c[1], c[2], c[3]);
    if (lane == 0) *reinterpret_cast<uint4*>(pc) = make_uint4(0, 0, 0, 0);
    if (lane == 63) *reinterpret_cast<uint4*>(pc + 260) = make_uint4(c[3], c[3], c[3], c[3]);
    int below = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) below += group_count<64>(c[j] < need);
    mb = below;
    wave_sync();
    // d = 4*lane + j: C[min(mb + d, 255)] - C[mb - d - 1]
    const int t = min(mb + 4 * lane, 255) + 4;
    const int s = max(mb - 4 * lane - 1, -1) + 4;
    int dbelow = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) dbelow += group_count<64>(pc[t + j] - pc[s - j] < need);
    D = dbelow;
}

__device__ __forceinline__ void wide_params(const uint32_t* pc, int mb, int D, float k, int n,
                                            WinParams& p, rfi_window_stats& s)
{
    float sig;
    const float t = threshold_of(D, k, sig);
    const int T = (int)floorf(t);
    const int m = mb - 128;
    const int lo = max(m - T, -128), hi = min(m + T, 127);
    const uint32_t inside = pc[4 + hi + 128] - pc[3 + lo + 128];
    p.lo = lo;
    p.hi = hi;
    p.m = m;
    p.sq8 = (int)__fmul_rn(sig, 256.0f);
    s.median = m;
    s.mad = D;
    s.n_flagged = (uint32_t)n - inside;
    s.threshold = t;
}

// ---------------------------------------------------------------------------
// Noise.  One Philox4x64-10 block (counter j >> 2) serves 4 consecutive
// samples: sample j takes word j & 3 and indexes the Q8 table with its 12
// most significant bits.
// ---------------------------------------------------------------------------
// 4 int8 noise samples starting at absolute index j0 (a multiple of 4):
// byte c is sample j0 + c.
__device__ __forceinline__ uint32_t noise_quad_i8(uint64_t j0, uint64_t seed, uint32_t key, int m,
                                                  int sq8)
{
    const Philox4x64 r = philox4x64_10(j0 >> 2, seed, key);
    uint32_t nb = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int g = c_q8[(uint32_t)(r.w[c] >> 52)];
        const int q = (sq8 * g + 32768) >> 16;  // |sq8 * g| < 2^31 for int8
        nb |= ((uint32_t)min(max(m + q, -128), 127) & 0xFFu) << (8 * c);
    }
    return nb;
}

// The flagged 4-sample parts (one Philox block each) of a workgroup's tile
// are pooled into one list, and one thread turns each entry into its
// merged part (noise in the flagged samples), so the draws of a workgroup
// occupy as few waves as the list needs and an isolated flagged sample
// costs one block.  A lane holds 4 load slots of P parts (4 / P dwords
// each); cf bit (slot * P + part) marks a part holding a flagged sample;
// merged(wave, lane, slot, part, x) returns the merged part from the input
// part x.  The list (1 KiB) and the parts (<= 2 KiB) live in LDS that the tile no
// longer needs once its windows' parameters are known (its histograms):
// nothing is written there before the first barrier below, which every
// wave reaches only after its selection.  The per-wave counts have storage
// of their own, as they are written before that barrier.
struct NoiseScratch {
    uint32_t* counts;  // [4]
    uint32_t* list;    // [256]
    uint4* data;       // [256], 16-byte aligned
};
constexpr int kNoiseAliasWords = 256 + 4 * 256;

template <int P> struct NoisePart;
template <> struct NoisePart<4> { using T = uint32_t; };
template <> struct NoisePart<2> { using T = uint2; };

// NT: threads of the workgroup (a multiple of 64, at most 256); the list
// holds NT parts a round.
template <int P, int NT = kBlock, class PartFn>
__device__ __forceinline__ void pool_noise(uint32_t (&v)[16], uint32_t cf, const NoiseScratch& ns,
                                           PartFn merged)
{
    using PartT = typename NoisePart<P>::T;
    constexpr int WPP = 4 / P;  // dwords per part
    constexpr int C = NT;       // parts per round
    PartT* data = reinterpret_cast<PartT*>(ns.data);
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const uint32_t cnt = __popc(cf);
    const uint32_t incl = group_incl_scan<64>(cnt);
    if (lane == 63) ns.counts[wave] = incl;
    __syncthreads();
    int wbase = 0, F = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int c = (int)ns.counts[w];
        wbase += w < wave ? c : 0;
        F += c;
    }
    const int base = wbase + (int)(incl - cnt);
    // With no entries the loop below has no barrier: close the counts reads
    // here so no wave reuses the scratch while another still reads it.
    if (F == 0) __syncthreads();
    for (int r0 = 0; r0 < F; r0 += C) {
        int e = base - r0;
#pragma unroll
        for (int q = 0; q < 4 * P; ++q) {
            if ((cf >> q) & 1u) {
                if (e >= 0 && e < C) {
                    ns.list[e] = (uint32_t)(wave << 8 | lane << 2 | (q / P)) | (uint32_t)(q % P) << 16;
                    if constexpr (P == 4) data[e] = v[q];
                    else data[e] = make_uint2(v[WPP * q], v[WPP * q + 1]);
                }
                ++e;
            }
        }
        __syncthreads();
        const int k = (int)threadIdx.x;
        if (k < min(C, F - r0)) {
            const uint32_t ent = ns.list[k];
            data[k] = merged((int)((ent >> 8) & 3u), (int)((ent >> 2) & 63u), (int)(ent & 3u),
                             (int)(ent >> 16), data[k]);
        }
        __syncthreads();
        e = base - r0;
#pragma unroll
        for (int q = 0; q < 4 * P; ++q) {
            if ((cf >> q) & 1u) {
                if (e >= 0 && e < C) {
                    if constexpr (P == 4) {
                        v[q] = data[e];
                    } else {
                        const uint2 t = data[e];
                        v[WPP * q] = t.x;
                        v[WPP * q + 1] = t.y;
                    }
                }
                ++e;
            }
        }
        __syncthreads();
    }
}

// pool_noise without its first barrier: each wave reserves its slots with
// one LDS atomic add on ns.counts[0], which the caller has zeroed before a
// workgroup barrier that precedes the call (the waves' slots then follow
// in the order of their adds).  The total is read after the barrier that
// closes the list writes.  A wave writes its list entries and parts as soon
// as it arrives, so the list and the parts must have storage of their own:
// unlike pool_noise's, they cannot alias memory that another wave of the
// workgroup may still be reading.
template <int P, class PartFn>
__device__ __forceinline__ void pool_noise_reserved(uint32_t (&v)[16], uint32_t cf, const NoiseScratch& ns,
                                                    PartFn merged)
{
    using PartT = typename NoisePart<P>::T;
    constexpr int WPP = 4 / P;
    constexpr int C = kBlock;
    PartT* data = reinterpret_cast<PartT*>(ns.data);
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const uint32_t cnt = __popc(cf);
    const uint32_t incl = group_incl_scan<64>(cnt);
    uint32_t wb = 0;
    if (lane == 63 && incl) wb = atomicAdd(&ns.counts[0], incl);
    wb = (uint32_t)__builtin_amdgcn_readlane((int)wb, 63);
    const int base = (int)(wb + incl - cnt);
    for (int r0 = 0;; r0 += C) {
        int e = base - r0;
#pragma unroll
        for (int q = 0; q < 4 * P; ++q) {
            if ((cf >> q) & 1u) {
                if (e >= 0 && e < C) {
                    ns.list[e] = (uint32_t)(wave << 8 | lane << 2 | (q / P)) | (uint32_t)(q % P) << 16;
                    if constexpr (P == 4) data[e] = v[q];
                    else data[e] = make_uint2(v[WPP * q], v[WPP * q + 1]);
                }
                ++e;
            }
        }
        __syncthreads();
        const int F = (int)ns.counts[0];  // every wave has added its count
        const int k = (int)threadIdx.x;
        if (k < min(C, F - r0)) {
            const uint32_t ent = ns.list[k];
            data[k] = merged((int)((ent >> 8) & 3u), (int)((ent >> 2) & 63u), (int)(ent & 3u),
                             (int)(ent >> 16), data[k]);
        }
        __syncthreads();
        e = base - r0;
#pragma unroll
        for (int q = 0; q < 4 * P; ++q) {
            if ((cf >> q) & 1u) {
                if (e >= 0 && e < C) {
                    if constexpr (P == 4) {
                        v[q] = data[e];
                    } else {
                        const uint2 t = data[e];
                        v[WPP * q] = t.x;
                        v[WPP * q + 1] = t.y;
                    }
                }
                ++e;
            }
        }
        __syncthreads();
        if (r0 + C >= F) break;
    }
}

// ---------------------------------------------------------------------------
// int8 tiles: 16 KiB of whole windows of one class W, 64 bytes per lane.
// ---------------------------------------------------------------------------
// Narrow windows: one 256-bin histogram per window, 12 words apart in bank
// order, so the same bin of the windows of a wave falls in different banks
// (12 measured 2-3 % faster than 8 at W 512, the same at W 1024 and 2048).
constexpr int kNarrowStride = 268;

template <int W, bool NS>
struct I8TileSmem {
    static constexpr int kWin = 16384 / W;
    static constexpr bool kWide = W >= 4096;
    static constexpr int kWPW = kWide ? W / 4096 : 1;  // waves per window
    // wide: per-wave replicated histograms; W = 4096 keeps its cumulative
    // counts in replica 0 of its wave, larger W in pc.
    // W = 512 runs its eight windows per wave in two rounds of four.
    static constexpr int kRounds = W == 512 ? 2 : 1;
    static constexpr int kHistWords = kWide ? 4 * kWaveHistWords : (kWin / kRounds) * kNarrowStride;
    static_assert(kHistWords >= kNoiseAliasWords, "noise scratch aliases the histograms");
    __align__(16) uint32_t hist[kHistWords];
    __align__(16) uint32_t tot[kWPW > 1 ? 4 * 256 : 0];  // each wave's bin totals
    WinParams prm[kWin];
    int32_t mad[kWin];  // statistics-only mode: each window's MAD
    uint32_t noise_counts[NS ? 4 : 0];
    __device__ NoiseScratch noise()
    {
        return NoiseScratch{noise_counts, hist, reinterpret_cast<uint4*>(hist + 256)};
    }
};

// Statistics record of one window produced by a tile, written by the caller
// once the tile's samples are stored.
struct TileStats {
    rfi_window_stats s;
    rfi_window_stats* dst;  // NULL: this lane writes nothing
};

__device__ __forceinline__ void write_stats(const TileStats& t)
{
    if (t.dst)
        gstore16(t.dst, make_uint4((uint32_t)t.s.median, (uint32_t)t.s.mad, t.s.n_flagged,
                                   __float_as_uint(t.s.threshold)));
}

// This lane's 64 bytes of a 16 KiB tile: four 16-byte loads at a 1 KiB
// stride, so each load instruction of the wave covers 1 KiB contiguously.
__device__ __forceinline__ void tile_load(const StreamView& d, int64_t first_byte, uint32_t (&v)[16])
{
    const uint8_t* xt = static_cast<const uint8_t*>(d.x) + first_byte + (threadIdx.x >> 6) * 4096 +
                        lane_id() * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 t = gload16_nt(xt + i * 1024);
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
    }
}

// Replacement of one lane's 16 dwords.  bounds(i) returns the window
// parameters of load slot i.  NOISE needs the pooled scratch.
template <int W, bool NS, int MODE, class Bounds>
__device__ __forceinline__ void i8_replace(const StreamView& d, int64_t first, uint64_t seed,
                                           I8TileSmem<W, NS>& sm, uint32_t (&v)[16], Bounds bounds)
{
    if constexpr (MODE == RFI_MODE_CLIP) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const WinParams p = bounds(i);
            const uint32_t lo = rep_i16(p.lo * 256), hi = rep_i16(p.hi * 256);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[4 * i + j] = clamp_i8x4(v[4 * i + j], lo, hi);
                sched_fence();
            }
        }
    } else if constexpr (MODE == RFI_MODE_ZERO) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const WinParams p = bounds(i);
            const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[4 * i + j] = byte_perm(0u, v[4 * i + j], flag_sel_i8x4(v[4 * i + j], lo_u, hi_u));
                sched_fence();
            }
        }
    } else {
        static_assert(NS, "noise needs its LDS scratch");
        uint32_t cf = 0;  // bit 4i + j: dword j of slot i holds a flagged sample
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const WinParams p = bounds(i);
            const uint32_t lo = rep_i16(p.lo * 256), hi = rep_i16(p.hi * 256);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                cf |= ((clamp_i8x4(v[4 * i + j], lo, hi) ^ v[4 * i + j]) != 0 ? 1u : 0u) << (4 * i + j);
            sched_fence();
        }
        if constexpr (NS) {
            const int64_t abs0 = d.abs_base + first;
            const uint32_t key1 = d.key;
            auto merged = [&](int wv, int ln, int slot, int part, uint32_t x) -> uint32_t {
                const int off = wv * 4096 + slot * 1024 + ln * 16 + part * 4;
                const WinParams p = sm.prm[off / W];
                const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
                const uint32_t nz = noise_quad_i8((uint64_t)(abs0 + off), seed, key1, p.m, p.sq8);
                return byte_perm(nz, x, flag_sel_i8x4(x, lo_u, hi_u));
            };
            pool_noise<4>(v, cf, sm.noise(), merged);
        }
    }
}

// Processes one int8 tile whose samples this lane already holds in v
// (tile_load), stores the output, and returns the statistics record this
// lane must write (see write_stats).
template <int W, bool NS, int MODE>
__device__ __forceinline__ TileStats i8_tile(const StreamView& d, int64_t first, uint64_t seed,
                                             I8TileSmem<W, NS>& sm, uint32_t (&v)[16])
{
    using Smem = I8TileSmem<W, NS>;
    constexpr uint32_t need = (W - 1) / 2 + 1;
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int wbase = wave * 4096;
    TileStats ts;
    ts.dst = nullptr;

    if constexpr (Smem::kWide) {
        constexpr int WPW = Smem::kWPW;
        const int wl = wave / WPW;
        uint32_t* h = sm.hist + wave * kWaveHistWords;
        if constexpr (WPW > 1) __syncthreads();  // the previous tile is done with tot and prm
        wide_hist_zero(h);
        wave_sync();
        uint32_t* hl = h + (lane & 3) * kRepStride;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            wide_hist_add(hl, v[q]);
            sched_fence();
        }
        wave_sync();
        uint32_t c[4];
        wide_hist_totals(h, c);
        // The cumulative counts overwrite replica 0 of the selecting wave,
        // whose reads were all issued above.
        uint32_t* pc = h;
        int mb = 0, D = 0;
        WinParams p;
        rfi_window_stats ws;
        if constexpr (WPW == 2) {
            // W 8192: both waves publish their totals; after one barrier each
            // wave adds its window's two and selects by itself (the same
            // values in both, no second exchange).
            *reinterpret_cast<uint4*>(sm.tot + wave * 256 + lane * 4) = make_uint4(c[0], c[1], c[2], c[3]);
            __syncthreads();
            const uint4 t0 = *reinterpret_cast<const uint4*>(sm.tot + (wl * 2) * 256 + lane * 4);
            const uint4 t1 = *reinterpret_cast<const uint4*>(sm.tot + (wl * 2 + 1) * 256 + lane * 4);
            c[0] = t0.x + t1.x;
            c[1] = t0.y + t1.y;
            c[2] = t0.z + t1.z;
            c[3] = t0.w + t1.w;
        } else if constexpr (WPW == 4) {
            // W 16384: the four waves' totals are added in LDS and one wave
            // selects (selecting in all four measured slower).
            if (threadIdx.x < 64) reinterpret_cast<uint4*>(sm.tot)[threadIdx.x] = make_uint4(0, 0, 0, 0);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 4; ++j) atomicAdd(&sm.tot[lane * 4 + j], c[j]);
            __syncthreads();
            if (wave == 0) {
                const uint4 t = *reinterpret_cast<const uint4*>(sm.tot + lane * 4);
                c[0] = t.x;
                c[1] = t.y;
                c[2] = t.z;
                c[3] = t.w;
            }
        }
        if (WPW < 4 || wave == 0) {
            wide_select(c, pc, need, mb, D);
            wide_params(pc, mb, D, d.k, W, p, ws);
        }
        if (wave % WPW == 0) {
            if (lane == 0) {
                sm.prm[wl] = p;
                if constexpr (MODE == kModeStats) sm.mad[wl] = D;
            }
            ts.s = ws;
            ts.dst = (lane == 0 && d.stats) ? d.stats + first / W + wl : nullptr;
        }
        if constexpr (WPW == 4) {
            __syncthreads();
            p = sm.prm[0];
        }
        // The record is complete: write it now rather than keep it in
        // registers through the replacement (the noise draws' peak).
        write_stats(ts);
        ts.dst = nullptr;
        if constexpr (MODE != kModeStats) i8_replace<W, NS, MODE>(d, first, seed, sm, v, [&](int) { return p; });
    } else {
        // Several windows per wave: one 256-bin histogram of x + 128 per
        // window.  W = 512 takes its eight windows per wave in two rounds
        // (loads 0-1, then 2-3) to halve the histogram space.
        constexpr int NWW = 4096 / W;           // windows per wave
        constexpr int ROUNDS = Smem::kRounds;
        constexpr int NWR = NWW / ROUNDS;       // windows per round
        constexpr int LPR = 4 / ROUNDS;         // loads per round
        constexpr int G = 64 / NWR;             // lanes per window in the scan
        uint32_t* hwave = sm.hist + wave * NWR * kNarrowStride;
        // A load's 1 KiB lies in at most two windows, so counting load i in
        // step i would send 32 or 64 lanes of a wave to one histogram and
        // serialise their same-bin atomics.  Lane groups count the loads of
        // a round in rotated order instead (lanes 8g .. 8g+7 mod 32 start at
        // load g for four loads per round, lanes 16g .. 16g+15 mod 32 at
        // load g for two), so each step spreads the wave over more windows.
        // The rotation uses masked selects with opaque masks, so it stays
        // bit-field inserts instead of becoming a per-lane indexed read.
        const int g = LPR == 4 ? (lane >> 3) & 3 : (lane >> 4) & 1;
        uint32_t m1 = (g & 1) ? ~0u : 0u, m2 = (g & 2) ? ~0u : 0u;
        asm volatile("" : "+v"(m1), "+v"(m2));
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if (r > 0) wave_sync();  // the previous round is done with the histograms
#pragma unroll
            for (int j = 0; j < NWR; ++j)
                reinterpret_cast<uint4*>(hwave + j * kNarrowStride)[lane] = make_uint4(0, 0, 0, 0);
            wave_sync();
            uint32_t q[4 * LPR];
#pragma unroll
            for (int t = 0; t < LPR; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int l0 = r * LPR + t, l1 = r * LPR + ((t + 1) % LPR);
                    q[4 * t + j] = bit_select(m1, v[4 * l1 + j], v[4 * l0 + j]);
                }
            if constexpr (LPR == 4) {
                uint32_t q2[16];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) q2[4 * t + j] = bit_select(m2, q[4 * ((t + 2) & 3) + j], q[4 * t + j]);
#pragma unroll
                for (int k = 0; k < 16; ++k) q[k] = q2[k];
            }
#pragma unroll
            for (int t = 0; t < LPR; ++t) {
                const int li = r * LPR + ((t + g) % LPR);
                uint32_t* hh = hwave + (((li * 1024 + lane * 16) / W) - r * NWR) * kNarrowStride;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t u = nphys4<G>(q[4 * t + j] ^ 0x80808080u);
                    atomicAdd(&hh[u & 0xFFu], 1u);
                    atomicAdd(&hh[(u >> 8) & 0xFFu], 1u);
                    atomicAdd(&hh[(u >> 16) & 0xFFu], 1u);
                    atomicAdd(&hh[u >> 24], 1u);
                    sched_fence();
                }
            }
            wave_sync();
            const int wl = wave * NWW + r * NWR + lane / G;
            uint32_t* hw = hwave + (lane / G) * kNarrowStride;
            int mb, D;
            select_i8<G>(hw, need, mb, D);
            WinParams p;
            rfi_window_stats ws;
            params_i8<G>(hw, mb, D, d.k, W, p, ws);
            // Lane r of the window's group keeps the statistics of round r.
            if ((lane & (G - 1)) == r) {
                sm.prm[wl] = p;
                if constexpr (MODE == kModeStats) sm.mad[wl] = D;
                ts.s = ws;
                ts.dst = d.stats ? d.stats + first / W + wl : nullptr;
            }
        }
        wave_sync();
        write_stats(ts);
        ts.dst = nullptr;
        if constexpr (MODE != kModeStats)
            i8_replace<W, NS, MODE>(d, first, seed, sm, v, [&](int i) {
                return sm.prm[(wbase + i * 1024 + lane * 16) / W];
            });
    }

    if constexpr (MODE != kModeStats) {
        uint8_t* yt = static_cast<uint8_t*>(d.y) + first + wbase + lane * 16;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            gstore16_nt(yt + i * 1024, make_uint4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]));
    }
    return ts;
}

// Mode dispatch: MODES is the set (bit m = mode m) compiled into a kernel.
template <int W, bool NS, int MODES>
__device__ __forceinline__ TileStats i8_tile_any(const StreamView& d, int64_t first, uint64_t seed,
                                                 I8TileSmem<W, NS>& sm, uint32_t (&v)[16])
{
    static_assert(!(MODES & 4) || NS, "noise needs its LDS scratch");
    if constexpr (MODES == (1 << kModeStats)) {
        return i8_tile<W, false, kModeStats>(d, first, seed, sm, v);
    } else if constexpr (MODES == 1) {
        return i8_tile<W, NS, RFI_MODE_ZERO>(d, first, seed, sm, v);
    } else if constexpr (MODES == 2) {
        return i8_tile<W, NS, RFI_MODE_CLIP>(d, first, seed, sm, v);
    } else if constexpr (MODES == 4) {
        return i8_tile<W, NS, RFI_MODE_NOISE>(d, first, seed, sm, v);
    } else {
        if ((MODES & 2) && d.mode == RFI_MODE_CLIP) return i8_tile<W, NS, RFI_MODE_CLIP>(d, first, seed, sm, v);
        if ((MODES & 1) && d.mode == RFI_MODE_ZERO) return i8_tile<W, NS, RFI_MODE_ZERO>(d, first, seed, sm, v);
        if constexpr ((MODES & 4) != 0) return i8_tile<W, NS, RFI_MODE_NOISE>(d, first, seed, sm, v);
        TileStats none;
        none.dst = nullptr;
        return none;
    }
}

// ---------------------------------------------------------------------------
// int8 generic window: any length, any alignment, optional head segment.
// One workgroup per window; two passes over the samples in global memory.
// ---------------------------------------------------------------------------
struct GenericSmem {
    union {
        uint32_t hist[4 * 256];                            // int16 radix: four digit histograms
        __align__(16) uint32_t whist[4 * kWaveHistWords];  // int8 register path: per-wave replicas
    };
    __align__(16) uint32_t tot[256];
    __align__(16) uint32_t pc[kPadC];
    WinParams prm;
    int32_t sel[4];
    uint32_t flagged;
};

template <typename T>
__device__ __forceinline__ int load_logical(const StreamView& d, int64_t i)
{
    return i < d.head_len ? (int)gload(static_cast<const T*>(d.x_head) + i)
                          : (int)gload(static_cast<const T*>(d.x) + (i - d.head_len));
}

// Noise sample for absolute index j (one Philox block per 4 samples).
__device__ __forceinline__ int noise_sample(int64_t j, uint64_t seed, uint32_t key, int m, int sq8,
                                            int vmin, int vmax)
{
    const Philox4x64 r = philox4x64_10((uint64_t)j >> 2, seed, key);
    const uint64_t word = pick4(r, (int)(j & 3));
    const int g = c_q8[(uint32_t)(word >> 52)];
    const int64_t q = ((int64_t)sq8 * g + 32768) >> 16;
    return (int)min(max((int64_t)m + q, (int64_t)vmin), (int64_t)vmax);
}

// Register path for a generic int8 window (zero, clip, statistics only,
// and noise where the instance allows it) with no head segment, 16-byte
// aligned input and output, and 512 <= n samples in at most four 16-byte
// chunks per thread: the aligned chunks covering [a, a + n) are loaded (four
// per lane), their in-window bytes counted into per-wave replicated histograms,
// the counts summed and selected as the wide tiles do, and the chunks
// replaced in registers and stored (whole chunks as one 16-byte store, the
// two edge chunks byte by byte, so a neighbouring window's bytes are never
// written).
constexpr int kGenericRegMin = 512;

// NOISE: noise-mode windows qualify too, when each dword of the stream holds
// one Philox block (absolute index of the stream's first sample a multiple
// of 4).
template <bool NOISE, int NT = kBlock>
__device__ __forceinline__ bool i8_generic_reg_ok(const StreamView& d, int64_t a, int n)
{
    if (d.head_len != 0 || n < kGenericRegMin) return false;
    if (d.mode == RFI_MODE_NOISE && (!NOISE || (d.abs_base & 3) != 0)) return false;
    if (((uintptr_t)d.x | (uintptr_t)d.y) & 15u) return false;
    // the last chunk may reach up to 15 bytes past the window: inside the
    // stream, or inside the packed layout's padding
    if (!d.padded && ((a + n + 15) & ~(int64_t)15) > d.length) return false;
    return ((a + n + 15) >> 4) - (a >> 4) <= 4 * NT;
}

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int b) { return (v >> (8 * b)) & 0xFFu; }

// NT: threads of the workgroup (256, or 64 / 128 for launches whose windows
// span at most 256 / 512 chunks, so that more windows are in flight per CU).
template <bool NOISE, int NT, class Smem>
__device__ void i8_generic_reg(const StreamView& d, int64_t w, int64_t a, int n, uint64_t seed, Smem& sm)
{
    const int tid = (int)threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint8_t* xb = static_cast<const uint8_t*>(d.x);
    uint8_t* yb = static_cast<uint8_t*>(d.y);
    const int64_t c0 = a >> 4, e = a + n;
    const int64_t nch = ((e + 15) >> 4) - c0;
    uint32_t v[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t c = tid + k * NT;
        uint4 t = make_uint4(0, 0, 0, 0);
        if (c < nch) t = gload16_nt(xb + (c0 + c) * 16);
        v[4 * k] = t.x;
        v[4 * k + 1] = t.y;
        v[4 * k + 2] = t.z;
        v[4 * k + 3] = t.w;
    }
    __syncthreads();  // the previous item is done with the scratch
    uint32_t* h = sm.whist + wave * kWaveHistWords;
    wide_hist_zero(h);
    if constexpr (NT > 64)
        for (int i = tid; i < 256; i += NT) sm.tot[i] = 0;
    __syncthreads();
    uint32_t* hl = h + (lane & 3) * kRepStride;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t c = tid + k * NT;
        if (c >= nch) continue;
        const int64_t cb = (c0 + c) * 16;
        if (cb >= a && cb + 16 <= e) {
#pragma unroll
            for (int j = 0; j < 4; ++j) wide_hist_add(hl, v[4 * k + j]);
        } else {
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (cb + b >= a && cb + b < e) atomicAdd(hl + byte_of(v[4 * k + b / 4], b % 4), 1u);
        }
    }
    wave_sync();
    uint32_t cnt[4];
    wide_hist_totals(h, cnt);
    if constexpr (NT > 64) {
#pragma unroll
        for (int j = 0; j < 4; ++j) atomicAdd(&sm.tot[lane * 4 + j], cnt[j]);
        __syncthreads();
        if (wave == 0) {
            const uint4 t = *reinterpret_cast<const uint4*>(sm.tot + lane * 4);
            cnt[0] = t.x;
            cnt[1] = t.y;
            cnt[2] = t.z;
            cnt[3] = t.w;
        }
    }
    if (wave == 0) {
        int mb, D;
        wide_select(cnt, sm.pc, (uint32_t)((n - 1) / 2 + 1), mb, D);
        WinParams p;
        rfi_window_stats s;
        wide_params(sm.pc, mb, D, d.k, n, p, s);
        if (lane == 0) {
            sm.prm = p;
            if (d.stats) d.stats[w] = s;
        }
    }
    __syncthreads();
    if (d.mode == kModeStats) return;
    const WinParams p = sm.prm;
    const uint32_t lo = rep_i16(p.lo * 256), hi = rep_i16(p.hi * 256);
    const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
    bool noise = false;
    if constexpr (NOISE) {
        if (d.mode == RFI_MODE_NOISE) {
            // One Philox block per dword holding a flagged sample (dword q
            // of a lane: chunk tid + (q / 4) NT, samples 4 (q % 4) ..), the
            // flagged dwords of the workgroup pooled so that the draws take
            // as few waves as there are flagged dwords.  The histograms are
            // dead once every wave holds the window's parameters.
            noise = true;
            uint32_t cf = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q)
                if (tid + (q >> 2) * NT < nch) cf |= ((clamp_i8x4(v[q], lo, hi) ^ v[q]) != 0 ? 1u : 0u) << q;
            const int64_t jb = d.abs_base + c0 * 16;
            if constexpr (NT >= 128) {
                auto merged = [&](int wv, int ln, int slot, int part, uint32_t x) -> uint32_t {
                    const int64_t j0 = jb + ((int64_t)(wv * 64 + ln) + (int64_t)slot * NT) * 16 + 4 * part;
                    const uint32_t nz = noise_quad_i8((uint64_t)j0, seed, d.key, p.m, p.sq8);
                    return byte_perm(nz, x, flag_sel_i8x4(x, lo_u, hi_u));
                };
                static_assert(sizeof(sm.whist) >= (16 + 2 * NT) * 4, "noise list in the histograms");
                pool_noise<4, NT>(v, cf,
                                  NoiseScratch{sm.whist, sm.whist + 16, reinterpret_cast<uint4*>(sm.whist + 16 + NT)},
                                  merged);
            } else {
                // One-wave workgroups (windows of at most 256 chunks) hold
                // few flagged dwords: each lane draws its own, in a loop over
                // them (no list, no barriers, fewer registers).
                while (cf) {
                    const int q = __builtin_ctz(cf);
                    cf &= cf - 1;
                    uint32_t x = 0;
#pragma unroll
                    for (int i = 0; i < 16; ++i) x = i == q ? v[i] : x;
                    const int64_t j0 = jb + (tid + (int64_t)(q >> 2) * NT) * 16 + 4 * (q & 3);
                    const uint32_t nz = noise_quad_i8((uint64_t)j0, seed, d.key, p.m, p.sq8);
                    x = byte_perm(nz, x, flag_sel_i8x4(x, lo_u, hi_u));
#pragma unroll
                    for (int i = 0; i < 16; ++i) v[i] = i == q ? x : v[i];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t c = tid + k * NT;
        if (c >= nch) continue;
        const int64_t cb = (c0 + c) * 16;
        uint32_t r[4];
        const bool clip = d.mode == RFI_MODE_CLIP;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = v[4 * k + j];
            r[j] = noise ? x : clip ? clamp_i8x4(x, lo, hi) : byte_perm(0u, x, flag_sel_i8x4(x, lo_u, hi_u));
        }
        if (cb >= a && cb + 16 <= e) {
            gstore16_nt(yb + cb, make_uint4(r[0], r[1], r[2], r[3]));
        } else {
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (cb + b >= a && cb + b < e) gstore(yb + cb + b, (uint8_t)byte_of(r[b / 4], b % 4));
        }
    }
}

// REG: the register path is compiled in (kernels that may see zero or clip
// windows).
// REG: zero/clip windows may take the register path; REG_NOISE: noise
// windows too (kept out of the fused kernels, whose register budget the
// inlined draw would raise).
template <bool REG = true, bool REG_NOISE = false, int NT = kBlock, class Smem = GenericSmem>
__device__ void i8_generic(const StreamView& d, int64_t w, uint64_t seed, Smem& sm)
{
    const int W = d.window;
    const int64_t a = w * (int64_t)W;
    const int n = (int)min((int64_t)W, d.length - a);
    if (REG && i8_generic_reg_ok<REG_NOISE, NT>(d, a, n)) {
        i8_generic_reg<REG_NOISE, NT>(d, w, a, n, seed, sm);
        return;
    }
    const int tid = (int)threadIdx.x;
    int8_t* y = static_cast<int8_t*>(d.y);
    __syncthreads();
    for (int i = tid; i < 256; i += NT) sm.hist[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += NT) atomicAdd(&sm.hist[load_logical<int8_t>(d, a + i) + 128], 1u);
    __syncthreads();
    if (tid < 64) {
        int mb, D;
        select_i8<64>(sm.hist, (uint32_t)((n - 1) / 2 + 1), mb, D);
        WinParams p;
        rfi_window_stats s;
        params_i8<64>(sm.hist, mb, D, d.k, n, p, s);
        if (tid == 0) {
            sm.prm = p;
            if (d.stats) d.stats[w] = s;
        }
    }
    __syncthreads();
    if (d.mode == kModeStats) return;
    const WinParams p = sm.prm;
    for (int i = tid; i < n; i += NT) {
        const int x = load_logical<int8_t>(d, a + i);
        int yv = x;
        if (x < p.lo || x > p.hi) {
            if (d.mode == RFI_MODE_ZERO) yv = 0;
            else if (d.mode == RFI_MODE_CLIP) yv = min(max(x, p.lo), p.hi);
            else yv = noise_sample(d.abs_base + a + i, seed, d.key, p.m, p.sq8, -128, 127);
        }
        gstore(y + a + i, (int8_t)yv);
    }
}

// Scratch of the generic kernels with NW = 1 or 2 waves: their replicated
// histograms (or the plain histogram of the two-pass path), the summed
// counts (two waves), the cumulative counts and the window's parameters
// (5.3 KB for one wave, so LDS admits 30 workgroups per CU; 10.6 KB for two).
template <int NW>
struct GenericSmemN {
    union {
        uint32_t hist[256];
        __align__(16) uint32_t whist[NW * kWaveHistWords];
    };
    __align__(16) uint32_t tot[NW > 1 ? 256 : 4];
    __align__(16) uint32_t pc[kPadC];
    WinParams prm;
};

// ---------------------------------------------------------------------------
// int16: radix select over two 8-bit digits.
// ---------------------------------------------------------------------------
// Find the bucket of rank `need` (1-based) in a 256-bin histogram whose bins
// are spread over R replicas (bin b, replica r at b * R + r).  Every lane of
// the wave gets the bucket and the count below it.  hw is left unchanged.
template <int R>
__device__ __forceinline__ void bucket_of(const uint32_t* hw, uint32_t need, int& bucket,
                                          uint32_t& below)
{
    const int lane = lane_id();
    uint32_t c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t* src = hw + (lane * 4 + j) * R;
        uint32_t s = 0;
        if constexpr (R >= 4) {
#pragma unroll
            for (int r = 0; r < R; r += 4) {
                const uint4 t = *reinterpret_cast<const uint4*>(src + r);
                s += t.x + t.y + t.z + t.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) s += src[r];
        }
        c[j] = s;
    }
#pragma unroll
    for (int j = 1; j < 4; ++j) c[j] += c[j - 1];
    const uint32_t incl = group_incl_scan<64>(c[3]);
    const uint32_t excl = incl - c[3];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] += excl;
    // Bins run in lane order and C is non-decreasing: the bucket holding
    // rank `need` is the number of bins with C < need.
    int nb = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) nb += group_count<64>(c[j] < need);
    bucket = min(nb, 255);  // 255 only if the histogram held fewer than `need`
    const int prev = bucket - 1;
    const int pj = prev & 3;
    const uint32_t mine = pj == 0 ? c[0] : pj == 1 ? c[1] : pj == 2 ? c[2] : c[3];
    const uint32_t got = (uint32_t)__builtin_amdgcn_readlane((int)mine, max(prev, 0) >> 2);
    below = prev >= 0 ? got : 0u;
}

__device__ __forceinline__ void zero_words(uint32_t* p, int words, int tid, int nthreads)
{
    for (int i = tid * 4; i < words; i += nthreads * 4)
        *reinterpret_cast<uint4*>(p + i) = make_uint4(0, 0, 0, 0);
}

// 4 int16 noise samples starting at absolute index j0 (a multiple of 4):
// dword k holds samples j0 + 2k (low half) and j0 + 2k + 1.
__device__ __forceinline__ uint2 noise_quad_i16(uint64_t j0, uint64_t seed, uint32_t key, int m,
                                                int sq8)
{
    const Philox4x64 r = philox4x64_10(j0 >> 2, seed, key);
    uint32_t o[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        uint32_t nb = 0;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int g = c_q8[(uint32_t)(r.w[2 * k + b] >> 52)];
            const int64_t q = ((int64_t)sq8 * g + 32768) >> 16;
            const int val = (int)min(max((int64_t)m + q, (int64_t)-32768), (int64_t)32767);
            nb |= ((uint32_t)val & 0xFFFFu) << (16 * b);
        }
        o[k] = nb;
    }
    return make_uint2(o[0], o[1]);
}

// int16 tile: radix selection with a 12-bit coarse digit and a 4-bit fine
// digit.  Sample values of a noise-dominated window sit within a few
// hundred of the median, so a coarse pass over the top 8 bits would send
// almost every sample to a handful of bins and serialise the LDS atomics;
// 4096 coarse bins (16 values each) spread them over hundreds.
// One copy of the coarse histogram: with the swizzle below the atomics of a
// Gaussian-like window spread over the banks well enough, and the smaller
// footprint (16 KiB) leaves room for more workgroups per CU than two
// copies did.
constexpr int kI16Reps = 1;  // replicas of the coarse histogram (replica = lane % R)

// Values of the full-resolution band of the fast path (one bin each).
constexpr int kI16Band = 4096;

struct I16TileSmem {
    // radix path: coarse counts h[bin * R + rep]; band path: one bin per
    // value of the band, then the bin of the samples above it
    __align__(16) uint32_t h[kI16Band + 16];
    uint32_t fine[2][16];  // fine digit inside the selected coarse bin
    uint32_t part[4];      // per-wave totals of the block scan
    int sel[2];            // selected coarse bin, count below it
    uint32_t flagged;
    uint32_t mad_below;    // samples with |x - m| below the MAD bracket
    uint32_t est[4];       // band path: the waves' median estimates
    uint32_t below;        // band path: samples below the band
    // The noise pool (pool_noise_reserved) writes its list while other
    // waves may still be searching the band's counts in h, so it has
    // storage of its own (3 KiB; 8 workgroups per CU still fit).
    uint32_t noise_counts[4];
    __align__(16) uint32_t noise_list[256];
    __align__(16) uint2 noise_data[256];
    __device__ NoiseScratch noise()
    {
        return NoiseScratch{noise_counts, noise_list, reinterpret_cast<uint4*>(noise_data)};
    }
};

// Physical word of histogram word w = bin * R + replica: the 16-byte
// chunks of each 64-word block are permuted by XOR with bits 6..9 of w, so
// that the selection's 16-byte row reads (lane t reads words 16Rt ..
// 16R(t+1) - 1) fall in distinct banks for 16 consecutive lanes; without it
// lanes 64 or 128 bytes apart meet in the same few banks.
__device__ __forceinline__ uint32_t i16_hidx(uint32_t w) { return w ^ (((w >> 6) & 15u) << 2); }

// Coarse bin holding rank `need` (1-based) of the 4096-bin histogram h, and
// the count of samples in lower bins, for the whole workgroup.  Thread t
// sums bins 16t .. 16t+15 over the replicas; ends with a barrier after
// which every thread may read sm.sel, and h holds the inclusive cumulative
// counts (h[bin] = samples in bins 0..bin; each thread rewrites only the
// bins it read).
__device__ __forceinline__ void i16_coarse_select(I16TileSmem& sm, uint32_t need)
{
    static_assert(kI16Reps == 1, "the cumulative counts are written one word per bin");
    constexpr int R = kI16Reps;
    const int tid = (int)threadIdx.x;
    const int lane = lane_id(), wave = tid >> 6;
    uint32_t c[16];
#pragma unroll
    for (int j = 0; j < 16 * R; j += 4) {
        const uint4 t = *reinterpret_cast<const uint4*>(sm.h + i16_hidx((uint32_t)(tid * 16 * R + j)));
        const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int bin = (j + q) / R;
            if ((j + q) % R == 0) c[bin] = w[q];
            else c[bin] += w[q];
        }
    }
#pragma unroll
    for (int j = 1; j < 16; ++j) c[j] += c[j - 1];
    const uint32_t incl = group_incl_scan<64>(c[15]);
    if (lane == 63) sm.part[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) off += w < wave ? sm.part[w] : 0u;
    const uint32_t excl = off + incl - c[15];
    if (excl < need && need <= excl + c[15]) {
        int cnt = 0;
        uint32_t below = excl;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t C = excl + c[j];
            cnt += C < need ? 1 : 0;
            below = C < need ? C : below;
        }
        sm.sel[0] = tid * 16 + cnt;
        sm.sel[1] = (int)below;
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4)
        *reinterpret_cast<uint4*>(sm.h + i16_hidx((uint32_t)(tid * 16 + j))) =
            make_uint4(excl + c[j], excl + c[j + 1], excl + c[j + 2], excl + c[j + 3]);
    __syncthreads();
}

// Lower end of the MAD bracket from the cumulative coarse counts of x + 32768
// (h after i16_coarse_select).  N(d) = #{|x - m| <= d} lies between the
// counts of the coarse bins inside and touching [M - d, M + d] (M = m +
// 32768); the smallest d whose touching count reaches `need` bounds the MAD
// from below, and the MAD is at most 15 above it (every bin touching
// [M - d, M + d] lies inside [M - d - 15, M + d + 15]).  A 64-way search by
// each wave over d in [0, 65535] (three rounds); reads only, no barrier.
__device__ __forceinline__ int i16_mad_lower(const I16TileSmem& sm, int M, uint32_t need)
{
    const int lane = lane_id();
    int lo = 0, span = 65536;
    while (span > 1) {
        const int step = (span + 63) >> 6;
        // sub-range `lane` is [lo + lane * step, lo + (lane + 1) * step - 1]
        const int right = min(lo + (lane + 1) * step - 1, lo + span - 1);
        bool ok = false;
        if (lo + lane * step < lo + span) {
            const int a = max(M - right, 0), c = min(M + right, 65535);
            const uint32_t hiC = sm.h[i16_hidx((uint32_t)(c >> 4))];
            const uint32_t loC = (a >> 4) > 0 ? sm.h[i16_hidx((uint32_t)((a >> 4) - 1))] : 0u;
            ok = hiC - loC >= need;
        }
        const uint64_t b = __ballot(ok);  // the last sub-range always qualifies
        const int f = (int)__builtin_ctzll(b);
        const int nlo = lo + f * step;
        span = min(step, lo + span - nlo);
        lo = nlo;
    }
    return lo;
}

// Fine digit (0..15) holding rank `need` of the 16-bin histogram f; every
// wave computes it (no barrier).
__device__ __forceinline__ int i16_fine_select(const uint32_t* f, uint32_t need)
{
    const int lane = lane_id();
    const uint32_t c = group_incl_scan<16>(lane < 16 ? f[lane & 15] : 0u);
    const uint64_t lt = __ballot(lane < 16 && c < need);
    return (int)__popcll(lt & 0xFFFFull);
}

__device__ __forceinline__ int lo16(uint32_t v) { return (int)(int16_t)(v & 0xFFFFu); }
__device__ __forceinline__ int hi16(uint32_t v) { return (int)(int16_t)(v >> 16); }

// int16 median and MAD by radix digits (the general path): a 12-bit coarse
// digit histogram, the coarse bin of the median, a 4-bit fine digit inside
// it, and the MAD from a 16-value bracket read off the coarse counts plus
// one filtered pass over |x - m|.  v: the tile's samples (16 dwords per
// lane); starts with a barrier (the scratch may still be read).
__device__ void i16_select_radix(const uint32_t (&v)[16], I16TileSmem& sm, int& m_out, int& D_out)
{
    constexpr int W = 8192;
    constexpr int R = kI16Reps;
    const int lane = lane_id();
    const int tid = (int)threadIdx.x;
    __syncthreads();
    zero_words(sm.h, 4096 * R, tid, kBlock);
    if (tid < 8) reinterpret_cast<uint4*>(&sm.fine[0][0])[tid] = make_uint4(0, 0, 0, 0);
    if (tid == 0) sm.mad_below = 0;
    __syncthreads();

    const uint32_t rep = (uint32_t)(lane & (R - 1));
    // Coarse digit of x + 32768: bits 4..15.
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t u = v[q] ^ 0x80008000u;
        atomicAdd(sm.h + i16_hidx(((u >> 4) & 0xFFFu) * R + rep), 1u);
        atomicAdd(sm.h + i16_hidx((u >> 20) * R + rep), 1u);
        sched_fence();
    }
    __syncthreads();
    constexpr uint32_t need = (W - 1) / 2 + 1;
    i16_coarse_select(sm, need);
    const int b1 = sm.sel[0];
    const uint32_t below1 = (uint32_t)sm.sel[1];
    // Fine digit inside coarse bin b1.  Words whose samples all lie outside
    // the bin in every lane are skipped with one wave-uniform test.
    const uint32_t B1 = ((uint32_t)b1 << 4) | ((uint32_t)b1 << 20);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t u = v[q] ^ 0x80008000u;
        const uint32_t t = u ^ B1;
        const bool in0 = (t & 0xFFF0u) == 0, in1 = (t & 0xFFF00000u) == 0;
        if (__ballot(in0 || in1) != 0) {
            if (in0) atomicAdd(&sm.fine[0][u & 0xFu], 1u);
            if (in1) atomicAdd(&sm.fine[0][(u >> 16) & 0xFu], 1u);
        }
    }
    __syncthreads();
    const int m = ((b1 << 4) | i16_fine_select(sm.fine[0], need - below1)) - 32768;
    // MAD: bracket [dlo, dlo + 15] from the coarse counts of x, then the
    // exact rank inside it from |x - m| of the samples (no second histogram
    // over 4096 bins).  The samples below the bracket are counted from
    // ballots (wave-uniform sums).
    const int dlo = i16_mad_lower(sm, m + 32768, need);
    const uint32_t m2 = rep_i16(m);
    const uint32_t dlo2 = rep_i16(dlo);
    uint32_t nbelow = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t dq = pk_absdiff_i16(v[q], m2);
        nbelow += (uint32_t)__popcll(__ballot((dq & 0xFFFFu) < (uint32_t)dlo)) +
                  (uint32_t)__popcll(__ballot(dq < ((uint32_t)dlo << 16)));
        pin_sgpr(nbelow);
        const uint32_t r = pk_sub_u16(dq, dlo2);  // wraps when below
        const bool in0 = (r & 0xFFFFu) < 16u, in1 = r < (16u << 16);
        if (__ballot(in0 || in1) != 0) {
            if (in0) atomicAdd(&sm.fine[1][r & 0xFu], 1u);
            if (in1) atomicAdd(&sm.fine[1][(r >> 16) & 0xFu], 1u);
        }
    }
    if (lane == 0) atomicAdd(&sm.mad_below, nbelow);
    __syncthreads();
    m_out = m;
    D_out = dlo + i16_fine_select(sm.fine[1], need - sm.mad_below);
}

// int16 median and MAD from one full-resolution histogram (the fast path).
// The band of kI16Band consecutive values of u = x + 32768 centred on an
// estimate of the median (the lower median of the four waves' sample
// medians, each over 64 of its samples) is counted at one bin per value,
// samples above it in one extra bin, samples below it by ballots.  The
// median is then read off the cumulative counts, and the MAD by a search
// over d of N(d) = #{m - d <= u <= m + d}, also read off them.  Returns
// false (every thread alike) when the median lies outside the band or the
// MAD reaches past it; the caller then selects by radix digits.  Exact
// either way: only where the counts are, not what they are, depends on
// the estimate.
__device__ bool i16_select_band(const uint32_t (&v)[16], I16TileSmem& sm, int& m_out, int& D_out)
{
    constexpr uint32_t need = 4096;  // rank floor((8192 - 1) / 2), 1-based
    const int lane = lane_id();
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    // This wave's estimate: the lower median of 64 of its samples (low
    // halves of dwords 0, 5, 10, 15 in lane groups of 16), by a bitwise
    // search on ballot counts.
    const uint32_t pick = lane < 16 ? v[0] : lane < 32 ? v[5] : lane < 48 ? v[10] : v[15];
    const uint32_t us = (pick ^ 0x8000u) & 0xFFFFu;
    uint32_t est = 0;
#pragma unroll
    for (int b = 15; b >= 8; --b) {
        const uint32_t t = est | (1u << b);
        est = __popcll(__ballot(us < t)) < 32 ? t : est;
    }
    est += 128;  // the middle of the 256-value bucket holding the estimate
    __syncthreads();  // the previous tile is done with the scratch
    zero_words(sm.h, kI16Band + 16, tid, kBlock);
    if (lane == 0) sm.est[wave] = est;
    if (tid == 0) {
        sm.below = 0;
        sm.flagged = 0;  // added to once the tile is replaced
        sm.noise_counts[0] = 0;  // the noise pool's slot reservations
    }
    __syncthreads();
    uint32_t e[4] = {sm.est[0], sm.est[1], sm.est[2], sm.est[3]};
    // lower median of the four estimates: the second smallest
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3 - i; ++j) {
            const uint32_t lo = min(e[j], e[j + 1]), hi = max(e[j], e[j + 1]);
            e[j] = lo;
            e[j + 1] = hi;
        }
    const int base = min(max((int)e[1] - kI16Band / 2, 0), 65536 - kI16Band);
    // u - base in each 16-bit half is x - (base - 32768) modulo 2^16.
    const uint32_t xb = (uint32_t)(base ^ 0x8000) & 0xFFFFu;
    const uint32_t xb2 = xb | (xb << 16);
    const int xs = base - 32768;  // the band's first sample value
    uint32_t below = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t x = v[q];
        // byte offset of each half's bin: (u - base) clamped to the extra
        // bin kI16Band, times 4
        const uint32_t t = pk_shl2_u16(pk_min_u16(pk_sub_u16(x, xb2), (uint32_t)kI16Band * 0x10001u));
        atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sm.h) + (t & 0xFFFFu)), 1u);
        atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sm.h) + (t >> 16)), 1u);
        below += (uint32_t)__popcll(__ballot((int)(int16_t)(x & 0xFFFFu) < xs)) +
                 (uint32_t)__popcll(__ballot((int32_t)x < xs * 65536));
        pin_sgpr(below);
        sched_fence();
    }
    if (lane == 0) atomicAdd(&sm.below, below);
    __syncthreads();
    const uint32_t bl = sm.below;
    // Thread t scans bins 16t .. 16t + 15, and rewrites them as inclusive
    // cumulative counts of the band (without the samples below it).
    uint32_t c[16];
#pragma unroll
    for (int j = 0; j < 16; j += 4) {
        const uint4 w = *reinterpret_cast<const uint4*>(sm.h + tid * 16 + j);
        c[j] = w.x;
        c[j + 1] = w.y;
        c[j + 2] = w.z;
        c[j + 3] = w.w;
    }
#pragma unroll
    for (int j = 1; j < 16; ++j) c[j] += c[j - 1];
    const uint32_t incl = group_incl_scan<64>(c[15]);
    if (lane == 63) sm.part[wave] = incl;
    __syncthreads();
    uint32_t off = 0, inside = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        off += w < wave ? sm.part[w] : 0u;
        inside += sm.part[w];
    }
    const uint32_t excl = bl + off + incl - c[15];
    if (excl < need && need <= excl + c[15]) {
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) cnt += excl + c[j] < need ? 1 : 0;
        sm.sel[0] = tid * 16 + cnt;
    }
#pragma unroll
    for (int j = 0; j < 16; j += 4)
        *reinterpret_cast<uint4*>(sm.h + tid * 16 + j) =
            make_uint4(excl + c[j], excl + c[j + 1], excl + c[j + 2], excl + c[j + 3]);
    __syncthreads();
    if (bl >= need || bl + inside < need) return false;  // the median is outside the band
    const int m = base + sm.sel[0];
    // C(u') = #{u <= u'} for u' in [base - 1, base + kI16Band - 1]
    auto C = [&](int u) -> uint32_t { return u < base ? bl : sm.h[u - base]; };
    const int dwin = min(base + kI16Band - 1 - m, m - base);
    if (C(m + dwin) - C(m - dwin - 1) < need) return false;  // the MAD reaches past the band
    // smallest d in [0, dwin] with N(d) >= need: 64-way search, each lane
    // testing the right end of its sub-range
    int lo = 0, span = dwin + 1;
    while (span > 1) {
        const int step = (span + 63) >> 6;
        const int right = min(lo + (lane + 1) * step - 1, lo + span - 1);
        const bool ok = lo + lane * step < lo + span && C(m + right) - C(m - right - 1) >= need;
        const int f = (int)__builtin_ctzll(__ballot(ok));  // the last sub-range always qualifies
        const int nlo = lo + f * step;
        span = min(step, lo + span - nlo);
        lo = nlo;
    }
    m_out = m - 32768;
    D_out = lo;
    return true;
}

// W = 8192 int16 samples = 16 KiB = one window per workgroup tile.
// MODES: bit m set if the launch has windows in mode m (one bit: the mode
// is fixed at compile time).
template <int MODES>
__device__ void i16_tile_8192(const StreamView& d, int64_t first, uint64_t seed, I16TileSmem& sm)
{
    constexpr int W = 8192;
    const int lane = lane_id();
    const int tid = (int)threadIdx.x;
    const int wbase = (tid >> 6) * 4096;  // bytes
    const uint8_t* xt = reinterpret_cast<const uint8_t*>(static_cast<const int16_t*>(d.x) + first) + wbase + lane * 16;

    uint32_t v[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 t = gload16_nt(xt + i * 1024);
        v[4 * i] = t.x;
        v[4 * i + 1] = t.y;
        v[4 * i + 2] = t.z;
        v[4 * i + 3] = t.w;
    }
    int m, D;
    if (!i16_select_band(v, sm, m, D)) i16_select_radix(v, sm, m, D);

    float sig;
    const float t = threshold_of(D, d.k, sig);
    const int T = (int)floorf(t);
    const int lo = max(m - T, -32768), hi = min(m + T, 32767);
    const uint32_t lo2 = rep_i16(lo), hi2 = rep_i16(hi);
    const int sq8 = (int)__fmul_rn(sig, 256.0f);
    const int mode = MODES == 1 ? RFI_MODE_ZERO : MODES == 2 ? RFI_MODE_CLIP : MODES == 4 ? RFI_MODE_NOISE : d.mode;
    uint32_t nflag = 0;  // wave-uniform (ballot counts)
    uint32_t cf = 0;     // bit 2i + h: dwords 2h, 2h + 1 of slot i hold a flagged sample
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t any = 0;
#pragma unroll
            for (int j = 2 * h; j < 2 * h + 2; ++j) {
                const int q = 4 * i + j;
                const uint32_t x = v[q];
                const uint32_t c = pk_clamp_i16(x, lo2, hi2);
                const uint32_t diff = c ^ x;  // non-zero halves: flagged samples
                nflag += (uint32_t)__popcll(__ballot((diff & 0xFFFFu) != 0)) +
                         (uint32_t)__popcll(__ballot(diff > 0xFFFFu));
                pin_sgpr(nflag);
                if (mode == RFI_MODE_CLIP) v[q] = c;
                else if (mode == RFI_MODE_ZERO) v[q] = x & ~pk_mask_nonzero_u16(diff);
                else any |= diff;
            }
            if (mode == RFI_MODE_NOISE) cf |= (any != 0 ? 1u : 0u) << (2 * i + h);
        }
    }
    if (mode == RFI_MODE_NOISE) {
        const int64_t abs0 = d.abs_base + first;
        const uint32_t key1 = d.key;
        auto merged = [&](int wv, int ln, int slot, int part, uint2 x) -> uint2 {
            // samples: 2048 per wave, 512 per load slot, 8 per lane, 4 per part
            const int off = wv * 2048 + slot * 512 + ln * 8 + part * 4;
            const uint2 nz = noise_quad_i16((uint64_t)(abs0 + off), seed, key1, m, sq8);
            const uint32_t m0 = nonzero_half_mask(pk_clamp_i16(x.x, lo2, hi2) ^ x.x);
            const uint32_t m1 = nonzero_half_mask(pk_clamp_i16(x.y, lo2, hi2) ^ x.y);
            return make_uint2((x.x & ~m0) | (nz.x & m0), (x.y & ~m1) | (nz.y & m1));
        };
        pool_noise_reserved<2>(v, cf, sm.noise(), merged);
    }
    // The store address is formed here from a fresh copy of the thread
    // index: kept live from the loads, its lane and wave offsets were spilled
    // to private memory and reloaded right before the stores.
    uint32_t t2 = (uint32_t)tid;
    asm volatile("" : "+v"(t2));
    uint8_t* yt = reinterpret_cast<uint8_t*>(static_cast<int16_t*>(d.y) + first) + (t2 >> 6) * 4096 + (t2 & 63) * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        gstore16_nt(yt + i * 1024, make_uint4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]));
    if (lane == 0) atomicAdd(&sm.flagged, nflag);
    __syncthreads();
    if (tid == 0 && d.stats) {
        rfi_window_stats s;
        s.median = m;
        s.mad = D;
        s.n_flagged = sm.flagged;
        s.threshold = t;
        d.stats[first / W] = s;
    }
}

// Generic int16 window: radix passes over global memory.
__device__ void i16_generic(const StreamView& d, int64_t w, uint64_t seed, GenericSmem& sm)
{
    const int W = d.window;
    const int64_t a = w * (int64_t)W;
    const int n = (int)min((int64_t)W, d.length - a);
    const int tid = (int)threadIdx.x;
    int16_t* y = static_cast<int16_t*>(d.y);
    uint32_t* h = sm.hist;
    const uint32_t need = (uint32_t)((n - 1) / 2 + 1);
    __syncthreads();
    for (int i = tid; i < 4 * 256; i += kBlock) h[i] = 0;
    if (tid == 0) sm.flagged = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kBlock)
        atomicAdd(&h[(uint32_t)(load_logical<int16_t>(d, a + i) + 32768) >> 8], 1u);
    __syncthreads();
    if (tid < 64) {
        int b;
        uint32_t below;
        bucket_of<1>(h, need, b, below);
        if (tid == 0) {
            sm.sel[0] = b;
            sm.sel[1] = (int)below;
        }
    }
    __syncthreads();
    const int b1 = sm.sel[0];
    const uint32_t below1 = (uint32_t)sm.sel[1];
    for (int i = tid; i < n; i += kBlock) {
        const uint32_t u = (uint32_t)(load_logical<int16_t>(d, a + i) + 32768);
        if ((int)(u >> 8) == b1) atomicAdd(&h[256 + (u & 0xFFu)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        int b;
        uint32_t below;
        bucket_of<1>(h + 256, need - below1, b, below);
        if (tid == 0) sm.sel[2] = ((b1 << 8) | b) - 32768;
    }
    __syncthreads();
    const int m = sm.sel[2];
    for (int i = tid; i < n; i += kBlock) {
        const uint32_t dv = (uint32_t)abs(load_logical<int16_t>(d, a + i) - m);
        atomicAdd(&h[512 + (dv >> 8)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        int b;
        uint32_t below;
        bucket_of<1>(h + 512, need, b, below);
        if (tid == 0) {
            sm.sel[0] = b;
            sm.sel[1] = (int)below;
        }
    }
    __syncthreads();
    const int b3 = sm.sel[0];
    const uint32_t below3 = (uint32_t)sm.sel[1];
    for (int i = tid; i < n; i += kBlock) {
        const uint32_t dv = (uint32_t)abs(load_logical<int16_t>(d, a + i) - m);
        if ((int)(dv >> 8) == b3) atomicAdd(&h[768 + (dv & 0xFFu)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        int b;
        uint32_t below;
        bucket_of<1>(h + 768, need - below3, b, below);
        if (tid == 0) sm.sel[3] = (b3 << 8) | b;
    }
    __syncthreads();
    const int D = sm.sel[3];
    float sig;
    const float t = threshold_of(D, d.k, sig);
    const int T = (int)floorf(t);
    const int lo = max(m - T, -32768), hi = min(m + T, 32767);
    const int sq8 = (int)__fmul_rn(sig, 256.0f);
    uint32_t nflag = 0;
    for (int i = tid; i < n; i += kBlock) {
        const int x = load_logical<int16_t>(d, a + i);
        int yv = x;
        if (x < lo || x > hi) {
            ++nflag;
            if (d.mode == RFI_MODE_ZERO) yv = 0;
            else if (d.mode == RFI_MODE_CLIP) yv = min(max(x, lo), hi);
            else yv = noise_sample(d.abs_base + a + i, seed, d.key, m, sq8, -32768, 32767);
        }
        gstore(y + a + i, (int16_t)yv);
    }
    nflag = group_sum<64>(nflag);
    if (lane_id() == 0) atomicAdd(&sm.flagged, nflag);
    __syncthreads();
    if (tid == 0 && d.stats) {
        rfi_window_stats s;
        s.median = m;
        s.mad = D;
        s.n_flagged = sm.flagged;
        s.threshold = t;
        d.stats[w] = s;
    }
}

// ---------------------------------------------------------------------------
// Kernels.  All loop over items with a grid stride, so the same kernel
// serves one-workgroup-per-item launches and persistent launches.
// ---------------------------------------------------------------------------
// Runs body(item_index) for this workgroup's items.  PERSIST: grid-stride
// loop; otherwise exactly one item per workgroup (no loop, so nothing is
// kept live across items).
template <bool PERSIST, class Body>
__device__ __forceinline__ void for_items(const LaunchArgs& a, Body body)
{
    if constexpr (PERSIST) {
        for (int64_t it = blockIdx.x; it < a.n_items; it += gridDim.x) body(it);
    } else {
        if ((int64_t)blockIdx.x < a.n_items) body((int64_t)blockIdx.x);
    }
}

// One or two tiles per workgroup.  With two, the second tile's loads are
// issued before the first tile is processed, so they are in flight while
// the first tile's histogram, selection and replacement run.
template <int CLS, int MODES, bool PERSIST, int TPW>
__global__ __launch_bounds__(kBlock) void k_i8_tiles(LaunchArgs a)
{
    constexpr int W = 512 << CLS;
    constexpr bool NOISE = (MODES & 4) != 0;
    __shared__ I8TileSmem<W, NOISE> sm;
    if constexpr (TPW == 1) {
        for_items<PERSIST>(a, [&](int64_t it) {
            const Item item = a.items[it];
            const StreamView d = resolve(a.streams[item.stream], a);
            uint32_t v[16];
            tile_load(d, item.first, v);
            write_stats(i8_tile_any<W, NOISE, MODES>(d, item.first, a.seed, sm, v));
        });
    } else {
        const int64_t it = 2 * (int64_t)blockIdx.x;
        if (it >= a.n_items) return;
        const bool two = it + 1 < a.n_items;
        const Item ia = a.items[it];
        const Item ib = a.items[two ? it + 1 : it];
        const StreamView da = resolve(a.streams[ia.stream], a);
        const StreamView db = resolve(a.streams[ib.stream], a);
        uint32_t va[16], vb[16];
        // Both loads are unconditional (the second repeats the first tile
        // when there is no second item): a branch around them would make
        // the first tile's waits cover the second tile's loads too.
        tile_load(da, ia.first, va);
        tile_load(db, ib.first, vb);
        const TileStats sa = i8_tile_any<W, NOISE, MODES>(da, ia.first, a.seed, sm, va);
        if (two) {
            if constexpr (W > 4096) __syncthreads();
            write_stats(i8_tile_any<W, NOISE, MODES>(db, ib.first, a.seed, sm, vb));
        }
        write_stats(sa);
    }
}

// NT = 64 or 128 threads per window, for launches whose windows all fit
// 4 * NT chunks (n <= 4066 or 8162 at any alignment): up to 30 or 15
// windows in flight per CU instead of the 8 of the 256-thread kernel.  One
// item per workgroup.
template <int NT, bool NOISE>
__global__ __launch_bounds__(NT, NOISE && NT >= 128 ? 8 : 0) void k_i8_generic_small(LaunchArgs a)
{
    __shared__ GenericSmemN<NT / 64> sm;
    if ((int64_t)blockIdx.x >= a.n_items) return;
    const Item item = a.items[blockIdx.x];
    const StreamView d = resolve(a.streams[item.stream], a);
    i8_generic<true, NOISE, NT>(d, item.first, a.seed, sm);
}

// NOISE: noise windows may take the register path (launched only for items
// that include noise streams: the draw costs registers the other modes'
// small windows would pay for in occupancy).
template <bool PERSIST, bool NOISE>
__global__ __launch_bounds__(kBlock, NOISE ? (PERSIST ? 4 : 8) : 0) void k_i8_generic(LaunchArgs a)
{
    __shared__ GenericSmem sm;
    for_items<PERSIST>(a, [&](int64_t it) {
        const Item item = a.items[it];
        const StreamView d = resolve(a.streams[item.stream], a);
        i8_generic<true, NOISE>(d, item.first, a.seed, sm);
    });
}

template <bool NS>
union I8FusedSmem {
    I8TileSmem<512, NS> c0;
    I8TileSmem<1024, NS> c1;
    I8TileSmem<2048, NS> c2;
    I8TileSmem<4096, NS> c3;
    I8TileSmem<8192, NS> c4;
    I8TileSmem<16384, NS> c5;
    GenericSmem g;
};

// Generic items of the all-modes fused kernel, which is too large for the
// compiler to inline the generic path: out of line, taking the descriptor's
// address and the launch's base addresses as scalars and resolving the
// stream itself.  Handing over the resolved stream (by reference, or by
// value, which the calling convention also passes through memory) made
// the caller store it to private memory before every item, tiles included:
// about 5 KiB of writes per wave.
template <bool REG, class Smem>
__device__ __noinline__ void i8_generic_item(const StreamDesc* sd, uint64_t x_base, uint64_t y_base,
                                             uint64_t stats_base, int32_t no_stats, int64_t w, uint64_t seed,
                                             Smem& sm)
{
    LaunchArgs la;
    la.x_base = x_base;
    la.y_base = y_base;
    la.stats_base = stats_base;
    la.no_stats = no_stats;
    const StreamView d = resolve(*sd, la);
    i8_generic<REG>(d, w, seed, sm);
}

// Every item kind and window class in one launch.  MODES: the modes of the
// launch's tiles (a kernel compiled for one mode needs fewer registers than
// one that branches over all three, and registers bound its occupancy);
// generic items take any mode.  The all-modes instance is bounded to four
// workgroups per CU (120 VGPRs, against 132 and three workgroups unbounded,
// a count set by the out-of-line generic item, which under the bound saves
// four callee-saved registers to private memory): on the 64-stream mixed
// batch 0.232 -> 0.214 ms in one launch; five workgroups (96 VGPRs)
// spilled in the tile code and lost it again.
// The one-mode instances keep the unbounded budget, which measured faster
// than five or seven workgroups per CU.
template <bool PERSIST, int MODES>
__global__ __launch_bounds__(kBlock, MODES == 7 ? 4 : 0) void k_i8_fused(LaunchArgs a)
{
    constexpr bool NS = (MODES & 4) != 0;
    __shared__ I8FusedSmem<NS> sm;
    for_items<PERSIST>(a, [&](int64_t it) {
        const Item item = a.items[it];
        if constexpr (MODES == 7) {
            if (item.kind == kItemGeneric) {
                i8_generic_item<true>(a.streams + item.stream, a.x_base, a.y_base, a.stats_base, a.no_stats,
                                      item.first, a.seed, sm.g);
                return;
            }
        }
        const StreamView d = resolve(a.streams[item.stream], a);
        if (item.kind == kItemGeneric) {
            i8_generic<(MODES & 3) != 0>(d, item.first, a.seed, sm.g);
            return;
        }
        // Items of different classes may follow each other: keep the LDS
        // of the previous item alive until every wave is done with it.
        __syncthreads();
        uint32_t v[16];
        tile_load(d, item.first, v);
        switch (i8_tile_class(d.window)) {
            case 0: write_stats(i8_tile_any<512, NS, MODES>(d, item.first, a.seed, sm.c0, v)); break;
            case 1: write_stats(i8_tile_any<1024, NS, MODES>(d, item.first, a.seed, sm.c1, v)); break;
            case 2: write_stats(i8_tile_any<2048, NS, MODES>(d, item.first, a.seed, sm.c2, v)); break;
            case 3: write_stats(i8_tile_any<4096, NS, MODES>(d, item.first, a.seed, sm.c3, v)); break;
            case 4: write_stats(i8_tile_any<8192, NS, MODES>(d, item.first, a.seed, sm.c4, v)); break;
            default: write_stats(i8_tile_any<16384, NS, MODES>(d, item.first, a.seed, sm.c5, v)); break;
        }
    });
}

// One tile per workgroup: eight workgroups per CU (the noise variant holds
// 63 VGPRs, against 68 and seven workgroups unbounded; 2.8 % faster in
// noise mode, zero and clip unchanged).  The persistent loop keeps more
// live (90-107 VGPRs): bounded the same way it spilled 88-120 bytes per
// lane and ran 27-31 % slower, so it keeps the unbounded budget.  (The int8
// tiles, bounded to 72 VGPRs, measured 2-3 % slower in noise mode.)
template <bool PERSIST, int MODES>
__global__ __launch_bounds__(kBlock, PERSIST ? 0 : 8) void k_i16_tiles(LaunchArgs a)
{
    __shared__ I16TileSmem sm;
    for_items<PERSIST>(a, [&](int64_t it) {
        const Item item = a.items[it];
        const StreamView d = resolve(a.streams[item.stream], a);
        i16_tile_8192<MODES>(d, item.first, a.seed, sm);
    });
}

template <bool PERSIST>
__global__ __launch_bounds__(kBlock) void k_i16_generic(LaunchArgs a)
{
    __shared__ GenericSmem sm;
    for_items<PERSIST>(a, [&](int64_t it) {
        const Item item = a.items[it];
        const StreamView d = resolve(a.streams[item.stream], a);
        i16_generic(d, item.first, a.seed, sm);
    });
}

union I16FusedSmem {
    I16TileSmem t;
    GenericSmem g;
};

template <bool PERSIST>
__global__ __launch_bounds__(kBlock) void k_i16_fused(LaunchArgs a)
{
    __shared__ I16FusedSmem sm;
    for_items<PERSIST>(a, [&](int64_t it) {
        const Item item = a.items[it];
        const StreamView d = resolve(a.streams[item.stream], a);
        if (item.kind == kItemGeneric) i16_generic(d, item.first, a.seed, sm.g);
        else i16_tile_8192<7>(d, item.first, a.seed, sm.t);
    });
}

// ---------------------------------------------------------------------------
// Several outputs from one read (int8 tiles): the tile's windows are
// selected once (statistics-only mode), then each output's parameters
// (its own k) are derived from the window's median and MAD and its
// replacement (its own mode) is applied to a copy of the tile and stored.
// Output o is the same as a single call with that output's k and mode.
// ---------------------------------------------------------------------------
template <int W>
struct I8MultiSmem {
    I8TileSmem<W, false> t;
    int32_t med[16384 / W];
    float thr[16384 / W];
    uint32_t nfl[16384 / W];
};

// Zero and clip outputs only: a noise output would keep a second copy of
// the tile and the pooled draws in registers, which costs more occupancy
// than a second read of the input (noise outputs are separate passes).
template <int CLS>
__global__ __launch_bounds__(kBlock) void k_i8_multi(MultiArgs ma)
{
    constexpr int W = 512 << CLS;
    constexpr int kWin = 16384 / W;
    __shared__ I8MultiSmem<W> sm;
    const LaunchArgs& a = ma.a;
    const Item item = a.items[blockIdx.x];
    const int tid = (int)threadIdx.x, lane = lane_id();
    const int wbase = (tid >> 6) * 4096;
    const StreamView d0 = resolve(a.streams[item.stream], a);
    uint32_t v[16];
    tile_load(d0, item.first, v);
    (void)i8_tile<W, false, kModeStats>(d0, item.first, a.seed, sm.t, v);
    __syncthreads();
    if (tid < kWin) sm.med[tid] = sm.t.prm[tid].m;
#pragma unroll 1
    for (int o = 0; o < ma.n_out; ++o) {
        LaunchArgs ao = a;
        ao.streams = ma.desc[o];
        ao.y_base = ma.y_base[o];
        ao.stats_base = ma.stats_base[o];
        ao.no_stats = ma.stats_base[o] == 0 ? 1 : 0;
        const StreamView d = resolve(ao.streams[item.stream], ao);
        __syncthreads();  // the previous output is done with prm and the scratch
        if (tid < kWin) {
            const int m = sm.med[tid];
            float sig;
            const float t = threshold_of(sm.t.mad[tid], d.k, sig);
            const int T = (int)floorf(t);
            WinParams p;
            p.lo = max(m - T, -128);
            p.hi = min(m + T, 127);
            p.m = m;
            p.sq8 = (int)__fmul_rn(sig, 256.0f);
            sm.t.prm[tid] = p;
            sm.thr[tid] = t;
            sm.nfl[tid] = 0;
        }
        __syncthreads();
        uint8_t* yt = static_cast<uint8_t*>(d.y) + item.first + wbase + lane * 16;
        {
            // zero / clip: slot by slot, four registers at a time
            const bool clip = d.mode == RFI_MODE_CLIP;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int win = (wbase + i * 1024 + lane * 16) / W;
                const WinParams p = sm.t.prm[win];
                const uint32_t lo = rep_i16(p.lo * 256), hi = rep_i16(p.hi * 256);
                const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
                uint32_t r[4], nf = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t xw = v[4 * i + j];
                    const uint32_t c = clamp_i8x4(xw, lo, hi);
                    nf += __popc(nonzero_byte_mask(c ^ xw)) >> 3;
                    r[j] = clip ? c : byte_perm(0u, xw, flag_sel_i8x4(xw, lo_u, hi_u));
                }
                if (nf) atomicAdd(&sm.nfl[win], nf);
                gstore16_nt(yt + i * 1024, make_uint4(r[0], r[1], r[2], r[3]));
            }
        }
        __syncthreads();
        if (tid < kWin && d.stats) {
            rfi_window_stats st;
            st.median = sm.med[tid];
            st.mad = sm.t.mad[tid];
            st.n_flagged = sm.nfl[tid];
            st.threshold = sm.thr[tid];
            d.stats[item.first / W + tid] = st;
        }
    }
}

// ---------------------------------------------------------------------------
// Median of MAD (Eq. (3)), int8: the MADs of the first pass are gathered,
// counted per stream in blocks of 64 windows, and each window's lower
// median of the MADs of its K-window history is found by a binary search
// over the 256 possible MAD values on those counts; a last pass applies
// Eqs. (1)-(2) with it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_mom_gather(const rfi_window_stats* __restrict__ stats,
                                                       int64_t total, uint8_t* __restrict__ mad)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g < total) mad[g] = (uint8_t)stats[g].mad;
}

// Two steps build row b of a stream's table, #{j < 64 b : mad_j <= v} for
// b = 0 .. ceil(nw / 64): per block of 64 windows (blockIdx.x = block b of
// stream blockIdx.y, thread v) the block's own count goes to row b + 1, then
// one workgroup per stream turns the rows into running sums.
__global__ __launch_bounds__(256) void k_mom_block_counts(const MomStream* __restrict__ streams,
                                                          const uint8_t* __restrict__ mad,
                                                          uint32_t* __restrict__ hcnt)
{
    const MomStream st = streams[blockIdx.y];
    const int64_t n = st.pre + st.nw;
    const int64_t j0 = (int64_t)blockIdx.x * kMomBlock;
    if (j0 >= n) return;
    __shared__ uint8_t m[kMomBlock];
    const int64_t j1 = min(j0 + kMomBlock, n);
    if ((int64_t)threadIdx.x < j1 - j0) m[threadIdx.x] = mad[st.eoff + j0 + threadIdx.x];
    __syncthreads();
    const uint32_t v = threadIdx.x;
    uint32_t c = 0;
    for (int j = 0; j < (int)(j1 - j0); ++j) c += m[j] <= v ? 1u : 0u;
    hcnt[(st.hoff + blockIdx.x + 1) * 256 + v] = c;
}

__global__ __launch_bounds__(256) void k_mom_counts(const MomStream* __restrict__ streams,
                                                    uint32_t* __restrict__ hcnt)
{
    const MomStream st = streams[blockIdx.x];
    uint32_t* row = hcnt + st.hoff * 256 + threadIdx.x;
    const int64_t nb = (st.pre + st.nw + kMomBlock - 1) / kMomBlock;
    uint32_t run = 0;
    row[0] = 0;
    // 16 rows per batch: their loads are in flight together
    for (int64_t b0 = 1; b0 <= nb; b0 += 16) {
        uint32_t t[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) t[i] = b0 + i <= nb ? row[(b0 + i) * 256] : 0u;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            run += t[i];
            if (b0 + i <= nb) row[(b0 + i) * 256] = run;
        }
    }
}

// The partial block of prefix p: entries [kMomBlock * (p / kMomBlock), p)
// of a MAD sequence, four to a dword (entry 4i + c in byte c of w[i]), the
// bytes from p on set to 255.  Only dwords holding an entry are read.
__device__ __forceinline__ void mom_partial(const uint8_t* m, int64_t p, uint32_t (&w)[16])
{
    const int64_t j0 = p / kMomBlock * kMomBlock;
    const int n = (int)(p - j0);  // 0 .. kMomBlock - 1
    const uintptr_t a = (uintptr_t)(m + j0);
    const uint32_t* base = reinterpret_cast<const uint32_t*>(a & ~(uintptr_t)3);
    const int off = (int)(a & 3);
    uint32_t r[17];
#pragma unroll
    for (int i = 0; i < 17; ++i) r[i] = 4 * i < off + n ? base[i] : 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t x = __builtin_amdgcn_alignbyte(r[i + 1], r[i], (uint32_t)off);
        const int valid = n - 4 * i;  // entries in this dword
        w[i] = valid >= 4 ? x : valid <= 0 ? ~0u : x | (~0u << (8 * valid));
    }
}

// Number of bytes <= v (v < 255) in w: each byte is subtracted from v in
// a 16-bit lane with bit 15 preset, which stays set exactly when the byte
// is at most v.
__device__ __forceinline__ uint32_t count_le(const uint32_t (&w)[16], int v)
{
    const uint32_t V = (uint32_t)v * 0x00010001u | 0x80008000u;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        c += __popc((V - (w[i] & 0x00FF00FFu)) & 0x80008000u);
        c += __popc((V - ((w[i] >> 8) & 0x00FF00FFu)) & 0x80008000u);
    }
    return c;
}

__global__ __launch_bounds__(kBlock) void k_mom_select(const MomStream* __restrict__ streams, int n_streams,
                                                       int64_t total, int32_t K,
                                                       const uint8_t* __restrict__ mad,
                                                       const uint32_t* __restrict__ hcnt,
                                                       const int32_t* __restrict__ hist_len,
                                                       int32_t* __restrict__ dm)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    int lo_s = 0, hi_s = n_streams - 1;  // last stream with woff <= g
    while (lo_s < hi_s) {
        const int mid = (lo_s + hi_s + 1) / 2;
        if (streams[mid].woff <= g) lo_s = mid;
        else hi_s = mid - 1;
    }
    const MomStream st = streams[lo_s];
    const int64_t w = g - st.woff;
    // sequence position of window w; the valid history starts pre - H back
    const int64_t p = st.pre + w;
    const int64_t H = st.pre > 0 ? min(max((int64_t)hist_len[lo_s], (int64_t)0), st.pre) : 0;
    const int64_t a = max(st.pre - H, p + 1 - (int64_t)K), b = p + 1;
    const uint32_t need = (uint32_t)((b - a - 1) / 2 + 1);
    const uint8_t* m = mad + st.eoff;
    const uint32_t* ha = hcnt + (st.hoff + a / kMomBlock) * 256;
    const uint32_t* hb = hcnt + (st.hoff + b / kMomBlock) * 256;
    // #{j < p : mad_j <= v} = block table row p / kMomBlock + partial block
    uint32_t wa[16], wb[16];
    mom_partial(m, a, wa);
    mom_partial(m, b, wb);
    int lo = 0, hi = 255;  // smallest v with #{a <= j < b : mad_j <= v} >= need
    while (lo < hi) {
        const int mid = (lo + hi) / 2;  // < 255
        if ((hb[mid] + count_le(wb, mid)) - (ha[mid] + count_le(wa, mid)) >= need) hi = mid;
        else lo = mid + 1;
    }
    dm[g] = lo;
}

// emad of streams with history slots (see launch_mom_extend).
__global__ __launch_bounds__(kBlock) void k_mom_extend(const MomStream* __restrict__ streams, int n_streams,
                                                       int64_t total_ext, const uint8_t* __restrict__ mad,
                                                       const uint8_t* __restrict__ hist,
                                                       uint8_t* __restrict__ emad)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= total_ext) return;
    int lo_s = 0, hi_s = n_streams - 1;  // last stream with eoff <= q
    while (lo_s < hi_s) {
        const int mid = (lo_s + hi_s + 1) / 2;
        if (streams[mid].eoff <= q) lo_s = mid;
        else hi_s = mid - 1;
    }
    const MomStream st = streams[lo_s];
    const int64_t i = q - st.eoff;
    emad[q] = i < st.pre ? hist[lo_s * st.pre + i] : mad[st.woff + (i - st.pre)];
}

// One workgroup per stream: the new right-aligned history, then its length.
__global__ __launch_bounds__(kBlock) void k_mom_history(const MomStream* __restrict__ streams,
                                                        const uint8_t* __restrict__ emad,
                                                        uint8_t* __restrict__ hist,
                                                        int32_t* __restrict__ hist_len)
{
    const MomStream st = streams[blockIdx.x];
    if (st.pre == 0) return;
    const int64_t H = min(max((int64_t)hist_len[blockIdx.x], (int64_t)0), st.pre);
    const int64_t Hn = min(st.pre, H + st.nw);
    // slot i (i >= pre - Hn) takes sequence entry nw + i
    for (int64_t i = st.pre - Hn + threadIdx.x; i < st.pre; i += kBlock)
        hist[blockIdx.x * st.pre + i] = emad[st.eoff + st.nw + i];
    __syncthreads();  // every thread has read hist_len
    if (threadIdx.x == 0) hist_len[blockIdx.x] = (int32_t)Hn;
}

struct MomSmem {
    WinParams prm[256];
    float thr[256];
    uint32_t flagged[256];
    uint32_t noise_counts[4];
    __align__(16) uint32_t noise_list[256];
    __align__(16) uint32_t noise_data[256];
    __device__ NoiseScratch noise()
    {
        return NoiseScratch{noise_counts, noise_list, reinterpret_cast<uint4*>(noise_data)};
    }
};

// One item: up to 256 whole windows (<= 16 KiB, or one window) of a stream,
// compiled per mode (the stream's mode is uniform over the workgroup).
template <int MODE>
__device__ __forceinline__ void mom_apply_item(const LaunchArgs& a, const MomItem& it, const StreamView& d,
                                               const int32_t* __restrict__ dm,
                                               const int64_t* __restrict__ stream_woff,
                                               rfi_window_stats* __restrict__ stats, MomSmem& sm)
{
    const int tid = (int)threadIdx.x;
    const int W = d.window;
    const int64_t g0 = stream_woff[it.stream] + it.first_window;
    if (tid < it.n_windows) {
        const int m = stats[g0 + tid].median;
        float sig;
        const float t = threshold_of(dm[g0 + tid], d.k, sig);
        const int T = (int)floorf(t);
        WinParams p;
        p.m = m;
        p.lo = max(m - T, -128);
        p.hi = min(m + T, 127);
        p.sq8 = (int)__fmul_rn(sig, 256.0f);
        sm.prm[tid] = p;
        sm.thr[tid] = t;
        sm.flagged[tid] = 0;
    }
    __syncthreads();
    const int64_t s0 = it.first_window * (int64_t)W;
    const int64_t s1 = min((it.first_window + it.n_windows) * (int64_t)W, d.length);
    const int8_t* x = static_cast<const int8_t*>(d.x);
    int8_t* y = static_cast<int8_t*>(d.y);
    if (s1 - s0 == 16384 && (W & 15) == 0) {
        // A whole 16 KiB tile of windows that are multiples of 16 samples:
        // every 16-byte chunk lies in one window.  All four loads of a lane
        // are issued before any store; noise goes through the workgroup pool.
        const int lane = tid & 63, wave = tid >> 6;
        const int64_t base = s0 + wave * 4096 + lane * 16;
        const int sh = __builtin_ctz((unsigned)W);  // W divides 16384: a power of two
        uint32_t v[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint4 t = gload16_nt(x + base + i * 1024);
            v[4 * i] = t.x;
            v[4 * i + 1] = t.y;
            v[4 * i + 2] = t.z;
            v[4 * i + 3] = t.w;
        }
        uint32_t cf = 0;  // bit 4i + q: dword q of chunk i holds a flagged sample
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int lw = (wave * 4096 + i * 1024 + lane * 16) >> sh;
            const WinParams p = sm.prm[lw];
            const uint32_t lo = rep_i16(p.lo * 256), hi = rep_i16(p.hi * 256);
            const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
            uint32_t nf = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t xw = v[4 * i + q];
                const uint32_t clipped = clamp_i8x4(xw, lo, hi);
                const uint32_t diff = clipped ^ xw;
                nf += __popc(nonzero_byte_mask(diff)) >> 3;
                cf |= (diff != 0 ? 1u : 0u) << (4 * i + q);
                if constexpr (MODE == RFI_MODE_CLIP) v[4 * i + q] = clipped;
                else if constexpr (MODE == RFI_MODE_ZERO)
                    v[4 * i + q] = byte_perm(0u, xw, flag_sel_i8x4(xw, lo_u, hi_u));
            }
            if (nf) atomicAdd(&sm.flagged[lw], nf);
        }
        if constexpr (MODE == RFI_MODE_NOISE) {
            const int64_t t0 = s0;
            auto merged = [&](int wv, int ln, int slot, int part, uint32_t xw) -> uint32_t {
                const int rel = wv * 4096 + slot * 1024 + ln * 16 + part * 4;
                const int64_t c = t0 + rel;
                const WinParams p = sm.prm[rel >> sh];
                const uint32_t lo_u = rep_i16((p.lo + 128) * 256), hi_u = rep_i16((p.hi + 128) * 256);
                const uint32_t nz = noise_quad_i8((uint64_t)(d.abs_base + c), a.seed, d.key, p.m, p.sq8);
                return byte_perm(nz, xw, flag_sel_i8x4(xw, lo_u, hi_u));
            };
            pool_noise<4>(v, cf, sm.noise(), merged);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            gstore16_nt(y + base + i * 1024, make_uint4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]));
    } else {
        // Other items (irregular W, stream tails): sample by sample.
#pragma unroll 1
        for (int64_t j = s0 + tid; j < s1; j += kBlock) {
            const int wl = (int)(j - s0) / W;
            const WinParams p = sm.prm[wl];
            const int xv = gload(x + j);
            int yv = xv;
            if (xv < p.lo || xv > p.hi) {
                atomicAdd(&sm.flagged[wl], 1u);
                if constexpr (MODE == RFI_MODE_ZERO) yv = 0;
                else if constexpr (MODE == RFI_MODE_CLIP) yv = min(max(xv, p.lo), p.hi);
                else yv = noise_sample(d.abs_base + j, a.seed, d.key, p.m, p.sq8, -128, 127);
            }
            gstore(y + j, (int8_t)yv);
        }
    }
    __syncthreads();
    if (tid < it.n_windows) {
        stats[g0 + tid].n_flagged = sm.flagged[tid];
        stats[g0 + tid].threshold = sm.thr[tid];
    }
}

__global__ __launch_bounds__(kBlock) void k_carry(const CarryItem* __restrict__ items)
{
    const CarryItem c = items[blockIdx.x];
    for (int i = (int)threadIdx.x; i < c.count; i += kBlock) {
        const int j = c.from + i;
        const uint64_t src = j < c.head_len ? c.head + (uint64_t)j * c.elem
                                            : c.body + (uint64_t)(j - c.head_len) * c.elem;
        const uint64_t dst = c.dst + (uint64_t)i * c.elem;
        if (c.elem == 1)
            gstore(reinterpret_cast<uint8_t*>(dst), gload(reinterpret_cast<const uint8_t*>(src)));
        else
            gstore(reinterpret_cast<uint16_t*>(dst), gload(reinterpret_cast<const uint16_t*>(src)));
    }
}

// ---------------------------------------------------------------------------
// Host launch wrappers.
// ---------------------------------------------------------------------------
// wg_per_cu > 0 caps the workgroups resident on one CU by padding each
// workgroup's LDS allocation (160 KiB per CU), an occupancy limit the
// autotuner can choose.
static thread_local int t_wg_per_cu = 0;

void set_wg_per_cu(int n) { t_wg_per_cu = n; }

static hipError_t launch(void (*k)(LaunchArgs), const LaunchArgs& a, int grid, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    if (grid < 1) grid = 1;
    size_t dyn = 0;
    if (t_wg_per_cu > 0) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k)) == hipSuccess) {
            const size_t want = (160u * 1024u) / (size_t)t_wg_per_cu;
            if (want > fa.sharedSizeBytes) dyn = ((want - fa.sharedSizeBytes) + 255) & ~(size_t)255;
            if (dyn + fa.sharedSizeBytes > 160u * 1024u) dyn = 0;
        }
    }
    LaunchArgs args = a;
    void* kargs[] = {&args};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(grid), dim3(kBlock), kargs, dyn, s);
}

template <int MODES, bool PERSIST, int T>
static void (*i8_tile_kernel_t(int cls))(LaunchArgs)
{
    switch (cls) {
        case 0: return k_i8_tiles<0, MODES, PERSIST, T>;
        case 1: return k_i8_tiles<1, MODES, PERSIST, T>;
        case 2: return k_i8_tiles<2, MODES, PERSIST, T>;
        case 3: return k_i8_tiles<3, MODES, PERSIST, T>;
        case 4: return k_i8_tiles<4, MODES, PERSIST, T>;
        case 5: return k_i8_tiles<5, MODES, PERSIST, T>;
        default: return nullptr;
    }
}

// Loop-free launches take one or two tiles per workgroup, persistent ones one.
template <int MODES, bool PERSIST>
static void (*i8_tile_kernel_m(int cls, int tpw))(LaunchArgs)
{
    if constexpr (PERSIST) return i8_tile_kernel_t<MODES, true, 1>(cls);
    else return tpw == 2 ? i8_tile_kernel_t<MODES, false, 2>(cls) : i8_tile_kernel_t<MODES, false, 1>(cls);
}

// modes: bit m set if some stream of the launch uses mode m.
template <bool PERSIST>
static void (*i8_tile_kernel_p(int cls, int modes, int tpw))(LaunchArgs)
{
    switch (modes) {
        case 1: return i8_tile_kernel_m<1, PERSIST>(cls, tpw);
        case 2: return i8_tile_kernel_m<2, PERSIST>(cls, tpw);
        case 3: return i8_tile_kernel_m<3, PERSIST>(cls, tpw);
        case 4: return i8_tile_kernel_m<4, PERSIST>(cls, tpw);
        case 1 << kModeStats: return i8_tile_kernel_m<1 << kModeStats, PERSIST>(cls, tpw);
        default: return i8_tile_kernel_m<7, PERSIST>(cls, tpw);
    }
}

static void (*i8_tile_kernel(int cls, int modes, bool persist, int tpw))(LaunchArgs)
{
    return persist ? i8_tile_kernel_p<true>(cls, modes, 1) : i8_tile_kernel_p<false>(cls, modes, tpw);
}

hipError_t launch_i8_tiles(int cls, int modes, int tpw, const LaunchArgs& a, int grid, hipStream_t s)
{
    // A grid that covers every item runs a loop-free variant with tpw
    // items per workgroup; a smaller grid runs the persistent variant.
    const bool persist = grid < a.n_items;
    if (tpw != 1 && tpw != 2) return hipErrorInvalidValue;
    auto k = i8_tile_kernel(cls, modes, persist, tpw);
    if (!k) return hipErrorInvalidValue;
    return launch(k, a, persist ? grid : (int)((a.n_items + tpw - 1) / tpw), s);
}
#define RFI_PICK(K, a, grid) ((grid) < (a).n_items ? K<true> : K<false>)
hipError_t launch_i8_generic(const LaunchArgs& a, int modes, int grid, hipStream_t s, int small_nt)
{
    const bool persist = grid < a.n_items;
    if ((small_nt == 64 || small_nt == 128) && !persist) {
        if (a.n_items <= 0) return hipSuccess;
        if (a.n_items > (1 << 30)) return hipErrorInvalidValue;
        const bool noise = (modes & 4) != 0;
        void (*k)(LaunchArgs) = small_nt == 64 ? (noise ? k_i8_generic_small<64, true> : k_i8_generic_small<64, false>)
                                               : (noise ? k_i8_generic_small<128, true> : k_i8_generic_small<128, false>);
        hipLaunchKernelGGL(k, dim3((unsigned)a.n_items), dim3((unsigned)small_nt), 0, s, a);
        return hipGetLastError();
    }
    void (*k)(LaunchArgs) = (modes & 4) ? (persist ? k_i8_generic<true, true> : k_i8_generic<false, true>)
                                        : (persist ? k_i8_generic<true, false> : k_i8_generic<false, false>);
    return launch(k, a, grid, s);
}
template <bool PERSIST>
static void (*i8_fused_kernel(int modes))(LaunchArgs)
{
    switch (modes) {
        case 1: return k_i8_fused<PERSIST, 1>;
        case 2: return k_i8_fused<PERSIST, 2>;
        case 4: return k_i8_fused<PERSIST, 4>;
        default: return k_i8_fused<PERSIST, 7>;
    }
}

hipError_t launch_i8_fused(int modes, const LaunchArgs& a, int grid, hipStream_t s)
{
    return launch(grid < a.n_items ? i8_fused_kernel<true>(modes) : i8_fused_kernel<false>(modes), a, grid, s);
}
template <bool PERSIST>
static void (*i16_tile_kernel(int modes))(LaunchArgs)
{
    switch (modes) {
        case 1: return k_i16_tiles<PERSIST, 1>;
        case 2: return k_i16_tiles<PERSIST, 2>;
        case 4: return k_i16_tiles<PERSIST, 4>;
        default: return k_i16_tiles<PERSIST, 7>;
    }
}

hipError_t launch_i16_tiles(int cls, int modes, const LaunchArgs& a, int grid, hipStream_t s)
{
    if (cls != 0) return hipErrorInvalidValue;
    return launch(grid < a.n_items ? i16_tile_kernel<true>(modes) : i16_tile_kernel<false>(modes), a, grid, s);
}
hipError_t launch_i16_generic(const LaunchArgs& a, int grid, hipStream_t s)
{
    return launch(RFI_PICK(k_i16_generic, a, grid), a, grid, s);
}
hipError_t launch_i16_fused(const LaunchArgs& a, int grid, hipStream_t s)
{
    return launch(RFI_PICK(k_i16_fused, a, grid), a, grid, s);
}
#undef RFI_PICK

hipError_t warm_fused(int elem_size, bool persist, hipStream_t s)
{
    LaunchArgs a{};  // no items: the workgroup returns at once
    void (*k)(LaunchArgs) = elem_size == 1 ? (persist ? i8_fused_kernel<true>(7) : i8_fused_kernel<false>(7))
                                           : (persist ? k_i16_fused<true> : k_i16_fused<false>);
    void* kargs[] = {&a};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(1), dim3(kBlock), kargs, 0, s);
}

__global__ __launch_bounds__(kBlock) void k_mom_apply(LaunchArgs a, const MomItem* __restrict__ items,
                                                      const int32_t* __restrict__ dm,
                                                      const int64_t* __restrict__ stream_woff,
                                                      const int64_t* __restrict__ abs_add,
                                                      rfi_window_stats* __restrict__ stats)
{
    __shared__ MomSmem sm;
    const MomItem it = items[blockIdx.x];
    StreamView d = resolve(a.streams[it.stream], a);
    if (abs_add) d.abs_base += abs_add[it.stream];
    if (d.mode == RFI_MODE_CLIP) mom_apply_item<RFI_MODE_CLIP>(a, it, d, dm, stream_woff, stats, sm);
    else if (d.mode == RFI_MODE_ZERO) mom_apply_item<RFI_MODE_ZERO>(a, it, d, dm, stream_woff, stats, sm);
    else mom_apply_item<RFI_MODE_NOISE>(a, it, d, dm, stream_woff, stats, sm);
}

hipError_t launch_i8_multi(int cls, const MultiArgs& ma, int grid, hipStream_t s)
{
    if (ma.a.n_items <= 0) return hipSuccess;
    void (*k)(MultiArgs) = nullptr;
    switch (cls) {
        case 0: k = k_i8_multi<0>; break;
        case 1: k = k_i8_multi<1>; break;
        case 2: k = k_i8_multi<2>; break;
        case 3: k = k_i8_multi<3>; break;
        case 4: k = k_i8_multi<4>; break;
        case 5: k = k_i8_multi<5>; break;
        default: return hipErrorInvalidValue;
    }
    MultiArgs args = ma;
    void* kargs[] = {&args};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(grid), dim3(kBlock), kargs, 0, s);
}

hipError_t launch_mom_gather(const rfi_window_stats* stats, int64_t total, uint8_t* mad, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mom_gather, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       stats, total, mad);
    return hipGetLastError();
}

hipError_t launch_mom_counts(const MomStream* streams, int n_streams, int64_t max_blocks, const uint8_t* mad,
                             uint32_t* hcnt, hipStream_t s)
{
    if (n_streams <= 0) return hipSuccess;
    if (max_blocks > 0) {
        if (max_blocks > (1 << 30) || n_streams > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_mom_block_counts, dim3((unsigned)max_blocks, (unsigned)n_streams), dim3(256), 0, s,
                           streams, mad, hcnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mom_counts, dim3(n_streams), dim3(256), 0, s, streams, hcnt);
    return hipGetLastError();
}

hipError_t launch_mom_select(const MomStream* streams, int n_streams, int64_t total, int32_t K,
                             const uint8_t* mad, const uint32_t* hcnt, const int32_t* hist_len, int32_t* dm,
                             hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mom_select, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       streams, n_streams, total, K, mad, hcnt, hist_len, dm);
    return hipGetLastError();
}

hipError_t launch_mom_extend(const MomStream* streams, int n_streams, int64_t total_ext, const uint8_t* mad,
                             const uint8_t* hist, uint8_t* emad, hipStream_t s)
{
    if (total_ext <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mom_extend, dim3((unsigned)((total_ext + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       streams, n_streams, total_ext, mad, hist, emad);
    return hipGetLastError();
}

hipError_t launch_mom_history(const MomStream* streams, int n_streams, const uint8_t* emad, uint8_t* hist,
                              int32_t* hist_len, hipStream_t s)
{
    if (n_streams <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mom_history, dim3((unsigned)n_streams), dim3(kBlock), 0, s, streams, emad, hist,
                       hist_len);
    return hipGetLastError();
}

hipError_t launch_mom_apply(const LaunchArgs& a, const MomItem* items, int64_t n_items, const int32_t* dm,
                            const int64_t* stream_woff, const int64_t* abs_add, rfi_window_stats* stats,
                            hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (n_items > (1 << 30)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mom_apply, dim3((unsigned)n_items), dim3(kBlock), 0, s, a, items, dm, stream_woff,
                       abs_add, stats);
    return hipGetLastError();
}

hipError_t launch_carry(const CarryItem* items, int n_items, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_carry, dim3(n_items), dim3(kBlock), 0, s, items);
    return hipGetLastError();
}

int persistent_grid(int elem_size, int cls, int modes, bool fused)
{
    void (*k)(LaunchArgs) = nullptr;
    if (elem_size == 1) {
        if (fused) k = i8_fused_kernel<true>(modes);
        else if (cls < 0) k = (modes & 4) ? k_i8_generic<true, true> : k_i8_generic<true, false>;
        else k = i8_tile_kernel(cls, modes, true, 1);
    } else {
        if (fused) k = k_i16_fused<true>;
        else if (cls < 0) k = k_i16_generic<true>;
        else k = i16_tile_kernel<true>(modes);
    }
    int per_cu = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return per_cu * cus;
}

}  // namespace rfi
