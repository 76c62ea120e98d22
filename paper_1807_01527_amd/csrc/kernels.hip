// gfx950 kernels of the ATVC hot path: slice open (lazy preserve), pair scan,
// slice close (window weights, AAT, super lists), restore join, sort, and
// the per-host estimate.  Wave64 throughout.  An AT is one byte while
// 2k < 256 and a 16-bit word beyond (the AT type T of the pool kernels); the
// streaming server's kernels use byte ATs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "atpool.hpp"

namespace atp {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t mod_mul_p(uint32_t a, uint32_t m) {
    // a*m mod (2^32 - 5): fold the high word twice (2^32 = 5 mod p), then one
    // conditional subtract (after two folds the value is below 2^32 + 25 < 2p).
    uint64_t x = (uint64_t)a * m;
    uint64_t y = (x >> 32) * 5ull + (x & 0xFFFFFFFFull);
    uint64_t y2 = (y >> 32) * 5ull + (y & 0xFFFFFFFFull);
    return (uint32_t)(y2 >= kPrime ? y2 - kPrime : y2);
}

// Section 4.1 IP mangling: bijection of 32-bit words, identity on [p, 2^32).
__device__ __forceinline__ uint32_t mangle(uint32_t a, uint32_t A) {
    return (uint64_t)a >= kPrime ? a : mod_mul_p(a, A);
}

__device__ __forceinline__ uint32_t block_of(uint32_t i, const Geometry& G) {
    if (G.blk_a == 0) return G.last_blk;
    uint32_t b = (uint32_t)(((uint64_t)i * G.blk_magic) >> 32);
    return b < G.last_blk ? b : G.last_blk;
}

__device__ __forceinline__ uint32_t act_of(uint32_t i, uint32_t c0, const Geometry& G) {
    uint32_t v = c0 + block_of(i, G);
    return v >= G.twok ? v - G.twok : v;
}

// act_of when every block holds at least two ATs (blk_a >= 2, so the magic
// multiplier fits 32 bits): one high multiply, and the wrap as an unsigned
// minimum (v < 4k: v - 2k wraps above v exactly when v < 2k).
__device__ __forceinline__ uint32_t act_of_narrow(uint32_t i, uint32_t c0, uint32_t magic, const Geometry& G) {
    const uint32_t b = min(__umulhi(i, magic), G.last_blk);
    const uint32_t v = c0 + b;
    return min(v, v - G.twok);
}

// Column x_j of LBS: c bits starting at bit sh[j], cyclic modulo W.  LL holds
// L twice (L | L << W) so one 64-bit shift reads across the wrap.
__device__ __forceinline__ uint32_t column(uint64_t LL, uint32_t sh, uint32_t mask) {
    return (uint32_t)(LL >> sh) & mask;
}

// Alg 1 on one AT: inactive value 2k, otherwise active when the distance
// from the block's timestamp is below k'.
__device__ __forceinline__ uint32_t is_active(uint32_t at, uint32_t act, uint32_t twok, uint32_t kq) {
    uint32_t d = act >= at ? act - at : act + twok - at;
    return (at != twok) & (d < kq);
}

// ATs of type T in a 32-bit word and in a 16-byte chunk; AT b of a word.
template <typename T>
constexpr uint32_t kPerWord = 4 / sizeof(T);
template <typename T>
constexpr uint32_t kPerChunk = 16 / sizeof(T);
template <typename T>
__device__ __forceinline__ uint32_t at_in_word(uint32_t w, uint32_t b) {
    return sizeof(T) == 1 ? (w >> (8 * b)) & 0xFFu : (w >> (16 * b)) & 0xFFFFu;
}
__device__ __forceinline__ uint32_t word_of(const uint4& v, uint32_t q) {
    return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}

template <typename T>
__device__ __forceinline__ uint32_t active_mask_word(uint32_t atw, uint32_t actw, uint32_t twok, uint32_t kq) {
    uint32_t m = 0;
#pragma unroll
    for (uint32_t b = 0; b < kPerWord<T>; b++)
        m |= is_active(at_in_word<T>(atw, b), at_in_word<T>(actw, b), twok, kq) << b;
    return m;
}

// bit e set when AT e of the chunk is active for k'
template <typename T>
__device__ __forceinline__ uint32_t active_mask_chunk(uint4 at, uint4 act, uint32_t twok, uint32_t kq) {
    constexpr uint32_t N = kPerWord<T>;
    return active_mask_word<T>(at.x, act.x, twok, kq) | (active_mask_word<T>(at.y, act.y, twok, kq) << N) |
           (active_mask_word<T>(at.z, act.z, twok, kq) << (2 * N)) |
           (active_mask_word<T>(at.w, act.w, twok, kq) << (3 * N));
}

__device__ __forceinline__ uint32_t active_mask16(uint4 at, uint4 act, uint32_t twok, uint32_t kq) {
    return active_mask_chunk<uint8_t>(at, act, twok, kq);
}

// Alg 1 on two ATs at a time in the 16-bit halves of a word (packed integer
// ops).  With d = act + 2k - at in [1, 4k) (exact while 4k <= 2^16), the
// distance is d mod 2k = min(d, d - 2k) (the second wraps high when d < 2k);
// the AT is inactive when at = 2k or the distance reaches k', and bit 15 of
// (x + 0x8000 - y) tests x >= y for x, y < 2^15 + y.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t w) { return __builtin_bit_cast(u16x2, w); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t both_halves(uint32_t v) { return v | (v << 16); }

// per 16-bit half: distance (in the low 15 bits) and the at = 2k flag (bit 15)
struct Alg1Halves {
    uint32_t dist;
    uint32_t off;
};
__device__ __forceinline__ Alg1Halves alg1_halves(uint32_t at2, uint32_t act2, uint32_t twok2, uint32_t c_at) {
    const u16x2 a = as_u16x2(at2);
    const u16x2 d = as_u16x2(act2) + as_u16x2(twok2) - a;
    const u16x2 m = __builtin_elementwise_min(d, d - as_u16x2(twok2));
    return {as_u32(m), as_u32(a + as_u16x2(c_at)) & 0x80008000u};
}
// number of inactive ATs among the two halves for window k' (c_kq = 0x8000 - k' in both halves)
__device__ __forceinline__ uint32_t inactive2(const Alg1Halves& h, uint32_t c_kq) {
    return __popc(((as_u32(as_u16x2(h.dist) + as_u16x2(c_kq))) | h.off) & 0x80008000u);
}
// Alg 1 on four byte ATs per 32-bit operation, while 4k <= 128 (k <= 32).
// With d = ACT + 2k - AT, in [0, 4k) so that no carry or borrow crosses a
// byte, an AT is active for window k' when AT != 2k and d < k' or
// 2k <= d < 2k + k' (the distance (ACT - AT) mod 2k is below k').  Bit 7 of
// every byte carries the comparisons: (d | 0x80) - c keeps bit 7 exactly
// when d >= c.
constexpr uint32_t kByteHigh = 0x80808080u, kByteOnes = 0x01010101u;
struct ByteLanes {
    uint32_t dh, live, ge2k;
};
__device__ __forceinline__ ByteLanes byte_lanes(uint32_t at4, uint32_t act4, uint32_t twok4) {
    const uint32_t dh = ((act4 + twok4) - at4) | kByteHigh;
    return {dh, ((at4 ^ twok4) | kByteHigh) - kByteOnes, dh - twok4};
}
// active ATs among the four for window k' (kq4 = k' and tkq4 = 2k + k' in every byte)
__device__ __forceinline__ uint32_t byte_active(const ByteLanes& b, uint32_t kq4, uint32_t tkq4) {
    return __popc((~(b.dh - kq4) | (b.ge2k & ~(b.dh - tkq4))) & b.live & kByteHigh);
}

// the 16-bit halves of a 16-byte chunk of ATs (bytes: even and odd bytes of every word apart)
template <typename T>
__device__ __forceinline__ void chunk_halves(uint4 v, uint32_t* h /* 8 or 4 */) {
    if (sizeof(T) == 1) {
#pragma unroll
        for (uint32_t q = 0; q < 4; q++) {
            const uint32_t w = word_of(v, q);
            h[2 * q] = w & 0x00FF00FFu;
            h[2 * q + 1] = (w >> 8) & 0x00FF00FFu;
        }
    } else {
        h[0] = v.x;
        h[1] = v.y;
        h[2] = v.z;
        h[3] = v.w;
    }
}

// per-position block timestamp table for the slice whose first block has C0
template <typename T>
__device__ void fill_act_lut(T* lut, uint32_t c0, const Geometry& G) {
    for (uint32_t i = threadIdx.x; i < G.g; i += blockDim.x) lut[i] = (T)act_of(i, c0, G);
    __syncthreads();
}

// ---------------------------------------------------------------- utilities

// n bytes set to the repeated 32-bit word v4 (n a multiple of 4 unless every
// byte of v4 is the same)
__global__ void k_fill_u8(uint8_t* __restrict__ p, uint64_t n, uint32_t v4) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 16;
    uint4 vv = make_uint4(v4, v4, v4, v4);
    for (uint64_t o = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; o < n; o += stride) {
        if (o + 16 <= n) *(uint4*)(p + o) = vv;
        else
            for (uint64_t q = o; q < n; q++) p[q] = (uint8_t)(v4 >> (8 * (q & 3)));
    }
}

__global__ void k_zero_u64(unsigned long long* p, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------- a1: open
// Alg 2 applied lazily: of the 2k blocks of every ATV only the two whose
// timestamp becomes 0 or k can change (Section 3); every other AT is left
// alone, which is exactly what Alg 2 does to it.  Work items are 16-byte
// chunks of one or two disjoint chunk spans per ATV; ATs outside the due
// blocks are written back unchanged.  pos0 is the AT index of the word's
// first AT.
template <typename T = uint8_t>
__device__ __forceinline__ uint32_t preserve_word(uint32_t v, uint32_t pos0, const PreserveSpans& S, uint32_t k,
                                                  uint32_t twok) {
    constexpr uint32_t B = 8 * sizeof(T);
    constexpr uint32_t M = sizeof(T) == 1 ? 0xFFu : 0xFFFFu;
    uint32_t nv = v;
#pragma unroll
    for (uint32_t b = 0; b < kPerWord<T>; b++) {
        const uint32_t pos = pos0 + b;
        const uint32_t at = at_in_word<T>(v, b);
        uint32_t out = at;
        if (pos >= S.r0lo && pos < S.r0hi && at <= k) out = twok;
        if (pos >= S.r1lo && pos < S.r1hi && ((at >= k && at < twok) || at == 0)) out = twok;
        nv = (nv & ~(M << (B * b))) | (out << (B * b));
    }
    return nv;
}

// One 16-byte chunk of a due range per thread: every chunk is independent, so
// the pass streams at memory speed.  ATs of a chunk outside the due blocks
// are written back unchanged.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_preserve(uint8_t* __restrict__ pool, uint64_t n_atv,
                                                     uint32_t log2g, uint32_t k, PreserveSpans S) {
    const uint32_t per = S.nw0 + S.nw1;  // 16-byte chunks per ATV
    const uint64_t total = n_atv * per;
    const uint32_t twok = 2 * k;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t atv = total < (1ull << 32) ? (uint32_t)it / per : it / per;
        const uint32_t ci = (uint32_t)(it - atv * per);
        const uint32_t chunk = ci < S.nw0 ? S.w0lo + ci : S.w1lo + (ci - S.nw0);
        uint4* p = reinterpret_cast<uint4*>(pool + ((atv << log2g) * sizeof(T))) + chunk;
        const uint4 v = *p;
        constexpr uint32_t CA = kPerChunk<T>, N = kPerWord<T>;
        uint4 nv;
        nv.x = preserve_word<T>(v.x, chunk * CA, S, k, twok);
        nv.y = preserve_word<T>(v.y, chunk * CA + N, S, k, twok);
        nv.z = preserve_word<T>(v.z, chunk * CA + 2 * N, S, k, twok);
        nv.w = preserve_word<T>(v.w, chunk * CA + 3 * N, S, k, twok);
        if (nv.x != v.x || nv.y != v.y || nv.z != v.z || nv.w != v.w) *p = nv;
    }
}

// ---------------------------------------------------------------- a2+a3: scan
// Alg 3 fused with the hashing of Section 4.1: f = A*aip mod p, frame = low u
// bits, columns from LBS, AT index BH(bip), value = that AT's block timestamp.
// The r byte stores need no atomics: every writer of an AT in a slice stores
// the same value.
template <int R, typename T>
__device__ __forceinline__ void scan_pair(T* __restrict__ pool, uint32_t a, uint32_t b,
                                          const Geometry& G, uint32_t c0) {
    uint32_t f = mangle(a, G.A);
    uint32_t z = f & G.umask;
    uint64_t L = (uint64_t)(f >> G.u);
    uint64_t LL = L | (L << G.W);
    uint32_t i = (uint32_t)((G.alpha * (uint64_t)b + G.beta) >> (64 - G.log2g));
    const T v = (T)act_of(i, c0, G);
    uint64_t zr = (uint64_t)z * R;
#pragma unroll
    for (int j = 0; j < R; j++) {
        uint32_t x = column(LL, G.sh[j], G.ncol_mask);
        uint64_t idx = ((((zr + j) << G.c) + x) << G.log2g) | i;
        pool[idx] = v;
    }
}

template <int R, bool VEC, typename T>
__global__ __launch_bounds__(kBlock) void k_ingest(T* __restrict__ pool, const uint32_t* __restrict__ aip,
                                                   const uint32_t* __restrict__ bip, uint64_t n, Geometry G,
                                                   uint32_t c0) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t done = 0;
    if (VEC) {
        const uint64_t n4 = n / 4;
        const uint4* a4 = reinterpret_cast<const uint4*>(aip);
        const uint4* b4 = reinterpret_cast<const uint4*>(bip);
        for (uint64_t q = tid; q < n4; q += stride) {
            uint4 a = a4[q];
            uint4 b = b4[q];
            scan_pair<R>(pool, a.x, b.x, G, c0);
            scan_pair<R>(pool, a.y, b.y, G, c0);
            scan_pair<R>(pool, a.z, b.z, G, c0);
            scan_pair<R>(pool, a.w, b.w, G, c0);
        }
        done = n4 * 4;
    }
    for (uint64_t q = done + tid; q < n; q += stride) scan_pair<R>(pool, aip[q], bip[q], G, c0);
}

// ---------------------------------------------------------------- a2+a3: binned scan
// Pass 1 hashes every pair once and appends a record to the bin of its frame
// group (frame mod 8): LBS (W bits) | frame >> 3 | AT index.  Pass 2 runs once
// per row: workgroup b works on bin b mod 8, and workgroups are handed to the
// 8 XCDs round robin, so each XCD's L2 only sees the byte stores of one
// (frame group, row) region of the pool -- a 2 MiB working set on the link
// geometry instead of the whole pool.
constexpr uint32_t kBins = 8;
constexpr uint32_t kSubs = 64;        // sub-runs per bin: spreads the run reservations over 512 counters
constexpr uint32_t kBinTile = 2048;   // pairs per block round

// Bin b, sub-run s holds records bins[(b * kSubs + s) * sub_cap + j], j < fill[b * kSubs + s];
// a block with index B only appends to sub-run B mod kSubs.  With n <= 8192
// tiles every block takes at most one tile, so a sub-run receives at most
// ceil(ceil(n / kBinTile) / kSubs) tiles <= n / kSubs + 32 + kBinTile pairs;
// sub_cap = ceil(n / kSubs) + 2 kBinTile covers that.
__global__ __launch_bounds__(kBlock) void k_bin_pairs(const uint32_t* __restrict__ aip, const uint32_t* __restrict__ bip,
                                                      uint64_t n, Geometry G, uint64_t* __restrict__ bins,
                                                      uint64_t sub_cap, unsigned long long* __restrict__ fill) {
    constexpr uint32_t kPer = kBinTile / kBlock;
    __shared__ uint32_t cnt[kBins];
    __shared__ unsigned long long base[kBins];
    const uint32_t sub = blockIdx.x % kSubs;
    for (uint64_t b0 = (uint64_t)blockIdx.x * kBinTile; b0 < n; b0 += (uint64_t)gridDim.x * kBinTile) {
        if (threadIdx.x < kBins) cnt[threadIdx.x] = 0;
        __syncthreads();
        uint64_t rec[kPer];
        uint32_t bin[kPer], slot[kPer];
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++) {
            const uint64_t q = b0 + (uint64_t)e * kBlock + threadIdx.x;
            bin[e] = kBins;
            if (q < n) {
                const uint32_t f = mangle(aip[q], G.A);
                const uint32_t z = f & G.umask;
                const uint32_t i = (uint32_t)((G.alpha * (uint64_t)bip[q] + G.beta) >> (64 - G.log2g));
                rec[e] = ((uint64_t)(f >> G.u) << 32) | ((uint64_t)(z >> 3) << 16) | i;
                bin[e] = z & (kBins - 1);
                slot[e] = atomicAdd(&cnt[bin[e]], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x < kBins)
            base[threadIdx.x] =
                cnt[threadIdx.x] ? atomicAdd(&fill[threadIdx.x * kSubs + sub], (unsigned long long)cnt[threadIdx.x])
                                 : 0ull;
        __syncthreads();
#pragma unroll
        for (uint32_t e = 0; e < kPer; e++)
            if (bin[e] < kBins) {
                const unsigned long long pos = base[bin[e]] + slot[e];
                if (pos < sub_cap) bins[((uint64_t)bin[e] * kSubs + sub) * sub_cap + pos] = rec[e];
            }
        __syncthreads();
    }
}

// The 64 sub-runs of a bin are scanned as one index space: each sub-run's
// length is rounded up to a multiple of 4 (sub_cap is one too), so a group of
// four consecutive indices never straddles two sub-runs; indices past a
// sub-run's fill are skipped.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_bins(const uint64_t* __restrict__ bins, uint64_t sub_cap,
                                                      const unsigned long long* __restrict__ fill,
                                                      T* __restrict__ pool, Geometry G, uint32_t c0, uint32_t row) {
    __shared__ unsigned long long pre[kSubs + 1];  // prefix of the rounded sub-run lengths
    __shared__ unsigned long long len[kSubs];      // records in each sub-run
    const uint32_t bin = blockIdx.x % kBins;
    const uint64_t bpb = gridDim.x / kBins;  // blocks per bin
    const uint64_t me = blockIdx.x / kBins;
    if (threadIdx.x < 64) {
        static_assert(kSubs == 64, "one lane per sub-run");
        const uint32_t s = threadIdx.x;
        const unsigned long long f = fill[bin * kSubs + s];
        const unsigned long long nb = f < sub_cap ? f : sub_cap;
        len[s] = nb;
        unsigned long long v = (nb + 3) & ~3ull;
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const unsigned long long t = __shfl_up(v, o, 64);
            if (s >= o) v += t;
        }
        pre[s + 1] = v;
        if (s == 0) pre[0] = 0;
    }
    __syncthreads();
    const uint64_t total = pre[kSubs];
    const uint32_t sh = G.sh[row];
    const uint64_t zr = (uint64_t)G.r;
    for (uint64_t q0 = (me * kBlock + threadIdx.x) * 4; q0 < total; q0 += bpb * kBlock * 4) {
        uint32_t s = 0;  // last sub-run with pre[s] <= q0
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1)
            if (pre[s + step] <= q0) s += step;
        const uint64_t local = q0 - pre[s];
        const uint64_t nb = len[s];
        const uint64_t* rec = bins + ((uint64_t)bin * kSubs + s) * sub_cap + local;
        uint64_t r4[4];
        if (local + 4 <= nb) {
            const ulonglong2 a = *reinterpret_cast<const ulonglong2*>(rec);
            const ulonglong2 b = *reinterpret_cast<const ulonglong2*>(rec + 2);
            r4[0] = a.x;
            r4[1] = a.y;
            r4[2] = b.x;
            r4[3] = b.y;
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++) r4[e] = local + e < nb ? rec[e] : ~0ull;
        }
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint64_t r = r4[e];
            if (r == ~0ull) continue;  // never a record: frame bits 16..31 stay below 0xFFFF
            const uint64_t L = r >> 32;
            const uint32_t z = (uint32_t)(((r >> 16) & 0xFFFFu) << 3) | bin;
            const uint32_t i = (uint32_t)(r & 0xFFFFu);
            const uint64_t LL = L | (L << G.W);
            const uint32_t x = column(LL, sh, G.ncol_mask);
            const uint64_t idx = (((((uint64_t)z * zr + row) << G.c) + x) << G.log2g) | i;
            pool[idx] = (T)act_of(i, c0, G);
        }
    }
}

// ---------------------------------------------------------------- a2+a3: tiled scan
// The pool is cut into tiles of 64 KiB (whole ATVs).  Pass 1 hashes every pair
// and writes, per block of kTileRecs AT stores (r per pair), its count of
// stores landing in each tile (a row of cnt).  Column scans over the blocks,
// in chunks of kTileChunk rows, and a scan of the tile totals give every
// (block, tile) run its place in the record array.  Pass 2 hashes again,
// groups the block's records (an AT's index inside its tile, 16 bits) by tile
// in LDS and writes each run contiguously.  Pass 3 runs one workgroup per
// tile: the tile is read into LDS, every record sets its AT to the value its
// index implies (its block timestamp), and the tile is written back.  The
// random stores hit LDS; HBM sees streams.
// a[j] <- a[(j + rot) mod R] for a lane-varying rot < R, as a barrel of
// fixed rotations (by 1, 2, 4) so that the array is only ever indexed by
// constants and stays in registers
template <int R>
__device__ __forceinline__ void rotate_rows(uint32_t (&a)[R], uint32_t rot) {
#pragma unroll
    for (int b = 1; b < R; b <<= 1) {
        const bool on = (rot & (uint32_t)b) != 0;
        uint32_t t[R];
#pragma unroll
        for (int j = 0; j < R; j++) t[j] = a[(j + b) % R];
#pragma unroll
        for (int j = 0; j < R; j++) a[j] = on ? t[j] : a[j];
    }
}

constexpr uint32_t kTileBytes = 1u << 16;
constexpr uint32_t kTileRecs = 16384;  // records per block in passes 1 and 2
static_assert(kTileRecs <= 0xFFFFu, "a block's count for one tile fits the 16-bit count table");
constexpr uint32_t kMaxTiles = 4096;
constexpr uint32_t kTileChunk = 64;    // rows (blocks) per chunk of the column scans
constexpr uint32_t kCountBlock = 1024;  // pass 1: four pairs per thread
constexpr uint32_t kColTiles = 64;      // tiles per block of the column passes (one wave wide)
constexpr uint32_t kApplyBlock = 1024;
constexpr uint32_t kScatterBlock = 1024;  // 16 waves; the scatter block holds 80 KiB of LDS, two per CU

// One job of a tiled launch (a pool, its pairs and its scratch); a launch of
// each pass covers up to kTileJobsMax jobs, the job given by one grid
// dimension, so that the passes of several pools fill the chip together.
struct TileJob {
    uint8_t* pool;
    const uint32_t* aip;
    const uint32_t* bip;
    uint16_t* rec;
    uint16_t* cnt;
    uint32_t* pre;
    uint32_t* csum;
    uint32_t* base;
    void* act;
    uint32_t* w_out;
    uint64_t n;
    Geometry G;
    PreserveSpans S;
    uint32_t c0, preserve, kq_w, n_tiles, nb, nchunk;
};
struct TileBatch {
    TileJob j[kTileJobsMax];
};

// log2 of the ATs per 64 KiB tile
__device__ __forceinline__ uint32_t tile_shift(const Geometry& G) { return 16u - (G.atb == 2 ? 1u : 0u); }

// The tiled scan only runs on pools of at most kMaxTiles * kTileBytes =
// 2^28 bytes, so ATV and AT indices fit 32 bits there: the index arithmetic
// of passes 1 and 2 is 32-bit (half the instructions of the 64-bit form).
static_assert((uint64_t)kMaxTiles * kTileBytes <= (1ull << 32), "tiled AT indices fit 32 bits");

// the r target AT indices of a pair (Alg 3), 32-bit
template <int R>
__device__ __forceinline__ void pair_targets(uint32_t a, uint32_t b, const Geometry& G, uint32_t* idx) {
    const uint32_t f = mangle(a, G.A);
    const uint32_t z = f & G.umask;
    const uint64_t L = (uint64_t)(f >> G.u);
    const uint64_t LL = L | (L << G.W);
    const uint32_t i = (uint32_t)((G.alpha * (uint64_t)b + G.beta) >> (64 - G.log2g));
    const uint32_t zc = (z * (uint32_t)R) << G.c;
#pragma unroll
    for (int j = 0; j < R; j++) {
        const uint32_t x = column(LL, G.sh[j], G.ncol_mask);
        idx[j] = ((zc + ((uint32_t)j << G.c) + x) << G.log2g) | i;
    }
}

// Workgroups are dealt to the 8 XCDs in turn (w -> XCD w mod 8).  This gives
// XCD x the x-th contiguous share of the logical blocks instead, in order, so
// that blocks running side by side on one XCD write neighbouring runs of each
// tile (pass 2): their partial cache lines meet in that XCD's L2 and leave it
// whole.  Pass 1 uses the same mapping, so a block's pairs are read by both
// passes on one XCD.
__device__ __forceinline__ uint32_t xcd_contiguous_block(uint32_t w, uint32_t nb) {
    constexpr uint32_t kXcds = 8;
    const uint32_t x = w % kXcds, l = w / kXcds, q = nb / kXcds, rem = nb % kXcds;
    return x * q + (x < rem ? x : rem) + l;
}

// The record passes (count, column scans, scatter) raise their waves' issue
// priority: a server runs them beside its close graph, and the next tile pass
// waits for them, not for the graph.
// Pass 1: block b's per-tile store counts -> cnt[b * n_tiles + tile], 16-bit
// (a block has at most kTileRecs stores; half the table traffic of every
// pass that reads it).  A tile
// holds whole ATVs (g <= the ATs of a tile), so a store's tile is its ATV's:
// it depends on aip alone and this pass never reads bip.
template <int R>
__global__ __launch_bounds__(kCountBlock) void k_tile_count(TileBatch J) {
    __builtin_amdgcn_s_setprio(3);
    const TileJob& TJ = J.j[blockIdx.y];
    const Geometry& G = TJ.G;
    const uint32_t* __restrict__ aip = TJ.aip;
    const uint64_t n = TJ.n;
    const uint32_t ts = tile_shift(G), n_tiles = TJ.n_tiles, c0 = TJ.c0;
    uint16_t* __restrict__ cnt = TJ.cnt;
    uint32_t* __restrict__ tot = TJ.csum + (uint64_t)TJ.nchunk * n_tiles;  // the row after the chunk sums
    void* __restrict__ act_table = TJ.w_out ? TJ.act : nullptr;
    __shared__ uint32_t hist[kMaxTiles];
    for (uint32_t t = threadIdx.x; t < n_tiles; t += kCountBlock) hist[t] = 0;
    {   // tile totals and the totals of every 64 tiles start at zero (the
        // column pass adds into them); the slice's block timestamp of every
        // AT position, for the tile pass
        const uint32_t tid = blockIdx.x * kCountBlock + threadIdx.x, nthr = gridDim.x * kCountBlock;
        for (uint32_t t = tid; t < n_tiles + kMaxTiles / kColTiles; t += nthr) tot[t] = 0;
        if (act_table)
            for (uint32_t i = tid; i < G.g; i += nthr) {
                if (G.atb == 2) static_cast<uint16_t*>(act_table)[i] = (uint16_t)act_of(i, c0, G);
                else static_cast<uint8_t*>(act_table)[i] = (uint8_t)act_of(i, c0, G);
            }
    }
    __syncthreads();
    constexpr uint32_t P = kTileRecs / R;
    const uint32_t blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
    if (blk >= TJ.nb) return;  // the grid covers the batch's largest job
    const uint64_t lo = (uint64_t)blk * P;
    const uint64_t hi = lo + P < n ? lo + P : n;
    const uint32_t atv_shift = ts - G.log2g;  // ATVs per tile = 2^atv_shift
    const uint32_t rot = threadIdx.x % R;
    // four pairs per thread per round, loads issued before use
    for (uint64_t q0 = lo + threadIdx.x; q0 < hi; q0 += 4 * kCountBlock) {
        uint32_t a4[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint64_t q = q0 + (uint64_t)e * kCountBlock;
            a4[e] = q < hi ? aip[q] : 0u;
        }
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (q0 + (uint64_t)e * kCountBlock >= hi) break;
            const uint32_t f = mangle(a4[e], G.A);
            const uint32_t z = f & G.umask;
            const uint64_t L = (uint64_t)(f >> G.u);
            const uint64_t LL = L | (L << G.W);
            const uint32_t zc = (z * (uint32_t)R) << G.c;
            uint32_t tile[R];
#pragma unroll
            for (int j = 0; j < R; j++) {
                const uint32_t atv = zc + ((uint32_t)j << G.c) + column(LL, G.sh[j], G.ncol_mask);
                tile[j] = atv >> atv_shift;
            }
            // lane l adds row (j + l) mod R at step j: lanes holding the same
            // frequent host then hit different counters in one instruction
            // instead of piling onto one
            rotate_rows<R>(tile, rot);
#pragma unroll
            for (int j = 0; j < R; j++) atomicAdd(&hist[tile[j]], 1u);
        }
    }
    __syncthreads();
    uint16_t* row = cnt + (uint64_t)blk * n_tiles;
    for (uint32_t t = threadIdx.x; t < n_tiles; t += kCountBlock) row[t] = (uint16_t)hist[t];
}

// Column sums of cnt over each chunk of kTileChunk rows -> csum[chunk][tile],
// and their totals over the chunks -> csum[nchunk][tile].  A block takes 64
// tiles of one chunk; each of its kColGroups waves sums kTileChunk /
// kColGroups rows (loads issued together) and the waves' sums meet in LDS.
// Rows of 64 tiles are 128-byte coalesced reads.
constexpr uint32_t kColGroups = kBlock / kColTiles;
constexpr uint32_t kColRows = kTileChunk / kColGroups;
static_assert(kColGroups * kColRows == kTileChunk, "a chunk splits evenly over the waves");

__global__ __launch_bounds__(kBlock) void k_tile_chunksum(TileBatch J) {
    __builtin_amdgcn_s_setprio(3);
    const TileJob& TJ = J.j[blockIdx.z];
    const uint16_t* __restrict__ cnt = TJ.cnt;
    const uint32_t nb = TJ.nb, n_tiles = TJ.n_tiles, nchunk = TJ.nchunk;
    uint32_t* __restrict__ csum = TJ.csum;
    if (blockIdx.y >= nchunk || blockIdx.x * kColTiles >= n_tiles) return;
    __shared__ uint32_t part[kColGroups][kColTiles];
    const uint32_t tl = threadIdx.x % kColTiles, rg = threadIdx.x / kColTiles;
    const uint32_t t = blockIdx.x * kColTiles + tl;
    const uint32_t c = blockIdx.y;
    const uint32_t b0 = c * kTileChunk + rg * kColRows;
    uint32_t v[kColRows];
#pragma unroll
    for (uint32_t e = 0; e < kColRows; e++)
        v[e] = (t < n_tiles && b0 + e < nb) ? cnt[(uint64_t)(b0 + e) * n_tiles + t] : 0u;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t e = 0; e < kColRows; e++) s += v[e];
    part[rg][tl] = s;
    __syncthreads();
    if (rg == 0) {  // the first wave: one lane per tile of the block
        // the row after the last chunk holds the tile totals, then the
        // totals of every kColTiles tiles (this block's share in one add)
        uint32_t* totals = csum + (uint64_t)nchunk * n_tiles;
        uint32_t tot = 0;
        if (t < n_tiles) {
#pragma unroll
            for (uint32_t g = 0; g < kColGroups; g++) tot += part[g][tl];
            csum[(uint64_t)c * n_tiles + t] = tot;
            atomicAdd(&totals[t], tot);
        }
        uint32_t gsum = tot;
        for (uint32_t o = 32; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o, 64);
        if (tl == 0) atomicAdd(&totals[n_tiles + blockIdx.x], gsum);
    }
}

// Exclusive scan of one block's values held as v (one per thread, NT
// threads); returns the thread's prefix and leaves the block total in *total.
template <uint32_t NT = kBlock>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch /* NT/64 + 1 */,
                                                         uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t x = v;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scratch[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < NT / 64; w++) {
            const uint32_t t = scratch[w];
            scratch[w] = s;
            s += t;
        }
        scratch[NT / 64] = s;
    }
    __syncthreads();
    const uint32_t r = scratch[wv] + x - v;
    *total = scratch[NT / 64];
    __syncthreads();
    return r;
}

// Start of every (block, tile) run in the record array -> pre[b][tile], and
// of every tile's records -> base[tile] (base[n_tiles] = all records).  A
// tile's records start after those of every earlier tile (the totals of the
// tiles before the block's 64, summed by the whole block, then a prefix over
// the 64); a chunk's runs start after the earlier chunks' (their column sums).
// Within the chunk the same split as the chunk sums: each wave's 16 rows,
// loads issued together, start after the rows of the waves before it.
__global__ __launch_bounds__(kBlock) void k_tile_rowpre(TileBatch J) {
    __builtin_amdgcn_s_setprio(3);
    const TileJob& TJ = J.j[blockIdx.z];
    const uint16_t* __restrict__ cnt = TJ.cnt;
    const uint32_t* __restrict__ csum = TJ.csum;
    const uint32_t nb = TJ.nb, n_tiles = TJ.n_tiles, nchunk = TJ.nchunk;
    uint32_t* __restrict__ pre = TJ.pre;
    uint32_t* __restrict__ base = TJ.base;
    if (blockIdx.y >= nchunk || blockIdx.x * kColTiles >= n_tiles) return;
    __shared__ uint32_t part[kColGroups][kColTiles];
    __shared__ uint32_t cp[kColGroups][kColTiles];
    __shared__ uint32_t red[kBlock / 64];
    __shared__ uint32_t tbase[kColTiles];
    const uint32_t tl = threadIdx.x % kColTiles, rg = threadIdx.x / kColTiles;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t t0 = blockIdx.x * kColTiles, t = t0 + tl;
    const uint32_t c = blockIdx.y;
    const uint32_t* tot = csum + (uint64_t)nchunk * n_tiles;
    const uint32_t b0 = c * kTileChunk + rg * kColRows;
    const bool col = t < n_tiles;
    uint32_t v[kColRows];
#pragma unroll
    for (uint32_t e = 0; e < kColRows; e++) v[e] = (col && b0 + e < nb) ? cnt[(uint64_t)(b0 + e) * n_tiles + t] : 0u;
    // records of the tiles before this block's: the totals of the earlier
    // groups of kColTiles tiles
    uint32_t before = 0;
    for (uint32_t q = threadIdx.x; q < blockIdx.x; q += kBlock) before += tot[n_tiles + q];
    for (uint32_t o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
    if (lane == 0) red[wv] = before;
    // this chunk's runs start after the earlier chunks' (split over the waves)
    uint32_t cs = 0;
    for (uint32_t q = rg; q < c; q += kColGroups) cs += col ? csum[(uint64_t)q * n_tiles + t] : 0u;
    cp[rg][tl] = cs;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t e = 0; e < kColRows; e++) s += v[e];
    part[rg][tl] = s;
    __syncthreads();
    if (wv == 0) {
        uint32_t b = 0;
        for (uint32_t w = 0; w < kBlock / 64; w++) b += red[w];
        const uint32_t tt = col ? tot[t] : 0u;
        uint32_t x = tt;  // inclusive prefix of the 64 tiles' totals
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        tbase[lane] = b + x - tt;
        if (c == 0 && col) {
            base[t] = b + x - tt;
            if (t == n_tiles - 1) base[n_tiles] = b + x;
        }
    }
    __syncthreads();
    if (!col) return;
    uint32_t run = tbase[tl];
    for (uint32_t g = 0; g < kColGroups; g++) run += cp[g][tl];
    for (uint32_t g = 0; g < rg; g++) run += part[g][tl];
#pragma unroll
    for (uint32_t e = 0; e < kColRows; e++) {
        if (b0 + e < nb) pre[(uint64_t)(b0 + e) * n_tiles + t] = run;
        run += v[e];
    }
}

// Pass 2: the block's records grouped by tile in LDS, then written run by run.
template <int R>
__global__ __launch_bounds__(kScatterBlock) void k_tile_scatter(TileBatch J) {
    __builtin_amdgcn_s_setprio(3);
    const TileJob& TJ = J.j[blockIdx.y];
    const Geometry& G = TJ.G;
    const uint32_t* __restrict__ aip = TJ.aip;
    const uint32_t* __restrict__ bip = TJ.bip;
    const uint64_t n = TJ.n;
    const uint32_t ts = tile_shift(G), n_tiles = TJ.n_tiles;
    const uint16_t* __restrict__ cnt = TJ.cnt;
    const uint32_t* __restrict__ pre = TJ.pre;
    uint16_t* __restrict__ rec = TJ.rec;
    // 80 KiB of LDS, so that two blocks share a CU: the staged records, then
    // one word per tile (its slot cursor, later its run's offset in rec);
    // the block scan's scratch sits where the records go, before they do
    extern __shared__ __align__(16) uint8_t smem_tile[];
    uint32_t* staged = reinterpret_cast<uint32_t*>(smem_tile);  // tile << 16 | in-tile index, grouped by tile
    uint32_t* cur = staged + kTileRecs;                         // slot cursors, then rec offset minus LDS start
    uint32_t* scratch = staged;
    constexpr uint32_t P = kTileRecs / R;
    constexpr uint32_t PPT = (P + kScatterBlock - 1) / kScatterBlock;  // pairs per thread
    const uint32_t blk = xcd_contiguous_block(blockIdx.x, gridDim.x);
    if (blk >= TJ.nb) return;  // the grid covers the batch's largest job
    const uint64_t lo = (uint64_t)blk * P;
    const uint64_t hi = lo + P < n ? lo + P : n;
    const uint32_t lmask = (1u << ts) - 1u;
    // hash the block's pairs once; the targets stay in registers
    uint32_t tgt[PPT][R];
    uint32_t a4[PPT], b4[PPT];
#pragma unroll
    for (uint32_t e = 0; e < PPT; e++) {
        const uint64_t q = lo + threadIdx.x + (uint64_t)e * kScatterBlock;
        a4[e] = q < hi ? aip[q] : 0u;
        b4[e] = q < hi ? bip[q] : 0u;
    }
#pragma unroll
    for (uint32_t e = 0; e < PPT; e++) {
        const bool ok = lo + threadIdx.x + (uint64_t)e * kScatterBlock < hi;
        uint32_t idx[R];
        pair_targets<R>(a4[e], b4[e], G, idx);
#pragma unroll
        for (int j = 0; j < R; j++) {
            // tile in the high half, in-tile index in the low half (ts <= 16)
            tgt[e][j] = ok ? ((idx[j] >> ts) << 16) | (idx[j] & lmask) : ~0u;
        }
    }
    // LDS run starts: exclusive scan of the block's counts (its row of the
    // count table), kMaxTiles / kScatterBlock consecutive tiles per thread
    constexpr uint32_t TPT = kMaxTiles / kScatterBlock;
    const uint32_t* prow = pre + (uint64_t)blk * n_tiles;
    const uint16_t* crow = cnt + (uint64_t)blk * n_tiles;
    uint32_t c[TPT], sum = 0;
#pragma unroll
    for (uint32_t e = 0; e < TPT; e++) {
        const uint32_t t = threadIdx.x * TPT + e;
        c[e] = t < n_tiles ? crow[t] : 0u;
        sum += c[e];
    }
    uint32_t total;
    uint32_t st = block_exclusive_scan<kScatterBlock>(sum, scratch, &total);
    uint32_t st0[TPT];
#pragma unroll
    for (uint32_t e = 0; e < TPT; e++) {
        const uint32_t t = threadIdx.x * TPT + e;
        st0[e] = st;
        if (t < n_tiles) cur[t] = st;
        st += c[e];
    }
    __syncthreads();
    // lane l takes its rows in the order (j + l) mod R, as in pass 1: lanes
    // holding one frequent host then move different tiles' cursors together
    const uint32_t rot = threadIdx.x % R;
#pragma unroll
    for (uint32_t e = 0; e < PPT; e++) {
        rotate_rows<R>(tgt[e], rot);
#pragma unroll
        for (int j = 0; j < R; j++) {
            const uint32_t v = tgt[e][j];
            if (v == ~0u) continue;
            staged[atomicAdd(&cur[v >> 16], 1u)] = v;
        }
    }
    __syncthreads();
    // the cursors become each run's offset in rec minus its LDS start
#pragma unroll
    for (uint32_t e = 0; e < TPT; e++) {
        const uint32_t t = threadIdx.x * TPT + e;
        if (t < n_tiles) cur[t] = prow[t] - st0[e];  // modulo 2^32; exact once a slot is added
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < total; i += kScatterBlock) {
        const uint32_t v = staged[i];
        rec[cur[v >> 16] + i] = (uint16_t)(v & 0xFFFFu);
    }
}

// Pass 3: one workgroup per tile applies the tile's records in LDS.  When the
// call opens the slice (preserve != 0) Alg 2 first runs here on the two due
// blocks of every ATV of the tile (the AT ranges of S), before any record:
// the same order as a separate opening pass, without its extra pool traffic.
// With w_out the pass also ends the slice's window count: every tile is
// visited (the call opened the slice) and, once its records are in, the k'-
// weight of each of its ATVs (Alg 1 with window kq_w) goes to w_out, which
// is what the close would compute if no other call adds to the slice.
template <typename T>
__global__ __launch_bounds__(kApplyBlock) void k_tile_apply(TileBatch J) {
    const TileJob& TJ = J.j[blockIdx.y];
    if (blockIdx.x >= TJ.n_tiles) return;  // the grid covers the batch's largest pool
    const Geometry& G = TJ.G;
    uint8_t* __restrict__ pool = TJ.pool;
    const uint16_t* __restrict__ rec = TJ.rec;
    const uint32_t* __restrict__ base = TJ.base;
    const uint32_t c0 = TJ.c0, preserve = TJ.preserve, kq_w = TJ.kq_w;
    const PreserveSpans& S = TJ.S;
    uint32_t* __restrict__ w_out = TJ.w_out;
    const T* __restrict__ act_table = static_cast<const T*>(TJ.act);
    extern __shared__ __align__(16) uint8_t smem_apply[];
    const uint32_t t = blockIdx.x;
    const uint32_t lo = base[t], hi = base[t + 1];
    if (lo == hi && !preserve) return;  // nothing lands here: the tile stays as it is
    uint4* lds = reinterpret_cast<uint4*>(smem_apply);
    uint4* src = reinterpret_cast<uint4*>(pool + (uint64_t)t * kTileBytes);
    // Everything the workgroup reads is requested before the first wait: the
    // tile (read and written once per call, so streamed past the caches), the
    // first records (a ragged head and tail record and one 16-byte chunk of
    // the aligned body per thread) and, for the window count, the block
    // timestamps of the thread's chunks.
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    constexpr uint32_t kPerThread = kTileBytes / 16 / kApplyBlock;
    static_assert(kPerThread * 16 * kApplyBlock == kTileBytes, "a tile is whole 16-byte chunks per thread");
    constexpr uint32_t CA = kPerChunk<T>;
    const uint32_t tid = threadIdx.x;
    u32x4* lds4 = reinterpret_cast<u32x4*>(smem_apply);
    u32x4* src4 = reinterpret_cast<u32x4*>(src);
    u32x4 v[kPerThread];
#pragma unroll
    for (uint32_t u = 0; u < kPerThread; u++) v[u] = __builtin_nontemporal_load(src4 + tid + u * kApplyBlock);
    const uint32_t a8 = (lo + 7u) & ~7u, b8 = hi & ~7u;
    const uint32_t n8 = a8 < b8 ? (b8 - a8) / 8 : 0;
    const uint4* rb = reinterpret_cast<const uint4*>(rec + a8);
    uint32_t r_head = ~0u, r_tail = ~0u;
    uint4 r_body = make_uint4(0, 0, 0, 0);
    if (n8) {
        if (lo + tid < a8) r_head = rec[lo + tid];
        if (b8 + tid < hi) r_tail = rec[b8 + tid];
        if (tid < n8) r_body = rb[tid];
    } else if (lo + tid < hi) {
        r_head = rec[lo + tid];  // a run shorter than 16 records: one each
    }
    uint4 acv[kPerThread];
    if (w_out) {
#pragma unroll
        for (uint32_t u = 0; u < kPerThread; u++)
            acv[u] = *reinterpret_cast<const uint4*>(act_table + (((tid + u * kApplyBlock) * CA) & (G.g - 1u)));
    }
#pragma unroll
    for (uint32_t u = 0; u < kPerThread; u++) lds4[tid + u * kApplyBlock] = v[u];
    __syncthreads();
    T* tl = reinterpret_cast<T*>(smem_apply);
    if (preserve) {
        const uint32_t n0 = S.r0hi - S.r0lo, n1 = S.r1hi - S.r1lo, per = n0 + n1;
        const uint32_t atvs = (kTileBytes / sizeof(T)) >> G.log2g;
        for (uint32_t q = tid; q < atvs * per; q += kApplyBlock) {
            const uint32_t v = q / per, e = q - v * per;
            const uint32_t pos = e < n0 ? S.r0lo + e : S.r1lo + (e - n0);
            T* a = tl + (v << G.log2g) + pos;
            const uint32_t at = *a;
            // Alg 2: the block whose timestamp becomes 0 clears ATs <= k, the
            // one whose timestamp becomes k clears k..2k-1 and 0
            if (e < n0 ? at <= G.k : ((at >= G.k && at < G.twok) || at == 0)) *a = (T)G.twok;
        }
        __syncthreads();
    }
    const uint32_t gmask = G.g - 1u;
    auto apply = [&](auto act) {
        if (r_head != ~0u) tl[r_head] = (T)act(r_head & gmask);
        if (r_tail != ~0u) tl[r_tail] = (T)act(r_tail & gmask);
        if (tid < n8) {
#pragma unroll
            for (uint32_t e = 0; e < 8; e++) {
                const uint32_t loc = (word_of(r_body, e / 2) >> (16 * (e & 1))) & 0xFFFFu;
                tl[loc] = (T)act(loc & gmask);
            }
        }
        // the rest of a long run, four chunks in flight per thread
        for (uint32_t q0 = tid + kApplyBlock; q0 < n8; q0 += 4 * kApplyBlock) {
            uint4 w[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const uint32_t q = q0 + u * kApplyBlock;
                w[u] = q < n8 ? rb[q] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                if (q0 + u * kApplyBlock >= n8) break;
#pragma unroll
                for (uint32_t e = 0; e < 8; e++) {
                    const uint32_t loc = (word_of(w[u], e / 2) >> (16 * (e & 1))) & 0xFFFFu;
                    tl[loc] = (T)act(loc & gmask);
                }
            }
        }
    };
    if (G.blk_a >= 2) {
        const uint32_t magic = (uint32_t)G.blk_magic;
        apply([&](uint32_t i) { return act_of_narrow(i, c0, magic, G); });
    } else {
        apply([&](uint32_t i) { return act_of(i, c0, G); });
    }
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kPerThread; u++) v[u] = lds4[tid + u * kApplyBlock];
#pragma unroll
    for (uint32_t u = 0; u < kPerThread; u++) __builtin_nontemporal_store(v[u], src4 + tid + u * kApplyBlock);
    if (w_out) {
        __shared__ uint32_t wl[kTileBytes / 16 / 64];  // per ATV, when an ATV spans more than 64 chunks
        const uint32_t cpa = G.g / CA;                // chunks per ATV (a power of two)
        const uint32_t seg = cpa < 64 ? cpa : 64;
        const uint32_t atvs = (kTileBytes / sizeof(T)) >> G.log2g;
        const uint64_t atv0 = (uint64_t)t * atvs;
        const uint32_t lane = threadIdx.x & 63u;
        if (cpa > 64) {
            for (uint32_t v = threadIdx.x; v < atvs; v += kApplyBlock) wl[v] = 0;
            __syncthreads();
        }
        const bool packed = G.twok <= 32768u;
        const bool bytes4 = sizeof(T) == 1 && G.twok <= 64u;
        const uint32_t twok2 = both_halves(G.twok), c_at = both_halves(0x8000u - G.twok);
        const uint32_t c_kq = both_halves(0x8000u - kq_w);
        const uint32_t twok4 = G.twok * kByteOnes, kq4 = kq_w * kByteOnes, tkq4 = (G.twok + kq_w) * kByteOnes;
#pragma unroll
        for (uint32_t u = 0; u < kPerThread; u++) {
            const uint32_t c = tid + u * kApplyBlock;
            const uint32_t pos = c * CA;                // AT index inside the tile
            const uint4 ac = acv[u];                    // block timestamps of positions pos mod g ..
            const uint4 d = lds[c];
            uint32_t act_n;
            if (bytes4) {
                act_n = 0;
#pragma unroll
                for (uint32_t q = 0; q < 4; q++)
                    act_n += byte_active(byte_lanes(word_of(d, q), word_of(ac, q), twok4), kq4, tkq4);
            } else if (packed) {
                constexpr uint32_t NH = 8 / sizeof(T);
                uint32_t ha[NH], hc[NH], ni = 0;
                chunk_halves<T>(d, ha);
                chunk_halves<T>(ac, hc);
#pragma unroll
                for (uint32_t q = 0; q < NH; q++) ni += inactive2(alg1_halves(ha[q], hc[q], twok2, c_at), c_kq);
                act_n = CA - ni;
            } else {
                act_n = __popc(active_mask_chunk<T>(d, ac, G.twok, kq_w));
            }
            for (uint32_t o = seg / 2; o > 0; o >>= 1) act_n += __shfl_xor(act_n, o, 64);
            if (lane % seg == 0) {
                const uint32_t v = pos >> G.log2g;
                if (cpa <= 64) w_out[atv0 + v] = act_n;
                else atomicAdd(&wl[v], act_n);
            }
        }
        if (cpa > 64) {
            __syncthreads();
            for (uint32_t v = threadIdx.x; v < atvs; v += kApplyBlock) w_out[atv0 + v] = wl[v];
        }
    }
}

// ---------------------------------------------------------------- a4: close
// One read of the pool: k'-weight of every ATV (Alg 1 per AT) for each of
// the Wn.n windows.  A group of lpa = min(64, g/CA) lanes covers one ATV with
// 16-byte loads of CA ATs; a wave covers 64/lpa ATVs per step.  Block
// timestamps come from an LDS table of g ATs.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_close(const T* __restrict__ pool, uint32_t* __restrict__ w,
                                                  uint64_t n_atv, Geometry G, uint32_t c0, CloseWindows Wn) {
    extern __shared__ __align__(16) uint8_t smem_close[];
    T* act_lut = reinterpret_cast<T*>(smem_close);
    fill_act_lut(act_lut, c0, G);
    constexpr uint32_t CA = kPerChunk<T>;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t lpa = G.g / CA < 64 ? G.g / CA : 64;
    const uint32_t apw = 64 / lpa;
    const uint32_t sub = lane / lpa, sl = lane % lpa;
    const uint32_t steps = G.g / (CA * lpa);
    // the packed form counts inactive ATs; it needs 4k <= 2^16.  Byte ATs with
    // 4k <= 128 count active ATs four per operation instead.
    const bool packed = G.twok <= 32768u;
    const bool bytes4 = sizeof(T) == 1 && G.twok <= 64u;
    const uint32_t twok2 = both_halves(G.twok), c_at = both_halves(0x8000u - G.twok);
    const uint32_t c_kq0 = both_halves(0x8000u - Wn.kq[0]);
    const uint32_t twok4 = G.twok * kByteOnes;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t base = wave * apw; base < n_atv; base += nwaves * apw) {
        const uint64_t atv = base + sub;
        uint32_t cnt[kMaxWindows];
#pragma unroll
        for (uint32_t j = 0; j < kMaxWindows; j++) cnt[j] = 0;
        if (atv < n_atv) {
            const T* p = pool + (atv << G.log2g);
            // four 16-byte loads in flight per lane
            for (uint32_t st0 = 0; st0 < steps; st0 += 4) {
                uint4 d[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; u++)
                    if (st0 + u < steps) d[u] = *reinterpret_cast<const uint4*>(p + ((st0 + u) * lpa + sl) * CA);
#pragma unroll
                for (uint32_t u = 0; u < 4; u++) {
                    if (st0 + u >= steps) break;
                    const uint4 ac = *reinterpret_cast<const uint4*>(act_lut + ((st0 + u) * lpa + sl) * CA);
                    if (bytes4) {
#pragma unroll
                        for (uint32_t q = 0; q < 4; q++) {
                            const ByteLanes b = byte_lanes(word_of(d[u], q), word_of(ac, q), twok4);
                            cnt[0] += byte_active(b, Wn.kq[0] * kByteOnes, (G.twok + Wn.kq[0]) * kByteOnes);
                            if (Wn.n > 1) {
#pragma unroll
                                for (uint32_t j = 1; j < kMaxWindows; j++)
                                    if (j < Wn.n)
                                        cnt[j] += byte_active(b, Wn.kq[j] * kByteOnes, (G.twok + Wn.kq[j]) * kByteOnes);
                            }
                        }
                    } else if (packed) {
                        constexpr uint32_t NH = 8 / sizeof(T);  // 16-bit halves per chunk
                        uint32_t ha[NH], hc[NH];
                        chunk_halves<T>(d[u], ha);
                        chunk_halves<T>(ac, hc);
#pragma unroll
                        for (uint32_t q = 0; q < NH; q++) {
                            const Alg1Halves hh = alg1_halves(ha[q], hc[q], twok2, c_at);
                            cnt[0] += inactive2(hh, c_kq0);
                            if (Wn.n > 1) {
#pragma unroll
                                for (uint32_t j = 1; j < kMaxWindows; j++)
                                    if (j < Wn.n) cnt[j] += inactive2(hh, both_halves(0x8000u - Wn.kq[j]));
                            }
                        }
                    } else if (Wn.n == 1) {
                        cnt[0] += __popc(active_mask_chunk<T>(d[u], ac, G.twok, Wn.kq[0]));
                    } else {
#pragma unroll
                        for (uint32_t j = 0; j < kMaxWindows; j++)
                            if (j < Wn.n) cnt[j] += __popc(active_mask_chunk<T>(d[u], ac, G.twok, Wn.kq[j]));
                    }
                }
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < kMaxWindows; j++) {
            if (j >= Wn.n) break;
            uint32_t c = packed && !bytes4 && atv < n_atv ? steps * CA - cnt[j] : cnt[j];  // the lane's active ATs
            for (uint32_t o = lpa / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            if (sl == 0 && atv < n_atv) w[(uint64_t)j * n_atv + atv] = c;
        }
    }
}

// Age histogram of every ATV in one read of the pool (Section 3: an AT holds
// the timestamp of the slice that last set it, so its age is the timestamp
// distance, and it counts in window k' exactly when that age is below k').
// hist[atv * k + a] = #{ATs of the ATV not inactive with age a}, a < k, so
// the k'-weight of every window k' <= k is a prefix sum of the ATV's row and
// no later window needs the pool again.  One wave per ATV, each with its own
// k bins in LDS; the wave also writes the kq-weight of the close's window.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_close_hist(const T* __restrict__ pool, uint16_t* __restrict__ hist,
                                                       uint32_t* __restrict__ w, uint64_t n_atv, Geometry G,
                                                       uint32_t c0, uint32_t kq) {
    extern __shared__ __align__(16) uint8_t smem_hist[];
    T* act_lut = reinterpret_cast<T*>(smem_hist);
    const uint32_t K = G.k;
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    uint32_t* bins = reinterpret_cast<uint32_t*>(smem_hist + ((G.g * sizeof(T) + 15u) & ~15u)) + wv * K;
    for (uint32_t a = lane; a < K; a += 64) bins[a] = 0;
    fill_act_lut(act_lut, c0, G);  // ends with a barrier
    constexpr uint32_t CA = kPerChunk<T>, N = kPerWord<T>;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + wv;
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t atv = wave; atv < n_atv; atv += nwaves) {
        const T* p = pool + (atv << G.log2g);
        for (uint32_t off = lane * CA; off < G.g; off += 64 * CA) {
            const uint4 d = *reinterpret_cast<const uint4*>(p + off);
            const uint4 ac = *reinterpret_cast<const uint4*>(act_lut + off);
#pragma unroll
            for (uint32_t b = 0; b < CA; b++) {
                const uint32_t at = at_in_word<T>(word_of(d, b / N), b % N);
                const uint32_t act = at_in_word<T>(word_of(ac, b / N), b % N);
                const uint32_t age = act >= at ? act - at : act + G.twok - at;
                if (at != G.twok && age < K) atomicAdd(&bins[age], 1u);
            }
        }
        // the wave's own LDS operations complete in order: its bins are whole
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t wk = 0;
        uint16_t* row = hist + atv * K;
        for (uint32_t a = lane; a < K; a += 64) {
            const uint32_t v = bins[a];
            row[a] = (uint16_t)v;  // v <= g <= 2^15
            wk += a < kq ? v : 0u;
            bins[a] = 0;
        }
        for (uint32_t o = 32; o > 0; o >>= 1) wk += __shfl_xor(wk, o, 64);
        if (lane == 0) w[atv] = wk;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// k'-weights of every ATV from the age histograms: the sum of the first k'
// bins of its row (one wave per ATV, coalesced reads of the row).
__global__ __launch_bounds__(kBlock) void k_hist_weights(const uint16_t* __restrict__ hist, uint32_t K,
                                                         uint64_t n_atv, uint32_t kq, uint32_t* __restrict__ w) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t atv = wave; atv < n_atv; atv += nwaves) {
        const uint16_t* row = hist + atv * K;
        uint32_t s = 0;
        for (uint32_t a = lane; a < kq; a += 64) s += row[a];
        for (uint32_t o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) w[atv] = s;
    }
}

// One workgroup per (frame, row): AAT = sum of the row's weights, and the
// ascending list of super columns (weight >= T) with its length.
__global__ __launch_bounds__(kBlock) void k_summarize(const uint32_t* __restrict__ w_all, uint64_t* __restrict__ aat_all,
                                                      uint32_t* __restrict__ sa_all, uint32_t* __restrict__ sa_cnt_all,
                                                      uint32_t* __restrict__ cnt_host, Geometry G, uint64_t n_atv,
                                                      uint32_t ngroups) {
    __shared__ uint32_t wave_cnt[kBlock / 64];
    __shared__ unsigned long long wave_sum[kBlock / 64];
    const uint32_t grp = blockIdx.x;
    const uint32_t* w = w_all + (uint64_t)blockIdx.y * n_atv;   // window blockIdx.y
    uint64_t* aat = aat_all + (uint64_t)blockIdx.y * ngroups;
    uint32_t* sa = sa_all + (uint64_t)blockIdx.y * n_atv;
    uint32_t* sa_cnt = sa_cnt_all + (uint64_t)blockIdx.y * ngroups;
    const uint64_t base = (uint64_t)grp << G.c;
    const uint32_t ncol = G.ncol_mask + 1;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint64_t sum = 0;
    uint32_t written = 0;
    for (uint32_t x0 = 0; x0 < ncol; x0 += kBlock) {
        uint32_t x = x0 + threadIdx.x;
        uint32_t wx = x < ncol ? w[base + x] : 0u;
        bool sup = x < ncol && wx >= G.T;
        sum += wx;
        uint64_t ball = __ballot(sup);
        uint32_t before = __popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wv] = __popcll(ball);
        __syncthreads();
        uint32_t off = written;
        for (uint32_t q = 0; q < wv; q++) off += wave_cnt[q];
        uint32_t tot = 0;
        for (uint32_t q = 0; q < kBlock / 64; q++) tot += wave_cnt[q];
        if (sup) sa[base + off + before] = x;
        written += tot;
        __syncthreads();
    }
    for (uint32_t o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane == 0) wave_sum[wv] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (uint32_t q = 0; q < kBlock / 64; q++) t += wave_sum[q];
        aat[grp] = t;
        sa_cnt[grp] = written;
        if (cnt_host) cnt_host[(uint64_t)blockIdx.y * ngroups + grp] = written;  // mapped host memory
    }
}

// ---------------------------------------------------------------- a5: restore
// Alg 4 as a pruned join.  One work item per (x_0, x_1) pair of a frame; rows
// 2..r-1 are added depth first, and a column is kept only if its bits agree
// with the LBS bits fixed so far -- so a tuple survives exactly when all its
// duplicate positions agree.  The survivor's LBS with the frame index gives f,
// unmangled into the address.
__device__ __forceinline__ uint32_t place(uint32_t x, uint32_t sh, const Geometry& G) {
    uint64_t t = (uint64_t)x << sh;
    return (uint32_t)((t | (t >> G.W)) & G.maskW);
}

__device__ __forceinline__ void emit(uint32_t L, uint32_t z, const Geometry& G, uint32_t* cand, uint64_t cap,
                                     unsigned long long* counter) {
    uint32_t F = G.u ? ((L << G.u) | z) : L;
    uint32_t a = mangle(F, G.Ainv);
    unsigned long long pos = atomicAdd(counter, 1ull);
    if (pos < cap) cand[pos] = a;
}

__global__ __launch_bounds__(kBlock) void k_restore_join(const uint32_t* __restrict__ sa,
                                                         const uint32_t* __restrict__ sa_cnt,
                                                         const uint64_t* __restrict__ prefix, uint64_t n_items,
                                                         Geometry G, uint32_t* __restrict__ cand, uint64_t cap,
                                                         unsigned long long* counter) {
    const uint32_t nframe = G.umask + 1, R = G.r;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n_items;
         it += (uint64_t)gridDim.x * blockDim.x) {
        // frame of this item: last z with prefix[z] <= it
        uint32_t lo = 0, hi = nframe;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (prefix[mid] <= it) lo = mid;
            else hi = mid;
        }
        const uint32_t z = lo;
        const uint64_t rem = it - prefix[z];
        const uint32_t* cnt = sa_cnt + (uint64_t)z * R;
        const uint64_t rowbase = (uint64_t)z * R << G.c;
        if (R == 1) {
            emit(place(sa[rowbase + rem], G.sh[0], G), z, G, cand, cap, counter);
            continue;
        }
        const uint32_t c1 = cnt[1];
        const uint32_t i0 = (uint32_t)(rem / c1), i1 = (uint32_t)(rem - (uint64_t)i0 * c1);
        uint32_t L = place(sa[rowbase + i0], G.sh[0], G);
        uint32_t M = G.win[0];
        uint32_t P = place(sa[rowbase + (1ull << G.c) + i1], G.sh[1], G);
        if ((P ^ L) & M & G.win[1]) continue;
        L |= P;
        M |= G.win[1];
        if (R == 2) {
            emit(L, z, G, cand, cap, counter);
            continue;
        }
        uint32_t Ls[kMaxRows], Ms[kMaxRows], idx[kMaxRows];
        uint32_t lvl = 2;
        Ls[2] = L;
        Ms[2] = M;
        idx[2] = 0;
        for (;;) {
            if (idx[lvl] >= cnt[lvl]) {
                if (lvl == 2) break;
                lvl--;
                idx[lvl]++;
                continue;
            }
            uint32_t Pq = place(sa[rowbase + ((uint64_t)lvl << G.c) + idx[lvl]], G.sh[lvl], G);
            if ((Pq ^ Ls[lvl]) & Ms[lvl] & G.win[lvl]) {
                idx[lvl]++;
                continue;
            }
            if (lvl == R - 1) {
                emit(Ls[lvl] | Pq, z, G, cand, cap, counter);
                idx[lvl]++;
            } else {
                Ls[lvl + 1] = Ls[lvl] | Pq;
                Ms[lvl + 1] = Ms[lvl] | G.win[lvl];
                lvl++;
                idx[lvl] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------- sort
// Bitonic sort of a power-of-two array: 2048-key tiles in LDS, global steps
// for strides of a tile or more.
constexpr uint32_t kTile = 2048;

__device__ __forceinline__ void cmp_swap_lds(uint32_t* s, uint32_t li, uint32_t lj, bool up) {
    uint32_t a = s[li], b = s[lj];
    if ((a > b) == up) {
        s[li] = b;
        s[lj] = a;
    }
}

// kfrom..kto: sizes of bitonic sequences merged inside the tile; if merge_only,
// only the j < kTile steps of size k = kfrom are run.
__global__ __launch_bounds__(kBlock) void k_bitonic_tile(uint32_t* __restrict__ keys, uint32_t kfrom,
                                                         uint32_t kto) {
    __shared__ uint32_t s[kTile];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (uint32_t q = threadIdx.x; q < kTile; q += kBlock) s[q] = keys[base + q];
    __syncthreads();
    for (uint32_t k = kfrom; k <= kto; k <<= 1) {
        for (uint32_t j = (k >> 1) < (kTile >> 1) ? (k >> 1) : (kTile >> 1); j > 0; j >>= 1) {
            for (uint32_t p = threadIdx.x; p < kTile / 2; p += kBlock) {
                uint32_t li = 2 * p - (p & (j - 1));
                uint32_t lj = li + j;
                bool up = ((base + li) & k) == 0;
                cmp_swap_lds(s, li, lj, up);
            }
            __syncthreads();
        }
    }
    for (uint32_t q = threadIdx.x; q < kTile; q += kBlock) keys[base + q] = s[q];
}

__global__ __launch_bounds__(kBlock) void k_bitonic_global(uint32_t* __restrict__ keys, uint64_t n, uint64_t k,
                                                           uint64_t j) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n / 2;
         p += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i = 2 * p - (p & (j - 1));
        uint64_t l = i + j;
        bool up = (i & k) == 0;
        uint32_t a = keys[i], b = keys[l];
        if ((a > b) == up) {
            keys[i] = b;
            keys[l] = a;
        }
    }
}

__global__ void k_small_sort(uint32_t* keys, uint32_t n) {
    // n <= kTile, power of two, single workgroup
    __shared__ uint32_t s[kTile];
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) s[q] = keys[q];
    __syncthreads();
    for (uint32_t k = 2; k <= n; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t p = threadIdx.x; p < n / 2; p += blockDim.x) {
                uint32_t li = 2 * p - (p & (j - 1));
                cmp_swap_lds(s, li, li + j, (li & k) == 0);
            }
            __syncthreads();
        }
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) keys[q] = s[q];
}

__global__ void k_pad_u32(uint32_t* keys, uint64_t from, uint64_t to) {
    for (uint64_t q = from + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < to;
         q += (uint64_t)gridDim.x * blockDim.x)
        keys[q] = 0xFFFFFFFFu;
}

// ---------------------------------------------------------------- a6: estimate
// Alg 5 + Eq 4.  One wave per host: lanes read 16-byte chunks of the host's r
// ATVs, AND the per-row active masks (Alg 1), count, reduce; lane 0 applies
// Eq 4 in FP64 with the same operation order as a plain evaluation (P_j
// exact, UP multiplied left to right, no contraction).
__device__ double eq4(uint32_t nat, uint32_t z, const uint64_t* __restrict__ aat, const Geometry& G,
                      uint8_t* flags_out) {
    uint8_t fl = 0;
    const double gd = (double)G.g;
    const double cells = (double)((uint64_t)G.g << G.c);
    double UP = 1.0;
    for (uint32_t j = 0; j < G.r; j++) {
        double Pj = (double)aat[(uint64_t)z * G.r + j] / cells;
        UP = (j == 0) ? Pj : UP * Pj;
    }
    const double one_minus = 1.0 - UP;
    double est;
    if (one_minus == 0.0) {
        est = __builtin_inf();
        fl |= AT_F_SAT;
    } else {
        uint32_t natc = nat;
        if (nat >= G.g) {
            natc = G.g - 1;
            fl |= AT_F_SAT;
        }
        const double q = (double)(G.g - natc) / (gd * one_minus);
        est = -gd * log(q);
        if (est < 0) fl |= AT_F_NEG;
    }
    if (est >= G.theta) fl |= AT_F_SUPER;
    *flags_out = fl;
    return est;
}

template <int R, typename T>
__global__ __launch_bounds__(kBlock) void k_estimate(const T* __restrict__ pool, const uint64_t* __restrict__ aat,
                                                     const uint32_t* __restrict__ aips, uint64_t n, Geometry G,
                                                     uint32_t c0q, uint32_t kq, double* __restrict__ est,
                                                     uint8_t* __restrict__ flags, uint32_t* __restrict__ nat_out) {
    extern __shared__ __align__(16) uint8_t smem_est[];
    T* act_lut = reinterpret_cast<T*>(smem_est);
    fill_act_lut(act_lut, c0q, G);
    constexpr uint32_t CA = kPerChunk<T>;
    const bool packed = G.twok <= 32768u;  // the packed form of Alg 1 needs 4k <= 2^16
    const uint32_t twok2 = both_halves(G.twok), c_at = both_halves(0x8000u - G.twok);
    const uint32_t c_kq = both_halves(0x8000u - kq);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t h = wave; h < n; h += nwaves) {
        const uint32_t a = aips[h];
        const uint32_t f = mangle(a, G.A);
        const uint32_t z = f & G.umask;
        const uint64_t L = (uint64_t)(f >> G.u);
        const uint64_t LL = L | (L << G.W);
        const T* rows[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            uint32_t x = column(LL, G.sh[j], G.ncol_mask);
            rows[j] = pool + (((((uint64_t)z * R + j) << G.c) + x) << G.log2g);
        }
        uint32_t cnt = 0;
        // up to four chunk positions per lane in flight, r loads each
        for (uint32_t off0 = lane * CA; off0 < G.g; off0 += 4 * 64 * CA) {
            uint4 d[4][R];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const uint32_t off = off0 + u * 64 * CA;
                if (off < G.g) {
#pragma unroll
                    for (int j = 0; j < R; j++) d[u][j] = *reinterpret_cast<const uint4*>(rows[j] + off);
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const uint32_t off = off0 + u * 64 * CA;
                if (off >= G.g) break;
                const uint4 ac = *reinterpret_cast<const uint4*>(act_lut + off);
                if (packed) {
                    // positions inactive in any row, then the active rest
                    constexpr uint32_t NH = 8 / sizeof(T);
                    uint32_t hc[NH], inact[NH];
                    chunk_halves<T>(ac, hc);
#pragma unroll
                    for (uint32_t q = 0; q < NH; q++) inact[q] = 0;
#pragma unroll
                    for (int j = 0; j < R; j++) {
                        uint32_t ha[NH];
                        chunk_halves<T>(d[u][j], ha);
#pragma unroll
                        for (uint32_t q = 0; q < NH; q++) {
                            const Alg1Halves hh = alg1_halves(ha[q], hc[q], twok2, c_at);
                            inact[q] |= (as_u32(as_u16x2(hh.dist) + as_u16x2(c_kq)) | hh.off) & 0x80008000u;
                        }
                    }
                    uint32_t ni = 0;
#pragma unroll
                    for (uint32_t q = 0; q < NH; q++) ni += __popc(inact[q]);
                    cnt += CA - ni;
                } else {
                    uint32_t m = ~0u;
#pragma unroll
                    for (int j = 0; j < R; j++) m &= active_mask_chunk<T>(d[u][j], ac, G.twok, kq);
                    cnt += __popc(m);
                }
            }
        }
        for (uint32_t o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) {
            uint8_t fl;
            double e = eq4(cnt, z, aat, G, &fl);
            if (est) est[h] = e;
            if (flags) flags[h] = fl;
            if (nat_out) nat_out[h] = cnt;
        }
    }
}


// ---------------------------------------------------------------- a7: features
// Occupancy-by-age features of a host (one workgroup per host, its 16-byte
// chunks of positions spread over the four waves): e_i = largest age over the
// host's r ATs at position i when all are active for the full window k.
// feat[d] = #{i : e_i = d}/g (d < min(k, 61)); feat[61] = min(ln(1 + max(plain,
// 0)), 20)/16 with plain the Eq 4 estimate for the close's k'; feat[62] =
// k/64; feat[63] = mean over rows of AAT/(g*2^c).  NAT(k') = #{i : e_i < k'}
// is counted in the same pass, so the plain estimate comes along.  The LDS
// histogram keeps ages below 64.
template <int R, typename T>
__global__ __launch_bounds__(kBlock) void k_features(const T* __restrict__ pool, const uint64_t* __restrict__ aat,
                                                     const uint32_t* __restrict__ aips, uint64_t n, Geometry G,
                                                     uint32_t c0q, uint32_t kq, float* __restrict__ feat,
                                                     double* __restrict__ est, uint8_t* __restrict__ flags) {
    extern __shared__ __align__(16) uint8_t smem_feat[];
    T* act_lut = reinterpret_cast<T*>(smem_feat);
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem_feat + ((G.g * sizeof(T) + 15u) & ~15u));  // 64 bins
    __shared__ uint32_t nat_w[kBlock / 64];
    // the first host's address is loaded while the table fills (it may sit
    // in host memory)
    uint32_t a_next = blockIdx.x < n ? aips[blockIdx.x] : 0u;
    fill_act_lut(act_lut, c0q, G);
    constexpr uint32_t CA = kPerChunk<T>, N = kPerWord<T>;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    for (uint64_t h = blockIdx.x; h < n; h += gridDim.x) {
        if (threadIdx.x < 64) hist[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t a = a_next;
        const uint32_t f = mangle(a, G.A);
        const uint32_t z = f & G.umask;
        const uint64_t L = (uint64_t)(f >> G.u);
        const uint64_t LL = L | (L << G.W);
        const T* rows[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            uint32_t x = column(LL, G.sh[j], G.ncol_mask);
            rows[j] = pool + (((((uint64_t)z * R + j) << G.c) + x) << G.log2g);
        }
        if (h + gridDim.x < n) a_next = aips[h + gridDim.x];
        // ages 0..15 are counted in registers, four 16-bit counts per word,
        // and summed over the wave before they reach the LDS histogram: the
        // ages of a window pile onto a few bins, and per-AT atomics on them
        // serialise.  A wave counts at most 64 * g / kBlock <= 8192 per bin.
        uint64_t h0 = 0, h1 = 0, h2 = 0, h3 = 0;
        uint32_t nat = 0;
        for (uint32_t off = threadIdx.x * CA; off < G.g; off += kBlock * CA) {
            uint4 d[R];
#pragma unroll
            for (int j = 0; j < R; j++) d[j] = *reinterpret_cast<const uint4*>(rows[j] + off);
            const uint4 ac = *reinterpret_cast<const uint4*>(act_lut + off);
#pragma unroll
            for (uint32_t b = 0; b < CA; b++) {
                const uint32_t actb = at_in_word<T>(word_of(ac, b / N), b % N);
                uint32_t e = 0, ok = 1;
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const uint32_t at = at_in_word<T>(word_of(d[j], b / N), b % N);
                    const uint32_t dist = actb >= at ? actb - at : actb + G.twok - at;
                    ok &= (at != G.twok) & (dist < G.k);
                    e = dist > e ? dist : e;
                }
                if (ok) {
                    nat += e < kq;
                    if (e < 16) {
                        const uint64_t inc = 1ull << ((e & 3u) * 16u);
                        const uint32_t q = e >> 2;
                        h0 += q == 0 ? inc : 0ull;
                        h1 += q == 1 ? inc : 0ull;
                        h2 += q == 2 ? inc : 0ull;
                        h3 += q == 3 ? inc : 0ull;
                    } else if (e < 64) {
                        atomicAdd(&hist[e], 1u);
                    }
                }
            }
        }
        for (uint32_t o = 32; o > 0; o >>= 1) {
            nat += __shfl_xor(nat, o, 64);
            h0 += __shfl_xor(h0, o, 64);
            h1 += __shfl_xor(h1, o, 64);
            h2 += __shfl_xor(h2, o, 64);
            h3 += __shfl_xor(h3, o, 64);
        }
        if (lane < 16) {
            const uint64_t hw = lane < 4 ? h0 : lane < 8 ? h1 : lane < 12 ? h2 : h3;
            const uint32_t c = (uint32_t)(hw >> ((lane & 3u) * 16u)) & 0xFFFFu;
            if (c) atomicAdd(&hist[lane], c);
        }
        if (lane == 0) nat_w[wv] = nat;
        __syncthreads();
        if (wv == 0) {
            uint32_t nat_all = 0;
#pragma unroll
            for (uint32_t w = 0; w < kBlock / 64; w++) nat_all += nat_w[w];
            const uint32_t hv = hist[lane];
            uint8_t fl = 0;
            double e_plain = 0.0;
            if (lane == 0) e_plain = eq4(nat_all, z, aat, G, &fl);
            e_plain = __shfl(e_plain, 0, 64);
            const uint32_t nd = G.k < 61 ? G.k : 61;
            float fv = lane < nd ? (float)((double)hv / (double)G.g) : 0.0f;
            if (lane == 61) {
                double lp = log(1.0 + (e_plain > 0 ? e_plain : 0.0));
                if (!(lp < 20.0)) lp = 20.0;
                fv = (float)(lp / 16.0);
            } else if (lane == 62) {
                fv = (float)((double)G.k / 64.0);
            } else if (lane == 63) {
                const double cells = (double)((uint64_t)G.g << G.c);
                double s2 = 0.0;
                for (uint32_t j = 0; j < G.r; j++) s2 += (double)aat[(uint64_t)z * G.r + j] / cells;
                fv = (float)(s2 / (double)G.r);
            }
            feat[h * 64 + lane] = fv;
            if (lane == 0) {
                if (est) est[h] = e_plain;
                if (flags) flags[h] = fl;
            }
        }
        __syncthreads();  // hist and nat_w are reused by the next host
    }
}

// ---------------------------------------------------------------- a9: serving
// Batched forms of the kernels above for many links per launch.  Every grid
// is fixed (the step graph is captured once); the work of a replay is read
// from the step descriptor and the device-side counters.  Links of one server
// share the geometry shape (r, c, s, u, g); k, seed and C0 are per link.

__device__ __forceinline__ uint32_t upper_index(const uint64_t* prefix, uint32_t n, uint64_t x) {
    // last i in [0, n) with prefix[i] <= x (prefix non-decreasing, prefix[0] = 0)
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_serve_preserve(const StepDesc* __restrict__ d,
                                                           const LinkSlot* __restrict__ L) {
    const uint32_t no = d->n_open;
    if (no == 0) return;
    const uint64_t total = d->open_prefix[no];
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t o = upper_index(d->open_prefix, no, it);
        const OpenDesc& od = d->open[o];
        const LinkSlot& ls = L[od.slot];
        const PreserveSpans& S = od.S;
        const uint32_t per_atv = S.nw0 + S.nw1;
        const uint64_t rem = it - d->open_prefix[o];
        const uint64_t atv = rem / per_atv;
        const uint32_t ci = (uint32_t)(rem - atv * per_atv);
        const uint32_t chunk = ci < S.nw0 ? S.w0lo + ci : S.w1lo + (ci - S.nw0);
        const uint32_t k = ls.G.k, twok = ls.G.twok;
        uint4* p = reinterpret_cast<uint4*>(ls.pool + (atv << ls.G.log2g)) + chunk;
        const uint4 v = *p;
        uint4 nv;
        nv.x = preserve_word(v.x, chunk * 16, S, k, twok);
        nv.y = preserve_word(v.y, chunk * 16 + 4, S, k, twok);
        nv.z = preserve_word(v.z, chunk * 16 + 8, S, k, twok);
        nv.w = preserve_word(v.w, chunk * 16 + 12, S, k, twok);
        if (nv.x != v.x || nv.y != v.y || nv.z != v.z || nv.w != v.w) *p = nv;
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_serve_ingest(const StepDesc* __restrict__ d, const LinkSlot* __restrict__ L) {
    const uint32_t nc = d->n_chunks;
    if (nc == 0) return;
    const uint64_t units = d->n_units;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t u = wave; u < units; u += nwaves) {
        // chunk c holds units [unit0_c, unit0_c + ceil(n_c / kServeUnit))
        uint32_t lo = 0, hi = nc;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (d->chunk[mid].unit0 <= u) lo = mid;
            else hi = mid;
        }
        const ChunkDesc& cd = d->chunk[lo];
        const LinkSlot& ls = L[cd.slot];
        const uint64_t q0 = (u - cd.unit0) * kServeUnit + lane * 4;
        if (q0 >= cd.n) continue;
        if (cd.vec && q0 + 4 <= cd.n) {
            const uint4 a = *reinterpret_cast<const uint4*>(cd.aip + q0);
            const uint4 b = *reinterpret_cast<const uint4*>(cd.bip + q0);
            scan_pair<R>(ls.pool, a.x, b.x, ls.G, cd.c0);
            scan_pair<R>(ls.pool, a.y, b.y, ls.G, cd.c0);
            scan_pair<R>(ls.pool, a.z, b.z, ls.G, cd.c0);
            scan_pair<R>(ls.pool, a.w, b.w, ls.G, cd.c0);
        } else {
            for (uint64_t q = q0; q < q0 + 4 && q < cd.n; q++) scan_pair<R>(ls.pool, cd.aip[q], cd.bip[q], ls.G, cd.c0);
        }
    }
}

// k'-weights of every ATV of every closing link; block timestamps are
// computed per byte (links differ in k and C0).
__global__ __launch_bounds__(kBlock) void k_serve_close(const StepDesc* __restrict__ d, const LinkSlot* __restrict__ L,
                                                        uint64_t n_atv, uint32_t log2g, uint8_t* __restrict__ act) {
    const uint32_t ncl = d->n_close;
    if (ncl == 0) return;
    {   // the block timestamp of every AT position, per close (read by the feature pass)
        const uint32_t g = 1u << log2g;
        const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x, nthr = (uint64_t)gridDim.x * kBlock;
        for (uint64_t q = tid; q < (uint64_t)ncl * g; q += nthr) {
            const uint32_t ci = (uint32_t)(q >> log2g), i = (uint32_t)(q & (g - 1u));
            act[q] = (uint8_t)act_of(i, d->close[ci].c0, L[d->close[ci].slot].G);
        }
    }
    bool all_ready = true;  // every slice's weights already counted by its tiled scan: nothing to read
    for (uint32_t ci = 0; ci < ncl; ci++) all_ready &= d->close[ci].ready != 0;
    if (all_ready) return;
    const uint32_t g = 1u << log2g;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t lpa = g / 16 < 64 ? g / 16 : 64;
    const uint32_t apw = 64 / lpa;
    const uint32_t sub = lane / lpa, sl = lane % lpa;
    const uint32_t steps = g / (16 * lpa);
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    const uint64_t total = (uint64_t)ncl * n_atv;
    for (uint64_t base = wave * apw; base < total; base += nwaves * apw) {
        const uint64_t gi = base + sub;
        uint32_t cnt = 0;
        const uint32_t ci = (uint32_t)(gi / n_atv);
        if (gi < total && !d->close[ci].ready) {
            const CloseDesc& cdsc = d->close[ci];
            const LinkSlot& ls = L[cdsc.slot];
            const uint64_t atv = gi - (uint64_t)ci * n_atv;
            const uint8_t* p = ls.pool + (atv << log2g);
            for (uint32_t st = 0; st < steps; st++) {
                const uint32_t off = (st * lpa + sl) * 16;
                const uint4 dv = *reinterpret_cast<const uint4*>(p + off);
                uint32_t acts[4];
#pragma unroll
                for (int wd = 0; wd < 4; wd++) {
                    uint32_t a4 = 0;
#pragma unroll
                    for (int b = 0; b < 4; b++) a4 |= act_of(off + 4 * wd + b, cdsc.c0, ls.G) << (8 * b);
                    acts[wd] = a4;
                }
                cnt += __popc(active_mask16(dv, make_uint4(acts[0], acts[1], acts[2], acts[3]), ls.G.twok, cdsc.kq));
            }
        }
        for (uint32_t o = lpa / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (sl == 0 && gi < total && !d->close[ci].ready) L[d->close[ci].slot].w[gi - (uint64_t)ci * n_atv] = cnt;
    }
}

__global__ __launch_bounds__(kBlock) void k_serve_summarize(const StepDesc* __restrict__ d,
                                                            const LinkSlot* __restrict__ L, uint32_t ngroups) {
    __shared__ uint32_t wave_cnt[kBlock / 64];
    __shared__ unsigned long long wave_sum[kBlock / 64];
    const uint32_t ci = blockIdx.x / ngroups, grp = blockIdx.x % ngroups;
    if (ci >= d->n_close) return;
    const LinkSlot& ls = L[d->close[ci].slot];
    const Geometry& G = ls.G;
    const uint64_t base = (uint64_t)grp << G.c;
    const uint32_t ncol = G.ncol_mask + 1;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint64_t sum = 0;
    uint32_t written = 0;
    for (uint32_t x0 = 0; x0 < ncol; x0 += kBlock) {
        const uint32_t x = x0 + threadIdx.x;
        const uint32_t wx = x < ncol ? ls.w[base + x] : 0u;
        const bool sup = x < ncol && wx >= G.T;
        sum += wx;
        const uint64_t ball = __ballot(sup);
        const uint32_t before = __popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wv] = __popcll(ball);
        __syncthreads();
        uint32_t off = written, tot = 0;
        for (uint32_t q = 0; q < kBlock / 64; q++) {
            if (q < wv) off += wave_cnt[q];
            tot += wave_cnt[q];
        }
        if (sup) ls.sa[base + off + before] = x;
        written += tot;
        __syncthreads();
    }
    for (uint32_t o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane == 0) wave_sum[wv] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (uint32_t q = 0; q < kBlock / 64; q++) t += wave_sum[q];
        ls.aat[grp] = t;
        ls.sa_cnt[grp] = written;
    }
}

// One wave per closing link, a lane per frame: restore items per frame (their
// prefix), U (a saturating sum) and the budget rule; then the items prefix
// over links (thread 0).
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) { return UINT64_MAX - a < b ? UINT64_MAX : a + b; }

__global__ void k_serve_restore_prep(const StepDesc* __restrict__ d, const LinkSlot* __restrict__ L,
                                     ServeState* __restrict__ S) {
    const uint32_t ncl = d->n_close;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    for (uint32_t ci = wv; ci < ncl; ci += nwv) {
        const LinkSlot& ls = L[d->close[ci].slot];
        const Geometry& G = ls.G;
        const uint32_t nframe = G.umask + 1;
        uint64_t U = 0, items = 0;
        if (lane == 0) ls.frame_prefix[0] = 0;
        for (uint32_t z0 = 0; z0 < nframe; z0 += 64) {
            const uint32_t z = z0 + lane;
            uint64_t prod = 0, it = 0;
            if (z < nframe) {
                prod = 1;
                bool empty = false;
                for (uint32_t j = 0; j < G.r; j++) {
                    const uint64_t cj = ls.sa_cnt[(uint64_t)z * G.r + j];
                    empty |= cj == 0;
                    prod = (prod == 0 || cj == 0) ? 0 : (prod > UINT64_MAX / cj ? UINT64_MAX : prod * cj);
                }
                it = empty ? 0 : ls.sa_cnt[(uint64_t)z * G.r];
                if (!empty && G.r >= 2) it *= ls.sa_cnt[(uint64_t)z * G.r + 1];
            }
            uint64_t x = it;  // inclusive prefix of the items over the lanes
            for (uint32_t o = 1; o < 64; o <<= 1) {
                const uint64_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (z < nframe) ls.frame_prefix[z + 1] = items + x;
            items += __shfl(x, 63, 64);
            for (uint32_t o = 32; o > 0; o >>= 1) prod = sat_add(prod, __shfl_xor(prod, o, 64));
            U = sat_add(U, prod);
        }
        if (lane == 0) {
            CloseOut& o = S->out[ci];
            o.U = U;
            o.rc = U > ls.tuple_budget ? AT_E_BUDGET : AT_OK;
            o.items = o.rc == AT_OK ? items : 0;
            o.cnt = 0;
            o.m = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        S->item_prefix[0] = 0;
        for (uint32_t ci = 0; ci < ncl; ci++) S->item_prefix[ci + 1] = S->item_prefix[ci] + S->out[ci].items;
    }
}

__global__ __launch_bounds__(kBlock) void k_serve_restore_join(const StepDesc* __restrict__ d,
                                                               const LinkSlot* __restrict__ L,
                                                               ServeState* __restrict__ S, uint32_t cap) {
    const uint32_t ncl = d->n_close;
    if (ncl == 0) return;
    const uint64_t total = S->item_prefix[ncl];
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t ci = upper_index(S->item_prefix, ncl, it);
        const LinkSlot& ls = L[d->close[ci].slot];
        const Geometry& G = ls.G;
        const uint32_t R = G.r;
        const uint64_t li = it - S->item_prefix[ci];
        const uint32_t z = upper_index(ls.frame_prefix, G.umask + 1, li);
        const uint64_t rem = li - ls.frame_prefix[z];
        const uint32_t* cnt = ls.sa_cnt + (uint64_t)z * R;
        const uint64_t rowbase = (uint64_t)z * R << G.c;
        unsigned long long* counter = &S->out[ci].cnt;
        if (R == 1) {
            emit(place(ls.sa[rowbase + rem], G.sh[0], G), z, G, ls.cand, cap, counter);
            continue;
        }
        const uint32_t c1 = cnt[1];
        const uint32_t i0 = (uint32_t)(rem / c1), i1 = (uint32_t)(rem - (uint64_t)i0 * c1);
        uint32_t Lb = place(ls.sa[rowbase + i0], G.sh[0], G);
        uint32_t M = G.win[0];
        const uint32_t P = place(ls.sa[rowbase + (1ull << G.c) + i1], G.sh[1], G);
        if ((P ^ Lb) & M & G.win[1]) continue;
        Lb |= P;
        M |= G.win[1];
        if (R == 2) {
            emit(Lb, z, G, ls.cand, cap, counter);
            continue;
        }
        uint32_t Ls[kMaxRows], Ms[kMaxRows], idx[kMaxRows];
        uint32_t lvl = 2;
        Ls[2] = Lb;
        Ms[2] = M;
        idx[2] = 0;
        for (;;) {
            if (idx[lvl] >= cnt[lvl]) {
                if (lvl == 2) break;
                lvl--;
                idx[lvl]++;
                continue;
            }
            const uint32_t Pq = place(ls.sa[rowbase + ((uint64_t)lvl << G.c) + idx[lvl]], G.sh[lvl], G);
            if ((Pq ^ Ls[lvl]) & Ms[lvl] & G.win[lvl]) {
                idx[lvl]++;
                continue;
            }
            if (lvl == R - 1) {
                emit(Ls[lvl] | Pq, z, G, ls.cand, cap, counter);
                idx[lvl]++;
            } else {
                Ls[lvl + 1] = Ls[lvl] | Pq;
                Ms[lvl + 1] = Ms[lvl] | G.win[lvl];
                lvl++;
                idx[lvl] = 0;
            }
        }
    }
}

// One workgroup per close: the candidate count, the cap rule and the close's
// slice of the host list (every workgroup derives the offsets of the closes
// before it from the restore's counts; workgroup 0 also records them), then
// its candidates sorted in LDS (cap <= kTile) and its watch hosts.
__global__ __launch_bounds__(kBlock) void k_serve_sort(const StepDesc* __restrict__ d, const LinkSlot* __restrict__ L,
                                                       ServeState* __restrict__ S, uint32_t* __restrict__ hosts,
                                                       uint32_t cap) {
    __shared__ uint32_t s[kTile];
    const uint32_t ci = blockIdx.x;
    const uint32_t ncl = d->n_close;
    if (ci >= ncl) return;
    // n_cand of a close: its count m when the restore ran (AT_OK) and m <= cap,
    // else 0.  Workgroup 0 may turn AT_OK into AT_E_OVERFLOW meanwhile, which
    // happens exactly when m > cap: both readings give 0.
    auto n_cand = [&](uint32_t c) -> uint32_t {
        const CloseOut& o = S->out[c];
        return (o.rc == AT_OK && o.cnt <= cap) ? (uint32_t)o.cnt : 0u;
    };
    uint64_t off = 0;
    for (uint32_t c = 0; c < ci; c++) off += n_cand(c) + L[d->close[c].slot].n_watch;
    const uint32_t n = n_cand(ci);
    const LinkSlot& ls = L[d->close[ci].slot];
    __syncthreads();  // every thread has read the counts before workgroup 0 writes them
    if (ci == 0 && threadIdx.x == 0) {
        uint64_t o2 = 0;
        for (uint32_t c = 0; c < ncl; c++) {
            CloseOut& o = S->out[c];
            const uint32_t nc = n_cand(c);
            o.m = o.cnt;
            if (o.rc == AT_OK && o.m > cap) o.rc = AT_E_OVERFLOW;
            o.n_cand = nc;
            o.host_off = (uint32_t)o2;
            o.n_hosts = nc + L[d->close[c].slot].n_watch;
            o2 += o.n_hosts;
        }
        S->n_hosts = o2;
    }
    uint32_t np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (uint32_t q = threadIdx.x; q < np2; q += blockDim.x) s[q] = q < n ? ls.cand[q] : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t k = 2; k <= np2; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t p = threadIdx.x; p < np2 / 2; p += blockDim.x) {
                const uint32_t li = 2 * p - (p & (j - 1));
                cmp_swap_lds(s, li, li + j, (li & k) == 0);
            }
            __syncthreads();
        }
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) hosts[off + q] = s[q];
    for (uint32_t q = threadIdx.x; q < ls.n_watch; q += blockDim.x) hosts[off + n + q] = ls.watch[q];
}

// Features and plain estimates of the host list (one wave per host).
template <int R>
__global__ __launch_bounds__(kBlock) void k_serve_features(const StepDesc* __restrict__ d,
                                                           const LinkSlot* __restrict__ L,
                                                           const ServeState* __restrict__ S,
                                                           const uint32_t* __restrict__ hosts,
                                                           const uint8_t* __restrict__ act_all,
                                                           float* __restrict__ feat,
                                                           double* __restrict__ est, uint8_t* __restrict__ pflags) {
    // per wave kHistCopies histograms of 128 ages (stride kHistStride, odd, so
    // that copies fall in different banks); lane l adds into copy l mod
    // kHistCopies, so lanes of equal age rarely hit one address
    constexpr uint32_t kHistCopies = 8, kHistStride = 129;
    __shared__ uint32_t hist_all[kBlock / 64][kHistCopies * kHistStride];
    uint32_t* hist_w = hist_all[threadIdx.x >> 6];
    uint32_t* hist = hist_w + (threadIdx.x & (kHistCopies - 1u)) * kHistStride;
    const uint32_t ncl = d->n_close;
    if (ncl == 0) return;
    const uint64_t nh = S->n_hosts;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t h = wave; h < nh; h += nwaves) {
        uint32_t ci = 0;
        while (ci + 1 < ncl && S->out[ci + 1].host_off <= h) ci++;
        const CloseDesc& cdsc = d->close[ci];
        const LinkSlot& ls = L[cdsc.slot];
        const Geometry& G = ls.G;
        for (uint32_t q = lane; q < kHistCopies * kHistStride; q += 64) hist_w[q] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t f = mangle(hosts[h], G.A);
        const uint32_t z = f & G.umask;
        const uint64_t Lw = (uint64_t)(f >> G.u);
        const uint64_t LL = Lw | (Lw << G.W);
        const uint8_t* rows[R];
#pragma unroll
        for (int j = 0; j < R; j++)
            rows[j] = ls.pool + (((((uint64_t)z * R + j) << G.c) + column(LL, G.sh[j], G.ncol_mask)) << G.log2g);
        // Two positions per packed 16-bit operation: per row the distance
        // (ACT - AT) mod 2k, with bit 15 set for an inactive AT, and its
        // maximum over the rows; the position counts (at age e) when e < k,
        // i.e. every row is active for the full window.
        const uint8_t* actp = act_all + ((uint64_t)ci << G.log2g);
        const uint32_t twok2 = both_halves(G.twok), c_at = both_halves(0x8000u - G.twok);
        for (uint32_t off = lane * 16; off < G.g; off += 64 * 16) {
            uint4 dv[R];
#pragma unroll
            for (int j = 0; j < R; j++) dv[j] = *reinterpret_cast<const uint4*>(rows[j] + off);
            const uint4 av = *reinterpret_cast<const uint4*>(actp + off);
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                const uint32_t aw = word_of(av, q);
                const uint32_t act_e = aw & 0x00FF00FFu, act_o = (aw >> 8) & 0x00FF00FFu;
                u16x2 e_e = {0, 0}, e_o = {0, 0};
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const uint32_t w = word_of(dv[j], q);
                    const Alg1Halves he = alg1_halves(w & 0x00FF00FFu, act_e, twok2, c_at);
                    const Alg1Halves ho = alg1_halves((w >> 8) & 0x00FF00FFu, act_o, twok2, c_at);
                    e_e = __builtin_elementwise_max(e_e, as_u16x2(he.dist | he.off));
                    e_o = __builtin_elementwise_max(e_o, as_u16x2(ho.dist | ho.off));
                }
                if (e_e.x < G.k) atomicAdd(&hist[e_e.x], 1u);
                if (e_o.x < G.k) atomicAdd(&hist[e_o.x], 1u);
                if (e_e.y < G.k) atomicAdd(&hist[e_e.y], 1u);
                if (e_o.y < G.k) atomicAdd(&hist[e_o.y], 1u);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t hv = 0, hv2 = 0;  // ages lane and lane + 64 over the copies
#pragma unroll
        for (uint32_t cpy = 0; cpy < kHistCopies; cpy++) {
            hv += hist_w[cpy * kHistStride + lane];
            hv2 += hist_w[cpy * kHistStride + lane + 64];
        }
        const uint32_t kq = cdsc.kq;
        uint32_t nat = (lane < kq ? hv : 0u) + (lane + 64 < kq ? hv2 : 0u);
        for (uint32_t o = 32; o > 0; o >>= 1) nat += __shfl_xor(nat, o, 64);
        uint8_t fl = 0;
        double e_plain = 0.0;
        if (lane == 0) e_plain = eq4(nat, z, ls.aat, G, &fl);
        e_plain = __shfl(e_plain, 0, 64);
        const uint32_t nd = G.k < 61 ? G.k : 61;
        float fv = lane < nd ? (float)((double)hv / (double)G.g) : 0.0f;
        if (lane == 61) {
            double lp = log(1.0 + (e_plain > 0 ? e_plain : 0.0));
            if (!(lp < 20.0)) lp = 20.0;
            fv = (float)(lp / 16.0);
        } else if (lane == 62) {
            fv = (float)((double)G.k / 64.0);
        } else if (lane == 63) {
            const double cells = (double)((uint64_t)G.g << G.c);
            double sacc = 0.0;
            for (uint32_t j = 0; j < G.r; j++) sacc += (double)ls.aat[(uint64_t)z * G.r + j] / cells;
            fv = (float)(sacc / (double)G.r);
        }
        feat[h * 64 + lane] = fv;
        if (lane == 0) {
            est[h] = e_plain;
            pflags[h] = fl;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// The step's results to mapped host memory (a step without a network): the
// state block, then per host of the list its address, plain estimate and
// flags.  Only the n_hosts rows in use cross the bus.
__global__ __launch_bounds__(kBlock) void k_serve_export(const StepDesc* __restrict__ d,
                                                         const ServeState* __restrict__ S,
                                                         const uint32_t* __restrict__ hosts,
                                                         const double* __restrict__ est,
                                                         const uint8_t* __restrict__ flags) {
    const ServeExport X = d->xp;
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t nthr = (uint64_t)gridDim.x * kBlock;
    constexpr uint32_t kWords = sizeof(ServeState) / 8;
    static_assert(sizeof(ServeState) % 8 == 0, "the state block copies as 8-byte words");
    const uint64_t* sw = reinterpret_cast<const uint64_t*>(S);
    uint64_t* dw = reinterpret_cast<uint64_t*>(X.state);
    for (uint64_t q = tid; q < kWords; q += nthr) dw[q] = sw[q];
    const uint64_t n = S->n_hosts < X.max_hosts ? S->n_hosts : X.max_hosts;
    for (uint64_t h = tid; h < n; h += nthr) {
        X.hosts[h] = hosts[h];
        X.est[h] = est[h];
        X.flags[h] = flags[h];
    }
}

// Comparator: the aging counters of ACE (Section 2.3) must all be decremented
// at every slice end -- one read and one write of the whole pool -- where the
// asynchronous timestamps only touch two blocks of each ATV (k_preserve).
// blockIdx.y = chunk; the chunk's pairs copied with a grid-stride loop
__global__ __launch_bounds__(kBlock) void k_gather_pairs(GatherList Lst, uint32_t* __restrict__ aip_out,
                                                         uint32_t* __restrict__ bip_out) {
    const uint32_t c = blockIdx.y;
    if (c >= Lst.n) return;
    const uint32_t* __restrict__ a = Lst.aip[c];
    const uint32_t* __restrict__ b = Lst.bip[c];
    const uint64_t n = Lst.cnt[c], off = Lst.off[c];
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (uint64_t)gridDim.x * kBlock) {
        aip_out[off + q] = a[q];
        bip_out[off + q] = b[q];
    }
}

// ---------------------------------------------------------------- f3: comparator
// ACE (Section 2.3) and the asynchronous timestamps side by side, each at its
// own width in packed fields: ceil(log2(k+1)) bits per ACE counter, one more
// per timestamp.  Sub-word fields have no byte of their own, so a pair's
// stores are atomic read-modify-writes of 32-bit words.  ACE sets a field to
// its largest value (all ones) with one OR.  A timestamp takes an AND that
// clears the bits its value lacks and an OR that sets those it has; every
// setter of a field within a slice writes the same value, so any interleaving
// of the two leaves that value, and fields of other positions are untouched.

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (uint64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

// ACE aging: a field that is not zero loses one.  Bit 0 of a field of
// x | x >> 1 | ... | x >> (bits - 1) is set exactly when the field is not
// zero (the shifts stay inside the field for that bit), and subtracting 1 from
// a nonzero field never borrows from the next.  Four words per thread.
__global__ __launch_bounds__(kBlock) void k_cmp_age(uint32_t* __restrict__ w, uint64_t n4, uint32_t bits, uint32_t lsb) {
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < n4; q += (uint64_t)gridDim.x * kBlock) {
        uint4 v = reinterpret_cast<uint4*>(w)[q];
        uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            uint32_t f = x[e];
            for (uint32_t b = 1; b < bits; b++) f |= x[e] >> b;
            x[e] -= f & lsb;
        }
        reinterpret_cast<uint4*>(w)[q] = make_uint4(x[0], x[1], x[2], x[3]);
    }
}

// Alg 3 on a packed pool: the r positions of each pair.
__global__ __launch_bounds__(kBlock) void k_cmp_set(uint32_t* __restrict__ words, const uint32_t* __restrict__ aip,
                                                    const uint32_t* __restrict__ bip, uint64_t n, Geometry G,
                                                    CmpLayout Lw, uint32_t ace, uint32_t c0) {
    const uint32_t fmask = (1u << Lw.bits) - 1u;
    for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += (uint64_t)gridDim.x * kBlock) {
        const uint32_t f = mangle(aip[q], G.A);
        const uint32_t z = f & G.umask;
        const uint64_t L = (uint64_t)(f >> G.u);
        const uint64_t LL = L | (L << G.W);
        const uint32_t i = (uint32_t)((G.alpha * (uint64_t)bip[q] + G.beta) >> (64 - G.log2g));
        const uint32_t wq = __umulhi(i, Lw.fmagic);
        const uint32_t sh = (i - wq * Lw.F) * Lw.bits;
        const uint32_t v = ace ? fmask : act_of(i, c0, G);
        for (uint32_t j = 0; j < G.r; j++) {
            const uint64_t atv = ((uint64_t)(z * G.r + j) << G.c) + column(LL, G.sh[j], G.ncol_mask);
            uint32_t* wp = words + atv * Lw.wv + wq;
            if (!ace) atomicAnd(wp, ~(fmask << sh) | (v << sh));
            atomicOr(wp, v << sh);
        }
    }
}

// Alg 2 on the packed timestamps of the two due blocks (their ACT becomes 0
// or k): one thread per word of the word spans of an ATV, a block holding as
// many ATVs as fit its 256 threads; only fields whose position lies in a due
// block change, and no two threads share a word.
__global__ __launch_bounds__(kBlock) void k_cmp_preserve(uint32_t* __restrict__ words, Geometry G, CmpLayout Lw,
                                                         uint32_t c0, PreserveSpans S, uint32_t s0lo, uint32_t s0n,
                                                         uint32_t s1lo, uint32_t s1n) {
    const uint32_t fmask = (1u << Lw.bits) - 1u;
    const uint32_t per = s0n + s1n;
    const bool wide = per >= kBlock;
    const uint32_t A = wide ? 1u : kBlock / per;  // ATVs per block
    const uint32_t a = wide ? 0u : threadIdx.x / per;
    const uint32_t e0 = wide ? threadIdx.x : threadIdx.x - a * per, estep = wide ? kBlock : per;
    if (a >= A) return;
    for (uint64_t atv = (uint64_t)blockIdx.x * A + a; atv < Lw.n_atv; atv += (uint64_t)gridDim.x * A) {
        for (uint32_t e = e0; e < per; e += estep) {
            const uint32_t wi = e < s0n ? s0lo + e : s1lo + (e - s0n);
            uint32_t* wp = words + atv * Lw.wv + wi;
            const uint32_t x = *wp;
            uint32_t y = x;
            for (uint32_t fl = 0; fl < Lw.F; fl++) {
                const uint32_t pos = wi * Lw.F + fl;
                const bool due = (pos >= S.r0lo && pos < S.r0hi) || (pos >= S.r1lo && pos < S.r1hi);
                const uint32_t sh = fl * Lw.bits;
                const uint32_t at = (x >> sh) & fmask;
                if (!due || at >= G.twok) continue;
                const uint32_t act = act_of(pos, c0, G);
                uint32_t since = act >= at ? act - at : act + G.twok - at;
                if (since == 0) since = G.twok;  // equal to the new ACT: set 2k slices ago
                if (since >= G.k) y = (y & ~(fmask << sh)) | (G.twok << sh);
            }
            if (y != x) *wp = y;
        }
    }
}

// k'-weight of every ATV of a packed pool (one wave per ATV): ACE fields of at
// least cmax - k' + 1, timestamps not inactive and less than k' slices old.
__global__ __launch_bounds__(kBlock) void k_cmp_close(const uint32_t* __restrict__ words, Geometry G, CmpLayout Lw,
                                                      uint32_t ace, uint32_t c0, uint32_t kq,
                                                      uint32_t* __restrict__ w) {
    const uint32_t fmask = (1u << Lw.bits) - 1u;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t atv = wave; atv < Lw.n_atv; atv += nwaves) {
        uint32_t cnt = 0;
        for (uint32_t wi = lane; wi < Lw.wv; wi += 64) {
            const uint32_t x = words[atv * Lw.wv + wi];
            for (uint32_t fl = 0; fl < Lw.F; fl++) {
                const uint32_t pos = wi * Lw.F + fl;
                if (pos >= G.g) break;
                const uint32_t v = (x >> (fl * Lw.bits)) & fmask;
                if (ace) {
                    cnt += v + kq > fmask;  // v >= cmax - k' + 1
                } else {
                    const uint32_t act = act_of(pos, c0, G);
                    const uint32_t d = act >= v ? act - v : act + G.twok - v;
                    cnt += (v != G.twok) & (d < kq);
                }
            }
        }
        for (uint32_t o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (lane == 0) w[atv] = cnt;
    }
}

// ---------------------------------------------------------------- probes
// Scatter roofline probe: the same input stream as the pair scan (8 B per
// item, 16-byte vector loads) and the same number of byte stores per item,
// but at uniformly random positions of a buffer of `bytes` (a power of two)
// -- the memory-side cost of the scan without its hashing and skew.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_scatter_probe(uint8_t* __restrict__ dst, uint64_t mask,
                                                          const uint32_t* __restrict__ a_in,
                                                          const uint32_t* __restrict__ b_in, uint64_t n) {
    const uint64_t n4 = n / 4;
    const uint4* a4 = reinterpret_cast<const uint4*>(a_in);
    const uint4* b4 = reinterpret_cast<const uint4*>(b_in);
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += (uint64_t)gridDim.x * blockDim.x) {
        uint4 a = a4[q], b = b4[q];
        uint32_t av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            uint64_t h = mix64(((uint64_t)av[e] << 32) | bv[e]);
#pragma unroll
            for (int j = 0; j < R; j++) dst[mix64(h + j) & mask] = (uint8_t)j;
        }
    }
}

uint32_t grid_for(uint64_t items, uint32_t cap) {
    uint64_t b = (items + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (uint32_t)(b < cap ? b : cap);
}


// Calls f(std::integral_constant<int, R>{}, T{}) for the handle's row count R
// (1..8) and AT type T (uint8_t, or uint16_t when G.atb == 2).
template <typename T, typename F>
hipError_t with_rows(uint32_t r, F&& f) {
    switch (r) {
        case 1: f(std::integral_constant<int, 1>{}, T{}); break;
        case 2: f(std::integral_constant<int, 2>{}, T{}); break;
        case 3: f(std::integral_constant<int, 3>{}, T{}); break;
        case 4: f(std::integral_constant<int, 4>{}, T{}); break;
        case 5: f(std::integral_constant<int, 5>{}, T{}); break;
        case 6: f(std::integral_constant<int, 6>{}, T{}); break;
        case 7: f(std::integral_constant<int, 7>{}, T{}); break;
        case 8: f(std::integral_constant<int, 8>{}, T{}); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
hipError_t with_rows_at(const Geometry& G, F&& f) {
    if (G.atb == 2) return with_rows<uint16_t>(G.r, f);
    if (G.atb == 1) return with_rows<uint8_t>(G.r, f);
    return hipErrorInvalidValue;
}

template <typename F>
hipError_t with_at(const Geometry& G, F&& f) {
    if (G.atb == 2) f(uint16_t{});
    else if (G.atb == 1) f(uint8_t{});
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

// ============================================================== launchers

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for((n + 15) / 16, 1u << 16)), dim3(kBlock), 0, st, p, n,
                       v * 0x01010101u);
    return hipGetLastError();
}

hipError_t launch_fill_pool(uint8_t* pool, uint64_t n_at, const Geometry& G, hipStream_t st) {
    if (n_at == 0) return hipSuccess;
    const uint64_t bytes = n_at * G.atb;
    const uint32_t v4 = G.atb == 2 ? G.twok * 0x00010001u : G.twok * 0x01010101u;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for((bytes + 15) / 16, 1u << 16)), dim3(kBlock), 0, st, pool, bytes, v4);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

PreserveSpans preserve_spans(const Geometry& G, uint32_t c0) {
    // blocks whose timestamp (c0 + b) mod 2k becomes 0 and k
    const uint32_t twok = G.twok, k = G.k;
    const uint32_t b0 = (twok - c0) % twok, b1 = (3 * k - c0) % twok;
    auto range = [&](uint32_t b, uint32_t& lo, uint32_t& hi) {
        if (G.blk_a == 0) {  // all ATs sit in the last block
            lo = 0;
            hi = (b == G.last_blk) ? G.g : 0;
        } else {
            lo = b * G.blk_a;
            hi = (b == G.last_blk) ? G.g : lo + G.blk_a;
        }
        if (hi <= lo) lo = hi = 0;
    };
    PreserveSpans S{};
    range(b0, S.r0lo, S.r0hi);
    range(b1, S.r1lo, S.r1hi);
    // 16-byte chunk spans (ca ATs each) of the two AT ranges, merged when
    // they share a chunk
    const uint32_t ca = 16 / G.atb;
    uint32_t sp[2][2];
    int ns = 0;
    if (S.r0hi > S.r0lo) { sp[ns][0] = S.r0lo / ca; sp[ns][1] = (S.r0hi + ca - 1) / ca; ns++; }
    if (S.r1hi > S.r1lo) { sp[ns][0] = S.r1lo / ca; sp[ns][1] = (S.r1hi + ca - 1) / ca; ns++; }
    if (ns == 2) {
        if (sp[0][0] > sp[1][0]) {
            uint32_t t0 = sp[0][0], t1 = sp[0][1];
            sp[0][0] = sp[1][0]; sp[0][1] = sp[1][1];
            sp[1][0] = t0; sp[1][1] = t1;
        }
        if (sp[1][0] <= sp[0][1]) {  // overlapping or adjacent chunk spans
            sp[0][1] = sp[1][1] > sp[0][1] ? sp[1][1] : sp[0][1];
            ns = 1;
        }
    }
    if (ns >= 1) { S.w0lo = sp[0][0]; S.nw0 = sp[0][1] - sp[0][0]; }
    if (ns == 2) { S.w1lo = sp[1][0]; S.nw1 = sp[1][1] - sp[1][0]; }
    return S;
}

hipError_t launch_preserve(uint8_t* pool, uint64_t n_atv, const Geometry& G, uint32_t c0, hipStream_t st) {
    const PreserveSpans S = preserve_spans(G, c0);
    const uint64_t items = n_atv * (S.nw0 + S.nw1);
    if (items == 0) return hipSuccess;
    return with_at(G, [&](auto t) {
        using T = decltype(t);
        hipLaunchKernelGGL(k_preserve<T>, dim3(grid_for(items, 1u << 16)), dim3(kBlock), 0, st, pool, n_atv, G.log2g,
                           G.k, S);
    });
}

hipError_t launch_ingest(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n, const Geometry& G,
                         uint32_t c0, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const bool vec = ((reinterpret_cast<uintptr_t>(aip) | reinterpret_cast<uintptr_t>(bip)) & 15u) == 0;
    const uint32_t grid = grid_for(vec ? (n + 3) / 4 : n, 1u << 20);
    return with_rows_at(G, [&](auto rc, auto t) {
        constexpr int R = decltype(rc)::value;
        using T = decltype(t);
        T* p = reinterpret_cast<T*>(pool);
        if (vec)
            hipLaunchKernelGGL((k_ingest<R, true, T>), dim3(grid), dim3(kBlock), 0, st, p, aip, bip, n, G, c0);
        else
            hipLaunchKernelGGL((k_ingest<R, false, T>), dim3(grid), dim3(kBlock), 0, st, p, aip, bip, n, G, c0);
    });
}

uint64_t binned_sub_cap(uint64_t n) { return ((n + kSubs - 1) / kSubs + 2 * kBinTile + 3) & ~3ull; }

hipError_t launch_ingest_binned(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n, const Geometry& G,
                                uint32_t c0, uint64_t* bins, uint64_t sub_cap, unsigned long long* fill,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (binned_sub_cap(n) > sub_cap || n > (uint64_t)8192 * kBinTile) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3((kBins * kSubs + kBlock - 1) / kBlock), dim3(kBlock), 0, st, fill,
                       kBins * kSubs);
    uint64_t blocks = (n + kBinTile - 1) / kBinTile;
    if (blocks > 8192) blocks = 8192;
    blocks = (blocks + kSubs - 1) / kSubs * kSubs;  // every sub-run gets the same number of blocks
    hipLaunchKernelGGL(k_bin_pairs, dim3((uint32_t)blocks), dim3(kBlock), 0, st, aip, bip, n, G, bins, sub_cap, fill);
    uint64_t per_bin = (n / kBins + 4 * kBlock - 1) / (4 * kBlock);
    if (per_bin < 1) per_bin = 1;
    if (per_bin > 512) per_bin = 512;
    return with_at(G, [&](auto t) {
        using T = decltype(t);
        for (uint32_t row = 0; row < G.r; row++)
            hipLaunchKernelGGL(k_scan_bins<T>, dim3((uint32_t)(kBins * per_bin)), dim3(kBlock), 0, st, bins, sub_cap,
                               fill, reinterpret_cast<T*>(pool), G, c0, row);
    });
}

bool tiled_fits(uint64_t pool_bytes) {
    return pool_bytes % kTileBytes == 0 && pool_bytes / kTileBytes >= 1 && pool_bytes / kTileBytes <= kMaxTiles;
}

TileSizes tiled_sizes(uint64_t n, uint64_t pool_bytes, const Geometry& G) {
    TileSizes z{};
    z.n_tiles = (uint32_t)(pool_bytes / kTileBytes);
    z.nb = (uint32_t)((n + kTileRecs / G.r - 1) / (kTileRecs / G.r));
    z.nchunk = (z.nb + kTileChunk - 1) / kTileChunk;
    z.recs = n * G.r;
    z.table = (uint64_t)z.nb * z.n_tiles;
    return z;
}

size_t tiled_lds_bytes(uint32_t n_tiles) {
    return kTileRecs * sizeof(uint32_t) + (((size_t)n_tiles + 3) & ~(size_t)3) * sizeof(uint32_t);
}

namespace {

// The batch's kernel arguments and grid extents (host side).
struct BatchPlan {
    TileBatch Bt;
    uint32_t max_nb, max_tiles, max_chunk;
};

hipError_t plan_batch(const TileJobSpec* js, uint32_t nj, BatchPlan* P) {
    if (nj == 0 || nj > kTileJobsMax) return hipErrorInvalidValue;
    TileBatch& Bt = P->Bt;
    Bt = TileBatch{};
    P->max_nb = P->max_tiles = P->max_chunk = 0;
    for (uint32_t q = 0; q < nj; q++) {
        const TileJobSpec& J = js[q];
        // one instance of each pass serves the batch: rows and AT width agree
        if (J.G.r != js[0].G.r || J.G.atb != js[0].G.atb) return hipErrorInvalidValue;
        if (J.w_out && !J.preserve) return hipErrorInvalidValue;  // the weights need every tile visited
        if (J.n == 0 || !tiled_fits(J.pool_bytes)) return hipErrorInvalidValue;
        const TileSizes z = tiled_sizes(J.n, J.pool_bytes, J.G);
        if (z.recs > J.B.rec_cap || z.table > J.B.table_cap || z.nchunk + 2 > J.B.chunk_cap)
            return hipErrorInvalidValue;
        TileJob& T = Bt.j[q];
        T.pool = J.pool;
        T.aip = J.aip;
        T.bip = J.bip;
        T.rec = J.B.rec;
        T.cnt = J.B.cnt;
        T.pre = J.B.pre;
        T.csum = J.B.csum;
        T.base = J.B.base;
        T.act = J.B.act;
        T.w_out = J.w_out;
        T.n = J.n;
        T.G = J.G;
        T.S = J.preserve ? preserve_spans(J.G, J.c0) : PreserveSpans{};
        T.c0 = J.c0;
        T.preserve = J.preserve ? 1u : 0u;
        T.kq_w = J.kq_w;
        T.n_tiles = z.n_tiles;
        T.nb = z.nb;
        T.nchunk = z.nchunk;
        P->max_nb = std::max(P->max_nb, z.nb);
        P->max_tiles = std::max(P->max_tiles, z.n_tiles);
        P->max_chunk = std::max(P->max_chunk, z.nchunk);
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_ingest_tiled_records(const TileJobSpec* js, uint32_t nj, hipStream_t st) {
    BatchPlan P;
    hipError_t e = plan_batch(js, nj, &P);
    if (e != hipSuccess) return e;
    // Passes 1 and 2 map blocks to XCDs by blockIdx.x alone: with several jobs
    // the row of blocks of each is a whole number of XCD rounds.
    const uint32_t gx = nj == 1 ? P.max_nb : (P.max_nb + 7u) & ~7u;
    const dim3 cols((P.max_tiles + kColTiles - 1) / kColTiles, P.max_chunk, nj);
    const Geometry& G0 = js[0].G;
    e = with_rows<uint8_t>(G0.r, [&](auto rc, auto) {
        constexpr int RR = decltype(rc)::value;
        hipLaunchKernelGGL((k_tile_count<RR>), dim3(gx, nj), dim3(kCountBlock), 0, st, P.Bt);
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_chunksum, cols, dim3(kBlock), 0, st, P.Bt);
    hipLaunchKernelGGL(k_tile_rowpre, cols, dim3(kBlock), 0, st, P.Bt);
    return with_rows<uint8_t>(G0.r, [&](auto rc, auto) {
        constexpr int RR = decltype(rc)::value;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile_scatter<RR>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)tiled_lds_bytes(kMaxTiles));
        hipLaunchKernelGGL((k_tile_scatter<RR>), dim3(gx, nj), dim3(kScatterBlock), tiled_lds_bytes(P.max_tiles),
                           st, P.Bt);
    });
}

hipError_t launch_ingest_tiled_apply(const TileJobSpec* js, uint32_t nj, hipStream_t st) {
    BatchPlan P;
    hipError_t e = plan_batch(js, nj, &P);
    if (e != hipSuccess) return e;
    return with_at(js[0].G, [&](auto t) {
        using T = decltype(t);
        hipLaunchKernelGGL(k_tile_apply<T>, dim3(P.max_tiles, nj), dim3(kApplyBlock), kTileBytes, st, P.Bt);
    });
}

hipError_t launch_ingest_tiled_batch(const TileJobSpec* js, uint32_t nj, hipStream_t st) {
    hipError_t e = launch_ingest_tiled_records(js, nj, st);
    return e == hipSuccess ? launch_ingest_tiled_apply(js, nj, st) : e;
}

hipError_t launch_ingest_tiled(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n,
                               uint64_t pool_bytes, const Geometry& G, uint32_t c0, const TileBufs& B, bool preserve,
                               uint32_t* w_out, uint32_t kq_w, hipStream_t st) {
    if (n == 0) return w_out && !preserve ? hipErrorInvalidValue : hipSuccess;
    const TileJobSpec J{pool, pool_bytes, aip, bip, n, G, c0, preserve, w_out, kq_w, B};
    return launch_ingest_tiled_batch(&J, 1, st);
}

hipError_t launch_close(const uint8_t* pool, uint32_t* w, uint64_t n_atv, const Geometry& G, uint32_t c0,
                        const CloseWindows& Wn, hipStream_t st) {
    const uint32_t ca = 16 / G.atb;  // ATs per 16-byte chunk
    const uint32_t lpa = G.g / ca < 64 ? G.g / ca : 64;
    const uint64_t atv_per_block = (kBlock / 64) * (64 / lpa);
    uint64_t blocks = (n_atv + atv_per_block - 1) / atv_per_block;
    if (blocks > 1024) blocks = 1024;  // every block fills a g-AT timestamp table first: amortise it
    return with_at(G, [&](auto t) {
        using T = decltype(t);
        hipLaunchKernelGGL(k_close<T>, dim3((uint32_t)blocks), dim3(kBlock), G.g * sizeof(T), st,
                           reinterpret_cast<const T*>(pool), w, n_atv, G, c0, Wn);
    });
}

hipError_t launch_close_hist(const uint8_t* pool, uint16_t* hist, uint32_t* w, uint64_t n_atv, const Geometry& G,
                             uint32_t c0, uint32_t kq, hipStream_t st) {
    if (G.k > kHistMaxK) return hipErrorInvalidValue;
    uint64_t blocks = (n_atv + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 2048) blocks = 2048;  // every block fills a g-AT timestamp table first
    const uint32_t lds = ((G.g * G.atb + 15u) & ~15u) + (kBlock / 64) * G.k * 4u;
    return with_at(G, [&](auto t) {
        using T = decltype(t);
        if (lds > 65536u)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_close_hist<T>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_close_hist<T>, dim3((uint32_t)blocks), dim3(kBlock), lds, st,
                           reinterpret_cast<const T*>(pool), hist, w, n_atv, G, c0, kq);
    });
}

hipError_t launch_hist_weights(const uint16_t* hist, uint32_t K, uint64_t n_atv, uint32_t kq, uint32_t* w,
                               hipStream_t st) {
    uint64_t blocks = (n_atv + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_hist_weights, dim3((uint32_t)blocks), dim3(kBlock), 0, st, hist, K, n_atv, kq, w);
    return hipGetLastError();
}

hipError_t launch_summarize(const uint32_t* w, uint64_t* aat, uint32_t* sa, uint32_t* sa_cnt, uint32_t* cnt_host,
                            const Geometry& G, uint64_t n_atv, uint32_t nwin, hipStream_t st) {
    const uint32_t groups = (G.umask + 1) * G.r;
    hipLaunchKernelGGL(k_summarize, dim3(groups, nwin), dim3(kBlock), 0, st, w, aat, sa, sa_cnt, cnt_host, G, n_atv,
                       groups);
    return hipGetLastError();
}

hipError_t launch_restore_join(const uint32_t* sa, const uint32_t* sa_cnt, const uint64_t* pair_prefix,
                               uint64_t n_items, const Geometry& G, uint32_t* cand, uint64_t cap,
                               unsigned long long* counter, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restore_join, dim3(grid_for(n_items, 1u << 16)), dim3(kBlock), 0, st, sa, sa_cnt,
                       pair_prefix, n_items, G, cand, cap, counter);
    return hipGetLastError();
}

hipError_t launch_sort_u32(uint32_t* keys, uint64_t m, uint64_t n_pow2, hipStream_t st) {
    if (m <= 1) return hipSuccess;
    if (n_pow2 > m)
        hipLaunchKernelGGL(k_pad_u32, dim3(grid_for(n_pow2 - m, 4096)), dim3(kBlock), 0, st, keys, m, n_pow2);
    if (n_pow2 <= kTile) {
        hipLaunchKernelGGL(k_small_sort, dim3(1), dim3(kBlock), 0, st, keys, (uint32_t)n_pow2);
        return hipGetLastError();
    }
    const uint32_t tiles = (uint32_t)(n_pow2 / kTile);
    hipLaunchKernelGGL(k_bitonic_tile, dim3(tiles), dim3(kBlock), 0, st, keys, 2u, kTile);
    for (uint64_t k = 2 * (uint64_t)kTile; k <= n_pow2; k <<= 1) {
        for (uint64_t j = k >> 1; j >= kTile; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3(grid_for(n_pow2 / 2, 1u << 16)), dim3(kBlock), 0, st, keys,
                               n_pow2, k, j);
        // remaining strides j < kTile of this k inside each tile
        hipLaunchKernelGGL(k_bitonic_tile, dim3(tiles), dim3(kBlock), 0, st, keys, (uint32_t)k, (uint32_t)k);
    }
    return hipGetLastError();
}

hipError_t launch_estimate(const uint8_t* pool, const uint64_t* aat, const uint32_t* aip, uint64_t n,
                           const Geometry& G, uint32_t c0q, uint32_t kq, double* est, uint8_t* flags, uint32_t* nat,
                           hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    return with_rows_at(G, [&](auto rc, auto t) {
        constexpr int R = decltype(rc)::value;
        using T = decltype(t);
        hipLaunchKernelGGL((k_estimate<R, T>), dim3((uint32_t)blocks), dim3(kBlock), G.g * sizeof(T), st,
                           reinterpret_cast<const T*>(pool), aat, aip, n, G, c0q, kq, est, flags, nat);
    });
}

hipError_t launch_features(const uint8_t* pool, const uint64_t* aat, const uint32_t* aip, uint64_t n,
                           const Geometry& G, uint32_t c0q, uint32_t kq, float* feat, double* est, uint8_t* flags,
                           hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = n;  // one workgroup per host
    if (blocks > 16384) blocks = 16384;
    const size_t shmem = ((G.g * G.atb + 15u) & ~15u) + 64 * sizeof(uint32_t);
    return with_rows_at(G, [&](auto rc, auto t) {
        constexpr int R = decltype(rc)::value;
        using T = decltype(t);
        hipLaunchKernelGGL((k_features<R, T>), dim3((uint32_t)blocks), dim3(kBlock), shmem, st,
                           reinterpret_cast<const T*>(pool), aat, aip, n, G, c0q, kq, feat, est, flags);
    });
}

constexpr uint32_t kServeGrid = 2048;  // persistent grid of the batched kernels
// The feature kernel takes one wave per host up to 32768 hosts a step: its
// waves are short, so the workgroups of kernels beside it (a server's record
// passes) get CUs as they free up, which a grid that keeps every CU for the
// whole kernel would not give them.
constexpr uint32_t kFeatGrid = 4 * kServeGrid;

hipError_t launch_serve_ingest_branch(const ServeBufs& B, const Geometry& shape, hipStream_t st) {
    hipLaunchKernelGGL(k_serve_preserve, dim3(kServeGrid), dim3(kBlock), 0, st, B.desc, B.slots);
#define AT_SERVE_ING(RR)                                                                                   \
    case RR:                                                                                               \
        hipLaunchKernelGGL((k_serve_ingest<RR>), dim3(kServeGrid * 2), dim3(kBlock), 0, st, B.desc, B.slots); \
        break;
    switch (shape.r) {
        AT_SERVE_ING(1)
        AT_SERVE_ING(2)
        AT_SERVE_ING(3)
        AT_SERVE_ING(4)
        AT_SERVE_ING(5)
        AT_SERVE_ING(6)
        AT_SERVE_ING(7)
        AT_SERVE_ING(8)
        default:
            return hipErrorInvalidValue;
    }
#undef AT_SERVE_ING
    return hipGetLastError();
}

hipError_t launch_serve_close_branch(const ServeBufs& B, const Geometry& shape, uint64_t n_atv, hipStream_t st) {
    const uint32_t ngroups = (shape.umask + 1) * shape.r;
    hipLaunchKernelGGL(k_serve_close, dim3(kServeGrid), dim3(kBlock), 0, st, B.desc, B.slots, n_atv, shape.log2g,
                       B.act);
    hipLaunchKernelGGL(k_serve_summarize, dim3(kServeMaxLinks * ngroups), dim3(kBlock), 0, st, B.desc, B.slots,
                       ngroups);
    hipLaunchKernelGGL(k_serve_restore_prep, dim3(1), dim3(1024), 0, st, B.desc, B.slots, B.state);
    hipLaunchKernelGGL(k_serve_restore_join, dim3(kServeGrid), dim3(kBlock), 0, st, B.desc, B.slots, B.state,
                       B.cand_cap);
    hipLaunchKernelGGL(k_serve_sort, dim3(kServeMaxLinks), dim3(kBlock), 0, st, B.desc, B.slots, B.state, B.hosts,
                       B.cand_cap);
#define AT_SERVE_FEAT(RR)                                                                                     \
    case RR:                                                                                                  \
        hipLaunchKernelGGL((k_serve_features<RR>), dim3(kFeatGrid), dim3(kBlock), 0, st, B.desc, B.slots, B.state,  \
                           B.hosts, B.act, B.feat, B.est, B.pflags);                                          \
        break;
    switch (shape.r) {
        AT_SERVE_FEAT(1)
        AT_SERVE_FEAT(2)
        AT_SERVE_FEAT(3)
        AT_SERVE_FEAT(4)
        AT_SERVE_FEAT(5)
        AT_SERVE_FEAT(6)
        AT_SERVE_FEAT(7)
        AT_SERVE_FEAT(8)
        default:
            return hipErrorInvalidValue;
    }
#undef AT_SERVE_FEAT
    return hipGetLastError();
}

hipError_t launch_serve_export(const ServeBufs& B, hipStream_t st) {
    hipLaunchKernelGGL(k_serve_export, dim3(64), dim3(kBlock), 0, st, B.desc, B.state, B.hosts, B.est, B.pflags);
    return hipGetLastError();
}

hipError_t launch_gather_pairs(const GatherList& Lst, uint32_t* aip_out, uint32_t* bip_out, hipStream_t st) {
    if (Lst.n == 0) return hipSuccess;
    if (Lst.n > kGatherMax) return hipErrorInvalidValue;
    uint64_t most = 0;
    for (uint32_t c = 0; c < Lst.n; c++) most = Lst.cnt[c] > most ? Lst.cnt[c] : most;
    const uint32_t gx = grid_for(most, 2048);
    hipLaunchKernelGGL(k_gather_pairs, dim3(gx, Lst.n), dim3(kBlock), 0, st, Lst, aip_out, bip_out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 1u << 16)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_cmp_age(uint32_t* words, uint64_t n, uint32_t bits, uint32_t lsb, hipStream_t st) {
    if (n == 0 || n % 4) return n ? hipErrorInvalidValue : hipSuccess;
    hipLaunchKernelGGL(k_cmp_age, dim3(grid_for(n / 4, 1u << 16)), dim3(kBlock), 0, st, words, n / 4, bits, lsb);
    return hipGetLastError();
}

hipError_t launch_cmp_set(uint32_t* words, const uint32_t* aip, const uint32_t* bip, uint64_t n, const Geometry& G,
                          const CmpLayout& Lw, bool ace, uint32_t c0, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cmp_set, dim3(grid_for(n, 1u << 16)), dim3(kBlock), 0, st, words, aip, bip, n, G, Lw,
                       (uint32_t)ace, c0);
    return hipGetLastError();
}

hipError_t launch_cmp_preserve(uint32_t* words, const Geometry& G, const CmpLayout& Lw, uint32_t c0,
                               const PreserveSpans& S, uint32_t s0lo, uint32_t s0n, uint32_t s1lo, uint32_t s1n,
                               hipStream_t st) {
    const uint32_t per = s0n + s1n;
    if (per == 0) return hipSuccess;
    const uint32_t A = per >= kBlock ? 1u : kBlock / per;
    uint64_t blocks = (Lw.n_atv + A - 1) / A;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_cmp_preserve, dim3((uint32_t)blocks), dim3(kBlock), 0, st, words, G, Lw, c0, S, s0lo, s0n,
                       s1lo, s1n);
    return hipGetLastError();
}

hipError_t launch_cmp_close(const uint32_t* words, const Geometry& G, const CmpLayout& Lw, bool ace, uint32_t c0,
                            uint32_t kq, uint32_t* w, hipStream_t st) {
    uint64_t blocks = (Lw.n_atv + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_cmp_close, dim3((uint32_t)blocks), dim3(kBlock), 0, st, words, G, Lw, (uint32_t)ace, c0, kq,
                       w);
    return hipGetLastError();
}

hipError_t launch_scatter_probe(uint8_t* dst, uint64_t bytes, const uint32_t* a, const uint32_t* b, uint64_t n,
                                uint32_t r, hipStream_t st) {
    if (n < 4) return hipSuccess;
    const uint32_t grid = grid_for(n / 4, 1u << 20);
    switch (r) {
        case 1: hipLaunchKernelGGL(k_scatter_probe<1>, dim3(grid), dim3(kBlock), 0, st, dst, bytes - 1, a, b, n); break;
        case 2: hipLaunchKernelGGL(k_scatter_probe<2>, dim3(grid), dim3(kBlock), 0, st, dst, bytes - 1, a, b, n); break;
        case 4: hipLaunchKernelGGL(k_scatter_probe<4>, dim3(grid), dim3(kBlock), 0, st, dst, bytes - 1, a, b, n); break;
        case 8: hipLaunchKernelGGL(k_scatter_probe<8>, dim3(grid), dim3(kBlock), 0, st, dst, bytes - 1, a, b, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace atp
