// Internal declarations of the gfx950 ATVC library: the constants every kernel
// needs (passed by value as a kernel argument) and the launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "at.h"

namespace atp {

constexpr uint64_t kPrime = 4294967291ull;  // 2^32 - 5, the mangling modulus
constexpr int kMaxRows = 8;

// Everything a kernel needs to hash a pair and locate its ATs.  Built once per
// handle on the host (see derive_geometry) and passed by value.
struct Geometry {
    uint32_t k, twok;        // window length and the AT inactive value 2k
    uint32_t r, c, s, u, W;  // rows, log2 columns, stride, log2 frames, 32-u
    uint32_t log2g, g;
    uint32_t ncol_mask;      // 2^c - 1
    uint32_t umask;          // 2^u - 1
    uint32_t T;              // super-ATV threshold
    uint32_t A, Ainv;        // mangling multiplier and its inverse mod p
    uint32_t blk_a;          // ATs in each of the first 2k-1 blocks (may be 0)
    uint32_t last_blk;       // 2k-1
    uint32_t atb;            // bytes per AT: 1 while 2k < 256, else 2
    uint64_t blk_magic;      // ceil(2^32 / blk_a): i / blk_a == (i*magic) >> 32 for i < 2^16
    uint64_t maskW;          // 2^W - 1
    uint64_t alpha, beta;    // BH multiply-add-shift
    uint32_t sh[kMaxRows];   // column j starts at LBS bit (s*j) mod W
    uint32_t win[kMaxRows];  // LBS bits covered by column j
    double theta;
};

Geometry derive_geometry(const at_params& p);  // from a handle's parameters (capi.hip)
int validate_params(const at_params& p);        // AT_OK or AT_E_INVAL, as at_create

// Lazy preserve work of one slice opening: the AT ranges of the two blocks
// whose timestamp becomes 0 and k, and the (one or two, disjoint) spans of
// 16-byte chunks covering them.
struct PreserveSpans {
    uint32_t r0lo, r0hi;  // AT range of the block with timestamp 0
    uint32_t r1lo, r1hi;  // AT range of the block with timestamp k
    uint32_t w0lo, nw0;   // span 0 of 16-byte chunks covering the ranges
    uint32_t w1lo, nw1;   // span 1 (may be empty; disjoint from span 0)
};
PreserveSpans preserve_spans(const Geometry& G, uint32_t c0);

// ---- launchers (kernels.hip); all asynchronous on `st` ---------------------
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t st);
// n_at ATs of a pool (G.atb bytes each) set to the inactive value 2k
hipError_t launch_fill_pool(uint8_t* pool, uint64_t n_at, const Geometry& G, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t st);
hipError_t launch_preserve(uint8_t* pool, uint64_t n_atv, const Geometry& G, uint32_t c0,
                           hipStream_t st);
hipError_t launch_ingest(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n,
                         const Geometry& G, uint32_t c0, hipStream_t st);
// Two-pass scan: pairs hashed once into 8 frame-group bins of 64 sub-runs
// each (8-byte records), then one pass per row with workgroup b on bin b mod 8.
// Scratch: bins of 8 * 64 * binned_sub_cap(n) records, fill of 512 counters.
constexpr uint32_t kScanBins = 8;
constexpr uint32_t kScanSubs = 64;
uint64_t binned_sub_cap(uint64_t n);
hipError_t launch_ingest_binned(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n, const Geometry& G,
                                uint32_t c0, uint64_t* bins, uint64_t sub_cap, unsigned long long* fill,
                                hipStream_t st);
// Tiled scan: the pool in 64 KiB tiles (at most 4096); the pairs' AT stores
// are counted and grouped per tile (16-bit in-tile indices), then one
// workgroup per tile applies them in LDS and writes the tile back.
struct TileSizes {
    uint32_t n_tiles, nb;  // tiles, blocks of the count/scatter passes
    uint32_t nchunk;       // chunks of blocks in the column scans
    uint64_t recs, table;  // records (n * r), nb * n_tiles
};
struct TileBufs {
    uint16_t* rec;   // rec_cap records
    uint16_t* cnt;   // table_cap: per-block tile counts
    uint32_t* pre;   // table_cap: per-(block, tile) run starts
    uint32_t* csum;  // chunk_cap * 4096: per-chunk column sums, then tile and 64-tile totals (nchunk + 2 rows)
    uint32_t* base;  // 4097 region starts
    uint8_t* act;    // g ATs: the slice's block timestamp per position (for the window count)
    uint64_t rec_cap, table_cap, chunk_cap;
};
bool tiled_fits(uint64_t pool_bytes);
TileSizes tiled_sizes(uint64_t n, uint64_t pool_bytes, const Geometry& G);
size_t tiled_lds_bytes(uint32_t n_tiles);  // dynamic LDS of the scatter pass
// preserve: the call opens the slice; Alg 2 on the due blocks runs inside the
// tile pass (every tile is visited) instead of a separate launch_preserve.
// w_out (needs preserve): the tile pass also writes every ATV's kq_w-weight
// after the call's stores, so a close with that window that follows this one
// call needs no pass over the pool.
hipError_t launch_ingest_tiled(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n,
                               uint64_t pool_bytes, const Geometry& G, uint32_t c0, const TileBufs& B, bool preserve,
                               uint32_t* w_out, uint32_t kq_w, hipStream_t st);
// Several tiled scans in one launch of each pass (a grid dimension per job):
// up to kTileJobsMax jobs that share r and the AT width, each one a call of
// launch_ingest_tiled with its own pool, pairs (n > 0) and scratch.
constexpr uint32_t kTileJobsMax = 8;
struct TileJobSpec {
    uint8_t* pool;
    uint64_t pool_bytes;
    const uint32_t* aip;
    const uint32_t* bip;
    uint64_t n;
    Geometry G;
    uint32_t c0;
    bool preserve;
    uint32_t* w_out;
    uint32_t kq_w;
    TileBufs B;
};
hipError_t launch_ingest_tiled_batch(const TileJobSpec* jobs, uint32_t n_jobs, hipStream_t st);
// The batch in its two halves: passes 1-2 with the column passes (they read
// the pairs and write only the scratch; the pools are untouched), then the
// tile pass (reads the scratch, reads and writes the pools).
hipError_t launch_ingest_tiled_records(const TileJobSpec* jobs, uint32_t n_jobs, hipStream_t st);
hipError_t launch_ingest_tiled_apply(const TileJobSpec* jobs, uint32_t n_jobs, hipStream_t st);
// Windows summarised by one close: weights for window j land in
// w[j * n_atv ...], AAT in aat[j * groups ...], super lists likewise.
constexpr uint32_t kMaxWindows = 8;
struct CloseWindows {
    uint32_t n;
    uint32_t kq[kMaxWindows];
};
hipError_t launch_close(const uint8_t* pool, uint32_t* w, uint64_t n_atv, const Geometry& G, uint32_t c0,
                        const CloseWindows& Wn, hipStream_t st);
// Packed comparator pools (f3): `bits`-bit fields, F = 32 / bits per word,
// ATV v's position i in word v * wv + i / F at bit (i % F) * bits.
struct CmpLayout {
    uint32_t bits, F, fmagic;  // fmagic = ceil(2^32 / F): i / F == umulhi(i, fmagic) for i < 2^16
    uint32_t wv;               // words per ATV
    uint64_t n_atv;
};
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
// ACE aging: every nonzero field of n words decreases by one
hipError_t launch_cmp_age(uint32_t* words, uint64_t n, uint32_t bits, uint32_t lsb, hipStream_t st);
// a pair's r positions: ACE (ace = true) sets the field to all ones, the
// packed timestamps set it to the ACT of the position's block
hipError_t launch_cmp_set(uint32_t* words, const uint32_t* aip, const uint32_t* bip, uint64_t n, const Geometry& G,
                          const CmpLayout& Lw, bool ace, uint32_t c0, hipStream_t st);
// lazy preserve (Alg 2) of the packed timestamps on the AT ranges of the two
// due blocks, one thread per word of the (merged) word spans
hipError_t launch_cmp_preserve(uint32_t* words, const Geometry& G, const CmpLayout& Lw, uint32_t c0,
                               const PreserveSpans& S, uint32_t s0lo, uint32_t s0n, uint32_t s1lo, uint32_t s1n,
                               hipStream_t st);
// per-ATV k'-weights of a packed pool
hipError_t launch_cmp_close(const uint32_t* words, const Geometry& G, const CmpLayout& Lw, bool ace, uint32_t c0,
                            uint32_t kq, uint32_t* w, hipStream_t st);
// Age-histogram close: hist[atv * k + a] (a < k) counts the ATVs' ATs of age
// a, w[atv] receives the kq-weight.  k <= kHistMaxK (LDS bins per wave).
constexpr uint32_t kHistMaxK = 1024;
hipError_t launch_close_hist(const uint8_t* pool, uint16_t* hist, uint32_t* w, uint64_t n_atv, const Geometry& G,
                             uint32_t c0, uint32_t kq, hipStream_t st);
// w[atv] = sum of the first kq bins of the ATV's histogram row of K bins
hipError_t launch_hist_weights(const uint16_t* hist, uint32_t K, uint64_t n_atv, uint32_t kq, uint32_t* w,
                               hipStream_t st);
// cnt_host (may be null): device-mapped host memory that also receives the
// super-list counts of every window, so the host reads them without a copy.
hipError_t launch_summarize(const uint32_t* w, uint64_t* aat, uint32_t* sa, uint32_t* sa_cnt, uint32_t* cnt_host,
                            const Geometry& G, uint64_t n_atv, uint32_t nwin, hipStream_t st);
hipError_t launch_restore_join(const uint32_t* sa, const uint32_t* sa_cnt, const uint64_t* pair_prefix,
                               uint64_t n_items, const Geometry& G, uint32_t* cand, uint64_t cap,
                               unsigned long long* counter, hipStream_t st);
hipError_t launch_sort_u32(uint32_t* keys, uint64_t m, uint64_t n_pow2, hipStream_t st);
hipError_t launch_estimate(const uint8_t* pool, const uint64_t* aat, const uint32_t* aip, uint64_t n,
                           const Geometry& G, uint32_t c0q, uint32_t kq, double* est, uint8_t* flags,
                           uint32_t* nat, hipStream_t st);

hipError_t launch_features(const uint8_t* pool, const uint64_t* aat, const uint32_t* aip, uint64_t n,
                           const Geometry& G, uint32_t c0q, uint32_t kq, float* feat, double* est, uint8_t* flags,
                           hipStream_t st);

// ---- learned correction (mlp.hip) ------------------------------------------
constexpr uint32_t kMlpDim = 64;
constexpr uint32_t kOffW1 = 0;
constexpr uint32_t kOffB1 = kMlpDim * kMlpDim;
constexpr uint32_t kOffW2 = kOffB1 + kMlpDim;
constexpr uint32_t kOffB2 = kOffW2 + kMlpDim * kMlpDim;
constexpr uint32_t kOffW3 = kOffB2 + kMlpDim;
constexpr uint32_t kOffB3 = kOffW3 + kMlpDim;
constexpr uint32_t kMlpParams = kOffB3 + 1;  // 8385
constexpr uint32_t kMlpChunk = 512;          // rows per weight-gradient partial

struct MlpDev {  // operands of the device network
    const uint16_t* W1b;
    const float* b1;
    const uint16_t* W2b;
    const float* b2;
    const uint16_t* w3b;
    const float* b3;
    const uint16_t* W2Tb;
};

struct MlpOut {  // bf16 operand copies refreshed from the FP32 master weights
    uint16_t* W1b;
    uint16_t* W2b;
    uint16_t* W2Tb;
    uint16_t* w3b;
};

struct MlpScratch {  // training activations, feature-major [64][nrows]
    uint16_t *XT, *H1T, *H2T, *dH1T, *dH2T;
    float *y, *dy, *partial, *grad;
};

struct AdamConst {
    float lr, b1, b2, one_minus_b1, one_minus_b2, c1, c2, eps;
};

hipError_t launch_mlp_forward(const float* X, uint64_t n, const MlpDev& P, float* y, hipStream_t st);

// The learned estimate's fallback rule applied to each network output as it
// is produced: z = y + 16 f[61]; estimate exp(z) inside [zlo, zhi], else the
// plain estimate with AT_F_FALLBACK; AT_F_SUPER when the estimate reaches
// theta; AT_F_SAT and AT_F_NEG kept from the plain flags.
struct LearnedEpilogue {
    const double* plain;
    const uint8_t* pflags;
    double zlo, zhi, theta;
    double* est;
    uint8_t* flags;
    double* plain_out;  // may be null: a copy of the plain estimates next to est
};
// Forward pass of the n feature rows X straight into L's estimates and flags.
hipError_t launch_mlp_forward_learned(const float* X, uint64_t n, const MlpDev& P, const LearnedEpilogue& L,
                                      hipStream_t st);
hipError_t launch_mlp_train_fwd_bwd(const float* X, const float* t, uint64_t n, uint64_t nrows, const MlpDev& P,
                                    const MlpScratch& S, hipStream_t st);
hipError_t launch_mlp_loss(const float* y, const float* t, uint64_t n, float* out, hipStream_t st);
// Xb[i] = X[idx[i]] (64 features), Tb[i] = lnn[idx[i]] - 16 * X[idx[i]][61]
hipError_t launch_mlp_gather(const float* X, const float* lnn, const int64_t* idx, uint64_t n, float* Xb, float* Tb,
                             hipStream_t st);
hipError_t launch_mlp_adam(float* w, float* m, float* v, const float* grad, const AdamConst& C, const MlpOut& O,
                           hipStream_t st);
hipError_t launch_mlp_refresh(const float* w, const MlpOut& O, hipStream_t st);

hipError_t launch_scatter_probe(uint8_t* dst, uint64_t bytes, const uint32_t* a, const uint32_t* b, uint64_t n,
                                uint32_t r, hipStream_t st);

// ---- serving: many links in one launch (kernels.hip, driven by serve.hip) --
constexpr uint32_t kServeMaxLinks = 64;
constexpr uint32_t kServeMaxChunks = 2048;
constexpr uint32_t kServeUnit = 256;  // pairs per wave work unit (4 per lane)

struct LinkSlot {  // device-resident description of one admitted link
    Geometry G;
    uint8_t* pool;
    uint32_t* w;
    uint64_t* aat;
    uint32_t* sa;
    uint32_t* sa_cnt;
    uint32_t* cand;           // restore candidates (capacity cand_cap)
    uint64_t* frame_prefix;   // 2^u + 1 restore items per frame, prefix
    const uint32_t* watch;    // hosts always estimated at close
    uint32_t n_watch;
    uint32_t pad;
    uint64_t tuple_budget;
};

struct OpenDesc {
    uint32_t slot, c0;
    PreserveSpans S;
};
struct ChunkDesc {
    const uint32_t* aip;
    const uint32_t* bip;
    uint64_t n;
    uint64_t unit0;  // first work unit of the chunk in the step's unit space
    uint32_t slot, c0, vec, pad;
};
struct CloseDesc {
    uint32_t slot, c0, kq;
    uint32_t ready;  // the slice's weights for window kq were written by its tiled scan: no pool pass
};

struct ServeState;
struct ServeExport {  // device addresses of the mapped host copies of a step's results
    ServeState* state;
    uint32_t* hosts;
    double* est;
    double* est_l;
    uint8_t* flags;
    uint64_t max_hosts;
};

struct StepDesc {  // one serving step, copied to the device before each replay
    uint32_t n_open, n_chunks, n_close, pad;
    uint64_t n_units;
    ServeExport xp;  // where the step's results go
    uint64_t open_prefix[kServeMaxLinks + 1];
    OpenDesc open[kServeMaxLinks];
    CloseDesc close[kServeMaxLinks];
    ChunkDesc chunk[kServeMaxChunks];
};

struct CloseOut {  // per close of a step
    uint64_t U;          // column tuples (Alg 4 enumeration size)
    uint64_t m;          // candidates found
    uint64_t items;      // restore join work items
    unsigned long long cnt;
    int32_t rc;          // AT_OK, AT_E_BUDGET or AT_E_OVERFLOW
    uint32_t n_cand;     // sorted candidates written to the host list
    uint32_t host_off;   // first entry in the step's host list
    uint32_t n_hosts;    // candidates + watch hosts
};

struct ServeState {
    CloseOut out[kServeMaxLinks];
    uint64_t item_prefix[kServeMaxLinks + 1];
    uint64_t n_hosts;
    uint64_t pad;
};

struct ServeBufs {  // device buffers of one server's step graph
    const StepDesc* desc;
    const LinkSlot* slots;
    ServeState* state;
    uint32_t* hosts;   // host list: per close, sorted candidates then watch hosts
    float* feat;       // hosts x 64
    double* est;       // plain estimates
    uint8_t* pflags;   // plain flags
    float* y;          // network output
    uint8_t* act;      // kServeMaxLinks x g: block timestamp of every AT position, per close
    uint64_t max_hosts;
    uint32_t cand_cap;
    uint32_t pad;
};

// Copy up to kGatherMax chunks of pairs into one contiguous pair of arrays
// (the chunks of one link that a serving step scans with the tiled scan).
constexpr uint32_t kGatherMax = 16;
struct GatherList {
    uint32_t n;
    const uint32_t* aip[kGatherMax];
    const uint32_t* bip[kGatherMax];
    uint64_t cnt[kGatherMax];
    uint64_t off[kGatherMax];  // destination offset of each chunk
};
hipError_t launch_gather_pairs(const GatherList& Lst, uint32_t* aip_out, uint32_t* bip_out, hipStream_t st);

hipError_t launch_serve_ingest_branch(const ServeBufs& B, const Geometry& shape, hipStream_t st);
hipError_t launch_serve_close_branch(const ServeBufs& B, const Geometry& shape, uint64_t n_atv, hipStream_t st);
// State block and the used host rows, with the plain estimates and flags, to
// the descriptor's export set (a step without a network).
hipError_t launch_serve_export(const ServeBufs& B, hipStream_t st);
// The same after the network's forward pass, the learned estimates computed on
// the way (its fallback rule for z outside [zlo, zhi]).
hipError_t launch_serve_export_learned(const ServeBufs& B, double zlo, double zhi, double theta, hipStream_t st);
hipError_t launch_mlp_forward_devn(const float* X, const uint64_t* n_dev, uint64_t nrows_max, const MlpDev& P, float* y,
                                   hipStream_t st);
}  // namespace atp
