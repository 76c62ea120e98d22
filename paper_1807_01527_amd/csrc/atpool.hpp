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
    uint32_t pad0;
    uint64_t blk_magic;      // ceil(2^32 / blk_a): i / blk_a == (i*magic) >> 32 for i < 2^16
    uint64_t maskW;          // 2^W - 1
    uint64_t alpha, beta;    // BH multiply-add-shift
    uint32_t sh[kMaxRows];   // column j starts at LBS bit (s*j) mod W
    uint32_t win[kMaxRows];  // LBS bits covered by column j
    double theta;
};

// ---- launchers (kernels.hip); all asynchronous on `st` ---------------------
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, uint32_t n, hipStream_t st);
hipError_t launch_preserve(uint8_t* pool, uint64_t n_atv, const Geometry& G, uint32_t c0,
                           hipStream_t st);
hipError_t launch_ingest(uint8_t* pool, const uint32_t* aip, const uint32_t* bip, uint64_t n,
                         const Geometry& G, uint32_t c0, hipStream_t st);
hipError_t launch_close(const uint8_t* pool, uint32_t* w, uint64_t n_atv, const Geometry& G,
                        uint32_t c0, uint32_t kq, hipStream_t st);
hipError_t launch_summarize(const uint32_t* w, uint64_t* aat, uint32_t* sa, uint32_t* sa_cnt,
                            const Geometry& G, hipStream_t st);
hipError_t launch_restore_join(const uint32_t* sa, const uint32_t* sa_cnt, const uint64_t* pair_prefix,
                               uint64_t n_items, const Geometry& G, uint32_t* cand, uint64_t cap,
                               unsigned long long* counter, hipStream_t st);
hipError_t launch_sort_u32(uint32_t* keys, uint64_t m, uint64_t n_pow2, hipStream_t st);
hipError_t launch_estimate(const uint8_t* pool, const uint64_t* aat, const uint32_t* aip, uint64_t n,
                           const Geometry& G, uint32_t c0q, uint32_t kq, double* est, uint8_t* flags,
                           uint32_t* nat, hipStream_t st);

hipError_t launch_scatter_probe(uint8_t* dst, uint64_t bytes, const uint32_t* a, const uint32_t* b, uint64_t n,
                                uint32_t r, hipStream_t st);

}  // namespace atp
