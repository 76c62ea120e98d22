/*
 * Exhaustive checks that pin the oracle to the mathematics rather than to
 * itself.  TEST INFRASTRUCTURE ONLY.  These loops run over all 2^32 values
 * and are split over host threads with OpenMP; the oracle itself stays
 * single-threaded.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* f is a bijection of 32-bit words iff unmangle(mangle(a)) == a for every a
 * (a left inverse on a finite set).  Returns the number of failures and the
 * first failing input. */
uint64_t oat_pin_bijection(const oat *o, uint32_t *first_bad)
{
    uint64_t bad = 0;
    uint32_t first = 0;
    int have = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t blk = 0; blk < (1ll << 16); blk++) {
        for (uint32_t lo = 0; lo < (1u << 16); lo++) {
            uint32_t a = ((uint32_t)blk << 16) | lo;
            if (oat_unmangle(o, oat_mangle(o, a)) != a) {
                bad++;
#pragma omp critical
                {
                    if (!have || a < first) {
                        first = a;
                        have = 1;
                    }
                }
            }
        }
    }
    *first_bad = first;
    return bad;
}

/* The restore set by definition: every 32-bit address whose r ATVs are all
 * super.  Enumerated through the mangled value F = f(a), which ranges over all
 * 2^32 words because f is a bijection; each F is split into frame and left
 * bits and its columns are read from a doubled copy of L.  Writes the
 * unmangled addresses (unsorted) to out (if cap allows) and returns the count. */
uint64_t oat_pin_restore_bruteforce(const oat *o, const uint8_t *super_flags, uint32_t r, uint32_t c,
                                    uint32_t s, uint32_t u, uint32_t *out, uint64_t cap)
{
    uint32_t W = 32 - u;
    uint64_t ncol = 1ull << c;
    uint64_t maskW = (W == 32) ? 0xFFFFFFFFull : ((1ull << W) - 1);
    uint64_t count = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t blk = 0; blk < (1ll << 16); blk++) {
        uint32_t local[4096];
        uint32_t nl = 0;
        for (uint32_t lo = 0; lo < (1u << 16); lo++) {
            uint32_t F = ((uint32_t)blk << 16) | lo;
            uint32_t z = u ? (F & ((1u << u) - 1)) : 0;
            uint64_t L = u ? (F >> u) : F;
            uint64_t LL = (L & maskW) | ((L & maskW) << W);
            int ok = 1;
            for (uint32_t j = 0; j < r && ok; j++) {
                uint32_t sh = (s * j) % W;
                uint64_t x = (LL >> sh) & (ncol - 1);
                ok = super_flags[((uint64_t)z * r + j) * ncol + x];
            }
            if (ok) {
                if (nl == 4096) {
                    uint64_t base;
#pragma omp atomic capture
                    { base = count; count += nl; }
                    for (uint32_t q = 0; q < nl; q++)
                        if (base + q < cap) out[base + q] = local[q];
                    nl = 0;
                }
                local[nl++] = oat_unmangle(o, F);
            }
        }
        if (nl) {
            uint64_t base;
#pragma omp atomic capture
            { base = count; count += nl; }
            for (uint32_t q = 0; q < nl; q++)
                if (base + q < cap) out[base + q] = local[q];
        }
    }
    return count;
}
