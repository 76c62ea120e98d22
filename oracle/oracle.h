/*
 * CPU oracle for the asynchronous-timestamp super-point method (ASSE,
 * "Distributed super point cardinality estimation under sliding time window
 * for high speed network").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded C that follows the
 * paper's definitions and algorithms step by step.  Only the tests, the
 * package smoke check and the CPU-baseline leg of the benchmark use it; the
 * product path never links or calls it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Readings of the paper taken where it is silent or garbled (see the design
 * notes for the full register):
 *   - prime p = 2^32 - 5; f(a) = A*a mod p for a < p, identity on [p, 2^32)
 *     (a bijection of 32-bit addresses; Section 4.1 leaves p open).
 *   - A, alpha, beta from SplitMix64(seed): A = 2^31 + (x0 mod (p - 2^31)),
 *     alpha = x1 | 1, beta = x2.
 *   - bit n of LBS(f, 32-u) is bit n of f >> u (LSB first); column x_j takes
 *     bits s*j .. s*j+c-1 of it, cyclically modulo W = 32-u (Section 4.1).
 *   - BH(b) = ((alpha*b + beta) mod 2^64) >> (64 - log2 g).
 *   - blocks of an ATV are contiguous; the first 2k-1 hold a = floor(g/2k)
 *     ATs, the last holds the rest (Section 3).
 *   - slice lifecycle: open(t) sets C0 = t mod 2k and runs preserveAT,
 *     pairs are scanned, close(t) summarises the window ending at t.
 *   - an AT holds 2k+1 values (ceil(log2(2k+1)) bits, Section 3); the oracle
 *     keeps every AT in a 16-bit word, so k <= 32767.
 */
#ifndef ASSE_ORACLE_H
#define ASSE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t k;            /* slices per window, 1..32767                  */
    uint32_t r, c, s, u;   /* rows, log2 columns, column stride, log2 frames */
    uint32_t log2g;        /* ATs per ATV = 2^log2g                        */
    double theta;          /* super point threshold                         */
    uint64_t seed;         /* hash parameter seed                           */
    uint64_t tuple_budget; /* restore guard; 0 -> 2^32                      */
} oat_params;

enum {
    OAT_OK = 0,
    OAT_E_INVAL = -1,
    OAT_E_STATE = -2,
    OAT_E_NOMEM = -3,
    OAT_E_OVERFLOW = -4,
    OAT_E_BUDGET = -6
};
enum { OAT_F_SAT = 1, OAT_F_NEG = 2, OAT_F_SUPER = 8 };

typedef struct oat oat;

int oat_create(const oat_params *p, oat **out);
void oat_destroy(oat *o);

/* Alg 1 (checkAT) and Alg 2 (preserveAT) on a single value. */
int oat_check_at(uint32_t k, uint32_t act, uint32_t at, uint32_t kprime);
uint32_t oat_preserve_at(uint32_t k, uint32_t act, uint32_t at);

/* Hashing primitives (Section 4.1). */
uint32_t oat_mangle(const oat *o, uint32_t a);
uint32_t oat_unmangle(const oat *o, uint32_t y);
void oat_rrh(const oat *o, uint32_t a, uint32_t *z, uint32_t *x /* r entries */);
uint32_t oat_bh(const oat *o, uint32_t b);
/* L (W bits) -> columns, and the literal round-trip tuple check of Alg 4. */
void oat_columns_of_L(const oat *o, uint32_t L, uint32_t *x);
int oat_tuple_to_L(const oat *o, const uint32_t *x, uint32_t *L);
/* The consecutive-row duplicate-position check written in Alg 4. */
int oat_tuple_dupcheck(const oat *o, const uint32_t *x);
uint32_t oat_block_of(const oat *o, uint32_t i);

/* Slice lifecycle: scan pairs, close a slice, query the closed window. */
int oat_ingest(oat *o, const uint32_t *aip, const uint32_t *bip, uint64_t n);
int oat_close(oat *o, uint32_t kprime);
int oat_requery(oat *o, uint32_t kprime);
/* Per-ATV age histograms of the closed window, n_atv x k counts. */
int oat_age_hist(const oat *o, uint32_t *out);
int oat_estimate(const oat *o, const uint32_t *aip, uint64_t n, double *est,
                 uint8_t *flags, uint32_t *nat);
int oat_restore(const oat *o, uint32_t *out, uint64_t cap, uint64_t *n_out);
int oat_tuple_count(const oat *o, uint64_t *U);
int oat_features(const oat *o, const uint32_t *aip, uint64_t n, float *feat /* n x 64 */);

/* ACE, the aging-counter comparator (Section 2.3): ceil(log2(k+1))-bit timeout
 * counters on the same cube and hashes; set to their largest value c when a
 * pair reaches them, decreased by one (down to 0) at every slice after the
 * first, active for window k' when at least c - k' + 1. */
typedef struct oat_ace oat_ace;
int oat_ace_create(const oat_params *p, oat_ace **out);
void oat_ace_destroy(oat_ace *a);
int oat_ace_ingest(oat_ace *a, const uint32_t *aip, const uint32_t *bip, uint64_t n);
int oat_ace_close(oat_ace *a, uint32_t kprime);
uint32_t oat_ace_bits(const oat_ace *a);
const uint16_t *oat_ace_counters(const oat_ace *a);  /* one per AT position */
const uint32_t *oat_ace_weights(const oat_ace *a);   /* per ATV, last close */

/* Introspection. */
uint64_t oat_pool_size(const oat *o);
const uint16_t *oat_pool(const oat *o);          /* AT values, one word each */
uint64_t oat_n_atv(const oat *o);
const uint32_t *oat_weights(const oat *o);     /* per ATV, last close       */
const uint64_t *oat_aat(const oat *o);         /* per (frame, row)          */
const uint8_t *oat_super(const oat *o);        /* per ATV, last close       */
void oat_constants(const oat *o, uint64_t *out /* p, A, Ainv, alpha, beta, T, W, blk_a */);
void oat_clock(const oat *o, uint64_t *out /* t, open, queryable, c0_query, kq */);

#ifdef __cplusplus
}
#endif
#endif
