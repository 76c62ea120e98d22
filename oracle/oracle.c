/*
 * CPU oracle for the asynchronous-timestamp super-point method.
 * TEST INFRASTRUCTURE ONLY -- see oracle.h for scope and readings.
 *
 * Everything here is deliberately literal: preserveAT is applied to every AT
 * of the pool at each slice opening (the eager form of Alg 2), checkAT is
 * evaluated per AT (Alg 1), columns are extracted bit by bit, and the restore
 * enumerates every column tuple (Alg 4).  Built with -O2 -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct oat {
    oat_params p;
    uint64_t prime, A, Ainv, alpha, beta;
    uint32_t W, g, ncol, nframe;
    uint32_t blk_a;   /* ATs in each of the first 2k-1 blocks */
    uint32_t T;       /* super-ATV threshold (integer)        */
    uint64_t n_atv, pool_size;
    uint16_t *at;     /* one 16-bit word per AT: values 0..2k, 2k <= 65534 */
    uint64_t t;       /* index of the current (or next) slice */
    int open;         /* slice t has been opened              */
    int queryable;    /* a closed window is held in the pool  */
    uint32_t c0;      /* C0 of the open slice                 */
    uint32_t c0_query, kq;
    uint32_t *w;
    uint64_t *aat;
    uint8_t *super;
};

/* ---- SplitMix64 (Steele, Lea, Flood 2014), used to derive hash parameters. */
static uint64_t splitmix_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)a * b) % m);
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = mulmod(r, b, m);
        b = mulmod(b, b, m);
        e >>= 1;
    }
    return r;
}

/* ---- Section 3: age of an AT.  An AT that is not inactive holds the ACT
 * of the slice that last set it, and the ACT advances by one per slice modulo
 * 2k, so the number of slices since then (modulo 2k) is the ACT difference. */
static uint32_t at_age(uint32_t k, uint32_t act, uint32_t at)
{
    uint32_t m = 2 * k;
    return act >= at ? act - at : act + m - at;
}

/* ---- checkAT (Alg 1, Section 3): active in the latest k' slices means not
 * inactive (value 2k) and set fewer than k' slices ago. */
int oat_check_at(uint32_t k, uint32_t act, uint32_t at, uint32_t kprime)
{
    if (at >= 2 * k) return 0;
    return at_age(k, act, at) < kprime;
}

/* ---- preserveAT (Alg 2, Section 3), applied at the start of a slice to an AT
 * whose block has just reached ACT `act`.  Only the blocks whose ACT becomes 0
 * or k are examined, so each AT is examined once every k slices.  At that
 * moment the AT must not survive if it was set k or more slices ago: a
 * value equal to the new ACT was written 2k slices back (the clock wrapped),
 * and any other value lies (act - value) mod 2k slices back.  Such an AT
 * becomes inactive; every younger one is left alone. */
uint32_t oat_preserve_at(uint32_t k, uint32_t act, uint32_t at)
{
    uint32_t inactive = 2 * k;
    if (at >= inactive) return at;
    if (act != 0 && act != k) return at;
    uint32_t since = at_age(k, act, at);
    if (since == 0) since = 2 * k;
    return since >= k ? inactive : at;
}

/* ---- Section 4.1: IP mangling f(a) = A*a mod p and its inverse. */
#define ORACLE_PRIME 4294967291ull /* 2^32 - 5 */

/* A, A^-1 < 2^32 and a < 2^32, so the product fits in 64 bits. */
uint32_t oat_mangle(const oat *o, uint32_t a)
{
    if ((uint64_t)a >= ORACLE_PRIME) return a;
    return (uint32_t)((o->A * (uint64_t)a) % ORACLE_PRIME);
}

uint32_t oat_unmangle(const oat *o, uint32_t y)
{
    if ((uint64_t)y >= ORACLE_PRIME) return y;
    return (uint32_t)((o->Ainv * (uint64_t)y) % ORACLE_PRIME);
}

/* bit n (LSB first) of the left W bits of f, i.e. of f >> u */
static uint32_t lbs_bit(uint32_t L, uint32_t n) { return (L >> n) & 1u; }

/* column x_j: c successive bits of LBS starting at s*j, wrapping modulo W */
void oat_columns_of_L(const oat *o, uint32_t L, uint32_t *x)
{
    for (uint32_t j = 0; j < o->p.r; j++) {
        uint32_t v = 0;
        for (uint32_t n = 0; n < o->p.c; n++) {
            uint32_t pos = (o->p.s * j + n) % o->W;
            v |= lbs_bit(L, pos) << n;
        }
        x[j] = v;
    }
}

void oat_rrh(const oat *o, uint32_t a, uint32_t *z, uint32_t *x)
{
    uint32_t f = oat_mangle(o, a);
    uint32_t frame = (o->p.u == 0) ? 0 : (f & ((1u << o->p.u) - 1u));
    uint32_t L = (o->p.u == 0) ? f : (f >> o->p.u);
    *z = frame;
    oat_columns_of_L(o, L, x);
}

/* BH: multiply-add-shift hash of bip into [0, g). */
uint32_t oat_bh(const oat *o, uint32_t b)
{
    uint64_t h = o->alpha * (uint64_t)b + o->beta;
    return (uint32_t)(h >> (64 - o->p.log2g));
}

/* Section 3: block of AT position i; the last block absorbs the remainder. */
uint32_t oat_block_of(const oat *o, uint32_t i)
{
    uint32_t last = 2 * o->p.k - 1;
    if (o->blk_a == 0) return last;
    uint32_t b = i / o->blk_a;
    return b < last ? b : last;
}

static uint32_t act_of(const oat *o, uint32_t c0, uint32_t i)
{
    return (c0 + oat_block_of(o, i)) % (2 * o->p.k);
}

static uint64_t atv_index(const oat *o, uint32_t z, uint32_t row, uint32_t x)
{
    return ((uint64_t)z * o->p.r + row) * o->ncol + x;
}

/* Concatenate the column bits of a tuple into L, then accept the tuple only if
 * extracting the columns of that L gives the tuple back (Alg 4's test that the
 * duplicate positions agree, in its plainest form). */
int oat_tuple_to_L(const oat *o, const uint32_t *x, uint32_t *L)
{
    uint32_t v = 0;
    for (uint32_t j = 0; j < o->p.r; j++)
        for (uint32_t n = 0; n < o->p.c; n++) {
            uint32_t pos = (o->p.s * j + n) % o->W;
            uint32_t bit = (x[j] >> n) & 1u;
            v = (v & ~(1u << pos)) | (bit << pos);
        }
    uint32_t back[64];
    oat_columns_of_L(o, v, back);
    for (uint32_t j = 0; j < o->p.r; j++)
        if (back[j] != x[j]) return 0;
    *L = v;
    return 1;
}

/* Alg 4's check as printed: bits of x_i at duplicate positions must equal
 * those of x_{(i+1) mod r} at the same positions of LBS. */
int oat_tuple_dupcheck(const oat *o, const uint32_t *x)
{
    uint32_t r = o->p.r, W = o->W;
    for (uint32_t i = 0; i < r; i++) {
        uint32_t i2 = (i + 1) % r;
        for (uint32_t n = 0; n < o->p.c; n++) {
            uint32_t pos = (o->p.s * i + n) % W;
            uint32_t n2 = (pos + W - (o->p.s * i2) % W) % W;
            if (n2 < o->p.c) {
                if (((x[i] >> n) & 1u) != ((x[i2] >> n2) & 1u)) return 0;
            }
        }
    }
    return 1;
}

int oat_create(const oat_params *p, oat **out)
{
    if (!p || !out) return OAT_E_INVAL;
    *out = NULL;
    uint32_t W = 32 - p->u;
    if (p->u >= 32 || p->k < 1 || p->k > 32767 || p->r < 1 || p->r > 64) return OAT_E_INVAL;
    if (p->s < 1 || p->s > p->c || p->c > W || p->c > 24) return OAT_E_INVAL;
    if (p->c + p->s * (p->r - 1) < W) return OAT_E_INVAL;       /* completeness */
    if (p->c * p->r <= W) return OAT_E_INVAL;                   /* redundancy   */
    if (p->s * (p->r - 1) >= W) return OAT_E_INVAL;
    if (p->log2g < 1 || p->log2g > 16 || !(p->theta > 0)) return OAT_E_INVAL;
    if ((uint64_t)p->c + p->u + p->log2g + 7 > 40) return OAT_E_INVAL; /* pool cap 2^40-ish */

    oat *o = (oat *)calloc(1, sizeof(oat));
    if (!o) return OAT_E_NOMEM;
    o->p = *p;
    if (o->p.tuple_budget == 0) o->p.tuple_budget = 1ull << 32;
    o->prime = ORACLE_PRIME;
    uint64_t st = p->seed;
    uint64_t x0 = splitmix_next(&st);
    uint64_t x1 = splitmix_next(&st);
    uint64_t x2 = splitmix_next(&st);
    o->A = (1ull << 31) + x0 % (o->prime - (1ull << 31));
    o->Ainv = powmod(o->A, o->prime - 2, o->prime);
    o->alpha = x1 | 1ull;
    o->beta = x2;
    o->W = W;
    o->g = 1u << p->log2g;
    o->ncol = 1u << p->c;
    o->nframe = 1u << p->u;
    o->blk_a = o->g / (2 * p->k);
    /* Section 4.2: a super ATV holds at least g - g*exp(-theta/g) active ATs */
    double thr = (double)o->g - (double)o->g * exp(-p->theta / (double)o->g);
    double Tc = ceil(thr);
    if (Tc < 0) Tc = 0;
    o->T = (uint32_t)Tc;
    o->n_atv = (uint64_t)o->nframe * p->r * o->ncol;
    o->pool_size = o->n_atv * o->g;
    o->at = (uint16_t *)malloc(o->pool_size * sizeof(uint16_t));
    o->w = (uint32_t *)calloc(o->n_atv, sizeof(uint32_t));
    o->aat = (uint64_t *)calloc((size_t)o->nframe * p->r, sizeof(uint64_t));
    o->super = (uint8_t *)calloc(o->n_atv, 1);
    if (!o->at || !o->w || !o->aat || !o->super) {
        oat_destroy(o);
        return OAT_E_NOMEM;
    }
    /* InitAT: every AT starts inactive (value 2k) */
    for (uint64_t q = 0; q < o->pool_size; q++) o->at[q] = (uint16_t)(2 * p->k);
    o->t = 0;
    o->open = 0;
    o->queryable = 0;
    *out = o;
    return OAT_OK;
}

void oat_destroy(oat *o)
{
    if (!o) return;
    free(o->at);
    free(o->w);
    free(o->aat);
    free(o->super);
    free(o);
}

/* Opening slice t: the ACT of every block advances (C0 = t mod 2k) and
 * preserveAT (Alg 2) runs on every AT of the pool. */
/* ACT of every AT position for the slice whose first block has ACT c0: the
 * same for every ATV (the blocks are positions within an ATV). */
static uint32_t *act_table(const oat *o, uint32_t c0)
{
    uint32_t *act = (uint32_t *)malloc((size_t)o->g * sizeof(uint32_t));
    if (act)
        for (uint32_t i = 0; i < o->g; i++) act[i] = act_of(o, c0, i);
    return act;
}

static void open_slice(oat *o)
{
    uint32_t k = o->p.k;
    o->c0 = (uint32_t)(o->t % (2 * k));
    uint32_t *act = act_table(o, o->c0);
    for (uint64_t v = 0; v < o->n_atv; v++) {
        uint16_t *atv = o->at + v * o->g;
        for (uint32_t i = 0; i < o->g; i++)
            atv[i] = (uint16_t)oat_preserve_at(k, act ? act[i] : act_of(o, o->c0, i), atv[i]);
    }
    free(act);
    o->open = 1;
    o->queryable = 0;
}

/* Alg 3: every pair sets, in each of the r ATVs selected by RRH(aip), the AT
 * chosen by BH(bip) to that AT's ACT. */
int oat_ingest(oat *o, const uint32_t *aip, const uint32_t *bip, uint64_t n)
{
    if (!o) return OAT_E_INVAL;
    if (!o->open) open_slice(o);
    uint32_t x[64], z;
    for (uint64_t q = 0; q < n; q++) {
        oat_rrh(o, aip[q], &z, x);
        uint32_t i = oat_bh(o, bip[q]);
        uint32_t act = act_of(o, o->c0, i);
        for (uint32_t j = 0; j < o->p.r; j++) {
            uint64_t v = atv_index(o, z, j, x[j]);
            o->at[v * o->g + i] = (uint16_t)act;
        }
    }
    return OAT_OK;
}

/* End of slice t: k'-weights of every ATV (Alg 1 per AT), AAT per (row,
 * frame) and the super-ATV flags (Section 4.2, 4.3). */
int oat_close(oat *o, uint32_t kprime)
{
    if (!o) return OAT_E_INVAL;
    if (kprime < 1 || kprime > o->p.k) return OAT_E_INVAL;
    if (!o->open) open_slice(o);
    memset(o->aat, 0, sizeof(uint64_t) * (size_t)o->nframe * o->p.r);
    uint32_t *act = act_table(o, o->c0);
    for (uint32_t z = 0; z < o->nframe; z++)
        for (uint32_t j = 0; j < o->p.r; j++)
            for (uint32_t x = 0; x < o->ncol; x++) {
                uint64_t v = atv_index(o, z, j, x);
                const uint16_t *atv = o->at + v * o->g;
                uint32_t w = 0;
                for (uint32_t i = 0; i < o->g; i++)
                    w += (uint32_t)oat_check_at(o->p.k, act ? act[i] : act_of(o, o->c0, i), atv[i], kprime);
                o->w[v] = w;
                o->aat[(uint64_t)z * o->p.r + j] += w;
                o->super[v] = (w >= o->T);
            }
    free(act);
    o->c0_query = o->c0;
    o->kq = kprime;
    o->t += 1;
    o->open = 0;
    o->queryable = 1;
    return OAT_OK;
}

/* Summaries of the window ending at the last closed slice for another k'
 * (1 <= k' <= k): same timestamps, same ACT, Alg 1 with the new k'.  The
 * clock does not move; later queries use this k'. */
int oat_requery(oat *o, uint32_t kprime)
{
    if (!o) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    if (kprime < 1 || kprime > o->p.k) return OAT_E_INVAL;
    memset(o->aat, 0, sizeof(uint64_t) * (size_t)o->nframe * o->p.r);
    for (uint32_t z = 0; z < o->nframe; z++)
        for (uint32_t j = 0; j < o->p.r; j++)
            for (uint32_t x = 0; x < o->ncol; x++) {
                uint64_t v = atv_index(o, z, j, x);
                const uint16_t *atv = o->at + v * o->g;
                uint32_t w = 0;
                for (uint32_t i = 0; i < o->g; i++)
                    w += (uint32_t)oat_check_at(o->p.k, act_of(o, o->c0_query, i), atv[i], kprime);
                o->w[v] = w;
                o->aat[(uint64_t)z * o->p.r + j] += w;
                o->super[v] = (w >= o->T);
            }
    o->kq = kprime;
    return OAT_OK;
}

/* Alg 5: NAT(aip) = number of positions i active in all r ATVs of aip. */
/* Age histogram of every ATV of the window ending at the last closed slice
 * (Section 3): out[v*k + a] = number of ATs of ATV v, in ATV index order,
 * that are not inactive and whose age -- the ACT distance since the slice
 * that set them -- is a, for a < k.  Such an AT is active for window k'
 * exactly when a < k', so every k'-weight is a prefix sum. */
int oat_age_hist(const oat *o, uint32_t *out)
{
    if (!o || !out) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    uint32_t k = o->p.k;
    memset(out, 0, sizeof(uint32_t) * (size_t)o->n_atv * k);
    for (uint64_t v = 0; v < o->n_atv; v++) {
        const uint16_t *atv = o->at + v * o->g;
        for (uint32_t i = 0; i < o->g; i++) {
            if (atv[i] >= 2 * k) continue;
            uint32_t a = at_age(k, act_of(o, o->c0_query, i), atv[i]);
            if (a < k) out[v * k + a] += 1;
        }
    }
    return OAT_OK;
}

static uint32_t nat_of(const oat *o, uint32_t z, const uint32_t *x)
{
    uint32_t nat = 0;
    for (uint32_t i = 0; i < o->g; i++) {
        int all = 1;
        for (uint32_t j = 0; j < o->p.r; j++) {
            uint64_t v = atv_index(o, z, j, x[j]);
            uint16_t at = o->at[v * o->g + i];
            if (!oat_check_at(o->p.k, act_of(o, o->c0_query, i), at, o->kq)) {
                all = 0;
                break;
            }
        }
        if (all) nat++;
    }
    return nat;
}

/* Eq 3/4: remove the expected false-active ATs (probability UP per AT that all
 * r rows are active by other hosts), then invert the linear estimator. */
static double estimate_one(const oat *o, uint32_t z, uint32_t nat, uint8_t *flags)
{
    uint8_t fl = 0;
    double gd = (double)o->g;
    double denom_cells = (double)((uint64_t)o->g * o->ncol);
    double UP = 1.0;
    for (uint32_t j = 0; j < o->p.r; j++) {
        double Pj = (double)o->aat[(uint64_t)z * o->p.r + j] / denom_cells;
        UP = (j == 0) ? Pj : UP * Pj;
    }
    double one_minus = 1.0 - UP;
    double est;
    if (one_minus == 0.0) {
        est = INFINITY;
        fl |= OAT_F_SAT;
    } else {
        uint32_t natc = nat;
        if (nat >= o->g) {
            natc = o->g - 1;
            fl |= OAT_F_SAT;
        }
        double q = (double)(o->g - natc) / (gd * one_minus);
        est = -gd * log(q);
        if (est < 0) fl |= OAT_F_NEG;
    }
    if (est >= o->p.theta) fl |= OAT_F_SUPER;
    *flags = fl;
    return est;
}

int oat_estimate(const oat *o, const uint32_t *aip, uint64_t n, double *est,
                 uint8_t *flags, uint32_t *nat)
{
    if (!o) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    uint32_t x[64], z;
    for (uint64_t q = 0; q < n; q++) {
        oat_rrh(o, aip[q], &z, x);
        uint32_t nt = nat_of(o, z, x);
        uint8_t fl;
        double e = estimate_one(o, z, nt, &fl);
        if (est) est[q] = e;
        if (flags) flags[q] = fl;
        if (nat) nat[q] = nt;
    }
    return OAT_OK;
}

static uint64_t sat_mul(uint64_t a, uint64_t b)
{
    if (a == 0 || b == 0) return 0;
    if (a > UINT64_MAX / b) return UINT64_MAX;
    return a * b;
}

/* U = sum over frames of the product of |SA(i,j)| over rows: the number of
 * column tuples Alg 4 enumerates. */
int oat_tuple_count(const oat *o, uint64_t *U)
{
    if (!o) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    uint64_t total = 0;
    for (uint32_t z = 0; z < o->nframe; z++) {
        uint64_t prod = 1;
        for (uint32_t j = 0; j < o->p.r; j++) {
            uint64_t cnt = 0;
            for (uint32_t x = 0; x < o->ncol; x++) cnt += o->super[atv_index(o, z, j, x)];
            prod = sat_mul(prod, cnt);
        }
        total = (UINT64_MAX - total < prod) ? UINT64_MAX : total + prod;
    }
    *U = total;
    return OAT_OK;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Alg 4: per frame, enumerate every tuple of super ATVs (one per row), keep
 * tuples whose duplicate positions agree, rebuild f = LBS || frame, unmangle. */
int oat_restore(const oat *o, uint32_t *out, uint64_t cap, uint64_t *n_out)
{
    if (!o || !n_out) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    uint64_t U;
    oat_tuple_count(o, &U);
    if (U > o->p.tuple_budget) {
        *n_out = U;
        return OAT_E_BUDGET;
    }
    uint32_t r = o->p.r;
    uint32_t **sa = (uint32_t **)calloc(r, sizeof(uint32_t *));
    uint32_t *cnt = (uint32_t *)calloc(r, sizeof(uint32_t));
    size_t outcap = 1024, m = 0;
    uint32_t *res = (uint32_t *)malloc(outcap * sizeof(uint32_t));
    for (uint32_t j = 0; j < r; j++) sa[j] = (uint32_t *)malloc(o->ncol * sizeof(uint32_t));
    uint32_t idx[64], x[64];
    for (uint32_t z = 0; z < o->nframe; z++) {
        int empty = 0;
        for (uint32_t j = 0; j < r; j++) {
            cnt[j] = 0;
            for (uint32_t xx = 0; xx < o->ncol; xx++)
                if (o->super[atv_index(o, z, j, xx)]) sa[j][cnt[j]++] = xx;
            if (cnt[j] == 0) empty = 1;
        }
        if (empty) continue;
        for (uint32_t j = 0; j < r; j++) idx[j] = 0;
        for (;;) {
            for (uint32_t j = 0; j < r; j++) x[j] = sa[j][idx[j]];
            uint32_t L;
            if (oat_tuple_to_L(o, x, &L)) {
                uint32_t f = (o->p.u == 0) ? L : ((L << o->p.u) | z);
                if (m == outcap) {
                    outcap *= 2;
                    res = (uint32_t *)realloc(res, outcap * sizeof(uint32_t));
                }
                res[m++] = oat_unmangle(o, f);
            }
            /* odometer over the tuple space, last row fastest */
            int j = (int)r - 1;
            while (j >= 0) {
                if (++idx[j] < cnt[j]) break;
                idx[j] = 0;
                j--;
            }
            if (j < 0) break;
        }
    }
    qsort(res, m, sizeof(uint32_t), cmp_u32);
    *n_out = m;
    int rc = OAT_OK;
    if (m > cap) rc = OAT_E_OVERFLOW;
    else if (out) memcpy(out, res, m * sizeof(uint32_t));
    for (uint32_t j = 0; j < r; j++) free(sa[j]);
    free(sa);
    free(cnt);
    free(res);
    return rc;
}

/* Occupancy-by-age features of a host (inputs of the learned correction):
 * e_i = the largest age over its r ATs at position i, or none if any of them
 * is inactive for the full window k;
 *   feat[d]  = #{i : e_i = d} / g                 for d < min(k, 61)
 *   feat[61] = min(ln(1 + max(plain, 0)), 20) / 16  (plain = Eq 4 estimate)
 *   feat[62] = k / 64
 *   feat[63] = (P_0 + ... + P_{r-1}) / r           (P_j as in Eq 4)
 * The histogram's prefix sums are NAT for every window k' <= k. */
int oat_features(const oat *o, const uint32_t *aip, uint64_t n, float *feat)
{
    if (!o) return OAT_E_INVAL;
    if (!o->queryable) return OAT_E_STATE;
    uint32_t k = o->p.k, x[64], z;
    uint32_t *hist = (uint32_t *)malloc(k * sizeof(uint32_t)); /* ages 0..k-1 */
    if (!hist) return OAT_E_NOMEM;
    for (uint64_t q = 0; q < n; q++) {
        oat_rrh(o, aip[q], &z, x);
        memset(hist, 0, k * sizeof(uint32_t));
        for (uint32_t i = 0; i < o->g; i++) {
            uint32_t act = act_of(o, o->c0_query, i);
            uint32_t e = 0;
            int inactive = 0;
            for (uint32_t j = 0; j < o->p.r; j++) {
                uint16_t at = o->at[atv_index(o, z, j, x[j]) * o->g + i];
                if (!oat_check_at(k, act, at, k)) {
                    inactive = 1;
                    break;
                }
                uint32_t age = (act + 2 * k - at) % (2 * k);
                if (age > e) e = age;
            }
            if (!inactive) hist[e]++;
        }
        uint8_t fl;
        double plain = estimate_one(o, z, nat_of(o, z, x), &fl);
        float *f = feat + q * 64;
        for (uint32_t d = 0; d < 64; d++) f[d] = 0.0f;
        for (uint32_t d = 0; d < k && d < 61; d++) f[d] = (float)((double)hist[d] / (double)o->g);
        double lp = log(1.0 + (plain > 0 ? plain : 0.0));
        if (!(lp < 20.0)) lp = 20.0;
        f[61] = (float)(lp / 16.0);
        f[62] = (float)((double)k / 64.0);
        double denom_cells = (double)((uint64_t)o->g * o->ncol);
        double s = 0;
        for (uint32_t j = 0; j < o->p.r; j++) s += (double)o->aat[(uint64_t)z * o->p.r + j] / denom_cells;
        f[63] = (float)(s / (double)o->p.r);
    }
    free(hist);
    return OAT_OK;
}

/* ---- ACE, the aging-counter estimator the paper compares against
 * (Section 2.3).  Every AT position of the same cube holds a timeout counter
 * of ceil(log2(k+1)) bits instead.  A pair sets the counters it reaches to
 * the largest value c = 2^bits - 1; every slice after the first starts by
 * decreasing every counter that is not zero.  At the close of slice t a
 * counter set in slice s holds c - (t - s) (until it reaches 0), so it is
 * active for window k' when it is at least c - k' + 1. */
struct oat_ace {
    oat *hash;          /* the same cube and hash functions; its ATs unused */
    uint32_t bits, cmax;
    uint16_t *cnt;      /* one counter per AT position, ATV-major */
    uint32_t *w;
    uint64_t t;
    int open;
};

int oat_ace_create(const oat_params *p, oat_ace **out)
{
    if (!out) return OAT_E_INVAL;
    *out = NULL;
    oat_ace *a = (oat_ace *)calloc(1, sizeof(oat_ace));
    if (!a) return OAT_E_NOMEM;
    int rc = oat_create(p, &a->hash);
    if (rc) {
        free(a);
        return rc;
    }
    a->bits = 1;
    while ((1u << a->bits) < p->k + 1) a->bits++;
    a->cmax = (1u << a->bits) - 1;
    a->cnt = (uint16_t *)calloc(a->hash->pool_size, sizeof(uint16_t));
    a->w = (uint32_t *)calloc(a->hash->n_atv, sizeof(uint32_t));
    if (!a->cnt || !a->w) {
        oat_ace_destroy(a);
        return OAT_E_NOMEM;
    }
    *out = a;
    return OAT_OK;
}

void oat_ace_destroy(oat_ace *a)
{
    if (!a) return;
    oat_destroy(a->hash);
    free(a->cnt);
    free(a->w);
    free(a);
}

static void ace_open(oat_ace *a)
{
    if (a->t > 0)
        for (uint64_t q = 0; q < a->hash->pool_size; q++)
            if (a->cnt[q] != 0) a->cnt[q] -= 1;
    a->open = 1;
}

int oat_ace_ingest(oat_ace *a, const uint32_t *aip, const uint32_t *bip, uint64_t n)
{
    if (!a) return OAT_E_INVAL;
    if (!a->open) ace_open(a);
    const oat *o = a->hash;
    uint32_t x[64], z;
    for (uint64_t q = 0; q < n; q++) {
        oat_rrh(o, aip[q], &z, x);
        uint32_t i = oat_bh(o, bip[q]);
        for (uint32_t j = 0; j < o->p.r; j++)
            a->cnt[atv_index(o, z, j, x[j]) * o->g + i] = (uint16_t)a->cmax;
    }
    return OAT_OK;
}

int oat_ace_close(oat_ace *a, uint32_t kprime)
{
    if (!a) return OAT_E_INVAL;
    const oat *o = a->hash;
    if (kprime < 1 || kprime > o->p.k) return OAT_E_INVAL;
    if (!a->open) ace_open(a);
    for (uint64_t v = 0; v < o->n_atv; v++) {
        uint32_t w = 0;
        for (uint32_t i = 0; i < o->g; i++) w += a->cnt[v * o->g + i] >= a->cmax - kprime + 1;
        a->w[v] = w;
    }
    a->t += 1;
    a->open = 0;
    return OAT_OK;
}

uint32_t oat_ace_bits(const oat_ace *a) { return a->bits; }
const uint16_t *oat_ace_counters(const oat_ace *a) { return a->cnt; }
const uint32_t *oat_ace_weights(const oat_ace *a) { return a->w; }

uint64_t oat_pool_size(const oat *o) { return o->pool_size; }
const uint16_t *oat_pool(const oat *o) { return o->at; }
uint64_t oat_n_atv(const oat *o) { return o->n_atv; }
const uint32_t *oat_weights(const oat *o) { return o->w; }
const uint64_t *oat_aat(const oat *o) { return o->aat; }
const uint8_t *oat_super(const oat *o) { return o->super; }

void oat_constants(const oat *o, uint64_t *out)
{
    out[0] = o->prime;
    out[1] = o->A;
    out[2] = o->Ainv;
    out[3] = o->alpha;
    out[4] = o->beta;
    out[5] = o->T;
    out[6] = o->W;
    out[7] = o->blk_a;
}

void oat_clock(const oat *o, uint64_t *out)
{
    out[0] = o->t;
    out[1] = (uint64_t)o->open;
    out[2] = (uint64_t)o->queryable;
    out[3] = o->c0_query;
    out[4] = o->kq;
}
