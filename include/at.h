/*
 * at.h -- C ABI of the MI355X (gfx950) asynchronous-timestamp super-point
 * library: sliding-window super point detection and cardinality estimation
 * with a cube of asynchronous timestamp vectors (ATVC), after J. Xu,
 * "Distributed super point cardinality estimation under sliding time window
 * for high speed network".
 *
 * Problem (Section 2.1, 2.2): every packet between the monitored network and
 * the outside yields a pair <aip, bip>; the cardinality of aip in a window is
 * the number of distinct bip seen with it; aip is a super point when that
 * number is at least theta.  Traffic is cut into equal time slices and the
 * window W(t, k) holds the k latest slices (Section 2.3).
 *
 * One handle = one link = one ATVC pool resident in device memory, driven on
 * one HIP stream that the caller owns.  Calls on one handle are not
 * thread-safe; distinct handles may be used from different threads.  Every
 * call returns AT_OK (0) or a negative error code; at_strerror() names it.
 *
 * Pool layout (device, owned by the handle): one byte per AT,
 *   AT[((z*r + y)*2^c + x)*g + i]
 * for frame z < 2^u, row y < r, column x < 2^c and AT position i < g, so each
 * ATV (g ATs) is contiguous.  An AT holds 0..2k; 2k means inactive.
 */
#ifndef AT_H
#define AT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct at_ctx at_ctx;

enum {
    AT_OK = 0,
    AT_E_INVAL = -1,    /* bad argument or parameter                          */
    AT_E_STATE = -2,    /* call not valid in the handle's current state       */
    AT_E_NOMEM = -3,    /* device or host allocation failed                   */
    AT_E_OVERFLOW = -4, /* result larger than the caller's capacity           */
    AT_E_DEVICE = -5,   /* a HIP runtime call or kernel launch failed         */
    AT_E_BUDGET = -6    /* restore would enumerate more column tuples than the
                           handle's tuple budget                              */
};

/* Per-host flags returned with each estimate. */
enum {
    AT_F_SAT = 1,      /* Eq 4 saturated: NAT reached g (NAT clamped to g-1) or
                          every AT of the frame is active (estimate +inf)     */
    AT_F_NEG = 2,      /* Eq 4 gave a negative value (NAT below g*UP)         */
    AT_F_FALLBACK = 4, /* learned correction unusable; plain estimate kept    */
    AT_F_SUPER = 8     /* estimate >= theta                                   */
};

typedef struct {
    uint32_t k;            /* slices per window, 1..127 (one byte per AT)      */
    uint32_t r;            /* rows: ATVs per host, 1..8                        */
    uint32_t c;            /* log2 of the columns per row, 1..20               */
    uint32_t s;            /* column stride in LBS bits, 1..c                  */
    uint32_t u;            /* log2 of the frames, 0..16                        */
    uint32_t log2g;        /* log2 of the ATs per ATV, 4..16                   */
    double theta;          /* super point threshold, > 0                       */
    uint64_t seed;         /* derives the mangling multiplier and the BH hash  */
    uint64_t tuple_budget; /* restore guard on column tuples; 0 means 2^32     */
} at_params;

/*
 * at_create -- allocate a pool of 2^(c+u) * r * 2^log2g bytes on the current
 * HIP device and set every AT to 2k (InitAT, Section 3).
 *
 * The geometry must allow the reversible hash of Section 4.1 (W = 32 - u):
 *   1 <= s <= c <= W,  c + s*(r-1) >= W (completeness: every bit of LBS lands
 *   in some column),  c*r > W (redundancy: some duplicate positions exist),
 *   s*(r-1) < W.
 * Hash parameters come from SplitMix64(seed): A = 2^31 + x0 mod (p - 2^31)
 * with p = 2^32 - 5, BH multiplier alpha = x1 | 1 and addend beta = x2.
 * hip_stream is a hipStream_t (NULL = the default stream) that every later
 * call on the handle is ordered on; the caller keeps it alive.
 * Errors: AT_E_INVAL (parameters), AT_E_NOMEM, AT_E_DEVICE.  On error *out is
 * NULL and nothing is left allocated.
 */
int at_create(const at_params *p, void *hip_stream, at_ctx **out);

/*
 * at_ingest_slice -- scan n pairs of the current slice (Alg 3, Section 4.1):
 * each pair sets, in each of the r ATVs named by RRH(aip), the AT chosen by
 * BH(bip) to that AT's current timestamp.  aip_dev and bip_dev are device
 * arrays of n uint32 each, owned by the caller and read asynchronously on the
 * handle's stream; they must stay valid until the stream passes this call.
 * The first ingest (or close) of a slice opens it: the block clock advances
 * (C0 = t mod 2k) and preserveAT (Alg 2) runs on the two blocks of every ATV
 * whose timestamp is 0 or k (Section 3).  Any number of calls per slice; pair
 * order, batch split and repeated pairs do not change the result.  n = 0 only
 * opens the slice.
 * Errors: AT_E_INVAL (null pointer with n > 0, or a pointer that is not device
 * memory), AT_E_DEVICE.
 */
int at_ingest_slice(at_ctx *h, const uint32_t *aip_dev, const uint32_t *bip_dev, uint64_t n);

/*
 * at_close_slice -- end the current slice t (opening it first if nothing was
 * ingested: an empty slice still slides the window) and summarise the window
 * of the k' latest slices, 1 <= k' <= k: per-ATV k'-weights |ATV|^k' (Alg 1),
 * active ATs per (row, frame) AAT(k', row, frame) and the super ATVs, those
 * whose weight reaches ceil(g - g*exp(-theta/g)) (Section 4.2, 4.3).  Then
 * t advances.  Asynchronous on the handle's stream.
 * Errors: AT_E_INVAL (k' outside [1, k]), AT_E_DEVICE.
 */
int at_close_slice(at_ctx *h, uint32_t kprime);

/*
 * at_estimate -- cardinality of each of n hosts over the window summarised by
 * the last close (Alg 5 and Eq 4, Section 4.3): NAT = ATs active in all r of
 * the host's ATVs, UP = product over rows of AAT/(g*2^c) in the host's frame,
 * estimate = -g*ln((g - NAT)/(g*(1 - UP))), computed in FP64.  NAT >= g is
 * clamped to g-1 and flagged AT_F_SAT; UP == 1 gives +inf with AT_F_SAT; a
 * negative value is returned as is with AT_F_NEG; AT_F_SUPER marks
 * estimate >= theta.  aip_host, est_out and flags_out are host arrays of n
 * entries owned by the caller.  Synchronous (waits for the handle's stream).
 * Errors: AT_E_STATE (no closed window, or a slice has been opened since the
 * last close), AT_E_INVAL, AT_E_NOMEM, AT_E_DEVICE.
 */
int at_estimate(at_ctx *h, const uint32_t *aip_host, uint64_t n, double *est_out,
                uint8_t *flags_out);

/*
 * at_restore -- candidate super points of the closed window (Alg 4, Section
 * 4.2): for every frame, every tuple of super ATVs (one per row) whose
 * duplicate-position bits agree gives LBS; f = LBS * 2^u + frame and the
 * address is f^-1 (unmangling).  The set equals the addresses whose r ATVs are
 * all super.  On AT_OK it writes the m candidates ascending to sip_out, and
 * their estimates and flags (as at_estimate) to est_out / flags_out (either
 * may be NULL), and sets *n_out = m.  Host buffers, owned by the caller.
 * Errors: AT_E_BUDGET when the number of tuples U = sum over frames of the
 * product of the rows' super-ATV counts exceeds the tuple budget (*n_out = U,
 * nothing written); AT_E_OVERFLOW when m > cap (*n_out = m, nothing written);
 * AT_E_STATE, AT_E_INVAL, AT_E_NOMEM, AT_E_DEVICE.  Synchronous.
 */
int at_restore(at_ctx *h, uint32_t *sip_out, double *est_out, uint8_t *flags_out, uint64_t cap,
               uint64_t *n_out);

/* at_destroy -- wait for the handle's stream, free the pool and every buffer.
 * The handle is invalid afterwards.  NULL is accepted. */
int at_destroy(at_ctx *h);

/* ---------------------------------------------------------------- extras */

/* Text for an error code. */
const char *at_strerror(int rc);

/* Pool size in bytes and number of ATVs. */
int at_pool_info(const at_ctx *h, uint64_t *pool_bytes, uint64_t *n_atv);

/* Synchronous copy of the whole pool (pool_bytes) to a host buffer. */
int at_read_pool(at_ctx *h, uint8_t *host_out);

/* Synchronous copy of the last close's summaries: per-ATV weights (n_atv
 * uint32) and AAT per (frame, row) (2^u * r uint64, index frame*r + row).
 * Either pointer may be NULL.  AT_E_STATE before the first close. */
int at_read_summary(at_ctx *h, uint32_t *w_host, uint64_t *aat_host);

/* Clock state: out[0] = t (slices closed so far), out[1] = 1 if slice t is
 * open, out[2] = 1 if a closed window can be queried, out[3] = C0 of that
 * window, out[4] = its k'. */
int at_clock(const at_ctx *h, uint64_t *out5);

/* Derived constants: out[0] = p, A, A^-1, alpha, beta, T (super threshold),
 * W = 32-u, a (ATs per block of the first 2k-1 blocks). */
int at_constants(const at_ctx *h, uint64_t *out8);

/* at_estimate plus NAT per host (nat_out, n uint32, may be NULL). */
int at_estimate_detail(at_ctx *h, const uint32_t *aip_host, uint64_t n, double *est_out,
                       uint8_t *flags_out, uint32_t *nat_out);

/* Stream-ordered, asynchronous estimate on device arrays (aip_dev, est_dev,
 * flags_dev, nat_dev of n entries; est/flags/nat may be NULL).  Valid in the
 * same state as at_estimate; the caller synchronises the stream. */
int at_estimate_dev(at_ctx *h, const uint32_t *aip_dev, uint64_t n, double *est_dev,
                    uint8_t *flags_dev, uint32_t *nat_dev);

/* Number of column tuples U that at_restore would enumerate (see above). */
int at_tuple_count(at_ctx *h, uint64_t *U);

/* Measurement probe, not part of the method: n items (n a multiple of 4,
 * a_dev/b_dev 16-byte aligned device arrays of n uint32, read like the pair
 * scan reads its input) each store r (1, 2, 4 or 8) bytes at uniformly random
 * positions of dst_dev (device, `bytes` a power of two).  It gives the
 * random-byte-store throughput of a buffer of the pool's size, the roofline
 * of at_ingest_slice.  Asynchronous on hip_stream. */
int at_probe_scatter(uint8_t *dst_dev, uint64_t bytes, const uint32_t *a_dev, const uint32_t *b_dev,
                     uint64_t n, uint32_t r, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* AT_H */
