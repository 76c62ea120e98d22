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
 * Pool layout (device, owned by the handle): one AT per element,
 *   AT[((z*r + y)*2^c + x)*g + i]
 * for frame z < 2^u, row y < r, column x < 2^c and AT position i < g, so each
 * ATV (g ATs) is contiguous.  An AT holds 0..2k; 2k means inactive.  That is
 * ceil(log2(2k+1)) bits (Section 3), stored in one byte while 2k < 256
 * (k <= 127) and in a little-endian 16-bit word otherwise (the paper's own run
 * uses k = 300).
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
    uint32_t k;            /* slices per window, 1..32767 (byte ATs to 127)    */
    uint32_t r;            /* rows: ATVs per host, 1..8                        */
    uint32_t c;            /* log2 of the columns per row, 1..20               */
    uint32_t s;            /* column stride in LBS bits, 1..c                  */
    uint32_t u;            /* log2 of the frames, 0..16                        */
    uint32_t log2g;        /* log2 of the ATs per ATV, 4..15                   */
    double theta;          /* super point threshold, > 0                       */
    uint64_t seed;         /* derives the mangling multiplier and the BH hash  */
    uint64_t tuple_budget; /* restore guard on column tuples; 0 means 2^32     */
} at_params;

/*
 * at_create -- allocate a pool of 2^(c+u) * r * 2^log2g ATs (1 byte each for
 * k <= 127, 2 bytes beyond) on the current HIP device and set every AT to 2k
 * (InitAT, Section 3).
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
 * t advances.  Asynchronous on the handle's stream; the per-(row, frame)
 * super-ATV counts are also stored in pinned host memory, where at_restore
 * and at_tuple_count wait for them instead of issuing a copy of their own.
 * Errors: AT_E_INVAL (k' outside [1, k]), AT_E_DEVICE.
 */
int at_close_slice(at_ctx *h, uint32_t kprime);

/* at_close_slice for several windows at once (the paper's "any k' <= k from
 * one state", Section 3): one read of the pool yields the k'-weights of every
 * ATV for each of the n windows kprimes[0..n-1] (1 <= n <= AT_MAX_WINDOWS,
 * each 1 <= k' <= k), then AAT and super lists per window.  Queries use
 * kprimes[0] until at_select_window picks another.  AT_E_INVAL otherwise. */
#define AT_MAX_WINDOWS 8
int at_close_slice_multi(at_ctx *h, const uint32_t *kprimes, uint32_t n);

/* Make estimates, restores and at_read_summary use the window k' of the last
 * close (one of its kprimes).  AT_E_STATE without a queryable window,
 * AT_E_INVAL if k' was not summarised. */
int at_select_window(at_ctx *h, uint32_t kprime);

/*
 * at_close_slice_hist -- at_close_slice(h, kprime) that, in the same single
 * read of the pool, also builds every ATV's age histogram (Section 3: an AT
 * set in the latest k' slices is active for every window k' <= k, and the
 * ATs' timestamps stay valid for all of them).  Bin a < k of an ATV counts
 * its ATs that are not inactive and were set a slices ago (timestamp
 * distance a modulo 2k), so |ATV|^k' is the sum of its first k' bins for
 * every k' <= k.  The histograms live in device memory, n_atv x k 16-bit
 * counts (allocated on first use, freed by at_destroy), and stay valid until
 * the next slice opens or another close runs.  Summaries, estimates and
 * restores then follow window kprime.
 * Errors: AT_E_INVAL (k' outside [1, k], or k > AT_HIST_MAX_K), AT_E_NOMEM,
 * AT_E_DEVICE.
 */
#define AT_HIST_MAX_K 1024
int at_close_slice_hist(at_ctx *h, uint32_t kprime);

/* Re-summarise the window held since the last at_close_slice_hist for any
 * k' in [1, k] from the histograms alone (no read of the pool): k'-weights,
 * AAT(k', row, frame) and super lists (Section 4.2, 4.3).  Estimates and
 * restores then use window k'.  AT_E_STATE unless the last close was
 * at_close_slice_hist and no slice has opened since; AT_E_INVAL for k'
 * outside [1, k]. */
int at_requery_window(at_ctx *h, uint32_t kprime);

/* Copy the last at_close_slice_hist's histograms (n_atv x k uint16, ATV-major
 * in ATV index order) to host memory; blocks until copied.  AT_E_STATE as for
 * at_requery_window. */
int at_read_age_hist(at_ctx *h, uint16_t *host_out);

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

/* Pool size in bytes and number of ATVs (bytes per AT = pool_bytes /
 * (n_atv * g): 1 for k <= 127, else 2). */
int at_pool_info(const at_ctx *h, uint64_t *pool_bytes, uint64_t *n_atv);

/* Synchronous copy of the whole pool (pool_bytes, the layout above) to a host
 * buffer. */
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

/* How at_ingest_slice scans (every mode gives the same pool):
 *   1 = direct: one pass, r AT stores per pair straight into the pool;
 *   2 = binned: pairs hashed once into 8 frame-group bins, then one pass per
 *       row in which workgroup b takes bin b mod 8, so each XCD's stores stay
 *       in one region of the pool (an extra 64 B of scratch per pair);
 *   3 = tiled: the pool in 64 KiB tiles; the calls' AT stores are counted and
 *       grouped per tile (2 B of scratch per store), then one workgroup per
 *       tile applies them in LDS and writes the tile back.  Needs a pool of
 *       whole tiles, at most 4096 of them (AT_E_INVAL otherwise);
 *   0 = automatic: tiled when the pool tiles and the call's r*n stores reach
 *       a twelfth of the pool's bytes, else binned when u >= 3, the pool is at
 *       least 32 MiB and the call has at least 65536 pairs, else direct.
 * Batches of up to 8M pairs at a time.  AT_E_INVAL for another mode. */
int at_set_scan_mode(at_ctx *h, int mode);


/*
 * at_ingest_slice_noalloc -- at_ingest_slice for callers that cannot
 * allocate device memory: code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, ordering and result as
 * at_ingest_slice (every scan gives the same pool); it calls no allocator.
 * When the scan mode picks the tiled scan, the call's records and tables live
 * in a fixed device array of AT_NOALLOC_SCRATCH_BYTES that the library keeps
 * on every GPU it runs on until the process ends; where at_ingest_slice would
 * bin, the direct scan (no scratch) runs.  n above AT_NOALLOC_MAX_PAIRS gives
 * AT_E_INVAL with nothing done: split larger slices over several calls.  All
 * calls on one GPU share that array and nothing in it needs clearing; calls
 * that overlap in time on one GPU (other handles' streams included) race.
 * Errors: as at_ingest_slice; AT_E_DEVICE if the array's address could not be
 * had when the handle was created.
 */
#define AT_NOALLOC_MAX_PAIRS (1ull << 20)
#define AT_NOALLOC_SCRATCH_BYTES (33ull << 20)
int at_ingest_slice_noalloc(at_ctx *h, const uint32_t *aip_dev, const uint32_t *bip_dev, uint64_t n);

/* ------------------------------------------------------ learned correction
 * Not in the paper: a small network that corrects the plain estimate from the
 * host's occupancy-by-age profile, with the plain estimate kept as fallback.
 *
 * Features of a host (AT_FEATURES = 64 floats), over the last closed window:
 * with e_i the largest age (ACT distance) of the host's r ATs at position i
 * when all r are active for the full window k (Alg 1 with k' = k),
 *   f[d]  = #{i : e_i = d} / g        for d < min(k, 61)   (0 above)
 *   f[61] = min(ln(1 + max(plain, 0)), 20) / 16, plain = the Eq 4 estimate
 *   f[62] = k / 64
 *   f[63] = mean over rows of AAT(k', row, frame) / (g * 2^c).
 * The prefix sum of f[0..k'-1] times g is NAT(k') of Alg 5.
 *
 * Network: 64 -> 64 -> 64 -> 1, ReLU.  Its output y corrects the plain
 * estimate's log feature: z = y + 16 * f[61] estimates ln n.  Parameters
 * (AT_MLP_NPARAM floats, FP32 master copy): W1[64][64] (row = output unit),
 * b1[64], W2[64][64], b2[64], w3[64], b3.  Features, weights and hidden
 * activations are rounded to bfloat16 (nearest even); products accumulate in
 * FP32 on the matrix cores.  Training minimises the mean squared error of ln n
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
 * Learned estimate = exp(z) when z is finite and within
 * [ln 16 - 0.5, ln 2^18 + 0.5], else the plain estimate with AT_F_FALLBACK. */
typedef struct at_mlp at_mlp;
#define AT_FEATURES 64
#define AT_MLP_NPARAM 8385

/* Features, plain estimates and their flags of n hosts (device arrays: aip_dev
 * n uint32; feat_dev n*64 float row-major; est_dev, flags_dev may be NULL).
 * Asynchronous on the handle's stream; valid in the same state as
 * at_estimate (AT_E_STATE otherwise). */
int at_features(at_ctx *h, const uint32_t *aip_dev, uint64_t n, float *feat_dev, double *est_dev,
                uint8_t *flags_dev);

/* A network on the given stream with all parameters zero.  AT_E_NOMEM. */
int at_mlp_create(void *hip_stream, at_mlp **out);
int at_mlp_destroy(at_mlp *m);
/* Copy AT_MLP_NPARAM host floats in (resets the optimiser) or out.  Sync. */
int at_mlp_set_params(at_mlp *m, const float *host_params);
int at_mlp_get_params(at_mlp *m, float *host_params);
/* y_dev[i] = network(x_dev[i*64 .. i*64+63]) for i < n.  Asynchronous. */
int at_mlp_forward(at_mlp *m, const float *x_dev, uint64_t n, float *y_dev);
/* Gradient of mean((y - t)^2) over the n rows (t: the target of y, i.e.
 * ln n - 16 * f[61] for the learned correction) into grad_dev (AT_MLP_NPARAM
 * floats, device, may be NULL); the loss to *loss_host if not NULL (then
 * synchronous). */
int at_mlp_grad(at_mlp *m, const float *x_dev, const float *t_dev, uint64_t n, float *grad_dev,
                float *loss_host);
/* A training batch on the network's stream: for i < n, row idx_dev[i] of the
 * n_all x 64 features x_dev into xb_dev[i*64 ..], and the network's target
 * tb_dev[i] = lnn_dev[idx_dev[i]] - 16 * x_dev[idx_dev[i]*64 + 61] (ln n
 * minus the plain estimate's log feature).  Device arrays; every idx_dev
 * entry must be a row of x_dev.  Asynchronous.  AT_E_INVAL for null pointers
 * with n > 0. */
int at_mlp_gather_batch(at_mlp *m, const float *x_dev, const float *lnn_dev, const int64_t *idx_dev, uint64_t n,
                        float *xb_dev, float *tb_dev);
/* One Adam step with the given gradient (device) and learning rate. */
int at_mlp_apply_grad(at_mlp *m, const float *grad_dev, float lr);
/* Gradient + Adam step on one batch; loss as in at_mlp_grad (before the step). */
int at_mlp_train_step(at_mlp *m, const float *x_dev, const float *t_dev, uint64_t n, float lr,
                      float *loss_host);
/* Learned estimates of n hosts with fallback (host arrays; plain_out, the
 * plain Eq 4 estimates, may be NULL).  Synchronous.  Flags: AT_F_SAT and
 * AT_F_NEG of the plain estimate, AT_F_FALLBACK, AT_F_SUPER of the returned
 * estimate. */
int at_estimate_learned(at_ctx *h, at_mlp *m, const uint32_t *aip_host, uint64_t n, double *est_out,
                        uint8_t *flags_out, double *plain_out);
/* The same on device arrays, asynchronous (plain_dev may be NULL). */
int at_estimate_learned_dev(at_ctx *h, at_mlp *m, const uint32_t *aip_dev, uint64_t n, double *est_dev,
                            uint8_t *flags_dev, double *plain_dev);
/* at_estimate_learned in two halves, so that a caller can queue the next
 * slice's at_ingest_slice (or any other call) while the estimates are being
 * computed.  _begin copies the n host addresses into the handle's own
 * pinned staging and queues the features, the network and the fallback,
 * which read the addresses from that staging and store their results there
 * (device-mapped host memory, no copy commands); it returns without
 * waiting.  The estimates are those of the window summarised by the last
 * close before _begin, whatever is queued afterwards.  _end waits for them
 * and writes n entries to est_out, flags_out and, if not NULL, plain_out
 * (the same values at_estimate_learned gives).  One _begin may be pending
 * per handle: a second _begin, or at_estimate_learned, before its _end gives
 * AT_E_STATE, as does _end without a pending _begin.  Other calls may run in
 * between.  Errors of _begin as at_estimate_learned; _end: AT_E_STATE,
 * AT_E_INVAL (null est_out or flags_out with n > 0; the pending estimate is
 * kept), AT_E_DEVICE (the pending estimate is dropped). */
int at_estimate_learned_begin(at_ctx *h, at_mlp *m, const uint32_t *aip_host, uint64_t n);
int at_estimate_learned_end(at_ctx *h, double *est_out, uint8_t *flags_out, double *plain_out);

/* ------------------------------------------------------ streaming server
 * Not in the paper: many links served by one device.  Every admitted link's
 * pool stays resident in device memory; links are admitted while the sum of
 * their footprints fits the HBM budget, later ones wait in FIFO order and are
 * admitted as others close.  Producers queue chunks of pairs and slice ends
 * per link at any time (thread-safe); each at_serve_step turns everything
 * queued so far into one batched step: the slices that open are preserved
 * and every queued chunk of every link is scanned in one launch, while the
 * slices whose chunks were all scanned in earlier steps are closed, restored
 * and estimated in a concurrent branch.  The step is a hipGraph captured
 * once and replayed with a new descriptor table each time.  A link whose
 * step holds as many pairs as its pool is large instead takes the tiled scan
 * (one launch for all such links of the step, ahead of the graph), and a
 * slice whose pairs and end it takes is scanned and closed in the same step.
 * The native thread (at_serve_start) plans a step made only of such scans
 * and their closes while the previous one runs, and queues its scans behind
 * the previous graph.
 *
 * All links of a server share the geometry shape (r, c, s, u, log2g, theta);
 * k and seed are per link.  Per closed slice the server returns the restore
 * outcome (AT_OK with up to cand_cap sorted candidates, AT_E_BUDGET with U,
 * or AT_E_OVERFLOW with m), the plain and learned estimates of the candidates
 * and of the link's watch hosts, and the latency from the slice end call to
 * the result being on the host. */
typedef struct at_serve at_serve;

typedef struct {
    uint64_t hbm_budget;   /* bytes of device memory the links may hold       */
    uint32_t max_links;    /* links resident at once, 1..64                    */
    uint32_t cand_cap;     /* restore candidates returned per close, 1..2048   */
    uint32_t watch_cap;    /* watch hosts per link, 0..16384                   */
    uint32_t r, c, s, u;   /* shared geometry (u <= 8)                         */
    uint32_t log2g;
    double theta;
} at_serve_config;

typedef struct {
    uint32_t link;         /* link id                                          */
    uint32_t kprime;       /* window of the close                              */
    uint64_t slice;        /* index of the closed slice                        */
    int32_t restore_rc;    /* AT_OK, AT_E_BUDGET or AT_E_OVERFLOW              */
    uint32_t n_cand;       /* candidates returned (0 unless restore_rc AT_OK)  */
    uint64_t n_out;        /* m candidates, or U when AT_E_BUDGET              */
    uint32_t n_watch;      /* watch-host estimates returned                    */
    uint32_t pad;
    double latency_ms;     /* slice end call -> result on the host             */
    double step_ms;        /* device time of the step that closed it          */
} at_serve_result;

int at_serve_create(const at_serve_config *cfg, at_serve **out);
int at_serve_destroy(at_serve *s);
/* Network used for the learned estimates (NULL: learned = plain, flagged
 * AT_F_FALLBACK).  The network must outlive its use by the server. */
int at_serve_set_mlp(at_serve *s, at_mlp *m);
/* Register a link: admitted at once (*admitted = 1) if its footprint fits the
 * budget and nobody waits, else queued (*admitted = 0).  AT_E_NOMEM if it can
 * never fit.  Served links use byte ATs: 1 <= k <= 127, else AT_E_INVAL. */
int at_serve_open_link(at_serve *s, uint32_t k, uint64_t seed, uint64_t tuple_budget, uint32_t *link_id,
                       int *admitted);
/* state: 0 waiting, 1 active, 2 closed; slices closed; queued events. */
int at_serve_link_state(at_serve *s, uint32_t link_id, int *state, uint64_t *slices_closed,
                        uint64_t *pending);
/* Release a link's memory (after the running step, and after any scans of
 * its pool already queued for the next) and admit waiting links. */
int at_serve_close_link(at_serve *s, uint32_t link_id);
/* Hosts estimated at every close of the link (host array, <= watch_cap). */
int at_serve_set_watch(at_serve *s, uint32_t link_id, const uint32_t *hosts_host, uint32_t n);
/* Queue a chunk of the link's current slice (device arrays of n uint32,
 * contents complete; they must stay valid until the step that scans them
 * returns).  AT_E_STATE unless the link is active. */
int at_serve_submit(at_serve *s, uint32_t link_id, const uint32_t *aip_dev, const uint32_t *bip_dev,
                    uint64_t n);
/* Queue the end of the link's current slice with window k' (1 <= k' <= k). */
int at_serve_end_slice(at_serve *s, uint32_t link_id, uint32_t kprime);
/* at_serve_submit of the slice's last chunk (n may be 0) and
 * at_serve_end_slice as one queue operation, so that no step can take the
 * chunk without its end: a step that scans a whole slice with the tiled scan
 * then also counts the slice's window weights, and the close reads no pool.
 * Latency is measured from this call. */
int at_serve_submit_last(at_serve *s, uint32_t link_id, const uint32_t *aip_dev, const uint32_t *bip_dev,
                         uint64_t n, uint32_t kprime);
/* Run one batched step (synchronous); *n_results = slices closed by it. */
int at_serve_step(at_serve *s, uint32_t *n_results);
/* Start a native thread that runs steps back to back while any link has
 * queued work and sleeps otherwise (AT_E_STATE if already running); stop
 * drains the queues, joins the thread and returns the first step error. */
int at_serve_start(at_serve *s);
int at_serve_stop(at_serve *s);
/* Pop the oldest result; arrays may be NULL; AT_E_STATE when none is ready,
 * AT_E_OVERFLOW when the capacities are too small (nothing popped). */
int at_serve_next_result(at_serve *s, at_serve_result *out, uint32_t *cand, double *cand_plain,
                         double *cand_learned, uint8_t *cand_flags, uint32_t cand_cap, double *watch_plain,
                         double *watch_learned, uint8_t *watch_flags, uint32_t watch_cap);
/* out[0] steps run, out[1] pairs scanned, out[2] bytes held by links,
 * out[3] links waiting for admission. */
int at_serve_stats(at_serve *s, uint64_t *out4);
/* Synchronous copy of an active link's pool to the host. */
int at_serve_read_pool(at_serve *s, uint32_t link_id, uint8_t *host_out);
/* Tiled scans run by the server so far: launches, the link scans they
 * covered (a step's tiled links share launches, up to 8 per launch, each a
 * grid row of every pass; a link's step of over 8M pairs takes launches of
 * its own), the pairs they scanned and their summed device time in ms (HIP
 * events around each launch on its stream).  A link's step goes to the tiled
 * scan, instead of the batched byte-store scan, when its r*n stores times 12
 * (30 once the resident pools exceed the 256 MiB last-level cache) reach its
 * pool's bytes and the pool is whole 64 KiB tiles, at most 4096.
 * planned_ahead: steps the native thread planned, and whose scans it queued,
 * before the previous step's graph had finished.  Any pointer may be NULL. */
int at_serve_tiled_stats(at_serve *s, uint64_t *calls, uint64_t *pairs, double *device_ms, uint64_t *jobs,
                         uint64_t *planned_ahead);

/*
 * The aging-counter comparator (Section 2.3 against Section 3).  ACE keeps a
 * timeout counter of ceil(log2(k+1)) bits at every AT position: a pair sets
 * the counters it reaches to their largest value c = 2^bits - 1, and every
 * slice after the first starts by decreasing every nonzero counter, so each
 * slice rewrites the whole pool.  A counter set s slices before a close holds
 * c - s and counts in window k' when it is at least c - k' + 1.  The
 * asynchronous timestamps need one bit more (2k+1 values) and their lazy
 * preserve (Alg 2) examines two of the 2k blocks of every ATV per slice.
 * Both are kept here at their own width, packed: F = floor(32 / bits) fields
 * per 32-bit word, position i of ATV v in word v * wv + i / F (wv =
 * ceil(g / F) words per ATV) at bits [(i % F) * bits, (i % F + 1) * bits),
 * unused fields and bits zero (timestamp fields start at 2k, inactive).
 * Sub-word fields take their stores as 32-bit atomics (ACE one OR, a
 * timestamp an AND and an OR).  The cube, hashes and block layout are those
 * of an at_ctx made with the same parameters, so the k'-weights of the two
 * kinds equal at_close_slice's.  Calls are asynchronous on hip_stream except
 * at_cmp_read.
 */
typedef struct at_cmp at_cmp;
enum { AT_CMP_ACE = 1, AT_CMP_AT = 2 };
/* kind AT_CMP_ACE or AT_CMP_AT.  AT_E_INVAL (parameters as at_create), AT_E_NOMEM. */
int at_cmp_create(const at_params *p, int kind, void *hip_stream, at_cmp **out);
int at_cmp_destroy(at_cmp *c);
/* out4 = {bits per field, fields per word F, words per ATV, words in all}. */
int at_cmp_info(const at_cmp *c, uint64_t *out4);
/* The slice's maintenance only (opening it if it is not): ACE ages every
 * counter (not before the first slice); the timestamps preserve their two
 * due blocks.  Later calls in the same slice do nothing. */
int at_cmp_open_slice(at_cmp *c);
/* Alg 3 on the packed pool: n pairs, aip_dev/bip_dev device arrays of n
 * uint32 (opens the slice first if needed). */
int at_cmp_ingest(at_cmp *c, const uint32_t *aip_dev, const uint32_t *bip_dev, uint64_t n);
/* End of the slice: per-ATV k'-weights, 1 <= k' <= k (AT_E_INVAL otherwise). */
int at_cmp_close(at_cmp *c, uint32_t kprime);
/* Copy the packed words (words_host: "words in all" uint32) and/or the last
 * close's weights (weights_host: one uint32 per ATV; AT_E_STATE before any
 * close, or once a slice has opened since) to host memory; blocks.  Either
 * pointer may be NULL. */
int at_cmp_read(at_cmp *c, uint32_t *words_host, uint32_t *weights_host);

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
