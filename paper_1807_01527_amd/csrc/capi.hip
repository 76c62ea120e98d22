// C ABI of the ATVC library: parameter validation, derived constants, the
// slice clock, device buffers and the sequencing of the kernels in
// kernels.hip.  All device work of a handle is ordered on its stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "at.h"
#include "atpool.hpp"

using atp::Geometry;

struct at_ctx {
    at_params p{};
    Geometry G{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t n_atv = 0, pool_bytes = 0;
    uint32_t nframe = 0, ngroups = 0;  // frames and (frame,row) groups
    // device state
    uint8_t* pool = nullptr;
    // summaries of up to kMaxWindows windows of the last close ...
    uint32_t* w_all = nullptr;
    uint64_t* aat_all = nullptr;
    uint32_t* sa_all = nullptr;
    uint32_t* sa_cnt_all = nullptr;
    uint32_t nwin = 0;
    uint32_t win_kq[atp::kMaxWindows] = {};
    uint16_t* hist = nullptr;     // per-ATV age histograms of the last close (k bins each), if it built them
    bool hist_valid = false;
    // ... and the one queries use
    uint32_t* w = nullptr;        // per ATV weight
    uint64_t* aat = nullptr;      // per (frame,row)
    uint32_t* sa = nullptr;       // per (frame,row): ascending super columns
    uint32_t* sa_cnt = nullptr;   // per (frame,row)
    unsigned long long* counter = nullptr;
    uint64_t* prefix = nullptr;   // nframe+1 restore item offsets
    // binned scan scratch
    uint64_t* bins = nullptr;
    uint64_t bins_cap = 0;
    unsigned long long* bin_fill = nullptr;
    atp::TileBufs tb{};           // tiled-scan scratch (grown on demand)
    uint8_t* pin = nullptr;       // pinned host staging of query inputs and outputs (grown on demand)
    uint64_t pin_cap = 0;
    uint32_t* pin_cnt = nullptr;  // pinned copy of the last close's super-ATV counts, every window,
    uint32_t* pin_cnt_dev = nullptr;  // stored there by the summary kernel through this mapping
    uint64_t pin_cnt_cap = 0;     // entries
    hipEvent_t cnt_ready = nullptr;  // recorded after the summary kernel
    uint8_t* pin_q = nullptr;     // pinned staging of the split learned estimate (its own, so other
    uint64_t pin_q_cap = 0;       // queries between _begin and _end cannot overwrite it); the kernels
    uint8_t* pin_q_dev = nullptr; // read the addresses from it and write the results into it directly
    hipEvent_t q_done = nullptr;  // recorded after the split estimate's copy back
    bool q_pending = false;
    uint64_t q_pending_n = 0;
    bool tiled_ok = false;        // the device has the LDS the tiled scan needs
    bool wfused = false;          // window-0 weights of the open slice already written by its one tiled call
    uint32_t wfused_kq = 0;
    int scan_mode = 0;            // 0 auto, 1 direct, 2 binned, 3 tiled
    uint8_t* scratch_dev = nullptr;  // this device's address of the no-alloc scratch array (or null)
    // grow-on-demand device scratch
    uint32_t* cand = nullptr;
    uint64_t cand_cap = 0;
    uint32_t* q_aip = nullptr;
    double* q_est = nullptr;
    uint8_t* q_flags = nullptr;
    uint32_t* q_nat = nullptr;
    float* q_feat = nullptr;      // n x 64 features
    double* q_plain = nullptr;
    uint64_t q_cap = 0;
    // slice clock
    uint64_t t = 0;
    bool open = false;
    bool queryable = false;
    uint32_t c0 = 0, c0_query = 0, kq = 0;
};

namespace {

uint64_t splitmix_next(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t pow_mod_p(uint64_t b, uint64_t e) {
    const uint64_t p = atp::kPrime;
    uint64_t r = 1;
    b %= p;
    while (e) {
        if (e & 1) r = (r * b) % p;  // operands < 2^32: products fit in 64 bits
        b = (b * b) % p;
        e >>= 1;
    }
    return r;
}

int validate(const at_params& p) {
    if (p.u > 16 || p.k < 1 || p.k > 32767 || p.r < 1 || p.r > (uint32_t)atp::kMaxRows) return AT_E_INVAL;
    const uint32_t W = 32 - p.u;
    if (p.c < 1 || p.c > 20 || p.s < 1 || p.s > p.c || p.c > W) return AT_E_INVAL;
    if (p.c + p.s * (p.r - 1) < W) return AT_E_INVAL;  // completeness
    if (p.c * p.r <= W) return AT_E_INVAL;             // redundancy
    if (p.s * (p.r - 1) >= W) return AT_E_INVAL;
    if (p.log2g < 4 || p.log2g > 15) return AT_E_INVAL;
    if (!(p.theta > 0) || !std::isfinite(p.theta)) return AT_E_INVAL;
    if ((uint64_t)p.c + p.u + p.log2g > 36) return AT_E_INVAL;  // pool <= r * 64 GiB
    return AT_OK;
}


int dev_err(hipError_t e) { return e == hipSuccess ? AT_OK : (e == hipErrorOutOfMemory ? AT_E_NOMEM : AT_E_DEVICE); }

template <typename T>
int dev_alloc(T** p, uint64_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? AT_E_NOMEM : AT_E_DEVICE;
    }
    return AT_OK;
}

void free_all(at_ctx* h) {
    void* bufs[] = {h->pool, h->w_all, h->aat_all, h->sa_all, h->sa_cnt_all, h->counter, h->prefix, h->cand,
                    h->q_aip, h->q_est, h->q_flags, h->q_nat, h->q_feat, h->q_plain, h->bins, h->bin_fill,
                    h->tb.rec, h->tb.cnt, h->tb.pre, h->tb.csum, h->tb.base, h->tb.act, h->hist};
    if (h->pin) (void)hipHostFree(h->pin);
    h->pin = nullptr;
    h->pin_cap = 0;
    if (h->pin_cnt) (void)hipHostFree(h->pin_cnt);
    h->pin_cnt = h->pin_cnt_dev = nullptr;
    if (h->pin_q) (void)hipHostFree(h->pin_q);
    h->pin_q = h->pin_q_dev = nullptr;
    if (h->cnt_ready) (void)hipEventDestroy(h->cnt_ready);
    h->cnt_ready = nullptr;
    if (h->q_done) (void)hipEventDestroy(h->q_done);
    h->q_done = nullptr;
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

bool device_accessible(const void* ptr) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
           attr.type == hipMemoryTypeUnified || (attr.type == hipMemoryTypeHost && attr.devicePointer != nullptr);
}

}  // namespace

// Scratch of at_ingest_slice_noalloc: the tiled scan's records and tables of
// one call, for callers that cannot allocate.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name
// is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns with that device current, kept per device.
static __device__ __align__(256) uint8_t scratch[AT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
uint8_t* scratch_addr[kMaxDevices] = {};

// Set-up, once per device (the caller has made `device` current): the
// array's address on that device, or null if it cannot be had.
uint8_t* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_addr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_addr[device] = static_cast<uint8_t*>(ptr);
    }
    return scratch_addr[device];
}

uint64_t up256(uint64_t x) { return (x + 255) & ~255ull; }

// The tiled scan's buffers for a call of z's size carved from the scratch
// array at base; returns the bytes used.
uint64_t carve_tiles(uint8_t* base, const atp::TileSizes& z, const Geometry& G, atp::TileBufs* tb) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t* p = base ? base + off : nullptr;
        off += up256(bytes);
        return p;
    };
    tb->rec = reinterpret_cast<uint16_t*>(take(z.recs * 2));
    tb->cnt = reinterpret_cast<uint16_t*>(take(z.table * 2));
    tb->pre = reinterpret_cast<uint32_t*>(take(z.table * 4));
    tb->csum = reinterpret_cast<uint32_t*>(take((uint64_t)(z.nchunk + 2) * 4096 * 4));
    tb->base = reinterpret_cast<uint32_t*>(take(4097 * 4));
    tb->act = take((uint64_t)G.g * G.atb);
    tb->rec_cap = z.recs;
    tb->table_cap = z.table;
    tb->chunk_cap = z.nchunk + 2;
    return off;
}

// Opening slice t: C0 = t mod 2k and Alg 2 on the due blocks.  With
// `deferred` the caller runs Alg 2 itself (the tiled scan does it in LDS).
int open_slice(at_ctx* h, bool deferred = false) {
    if (h->open) return AT_OK;
    h->c0 = (uint32_t)(h->t % h->G.twok);
    if (!deferred && atp::launch_preserve(h->pool, h->n_atv, h->G, h->c0, h->stream) != hipSuccess)
        return AT_E_DEVICE;
    h->open = true;
    h->queryable = false;
    return AT_OK;
}

uint64_t up64(uint64_t x) { return (x + 63) & ~63ull; }

// Byte offsets of the results of a split learned estimate of n hosts in its
// pinned staging, after the addresses.
struct OutLayout {
    uint64_t est, plain, flags, total;
};
OutLayout out_layout(uint64_t n) {
    OutLayout O{};
    O.est = 0;
    O.plain = up64(8 * n);
    O.flags = up64(O.plain + 8 * n);
    O.total = up64(O.flags + n);
    return O;
}

int ensure_query(at_ctx* h, uint64_t n) {
    if (n <= h->q_cap) return AT_OK;
    // a pending split estimate still reads and writes these buffers
    if (h->q_pending && hipEventSynchronize(h->q_done) != hipSuccess) return AT_E_DEVICE;
    uint64_t cap = std::max<uint64_t>(n, 1024);
    if (h->q_aip) (void)hipFree(h->q_aip);
    if (h->q_est) (void)hipFree(h->q_est);
    if (h->q_flags) (void)hipFree(h->q_flags);
    if (h->q_nat) (void)hipFree(h->q_nat);
    if (h->q_feat) (void)hipFree(h->q_feat);
    if (h->q_plain) (void)hipFree(h->q_plain);
    h->q_aip = nullptr;
    h->q_est = nullptr;
    h->q_flags = nullptr;
    h->q_nat = nullptr;
    h->q_feat = nullptr;
    h->q_plain = nullptr;
    h->q_cap = 0;
    int rc;
    if ((rc = dev_alloc(&h->q_aip, cap)) || (rc = dev_alloc(&h->q_est, cap)) || (rc = dev_alloc(&h->q_flags, cap)) ||
        (rc = dev_alloc(&h->q_nat, cap)) || (rc = dev_alloc(&h->q_feat, cap * 64)) ||
        (rc = dev_alloc(&h->q_plain, cap)))
        return rc;
    h->q_cap = cap;
    return AT_OK;
}

uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a > UINT64_MAX / b) return UINT64_MAX;
    return a * b;
}

// Pinned staging: copies between the caller's (pageable) host buffers and the
// device go through it, so they run as asynchronous DMA and one call waits
// once.  Grown on demand; one region per field.
int ensure_pinned(at_ctx* h, uint64_t bytes) {
    if (bytes <= h->pin_cap) return AT_OK;
    if (h->pin) (void)hipHostFree(h->pin);
    h->pin = nullptr;
    h->pin_cap = 0;
    const uint64_t cap = std::max<uint64_t>((bytes + 65535) & ~65535ull, 1u << 20);
    if (hipHostMalloc((void**)&h->pin, cap, hipHostMallocDefault) != hipSuccess) {
        h->pin = nullptr;
        (void)hipGetLastError();
        return AT_E_NOMEM;
    }
    h->pin_cap = cap;
    return AT_OK;
}

// Byte offsets of the staging regions for n hosts (64-byte aligned).
struct PinLayout {
    uint64_t aip, est, nat, flags, total;
};
PinLayout pin_layout(uint64_t n) {
    PinLayout L{};
    L.aip = 0;
    L.est = up64(L.aip + 4 * n);
    L.nat = up64(L.est + 8 * n);
    L.flags = up64(L.nat + 4 * n);
    L.total = up64(L.flags + n);
    return L;
}

// The selected window's super-ATV counts, as the last close's summary stored them in mapped host memory.
int read_counts(at_ctx* h, std::vector<uint32_t>& cnt) {
    cnt.assign(h->ngroups, 0);
    const hipError_t e = hipEventSynchronize(h->cnt_ready);
    if (e != hipSuccess) return dev_err(e);
    std::memcpy(cnt.data(), h->pin_cnt + (h->sa_cnt - h->sa_cnt_all), h->ngroups * sizeof(uint32_t));
    return AT_OK;
}

// Room for the counts of n windows; waits for the last summary's stores into the old buffer first.
int ensure_pin_cnt(at_ctx* h, uint64_t entries) {
    if (entries <= h->pin_cnt_cap) return AT_OK;
    if (h->pin_cnt) {
        if (hipEventSynchronize(h->cnt_ready) != hipSuccess) return AT_E_DEVICE;
        (void)hipHostFree(h->pin_cnt);
    }
    h->pin_cnt = h->pin_cnt_dev = nullptr;
    h->pin_cnt_cap = 0;
    if (hipHostMalloc((void**)&h->pin_cnt, entries * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        h->pin_cnt = nullptr;
        (void)hipGetLastError();
        return AT_E_NOMEM;
    }
    if (hipHostGetDevicePointer((void**)&h->pin_cnt_dev, h->pin_cnt, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h->pin_cnt);
        h->pin_cnt = h->pin_cnt_dev = nullptr;
        return AT_E_DEVICE;
    }
    h->pin_cnt_cap = entries;
    return AT_OK;
}

// Staging of the split learned estimate; only grown while none is pending.
int ensure_pin_q(at_ctx* h, uint64_t bytes) {
    if (bytes <= h->pin_q_cap) return AT_OK;
    if (h->pin_q) (void)hipHostFree(h->pin_q);
    h->pin_q = h->pin_q_dev = nullptr;
    h->pin_q_cap = 0;
    const uint64_t cap = std::max<uint64_t>((bytes + 65535) & ~65535ull, 1u << 16);
    if (hipHostMalloc((void**)&h->pin_q, cap, hipHostMallocDefault) != hipSuccess) {
        h->pin_q = nullptr;
        (void)hipGetLastError();
        return AT_E_NOMEM;
    }
    if (hipHostGetDevicePointer((void**)&h->pin_q_dev, h->pin_q, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h->pin_q);
        h->pin_q = h->pin_q_dev = nullptr;
        return AT_E_DEVICE;
    }
    h->pin_q_cap = cap;
    return AT_OK;
}

uint64_t tuple_count(const at_ctx* h, const std::vector<uint32_t>& cnt) {
    uint64_t total = 0;
    for (uint32_t z = 0; z < h->nframe; z++) {
        uint64_t prod = 1;
        for (uint32_t j = 0; j < h->p.r; j++) prod = sat_mul(prod, cnt[(uint64_t)z * h->p.r + j]);
        total = (UINT64_MAX - total < prod) ? UINT64_MAX : total + prod;
    }
    return total;
}

}  // namespace

namespace atp {

int validate_params(const at_params& p) { return validate(p); }

// Hash constants and block layout of a handle, from its parameters (Section 3,
// Section 4.1); at_create and the streaming server both use it.
Geometry derive_geometry(const at_params& p) {
    Geometry G{};
    G.k = p.k;
    G.twok = 2 * p.k;
    G.atb = G.twok < 256 ? 1 : 2;  // AT bytes: 2k + 1 values per AT
    G.r = p.r;
    G.c = p.c;
    G.s = p.s;
    G.u = p.u;
    G.W = 32 - p.u;
    G.log2g = p.log2g;
    G.g = 1u << p.log2g;
    G.ncol_mask = (1u << p.c) - 1u;
    G.umask = (1u << p.u) - 1u;
    uint64_t st = p.seed;
    const uint64_t x0 = splitmix_next(st), x1 = splitmix_next(st), x2 = splitmix_next(st);
    const uint64_t A = (1ull << 31) + x0 % (atp::kPrime - (1ull << 31));
    G.A = (uint32_t)A;
    G.Ainv = (uint32_t)pow_mod_p(A, atp::kPrime - 2);
    G.alpha = x1 | 1ull;
    G.beta = x2;
    G.blk_a = G.g / G.twok;
    G.last_blk = G.twok - 1;
    G.blk_magic = G.blk_a ? (((1ull << 32) + G.blk_a - 1) / G.blk_a) : 0;
    G.maskW = G.W == 32 ? 0xFFFFFFFFull : ((1ull << G.W) - 1);
    for (uint32_t j = 0; j < (uint32_t)atp::kMaxRows; j++) {
        G.sh[j] = j < p.r ? (p.s * j) % G.W : 0;
        if (j < p.r) {
            uint64_t t = (uint64_t)G.ncol_mask << G.sh[j];
            G.win[j] = (uint32_t)((t | (t >> G.W)) & G.maskW);
        }
    }
    // Section 4.2: super ATVs hold at least g - g*exp(-theta/g) active ATs
    const double thr = (double)G.g - (double)G.g * std::exp(-p.theta / (double)G.g);
    double Tc = std::ceil(thr);
    if (Tc < 0) Tc = 0;
    G.T = (uint32_t)Tc;
    G.theta = p.theta;
    return G;
}

}  // namespace atp

extern "C" {

const char* at_strerror(int rc) {
    switch (rc) {
        case AT_OK: return "ok";
        case AT_E_INVAL: return "invalid argument";
        case AT_E_STATE: return "call not valid in the current state";
        case AT_E_NOMEM: return "out of memory";
        case AT_E_OVERFLOW: return "result exceeds capacity";
        case AT_E_DEVICE: return "HIP device error";
        case AT_E_BUDGET: return "restore tuple budget exceeded";
        default: return "unknown error";
    }
}

int at_create(const at_params* p, void* hip_stream, at_ctx** out) {
    if (!out) return AT_E_INVAL;
    *out = nullptr;
    if (!p) return AT_E_INVAL;
    int rc = validate(*p);
    if (rc) return rc;
    at_ctx* h = new (std::nothrow) at_ctx();
    if (!h) return AT_E_NOMEM;
    h->p = *p;
    if (h->p.tuple_budget == 0) h->p.tuple_budget = 1ull << 32;
    h->G = atp::derive_geometry(h->p);
    h->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return AT_E_DEVICE;
    }
    h->scratch_dev = scratch_on(h->device);  // null: at_ingest_slice_noalloc answers AT_E_DEVICE
    h->nframe = 1u << p->u;
    h->ngroups = h->nframe * p->r;
    h->n_atv = (uint64_t)h->ngroups << p->c;
    h->pool_bytes = (h->n_atv << p->log2g) * h->G.atb;
    const uint64_t W = atp::kMaxWindows;
    if ((rc = dev_alloc(&h->pool, h->pool_bytes)) || (rc = dev_alloc(&h->w_all, W * h->n_atv)) ||
        (rc = dev_alloc(&h->aat_all, W * h->ngroups)) || (rc = dev_alloc(&h->sa_all, W * h->n_atv)) ||
        (rc = dev_alloc(&h->sa_cnt_all, W * h->ngroups)) || (rc = dev_alloc(&h->counter, 1)) ||
        (rc = dev_alloc(&h->prefix, h->nframe + 1))) {
        free_all(h);
        delete h;
        return rc;
    }
    if (hipEventCreateWithFlags(&h->cnt_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->q_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        free_all(h);
        delete h;
        return AT_E_DEVICE;
    }
    if ((rc = ensure_pin_cnt(h, h->ngroups))) {
        free_all(h);
        delete h;
        return rc;
    }
    // InitAT (Section 3): every AT starts inactive
    hipError_t e = atp::launch_fill_pool(h->pool, h->n_atv << p->log2g, h->G, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return AT_E_DEVICE;
    }
    h->w = h->w_all;
    h->aat = h->aat_all;
    h->sa = h->sa_all;
    h->sa_cnt = h->sa_cnt_all;
    int lds = 0;
    h->tiled_ok = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess &&
                  (size_t)lds >= atp::tiled_lds_bytes(4096) + 1024;
    *out = h;
    return AT_OK;
}

int at_destroy(at_ctx* h) {
    if (!h) return AT_OK;
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return AT_OK;
}

// The binned scan pays two extra 8-byte passes per pair to keep each XCD's
// byte stores inside one (frame group, row) region; worth it when the pool is
// far larger than an L2 and there are at least 8 frames.
constexpr uint64_t kBinBatch = 8u << 20;  // pairs per binned sub-batch

// The tiled scan reads and writes the whole pool once per call, so it pays
// when the call's r*n byte stores are many next to the pool: each random
// store costs a partial-line write-back of about 30 bytes otherwise.
enum ScanPath { kDirect = 1, kBinned = 2, kTiled = 3 };

int scan_path(const at_ctx* h, uint64_t n) {
    if (h->scan_mode != 0) return h->scan_mode;
    if (h->tiled_ok && atp::tiled_fits(h->pool_bytes) && n * h->p.r * 12 >= h->pool_bytes) return kTiled;
    if (h->p.u >= 3 && h->pool_bytes >= (32ull << 20) && n >= 65536) return kBinned;
    return kDirect;
}

int ingest_tiled_buffers(at_ctx* h, uint64_t n);

// The tiled launches of a call with the given scratch.
int ingest_tiled_with(at_ctx* h, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n, bool preserve,
                      const atp::TileBufs& tb) {
    // a single batch that opens the slice also writes the full window's weights
    const bool weights = preserve && n <= kBinBatch;
    for (uint64_t off = 0; off < n; off += kBinBatch) {
        const uint64_t m = std::min<uint64_t>(kBinBatch, n - off);
        if (atp::launch_ingest_tiled(h->pool, aip_dev + off, bip_dev + off, m, h->pool_bytes, h->G, h->c0, tb,
                                     preserve && off == 0, weights ? h->w_all : nullptr, h->p.k,
                                     h->stream) != hipSuccess)
            return AT_E_DEVICE;
    }
    h->wfused = weights;
    h->wfused_kq = h->p.k;
    return AT_OK;
}

int ingest_tiled(at_ctx* h, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n, bool preserve) {
    int rc = ingest_tiled_buffers(h, n);
    if (rc) {
        // the slice is open already: its preserve must not be lost
        if (preserve && atp::launch_preserve(h->pool, h->n_atv, h->G, h->c0, h->stream) != hipSuccess)
            return AT_E_DEVICE;
        return rc;
    }
    return ingest_tiled_with(h, aip_dev, bip_dev, n, preserve, h->tb);
}

int ingest_tiled_buffers(at_ctx* h, uint64_t n) {
    int rc;
    const atp::TileSizes z = atp::tiled_sizes(std::min<uint64_t>(n, kBinBatch), h->pool_bytes, h->G);
    if (z.recs > h->tb.rec_cap) {
        if (h->tb.rec) (void)hipFree(h->tb.rec);
        h->tb.rec = nullptr;
        h->tb.rec_cap = 0;
        if ((rc = dev_alloc(&h->tb.rec, z.recs))) return rc;
        h->tb.rec_cap = z.recs;
    }
    if (z.table > h->tb.table_cap) {
        if (h->tb.cnt) (void)hipFree(h->tb.cnt);
        if (h->tb.pre) (void)hipFree(h->tb.pre);
        h->tb.cnt = nullptr;
        h->tb.pre = nullptr;
        h->tb.table_cap = 0;
        if ((rc = dev_alloc(&h->tb.cnt, z.table)) || (rc = dev_alloc(&h->tb.pre, z.table))) return rc;
        h->tb.table_cap = z.table;
    }
    if (z.nchunk + 2 > h->tb.chunk_cap) {
        if (h->tb.csum) (void)hipFree(h->tb.csum);
        h->tb.csum = nullptr;
        h->tb.chunk_cap = 0;
        if ((rc = dev_alloc(&h->tb.csum, (uint64_t)(z.nchunk + 2) * 4096))) return rc;
        h->tb.chunk_cap = z.nchunk + 2;
    }
    if (!h->tb.base && (rc = dev_alloc(&h->tb.base, 4097))) return rc;
    if (!h->tb.act && (rc = dev_alloc(&h->tb.act, (uint64_t)h->G.g * h->G.atb))) return rc;
    return AT_OK;
}

int at_ingest_slice(at_ctx* h, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n) {
    if (!h) return AT_E_INVAL;
    if (n > 0) {
        if (!aip_dev || !bip_dev) return AT_E_INVAL;
        if (!device_accessible(aip_dev) || !device_accessible(bip_dev)) return AT_E_INVAL;
    }
    const int path = n ? scan_path(h, n) : 0;
    // a tiled call that opens the slice runs the opening preserve in its tile pass
    const bool fuse = !h->open && path == kTiled;
    int rc = open_slice(h, fuse);
    if (rc) return rc;
    if (n == 0) return AT_OK;
    h->wfused = false;  // any stores after the fused count make it stale
    if (path == kTiled) return ingest_tiled(h, aip_dev, bip_dev, n, fuse);
    if (path == kDirect)
        return atp::launch_ingest(h->pool, aip_dev, bip_dev, n, h->G, h->c0, h->stream) == hipSuccess ? AT_OK
                                                                                                     : AT_E_DEVICE;
    const uint64_t sub_cap = atp::binned_sub_cap(std::min<uint64_t>(n, kBinBatch));
    if (sub_cap > h->bins_cap) {
        if (h->bins) (void)hipFree(h->bins);
        h->bins = nullptr;
        h->bins_cap = 0;
        if ((rc = dev_alloc(&h->bins, (uint64_t)atp::kScanBins * atp::kScanSubs * sub_cap))) return rc;
        h->bins_cap = sub_cap;
    }
    if (!h->bin_fill && (rc = dev_alloc(&h->bin_fill, atp::kScanBins * atp::kScanSubs))) return rc;
    for (uint64_t off = 0; off < n; off += kBinBatch) {
        const uint64_t m = std::min<uint64_t>(kBinBatch, n - off);
        if (atp::launch_ingest_binned(h->pool, aip_dev + off, bip_dev + off, m, h->G, h->c0, h->bins, h->bins_cap,
                                      h->bin_fill, h->stream) != hipSuccess)
            return AT_E_DEVICE;
    }
    return AT_OK;
}

int at_ingest_slice_noalloc(at_ctx* h, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n) {
    if (!h || n > AT_NOALLOC_MAX_PAIRS) return AT_E_INVAL;
    if (n > 0) {
        if (!aip_dev || !bip_dev) return AT_E_INVAL;
        if (!device_accessible(aip_dev) || !device_accessible(bip_dev)) return AT_E_INVAL;
    }
    int path = n ? scan_path(h, n) : 0;
    if (path == kBinned) path = kDirect;  // the binned scan's bins are not in the scratch array
    atp::TileBufs tb{};
    if (path == kTiled) {
        // checked before the slice opens: a tiled call that opens it owns its preserve
        if (!h->scratch_dev) return AT_E_DEVICE;
        const atp::TileSizes z = atp::tiled_sizes(n, h->pool_bytes, h->G);
        if (carve_tiles(h->scratch_dev, z, h->G, &tb) > AT_NOALLOC_SCRATCH_BYTES) return AT_E_INVAL;
    }
    const bool fuse = !h->open && path == kTiled;
    int rc = open_slice(h, fuse);
    if (rc) return rc;
    if (n == 0) return AT_OK;
    h->wfused = false;
    if (path == kTiled) return ingest_tiled_with(h, aip_dev, bip_dev, n, fuse, tb);
    return atp::launch_ingest(h->pool, aip_dev, bip_dev, n, h->G, h->c0, h->stream) == hipSuccess ? AT_OK
                                                                                                 : AT_E_DEVICE;
}

int at_set_scan_mode(at_ctx* h, int mode) {
    if (!h || mode < 0 || mode > 3) return AT_E_INVAL;
    if (mode == 3 && !(h->tiled_ok && atp::tiled_fits(h->pool_bytes))) return AT_E_INVAL;
    h->scan_mode = mode;
    return AT_OK;
}

namespace {
void use_window(at_ctx* h, uint32_t j) {
    h->w = h->w_all + (uint64_t)j * h->n_atv;
    h->aat = h->aat_all + (uint64_t)j * h->ngroups;
    h->sa = h->sa_all + (uint64_t)j * h->n_atv;
    h->sa_cnt = h->sa_cnt_all + (uint64_t)j * h->ngroups;
    h->kq = h->win_kq[j];
}
}  // namespace

int at_close_slice_multi(at_ctx* h, const uint32_t* kprimes, uint32_t n) {
    if (!h || !kprimes || n < 1 || n > atp::kMaxWindows) return AT_E_INVAL;
    atp::CloseWindows Wn{};
    Wn.n = n;
    for (uint32_t j = 0; j < n; j++) {
        if (kprimes[j] < 1 || kprimes[j] > h->p.k) return AT_E_INVAL;
        Wn.kq[j] = kprimes[j];
    }
    int rc = ensure_pin_cnt(h, (uint64_t)n * h->ngroups);
    if (rc) return rc;
    rc = open_slice(h);
    if (rc) return rc;
    // the slice's one tiled call already counted window k: no pass over the pool
    const bool counted = n == 1 && h->wfused && kprimes[0] == h->wfused_kq;
    h->wfused = false;
    h->hist_valid = false;
    hipError_t e = counted ? hipSuccess
                           : atp::launch_close(h->pool, h->w_all, h->n_atv, h->G, h->c0, Wn, h->stream);
    if (e == hipSuccess)
        e = atp::launch_summarize(h->w_all, h->aat_all, h->sa_all, h->sa_cnt_all, h->pin_cnt_dev, h->G, h->n_atv, n,
                                  h->stream);
    if (e == hipSuccess) e = hipEventRecord(h->cnt_ready, h->stream);
    if (e != hipSuccess) return AT_E_DEVICE;
    h->nwin = n;
    for (uint32_t j = 0; j < n; j++) h->win_kq[j] = kprimes[j];
    h->c0_query = h->c0;
    use_window(h, 0);
    h->t += 1;
    h->open = false;
    h->queryable = true;
    return AT_OK;
}

int at_close_slice(at_ctx* h, uint32_t kprime) {
    if (!h) return AT_E_INVAL;
    return at_close_slice_multi(h, &kprime, 1);
}

int at_close_slice_hist(at_ctx* h, uint32_t kprime) {
    static_assert(atp::kHistMaxK == AT_HIST_MAX_K, "one histogram limit");
    if (!h || kprime < 1 || kprime > h->p.k || h->p.k > AT_HIST_MAX_K) return AT_E_INVAL;
    int rc = ensure_pin_cnt(h, h->ngroups);
    if (rc) return rc;
    if (!h->hist && (rc = dev_alloc(&h->hist, h->n_atv * h->p.k))) return rc;
    rc = open_slice(h);
    if (rc) return rc;
    h->wfused = false;
    h->hist_valid = false;
    hipError_t e = atp::launch_close_hist(h->pool, h->hist, h->w_all, h->n_atv, h->G, h->c0, kprime, h->stream);
    if (e == hipSuccess)
        e = atp::launch_summarize(h->w_all, h->aat_all, h->sa_all, h->sa_cnt_all, h->pin_cnt_dev, h->G, h->n_atv, 1,
                                  h->stream);
    if (e == hipSuccess) e = hipEventRecord(h->cnt_ready, h->stream);
    if (e != hipSuccess) return AT_E_DEVICE;
    h->nwin = 1;
    h->win_kq[0] = kprime;
    h->c0_query = h->c0;
    use_window(h, 0);
    h->t += 1;
    h->open = false;
    h->queryable = true;
    h->hist_valid = true;
    return AT_OK;
}

int at_requery_window(at_ctx* h, uint32_t kprime) {
    if (!h || kprime < 1 || kprime > h->p.k) return AT_E_INVAL;
    if (!h->queryable || !h->hist_valid) return AT_E_STATE;
    hipError_t e = atp::launch_hist_weights(h->hist, h->p.k, h->n_atv, kprime, h->w_all, h->stream);
    if (e == hipSuccess)
        e = atp::launch_summarize(h->w_all, h->aat_all, h->sa_all, h->sa_cnt_all, h->pin_cnt_dev, h->G, h->n_atv, 1,
                                  h->stream);
    if (e == hipSuccess) e = hipEventRecord(h->cnt_ready, h->stream);
    if (e != hipSuccess) return AT_E_DEVICE;
    h->nwin = 1;
    h->win_kq[0] = kprime;
    use_window(h, 0);
    return AT_OK;
}

int at_read_age_hist(at_ctx* h, uint16_t* host_out) {
    if (!h || !host_out) return AT_E_INVAL;
    if (!h->queryable || !h->hist_valid) return AT_E_STATE;
    hipError_t e = hipMemcpyAsync(host_out, h->hist, h->n_atv * h->p.k * sizeof(uint16_t), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return dev_err(e);
}

int at_select_window(at_ctx* h, uint32_t kprime) {
    if (!h) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    for (uint32_t j = 0; j < h->nwin; j++)
        if (h->win_kq[j] == kprime) {
            use_window(h, j);
            return AT_OK;
        }
    return AT_E_INVAL;
}

int at_estimate_dev(at_ctx* h, const uint32_t* aip_dev, uint64_t n, double* est_dev, uint8_t* flags_dev,
                    uint32_t* nat_dev) {
    if (!h) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    if (n == 0) return AT_OK;
    if (!aip_dev) return AT_E_INVAL;
    hipError_t e = atp::launch_estimate(h->pool, h->aat, aip_dev, n, h->G, h->c0_query, h->kq, est_dev, flags_dev,
                                        nat_dev, h->stream);
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int at_estimate_detail(at_ctx* h, const uint32_t* aip_host, uint64_t n, double* est_out, uint8_t* flags_out,
                       uint32_t* nat_out) {
    if (!h) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    if (n == 0) return AT_OK;
    if (!aip_host) return AT_E_INVAL;
    int rc = ensure_query(h, n);
    const PinLayout L = pin_layout(n);
    if (!rc) rc = ensure_pinned(h, L.total);
    if (rc) return rc;
    std::memcpy(h->pin + L.aip, aip_host, n * sizeof(uint32_t));
    hipError_t e = hipMemcpyAsync(h->q_aip, h->pin + L.aip, n * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = atp::launch_estimate(h->pool, h->aat, h->q_aip, n, h->G, h->c0_query, h->kq, h->q_est, h->q_flags,
                                 h->q_nat, h->stream);
    if (e == hipSuccess && est_out)
        e = hipMemcpyAsync(h->pin + L.est, h->q_est, n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && flags_out)
        e = hipMemcpyAsync(h->pin + L.flags, h->q_flags, n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && nat_out)
        e = hipMemcpyAsync(h->pin + L.nat, h->q_nat, n * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_err(e);
    if (est_out) std::memcpy(est_out, h->pin + L.est, n * sizeof(double));
    if (flags_out) std::memcpy(flags_out, h->pin + L.flags, n);
    if (nat_out) std::memcpy(nat_out, h->pin + L.nat, n * sizeof(uint32_t));
    return AT_OK;
}

int at_estimate(at_ctx* h, const uint32_t* aip_host, uint64_t n, double* est_out, uint8_t* flags_out) {
    return at_estimate_detail(h, aip_host, n, est_out, flags_out, nullptr);
}

int at_tuple_count(at_ctx* h, uint64_t* U) {
    if (!h || !U) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    std::vector<uint32_t> cnt;
    int rc = read_counts(h, cnt);
    if (rc) return rc;
    *U = tuple_count(h, cnt);
    return AT_OK;
}

int at_restore(at_ctx* h, uint32_t* sip_out, double* est_out, uint8_t* flags_out, uint64_t cap, uint64_t* n_out) {
    if (!h || !n_out) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    std::vector<uint32_t> cnt;
    int rc = read_counts(h, cnt);
    if (rc) return rc;
    const uint64_t U = tuple_count(h, cnt);
    if (U > h->p.tuple_budget) {
        *n_out = U;
        return AT_E_BUDGET;
    }
    // work items: (x0, x1) pairs per frame (single columns when r == 1)
    std::vector<uint64_t> prefix(h->nframe + 1, 0);
    for (uint32_t z = 0; z < h->nframe; z++) {
        uint64_t items = cnt[(uint64_t)z * h->p.r];
        if (h->p.r >= 2) items *= cnt[(uint64_t)z * h->p.r + 1];
        bool empty = false;
        for (uint32_t j = 0; j < h->p.r; j++) empty |= cnt[(uint64_t)z * h->p.r + j] == 0;
        prefix[z + 1] = prefix[z] + (empty ? 0 : items);
    }
    const uint64_t n_items = prefix[h->nframe];
    // candidates are at most U (distinct tuples give distinct addresses)
    uint64_t need = std::min<uint64_t>(U, cap);
    uint64_t pow2 = 1;
    while (pow2 < need) pow2 <<= 1;
    if (pow2 > h->cand_cap) {
        if (h->cand) (void)hipFree(h->cand);
        h->cand = nullptr;
        h->cand_cap = 0;
        if ((rc = dev_alloc(&h->cand, pow2))) return rc;
        h->cand_cap = pow2;
    }
    const uint64_t pre_bytes = prefix.size() * sizeof(uint64_t);
    if ((rc = ensure_pinned(h, pre_bytes + 64))) return rc;
    std::memcpy(h->pin + 64, prefix.data(), pre_bytes);
    hipError_t e = hipMemcpyAsync(h->prefix, h->pin + 64, pre_bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = atp::launch_zero_u64(h->counter, 1, h->stream);
    if (e == hipSuccess)
        e = atp::launch_restore_join(h->sa, h->sa_cnt, h->prefix, n_items, h->G, h->cand, need, h->counter,
                                     h->stream);
    unsigned long long m = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(h->pin, h->counter, sizeof(m), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_err(e);
    std::memcpy(&m, h->pin, sizeof(m));
    *n_out = m;
    if (m > cap) return AT_E_OVERFLOW;
    if (m == 0) return AT_OK;
    uint64_t mp2 = 1;
    while (mp2 < m) mp2 <<= 1;
    if ((rc = ensure_query(h, m))) return rc;
    const PinLayout L = pin_layout(m);  // candidates in the aip region
    if ((rc = ensure_pinned(h, L.total))) return rc;
    e = atp::launch_sort_u32(h->cand, m, mp2, h->stream);
    if (e == hipSuccess && (est_out || flags_out))
        e = atp::launch_estimate(h->pool, h->aat, h->cand, m, h->G, h->c0_query, h->kq, h->q_est, h->q_flags,
                                 nullptr, h->stream);
    if (e == hipSuccess && sip_out)
        e = hipMemcpyAsync(h->pin + L.aip, h->cand, m * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && est_out)
        e = hipMemcpyAsync(h->pin + L.est, h->q_est, m * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && flags_out)
        e = hipMemcpyAsync(h->pin + L.flags, h->q_flags, m, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_err(e);
    if (sip_out) std::memcpy(sip_out, h->pin + L.aip, m * sizeof(uint32_t));
    if (est_out) std::memcpy(est_out, h->pin + L.est, m * sizeof(double));
    if (flags_out) std::memcpy(flags_out, h->pin + L.flags, m);
    return AT_OK;
}

int at_pool_info(const at_ctx* h, uint64_t* pool_bytes, uint64_t* n_atv) {
    if (!h) return AT_E_INVAL;
    if (pool_bytes) *pool_bytes = h->pool_bytes;
    if (n_atv) *n_atv = h->n_atv;
    return AT_OK;
}

int at_read_pool(at_ctx* h, uint8_t* host_out) {
    if (!h || !host_out) return AT_E_INVAL;
    hipError_t e = hipMemcpyAsync(host_out, h->pool, h->pool_bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return dev_err(e);
}

int at_read_summary(at_ctx* h, uint32_t* w_host, uint64_t* aat_host) {
    if (!h) return AT_E_INVAL;
    if (h->t == 0) return AT_E_STATE;
    hipError_t e = hipSuccess;
    if (w_host) e = hipMemcpyAsync(w_host, h->w, h->n_atv * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && aat_host)
        e = hipMemcpyAsync(aat_host, h->aat, h->ngroups * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return dev_err(e);
}

int at_clock(const at_ctx* h, uint64_t* out5) {
    if (!h || !out5) return AT_E_INVAL;
    out5[0] = h->t;
    out5[1] = h->open;
    out5[2] = h->queryable;
    out5[3] = h->c0_query;
    out5[4] = h->kq;
    return AT_OK;
}

int at_constants(const at_ctx* h, uint64_t* out8) {
    if (!h || !out8) return AT_E_INVAL;
    out8[0] = atp::kPrime;
    out8[1] = h->G.A;
    out8[2] = h->G.Ainv;
    out8[3] = h->G.alpha;
    out8[4] = h->G.beta;
    out8[5] = h->G.T;
    out8[6] = h->G.W;
    out8[7] = h->G.blk_a;
    return AT_OK;
}

int at_probe_scatter(uint8_t* dst_dev, uint64_t bytes, const uint32_t* a_dev, const uint32_t* b_dev, uint64_t n,
                     uint32_t r, void* hip_stream) {
    if (!dst_dev || !a_dev || !b_dev || bytes == 0 || (bytes & (bytes - 1)) || (n % 4) ||
        ((reinterpret_cast<uintptr_t>(a_dev) | reinterpret_cast<uintptr_t>(b_dev)) & 15u))
        return AT_E_INVAL;
    if (!(r == 1 || r == 2 || r == 4 || r == 8)) return AT_E_INVAL;
    if (!device_accessible(dst_dev) || !device_accessible(a_dev) || !device_accessible(b_dev)) return AT_E_INVAL;
    return atp::launch_scatter_probe(dst_dev, bytes, a_dev, b_dev, n, r, (hipStream_t)hip_stream) == hipSuccess
               ? AT_OK
               : AT_E_DEVICE;
}

}  // extern "C"

// ============================================================== learned correction

struct at_mlp {
    hipStream_t stream = nullptr;
    float* w = nullptr;  // FP32 master parameters (kMlpParams)
    float* m = nullptr;  // Adam moments
    float* v = nullptr;
    uint16_t* W1b = nullptr;
    uint16_t* W2b = nullptr;
    uint16_t* W2Tb = nullptr;
    uint16_t* w3b = nullptr;
    float* loss = nullptr;
    uint64_t step = 0;
    atp::MlpScratch S{};
    uint64_t s_rows = 0;
};

namespace {

atp::MlpDev mlp_dev(const at_mlp* M) {
    return atp::MlpDev{M->W1b, M->w + atp::kOffB1, M->W2b, M->w + atp::kOffB2, M->w3b, M->w + atp::kOffB3, M->W2Tb};
}

atp::MlpOut mlp_out(at_mlp* M) { return atp::MlpOut{M->W1b, M->W2b, M->W2Tb, M->w3b}; }

void mlp_free_scratch(at_mlp* M) {
    void* b[] = {M->S.XT, M->S.H1T, M->S.H2T, M->S.dH1T, M->S.dH2T, M->S.y, M->S.dy, M->S.partial, M->S.grad};
    for (void* p : b)
        if (p) (void)hipFree(p);
    M->S = atp::MlpScratch{};
    M->s_rows = 0;
}

int mlp_ensure(at_mlp* M, uint64_t nrows) {
    if (nrows <= M->s_rows) return AT_OK;
    mlp_free_scratch(M);
    int rc;
    const uint64_t T = 64 * nrows;
    if ((rc = dev_alloc(&M->S.XT, T)) || (rc = dev_alloc(&M->S.H1T, T)) || (rc = dev_alloc(&M->S.H2T, T)) ||
        (rc = dev_alloc(&M->S.dH1T, T)) || (rc = dev_alloc(&M->S.dH2T, T)) || (rc = dev_alloc(&M->S.y, nrows)) ||
        (rc = dev_alloc(&M->S.dy, nrows)) || (rc = dev_alloc(&M->S.partial, nrows / atp::kMlpChunk * atp::kMlpParams)) ||
        (rc = dev_alloc(&M->S.grad, atp::kMlpParams))) {
        mlp_free_scratch(M);
        return rc;
    }
    M->s_rows = nrows;
    return AT_OK;
}

// forward + backward + reduction into M->S.grad (and optionally the loss)
int mlp_grad(at_mlp* M, const float* x_dev, const float* t_dev, uint64_t n) {
    const uint64_t nrows = (n + atp::kMlpChunk - 1) / atp::kMlpChunk * atp::kMlpChunk;
    int rc = mlp_ensure(M, nrows);
    if (rc) return rc;
    hipError_t e = atp::launch_mlp_train_fwd_bwd(x_dev, t_dev, n, nrows, mlp_dev(M), M->S, M->stream);
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int mlp_adam(at_mlp* M, const float* grad, float lr) {
    M->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    atp::AdamConst C{lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2),
                     (float)(1.0 - std::pow(b1, (double)M->step)), (float)(1.0 - std::pow(b2, (double)M->step)), 1e-8f};
    return atp::launch_mlp_adam(M->w, M->m, M->v, grad, C, mlp_out(M), M->stream) == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int read_loss(at_mlp* M, const float* t_dev, uint64_t n, float* loss_host) {
    hipError_t e = atp::launch_mlp_loss(M->S.y, t_dev, n, M->loss, M->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(loss_host, M->loss, sizeof(float), hipMemcpyDeviceToHost, M->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
    return dev_err(e);
}

}  // namespace

namespace atp {
bool mlp_operands(const at_mlp* m, MlpDev* out) {
    if (!m) return false;
    *out = mlp_dev(m);
    return true;
}
}  // namespace atp

extern "C" {

int at_mlp_create(void* hip_stream, at_mlp** out) {
    if (!out) return AT_E_INVAL;
    *out = nullptr;
    at_mlp* M = new (std::nothrow) at_mlp();
    if (!M) return AT_E_NOMEM;
    M->stream = (hipStream_t)hip_stream;
    int rc;
    if ((rc = dev_alloc(&M->w, atp::kMlpParams)) || (rc = dev_alloc(&M->m, atp::kMlpParams)) ||
        (rc = dev_alloc(&M->v, atp::kMlpParams)) || (rc = dev_alloc(&M->W1b, 64 * 64)) ||
        (rc = dev_alloc(&M->W2b, 64 * 64)) || (rc = dev_alloc(&M->W2Tb, 64 * 64)) || (rc = dev_alloc(&M->w3b, 64)) ||
        (rc = dev_alloc(&M->loss, 1))) {
        at_mlp_destroy(M);
        return rc;
    }
    std::vector<float> zero(atp::kMlpParams, 0.0f);
    hipError_t e = hipMemcpyAsync(M->w, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M->m, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M->v, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = atp::launch_mlp_refresh(M->w, mlp_out(M), M->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
    if (e != hipSuccess) {
        at_mlp_destroy(M);
        return AT_E_DEVICE;
    }
    *out = M;
    return AT_OK;
}

int at_mlp_destroy(at_mlp* M) {
    if (!M) return AT_OK;
    (void)hipStreamSynchronize(M->stream);
    mlp_free_scratch(M);
    void* b[] = {M->w, M->m, M->v, M->W1b, M->W2b, M->W2Tb, M->w3b, M->loss};
    for (void* p : b)
        if (p) (void)hipFree(p);
    delete M;
    return AT_OK;
}

int at_mlp_set_params(at_mlp* M, const float* host_params) {
    if (!M || !host_params) return AT_E_INVAL;
    std::vector<float> zero(atp::kMlpParams, 0.0f);
    hipError_t e = hipMemcpyAsync(M->w, host_params, atp::kMlpParams * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M->m, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(M->v, zero.data(), zero.size() * 4, hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) e = atp::launch_mlp_refresh(M->w, mlp_out(M), M->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
    M->step = 0;
    return dev_err(e);
}

int at_mlp_get_params(at_mlp* M, float* host_params) {
    if (!M || !host_params) return AT_E_INVAL;
    hipError_t e = hipMemcpyAsync(host_params, M->w, atp::kMlpParams * 4, hipMemcpyDeviceToHost, M->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
    return dev_err(e);
}

int at_mlp_forward(at_mlp* M, const float* x_dev, uint64_t n, float* y_dev) {
    if (!M || (n && (!x_dev || !y_dev))) return AT_E_INVAL;
    return atp::launch_mlp_forward(x_dev, n, mlp_dev(M), y_dev, M->stream) == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int at_mlp_grad(at_mlp* M, const float* x_dev, const float* t_dev, uint64_t n, float* grad_dev, float* loss_host) {
    if (!M || !x_dev || !t_dev || n == 0) return AT_E_INVAL;
    int rc = mlp_grad(M, x_dev, t_dev, n);
    if (rc) return rc;
    if (grad_dev) {
        hipError_t e = hipMemcpyAsync(grad_dev, M->S.grad, atp::kMlpParams * 4, hipMemcpyDeviceToDevice, M->stream);
        if (e != hipSuccess) return AT_E_DEVICE;
    }
    return loss_host ? read_loss(M, t_dev, n, loss_host) : AT_OK;
}

int at_mlp_apply_grad(at_mlp* M, const float* grad_dev, float lr) {
    if (!M || !grad_dev || !(lr > 0)) return AT_E_INVAL;
    return mlp_adam(M, grad_dev, lr);
}

int at_mlp_train_step(at_mlp* M, const float* x_dev, const float* t_dev, uint64_t n, float lr, float* loss_host) {
    if (!M || !x_dev || !t_dev || n == 0 || !(lr > 0)) return AT_E_INVAL;
    int rc = mlp_grad(M, x_dev, t_dev, n);
    if (rc) return rc;
    if (loss_host && (rc = read_loss(M, t_dev, n, loss_host))) return rc;
    return mlp_adam(M, M->S.grad, lr);
}

int at_mlp_gather_batch(at_mlp* M, const float* x_dev, const float* lnn_dev, const int64_t* idx_dev, uint64_t n,
                        float* xb_dev, float* tb_dev) {
    if (!M || (n && (!x_dev || !lnn_dev || !idx_dev || !xb_dev || !tb_dev))) return AT_E_INVAL;
    return atp::launch_mlp_gather(x_dev, lnn_dev, idx_dev, n, xb_dev, tb_dev, M->stream) == hipSuccess ? AT_OK
                                                                                                   : AT_E_DEVICE;
}

int at_features(at_ctx* h, const uint32_t* aip_dev, uint64_t n, float* feat_dev, double* est_dev, uint8_t* flags_dev) {
    if (!h || (n && (!aip_dev || !feat_dev))) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    hipError_t e = atp::launch_features(h->pool, h->aat, aip_dev, n, h->G, h->c0_query, h->kq, feat_dev, est_dev,
                                        flags_dev, h->stream);
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int at_estimate_learned_dev(at_ctx* h, at_mlp* M, const uint32_t* aip_dev, uint64_t n, double* est_dev,
                            uint8_t* flags_dev, double* plain_dev) {
    if (!h || !M || (n && (!aip_dev || !est_dev || !flags_dev))) return AT_E_INVAL;
    if (!h->queryable) return AT_E_STATE;
    if (n == 0) return AT_OK;
    int rc = ensure_query(h, n);
    if (rc) return rc;
    // the plain estimates stay in device memory for the fallback (the outputs
    // may be mapped host memory); the network's epilogue copies them out
    hipError_t e = atp::launch_features(h->pool, h->aat, aip_dev, n, h->G, h->c0_query, h->kq, h->q_feat,
                                        h->q_plain, h->q_flags, h->stream);
    if (e == hipSuccess) {
        const atp::LearnedEpilogue L{h->q_plain, h->q_flags, std::log(16.0) - 0.5, std::log(262144.0) + 0.5,
                                     h->p.theta, est_dev, flags_dev, plain_dev};
        e = atp::launch_mlp_forward_learned(h->q_feat, n, mlp_dev(M), L, h->stream);
    }
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

int at_estimate_learned_begin(at_ctx* h, at_mlp* M, const uint32_t* aip_host, uint64_t n) {
    if (!h || !M || (n && !aip_host)) return AT_E_INVAL;
    if (!h->queryable || h->q_pending) return AT_E_STATE;
    if (n > 0) {
        const uint64_t off = up64(4 * n);  // results follow the addresses in the staging
        const OutLayout O = out_layout(n);
        int rc = ensure_query(h, n);
        if (!rc) rc = ensure_pin_q(h, off + O.total);
        if (rc) return rc;
        // the kernels read the addresses from the staging and store the
        // results there: no copy commands between them and the host
        std::memcpy(h->pin_q, aip_host, n * sizeof(uint32_t));
        uint8_t* res = h->pin_q_dev + off;
        rc = at_estimate_learned_dev(h, M, reinterpret_cast<const uint32_t*>(h->pin_q_dev), n,
                                     reinterpret_cast<double*>(res + O.est), res + O.flags,
                                     reinterpret_cast<double*>(res + O.plain));
        if (rc) return rc;
        if (hipEventRecord(h->q_done, h->stream) != hipSuccess) return AT_E_DEVICE;
    }
    h->q_pending = true;
    h->q_pending_n = n;
    return AT_OK;
}

int at_estimate_learned_end(at_ctx* h, double* est_out, uint8_t* flags_out, double* plain_out) {
    if (!h) return AT_E_INVAL;
    if (!h->q_pending) return AT_E_STATE;
    const uint64_t n = h->q_pending_n;
    if (n && (!est_out || !flags_out)) return AT_E_INVAL;
    h->q_pending = false;
    if (n == 0) return AT_OK;
    const hipError_t e = hipEventSynchronize(h->q_done);
    if (e != hipSuccess) return dev_err(e);
    const uint8_t* res = h->pin_q + up64(4 * n);
    const OutLayout O = out_layout(n);
    std::memcpy(est_out, res + O.est, n * sizeof(double));
    std::memcpy(flags_out, res + O.flags, n);
    if (plain_out) std::memcpy(plain_out, res + O.plain, n * sizeof(double));
    return AT_OK;
}

int at_estimate_learned(at_ctx* h, at_mlp* M, const uint32_t* aip_host, uint64_t n, double* est_out,
                        uint8_t* flags_out, double* plain_out) {
    if (!h || !M || (n && (!aip_host || !est_out || !flags_out))) return AT_E_INVAL;
    if (!h->queryable || h->q_pending) return AT_E_STATE;
    if (n == 0) return AT_OK;
    const int rc = at_estimate_learned_begin(h, M, aip_host, n);
    if (rc) return rc;
    return at_estimate_learned_end(h, est_out, flags_out, plain_out);
}

}  // extern "C"
