// The aging-counter comparator: ACE counters and the asynchronous timestamps,
// each packed at its own width, on the cube and hashes of an at_ctx with the
// same parameters (at_cmp_* in at.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>

#include "at.h"
#include "atpool.hpp"

using atp::CmpLayout;
using atp::Geometry;

struct at_cmp {
    at_params p{};
    Geometry G{};
    int kind = 0;
    hipStream_t stream = nullptr;
    CmpLayout L{};
    uint64_t n_words = 0;  // ATVs * words per ATV
    uint64_t alloc = 0;    // words allocated: n_words rounded up to whole 16-byte units
    uint32_t* words = nullptr;
    uint32_t* w = nullptr;
    uint64_t t = 0;
    bool open = false;
    bool closed = false;
    uint32_t c0 = 0, c0_query = 0;
};

namespace {

uint32_t width_of(uint32_t values) {  // bits holding 0 .. values - 1
    uint32_t b = 1;
    while ((1u << b) < values) b++;
    return b;
}

int open_slice(at_cmp* h) {
    if (h->open) return AT_OK;
    hipError_t e = hipSuccess;
    if (h->kind == AT_CMP_ACE) {
        // every counter ages at each slice after the first
        uint32_t lsb = 0;
        for (uint32_t f = 0; f < h->L.F; f++) lsb |= 1u << (f * h->L.bits);
        if (h->t > 0) e = atp::launch_cmp_age(h->words, h->alloc, h->L.bits, lsb, h->stream);
    } else {
        h->c0 = (uint32_t)(h->t % h->G.twok);
        const atp::PreserveSpans S = atp::preserve_spans(h->G, h->c0);
        // word spans of the two due AT ranges, merged when they share a word
        uint32_t sp[2][2];
        int ns = 0;
        if (S.r0hi > S.r0lo) { sp[ns][0] = S.r0lo / h->L.F; sp[ns][1] = (S.r0hi + h->L.F - 1) / h->L.F; ns++; }
        if (S.r1hi > S.r1lo) { sp[ns][0] = S.r1lo / h->L.F; sp[ns][1] = (S.r1hi + h->L.F - 1) / h->L.F; ns++; }
        if (ns == 2) {
            if (sp[0][0] > sp[1][0]) std::swap(sp[0], sp[1]);
            if (sp[1][0] < sp[0][1]) {
                sp[0][1] = std::max(sp[0][1], sp[1][1]);
                ns = 1;
            }
        }
        const uint32_t s0lo = ns > 0 ? sp[0][0] : 0, s0n = ns > 0 ? sp[0][1] - sp[0][0] : 0;
        const uint32_t s1lo = ns > 1 ? sp[1][0] : 0, s1n = ns > 1 ? sp[1][1] - sp[1][0] : 0;
        e = atp::launch_cmp_preserve(h->words, h->G, h->L, h->c0, S, s0lo, s0n, s1lo, s1n, h->stream);
    }
    if (e != hipSuccess) return AT_E_DEVICE;
    h->open = true;
    h->closed = false;
    return AT_OK;
}

}  // namespace

extern "C" {

int at_cmp_create(const at_params* p, int kind, void* hip_stream, at_cmp** out) {
    if (!out) return AT_E_INVAL;
    *out = nullptr;
    if (!p || (kind != AT_CMP_ACE && kind != AT_CMP_AT) || atp::validate_params(*p)) return AT_E_INVAL;
    at_cmp* h = new (std::nothrow) at_cmp;
    if (!h) return AT_E_NOMEM;
    h->p = *p;
    h->G = atp::derive_geometry(*p);
    h->kind = kind;
    h->stream = (hipStream_t)hip_stream;
    // ACE counters hold 0..k: ceil(log2(k+1)) bits, their largest value all
    // ones (at least k).  Timestamps hold 0..2k: one bit more.
    h->L.bits = kind == AT_CMP_ACE ? width_of(p->k + 1) : width_of(2 * p->k + 1);
    h->L.F = 32 / h->L.bits;
    h->L.fmagic = (uint32_t)((((uint64_t)1 << 32) + h->L.F - 1) / h->L.F);
    h->L.wv = (h->G.g + h->L.F - 1) / h->L.F;
    h->L.n_atv = ((uint64_t)1 << (p->c + p->u)) * p->r;
    h->n_words = h->L.n_atv * h->L.wv;
    h->alloc = (h->n_words + 3) & ~3ull;
    int rc = AT_OK;
    if (hipMalloc((void**)&h->words, h->alloc * 4) != hipSuccess ||
        hipMalloc((void**)&h->w, h->L.n_atv * 4) != hipSuccess) {
        (void)hipGetLastError();
        rc = AT_E_NOMEM;
    }
    uint32_t fill = 0;  // ACE counters start at 0; timestamps inactive (2k) in every field
    if (kind == AT_CMP_AT)
        for (uint32_t f = 0; f < h->L.F; f++) fill |= h->G.twok << (f * h->L.bits);
    if (!rc && (atp::launch_fill_u32(h->words, h->n_words, fill, h->stream) != hipSuccess ||
                atp::launch_fill_u32(h->words + h->n_words, h->alloc - h->n_words, 0, h->stream) != hipSuccess))
        rc = AT_E_DEVICE;
    if (rc) {
        at_cmp_destroy(h);
        return rc;
    }
    *out = h;
    return AT_OK;
}

int at_cmp_destroy(at_cmp* h) {
    if (!h) return AT_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->words) (void)hipFree(h->words);
    if (h->w) (void)hipFree(h->w);
    delete h;
    return AT_OK;
}

int at_cmp_info(const at_cmp* h, uint64_t* out4) {
    if (!h || !out4) return AT_E_INVAL;
    out4[0] = h->L.bits;
    out4[1] = h->L.F;
    out4[2] = h->L.wv;
    out4[3] = h->n_words;
    return AT_OK;
}

int at_cmp_open_slice(at_cmp* h) {
    if (!h) return AT_E_INVAL;
    return open_slice(h);
}

int at_cmp_ingest(at_cmp* h, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n) {
    if (!h || (n && (!aip_dev || !bip_dev))) return AT_E_INVAL;
    int rc = open_slice(h);
    if (rc || n == 0) return rc;
    return atp::launch_cmp_set(h->words, aip_dev, bip_dev, n, h->G, h->L, h->kind == AT_CMP_ACE, h->c0, h->stream) ==
                   hipSuccess
               ? AT_OK
               : AT_E_DEVICE;
}

int at_cmp_close(at_cmp* h, uint32_t kprime) {
    if (!h || kprime < 1 || kprime > h->p.k) return AT_E_INVAL;
    int rc = open_slice(h);
    if (rc) return rc;
    if (atp::launch_cmp_close(h->words, h->G, h->L, h->kind == AT_CMP_ACE, h->c0, kprime, h->w, h->stream) !=
        hipSuccess)
        return AT_E_DEVICE;
    h->c0_query = h->c0;
    h->t += 1;
    h->open = false;
    h->closed = true;
    return AT_OK;
}

int at_cmp_read(at_cmp* h, uint32_t* words_host, uint32_t* weights_host) {
    if (!h) return AT_E_INVAL;
    if (weights_host && !h->closed) return AT_E_STATE;
    hipError_t e = hipSuccess;
    if (words_host) e = hipMemcpyAsync(words_host, h->words, h->n_words * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && weights_host)
        e = hipMemcpyAsync(weights_host, h->w, h->L.n_atv * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

}  // extern "C"
