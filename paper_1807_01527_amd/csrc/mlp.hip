// Learned correction of the plain estimate: a 64 -> 64 -> 64 -> 1 ReLU
// network over the 64 occupancy features of a host, predicting ln n.
// Weights and activations are bfloat16 and products accumulate in FP32 on the
// CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16); biases, the output and the
// optimiser state are FP32.  One wave owns 16 rows (hosts) at a time.
//
// MFMA 16x16x32 operand layout (lane l, q = l / 16, m = l % 16):
//   A (16 x 32): lane holds A[m][8q .. 8q+7]
//   B (32 x 16): lane holds B[8q .. 8q+7][m]
//   D (16 x 16): lane holds D[4q .. 4q+3][m]
#include <hip/hip_runtime.h>

#include <cstdint>

#include "atpool.hpp"

namespace atp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int D = kMlpDim;

__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 4 consecutive rows of one column, feature-major [col][row] (8-byte store)
__device__ __forceinline__ void store4_T(uint16_t* T, uint64_t ldT, uint32_t col, uint64_t row0, const uint16_t v[4]) {
    uint2 pk;
    pk.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    pk.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    *reinterpret_cast<uint2*>(T + (uint64_t)col * ldT + row0) = pk;
}

__device__ __forceinline__ void load4_T(const uint16_t* T, uint64_t ldT, uint32_t col, uint64_t row0, uint16_t v[4]) {
    uint2 pk = *reinterpret_cast<const uint2*>(T + (uint64_t)col * ldT + row0);
    v[0] = (uint16_t)(pk.x & 0xFFFFu);
    v[1] = (uint16_t)(pk.x >> 16);
    v[2] = (uint16_t)(pk.y & 0xFFFFu);
    v[3] = (uint16_t)(pk.y >> 16);
}

// The fallback rule for row i (see LearnedEpilogue), shared by the fused
// epilogue and the serving export.
__device__ __forceinline__ void learned_store(const double* __restrict__ plain, const uint8_t* __restrict__ pflags,
                                              double zlo, double zhi, double theta, uint64_t i, float y, float f61,
                                              double* __restrict__ est, uint8_t* __restrict__ flags) {
    const double z = (double)y + 16.0 * (double)f61;
    uint8_t fl = pflags[i] & (uint8_t)(AT_F_SAT | AT_F_NEG);
    double e;
    if (!(z >= zlo && z <= zhi)) {
        e = plain[i];
        fl |= AT_F_FALLBACK;
    } else {
        e = exp(z);
    }
    if (e >= theta) fl |= AT_F_SUPER;
    est[i] = e;
    flags[i] = fl;
}

// Forward pass.  nrows is a multiple of 64, so every wave of a block runs the
// same number of iterations and block barriers are safe.  TRAIN also stores
// the bf16 input and hidden activations feature-major for the backward pass.
// n_dev, when given, holds the row count (written by an earlier kernel of the
// same graph); n is then only the capacity.  With L.est set (inference only)
// each output goes through the learned estimate's fallback rule instead of
// to y.
template <bool TRAIN>
__global__ __launch_bounds__(kBlock) void k_mlp_fwd(const float* __restrict__ X, uint64_t n, uint64_t nrows,
                                                    MlpDev P, float* __restrict__ y, uint16_t* __restrict__ XT,
                                                    uint16_t* __restrict__ H1T, uint16_t* __restrict__ H2T,
                                                    uint64_t ldT, const uint64_t* __restrict__ n_dev,
                                                    LearnedEpilogue L) {
    __shared__ __align__(16) uint16_t hs[kBlock / 64][16][D + 8];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t m = lane & 15u, q = lane >> 4;
    if (n_dev) n = *n_dev < n ? *n_dev : n;
    for (uint64_t r0 = ((uint64_t)blockIdx.x * 4 + wv) * 16; r0 < nrows; r0 += (uint64_t)gridDim.x * 64) {
        if (!TRAIN && r0 - 16 * wv >= n) continue;  // the whole block is past the last row
        const uint64_t row = r0 + m;
        bf16x8 A[2];
#pragma unroll
        for (int kk = 0; kk < 2; kk++) {
            uint16_t hv[8];
            if (row < n) {
                const float4* src = reinterpret_cast<const float4*>(X + row * D + 32 * kk + 8 * q);
                float4 a = src[0], b = src[1];
                float xv[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
                for (int e = 0; e < 8; e++) hv[e] = f2bf(xv[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; e++) hv[e] = 0;
            }
            if (TRAIN) {
#pragma unroll
                for (int e = 0; e < 8; e++) XT[(uint64_t)(32 * kk + 8 * q + e) * ldT + row] = hv[e];
            }
            u32x4 pk = {(uint32_t)hv[0] | ((uint32_t)hv[1] << 16), (uint32_t)hv[2] | ((uint32_t)hv[3] << 16),
                        (uint32_t)hv[4] | ((uint32_t)hv[5] << 16), (uint32_t)hv[6] | ((uint32_t)hv[7] << 16)};
            A[kk] = __builtin_bit_cast(bf16x8, pk);
        }
        // layer 1
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; kk++) acc = mfma(A[kk], load8(P.W1b + (16 * nt + m) * D + 32 * kk + 8 * q), acc);
            const uint32_t col = 16 * nt + m;
            uint16_t hb[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                float z = acc[e] + P.b1[col];
                hb[e] = f2bf(z > 0.f ? z : 0.f);
                hs[wv][4 * q + e][col] = hb[e];
            }
            if (TRAIN) store4_T(H1T, ldT, col, r0 + 4 * q, hb);
        }
        __syncthreads();
        bf16x8 A2[2];
#pragma unroll
        for (int kk = 0; kk < 2; kk++) A2[kk] = load8(&hs[wv][m][32 * kk + 8 * q]);
        // layer 2 and the output dot product
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; kk++) acc = mfma(A2[kk], load8(P.W2b + (16 * nt + m) * D + 32 * kk + 8 * q), acc);
            const uint32_t col = 16 * nt + m;
            const float w3 = bf2f(P.w3b[col]);
            uint16_t hb[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                float z = acc[e] + P.b2[col];
                hb[e] = f2bf(z > 0.f ? z : 0.f);
                part[e] += bf2f(hb[e]) * w3;
            }
            if (TRAIN) store4_T(H2T, ldT, col, r0 + 4 * q, hb);
        }
#pragma unroll
        for (int e = 0; e < 4; e++)
            for (uint32_t o = 1; o < 16; o <<= 1) part[e] += __shfl_xor(part[e], o, 64);
        if (!TRAIN && L.est) {
            // every lane of a 16-lane group holds its four sums after the
            // butterfly: lanes m < 4 take one row each, in parallel
            if (m < 4) {
                const float pv = m == 0 ? part[0] : m == 1 ? part[1] : m == 2 ? part[2] : part[3];
                const uint64_t rr = r0 + 4 * q + m;
                if (rr < n) {
                    learned_store(L.plain, L.pflags, L.zlo, L.zhi, L.theta, rr, pv + P.b3[0], X[rr * D + 61], L.est,
                                  L.flags);
                    if (L.plain_out) L.plain_out[rr] = L.plain[rr];
                }
            }
        } else if (m == 0) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint64_t rr = r0 + 4 * q + e;
                if (TRAIN || rr < n) y[rr] = part[e] + P.b3[0];
            }
        }
        __syncthreads();
    }
}

// Backward pass over rows: dy = scale*(y - t) (0 for padding rows), then
// dh2 = dy * w3 on active units, dh1 = (dh2 W2) on active units; both stored
// bf16 feature-major for the weight gradients.
__global__ __launch_bounds__(kBlock) void k_mlp_bwd(const float* __restrict__ y, const float* __restrict__ t, uint64_t n,
                                                    uint64_t nrows, float scale, MlpDev P,
                                                    const uint16_t* __restrict__ H1T, const uint16_t* __restrict__ H2T,
                                                    uint16_t* __restrict__ dH1T, uint16_t* __restrict__ dH2T,
                                                    float* __restrict__ dy_out, uint64_t ldT) {
    __shared__ __align__(16) uint16_t hs[kBlock / 64][16][D + 8];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t m = lane & 15u, q = lane >> 4;
    for (uint64_t r0 = ((uint64_t)blockIdx.x * 4 + wv) * 16; r0 < nrows; r0 += (uint64_t)gridDim.x * 64) {
        float dyv[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint64_t rr = r0 + 4 * q + e;
            dyv[e] = rr < n ? scale * (y[rr] - t[rr]) : 0.f;
            if (m == 0) dy_out[rr] = dyv[e];
        }
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            const uint32_t col = 16 * nt + m;
            const float w3 = bf2f(P.w3b[col]);
            uint16_t h2[4], db[4];
            load4_T(H2T, ldT, col, r0 + 4 * q, h2);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                float d = bf2f(h2[e]) > 0.f ? dyv[e] * w3 : 0.f;
                db[e] = f2bf(d);
                hs[wv][4 * q + e][col] = db[e];
            }
            store4_T(dH2T, ldT, col, r0 + 4 * q, db);
        }
        __syncthreads();
        bf16x8 A[2];
#pragma unroll
        for (int kk = 0; kk < 2; kk++) A[kk] = load8(&hs[wv][m][32 * kk + 8 * q]);
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
            // B[o][i] = W2[o][i], read from the transposed copy W2T[i][o]
#pragma unroll
            for (int kk = 0; kk < 2; kk++) acc = mfma(A[kk], load8(P.W2Tb + (16 * nt + m) * D + 32 * kk + 8 * q), acc);
            const uint32_t col = 16 * nt + m;
            uint16_t h1[4], db[4];
            load4_T(H1T, ldT, col, r0 + 4 * q, h1);
#pragma unroll
            for (int e = 0; e < 4; e++) db[e] = f2bf(bf2f(h1[e]) > 0.f ? acc[e] : 0.f);
            store4_T(dH1T, ldT, col, r0 + 4 * q, db);
        }
        __syncthreads();
    }
}

// Weight gradients of one chunk of kMlpChunk rows: dW1 = dH1^T X and
// dW2 = dH2^T H1 on the matrix cores (the batch is the contraction), and the
// bias / output-layer sums on the vector units.  Each chunk writes every
// parameter slot of its own partial row once, so the reduction order is fixed.
__global__ __launch_bounds__(kBlock) void k_mlp_wgrad(const uint16_t* __restrict__ XT, const uint16_t* __restrict__ H1T,
                                                      const uint16_t* __restrict__ H2T, const uint16_t* __restrict__ dH1T,
                                                      const uint16_t* __restrict__ dH2T, const float* __restrict__ dy,
                                                      uint64_t ldT, float* __restrict__ partial) {
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t m = lane & 15u, q = lane >> 4;
    const uint64_t b0 = (uint64_t)blockIdx.x * kMlpChunk;
    float* out = partial + (uint64_t)blockIdx.x * kMlpParams;
    for (uint32_t T = wv; T < 32; T += kBlock / 64) {
        const uint32_t mat = T / 16, ot = (T % 16) / 4, it = T % 4;
        const uint16_t* Aop = mat ? dH2T : dH1T;
        const uint16_t* Bop = mat ? H1T : XT;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (uint32_t ks = 0; ks < kMlpChunk / 32; ks++) {
            const uint64_t b = b0 + 32 * ks + 8 * q;
            acc = mfma(load8(Aop + (uint64_t)(16 * ot + m) * ldT + b), load8(Bop + (uint64_t)(16 * it + m) * ldT + b),
                       acc);
        }
        const uint32_t base = mat ? kOffW2 : kOffW1;
#pragma unroll
        for (int e = 0; e < 4; e++) out[base + (16 * ot + 4 * q + e) * D + 16 * it + m] = acc[e];
    }
    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        float s = 0.f;
        for (uint32_t b = 0; b < kMlpChunk; b++) s += bf2f(dH1T[(uint64_t)tid * ldT + b0 + b]);
        out[kOffB1 + tid] = s;
    } else if (tid < 128) {
        const uint32_t o = tid - 64;
        float s = 0.f;
        for (uint32_t b = 0; b < kMlpChunk; b++) s += bf2f(dH2T[(uint64_t)o * ldT + b0 + b]);
        out[kOffB2 + o] = s;
    } else if (tid < 192) {
        const uint32_t i = tid - 128;
        float s = 0.f;
        for (uint32_t b = 0; b < kMlpChunk; b++) s += dy[b0 + b] * bf2f(H2T[(uint64_t)i * ldT + b0 + b]);
        out[kOffW3 + i] = s;
    } else if (tid == 192) {
        float s = 0.f;
        for (uint32_t b = 0; b < kMlpChunk; b++) s += dy[b0 + b];
        out[kOffB3] = s;
    }
}

__global__ void k_mlp_reduce(const float* __restrict__ partial, uint32_t nchunks, float* __restrict__ grad) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float s = 0.f;
    for (uint32_t c = 0; c < nchunks; c++) s += partial[(uint64_t)c * kMlpParams + p];
    grad[p] = s;
}

__global__ void k_mlp_loss(const float* __restrict__ y, const float* __restrict__ t, uint64_t n, float* __restrict__ out) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double d = (double)y[i] - (double)t[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(red[0] / (double)n);
}

// Copy master weights into the bf16 operand copies (W1, W2, W2^T, w3).
__device__ __forceinline__ void refresh_bf16(uint32_t p, float w, const MlpOut& O) {
    if (p < kOffB1) {
        O.W1b[p] = f2bf(w);
    } else if (p >= kOffW2 && p < kOffB2) {
        const uint32_t idx = p - kOffW2, o = idx / D, i = idx % D;
        const uint16_t b = f2bf(w);
        O.W2b[idx] = b;
        O.W2Tb[i * D + o] = b;
    } else if (p >= kOffW3 && p < kOffB3) {
        O.w3b[p - kOffW3] = f2bf(w);
    }
}

// A training batch: rows idx[i] of the features and the network's target
// for each, ln n minus the plain estimate's log feature (16 * f[61]).  One
// wave per row; lane l copies feature l.
__global__ __launch_bounds__(kBlock) void k_mlp_gather(const float* __restrict__ X, const float* __restrict__ lnn,
                                                       const int64_t* __restrict__ idx, uint64_t n,
                                                       float* __restrict__ Xb, float* __restrict__ Tb) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t i = wave; i < n; i += nwaves) {
        const uint64_t r = (uint64_t)idx[i];
        const float x = X[r * 64 + lane];
        Xb[i * 64 + lane] = x;
        if (lane == 61) Tb[i] = lnn[r] - 16.0f * x;
    }
}

__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ mo, float* __restrict__ ve,
                           const float* __restrict__ grad, AdamConst C, MlpOut O) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float m = C.b1 * mo[p] + C.one_minus_b1 * g;
    const float v = C.b2 * ve[p] + C.one_minus_b2 * (g * g);
    const float mh = m / C.c1;
    const float vh = v / C.c2;
    const float nw = w[p] - C.lr * (mh / (sqrtf(vh) + C.eps));
    mo[p] = m;
    ve[p] = v;
    w[p] = nw;
    refresh_bf16(p, nw, O);
}

__global__ void k_mlp_refresh(const float* __restrict__ w, MlpOut O) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) refresh_bf16(p, w[p], O);
}

// Learned estimate with the plain one as fallback.  The network predicts the
// correction to the plain estimate's log feature: z = y + 16*f[61] estimates
// ln n.  exp(z) is returned when z is finite and inside [zlo, zhi] (the
// trained range of ln n), else the plain estimate with AT_F_FALLBACK.
// AT_F_SUPER is recomputed for the returned estimate.
// A serving step's results to the mapped host copy its descriptor names, with
// the learned estimates computed on the way: the state block, then per host of
// the list its address, plain estimate, learned estimate (the fallback rule
// above) and flags.
__global__ void k_serve_export_learned(const StepDesc* __restrict__ d, const ServeState* __restrict__ S,
                                       const uint32_t* __restrict__ hosts, const float* __restrict__ y,
                                       const float* __restrict__ feat, const double* __restrict__ plain,
                                       const uint8_t* __restrict__ pflags, double zlo, double zhi, double theta) {
    const ServeExport X = d->xp;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
    constexpr uint32_t kWords = sizeof(ServeState) / 8;
    static_assert(sizeof(ServeState) % 8 == 0, "the state block copies as 8-byte words");
    const uint64_t* sw = reinterpret_cast<const uint64_t*>(S);
    uint64_t* dw = reinterpret_cast<uint64_t*>(X.state);
    for (uint64_t q = tid; q < kWords; q += nthr) dw[q] = sw[q];
    const uint64_t n = S->n_hosts < X.max_hosts ? S->n_hosts : X.max_hosts;
    for (uint64_t h = tid; h < n; h += nthr) {
        X.hosts[h] = hosts[h];
        X.est[h] = plain[h];
        learned_store(plain, pflags, zlo, zhi, theta, h, y[h], feat[h * kMlpDim + 61], X.est_l, X.flags);
    }
}

}  // namespace

hipError_t launch_serve_export_learned(const ServeBufs& B, double zlo, double zhi, double theta, hipStream_t st) {
    hipLaunchKernelGGL(k_serve_export_learned, dim3(64), dim3(kBlock), 0, st, B.desc, B.state, B.hosts, B.y, B.feat,
                       B.est, B.pflags, zlo, zhi, theta);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* X, uint64_t n, const MlpDev& P, float* y, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint64_t nrows = (n + 63) / 64 * 64;
    uint64_t blocks = nrows / 64;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, X, n, nrows, P, y, nullptr,
                       nullptr, nullptr, (uint64_t)0, (const uint64_t*)nullptr, LearnedEpilogue{});
    return hipGetLastError();
}

hipError_t launch_mlp_forward_learned(const float* X, uint64_t n, const MlpDev& P, const LearnedEpilogue& L,
                                      hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (!L.est || !L.flags || !L.plain || !L.pflags) return hipErrorInvalidValue;
    const uint64_t nrows = (n + 63) / 64 * 64;
    uint64_t blocks = nrows / 64;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, X, n, nrows, P, (float*)nullptr,
                       nullptr, nullptr, nullptr, (uint64_t)0, (const uint64_t*)nullptr, L);
    return hipGetLastError();
}

hipError_t launch_mlp_forward_devn(const float* X, const uint64_t* n_dev, uint64_t nrows_max, const MlpDev& P,
                                   float* y, hipStream_t st) {
    const uint64_t nrows = (nrows_max + 63) / 64 * 64;
    uint64_t blocks = nrows / 64;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, X, nrows_max, nrows, P, y,
                       nullptr, nullptr, nullptr, (uint64_t)0, n_dev, LearnedEpilogue{});
    return hipGetLastError();
}

hipError_t launch_mlp_train_fwd_bwd(const float* X, const float* t, uint64_t n, uint64_t nrows, const MlpDev& P,
                                    const MlpScratch& S, hipStream_t st) {
    uint64_t blocks = nrows / 64;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_mlp_fwd<true>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, X, n, nrows, P, S.y, S.XT,
                       S.H1T, S.H2T, nrows, (const uint64_t*)nullptr, LearnedEpilogue{});
    hipLaunchKernelGGL(k_mlp_bwd, dim3((uint32_t)blocks), dim3(kBlock), 0, st, S.y, t, n, nrows, 2.0f / (float)n, P,
                       S.H1T, S.H2T, S.dH1T, S.dH2T, S.dy, nrows);
    const uint32_t nchunks = (uint32_t)(nrows / kMlpChunk);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(nchunks), dim3(kBlock), 0, st, S.XT, S.H1T, S.H2T, S.dH1T, S.dH2T, S.dy,
                       nrows, S.partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, S.partial, nchunks,
                       S.grad);
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const float* X, const float* lnn, const int64_t* idx, uint64_t n, float* Xb, float* Tb,
                             hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mlp_gather, dim3((uint32_t)blocks), dim3(kBlock), 0, st, X, lnn, idx, n, Xb, Tb);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* y, const float* t, uint64_t n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kBlock), 0, st, y, t, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, float* m, float* v, const float* grad, const AdamConst& C, const MlpOut& O,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, w, m, v, grad, C, O);
    return hipGetLastError();
}

hipError_t launch_mlp_refresh(const float* w, const MlpOut& O, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_refresh, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st, w, O);
    return hipGetLastError();
}

}  // namespace atp
