// Learned subgraph scorer: a three-layer MLP (kScorerIn -> 256 -> 256 -> 1,
// ReLU) with BF16 weights and activations and FP32 accumulation.  The two
// wide layers and their gradients run on the matrix cores
// (v_mfma_f32_32x32x16_bf16); the 256 -> 1 head, the loss, the bias sums
// and the Adam update are plain FP32 vector code.  It scores candidate
// unions of UnionDP's partition phase (Section 4.2) and is trained on plans
// the exact DP produces (mpdp_scorer.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "mpdp.h"
#include "mpdp_scorer.h"

namespace {

constexpr int kIn = MPDP_SCORER_IN;
constexpr int kHid = MPDP_SCORER_HIDDEN;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(uint16_t)))) uint16_t u16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Device parameter block: FP32 master values, BF16 working copies,
// gradients and Adam moments, all in one allocation (offsets: scorer_layout).
struct Params {
    float *w1, *b1, *w2, *b2, *w3, *b3;           // master
    uint16_t *w1h, *w2h, *w3h;                     // bf16 copies used by the forward pass
    float *g;                                      // gradients, same order as the master values
    float *m, *v;                                  // Adam moments
};

constexpr size_t kN1 = (size_t)kIn * kHid, kN2 = (size_t)kHid * kHid, kN3 = kHid;
constexpr size_t kNParams = kN1 + kHid + kN2 + kHid + kN3 + 1;

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t master, bf, grad, m, v, total;
};

Layout scorer_layout() {
    Layout L{};
    size_t o = 0;
    L.master = o; o = up256(o + 4 * kNParams);
    L.bf = o;     o = up256(o + 2 * (kN1 + kN2 + kN3));
    L.grad = o;   o = up256(o + 4 * kNParams);
    L.m = o;      o = up256(o + 4 * kNParams);
    L.v = o;      o = up256(o + 4 * kNParams);
    L.total = o;
    return L;
}

Params params_at(void *base) {
    const Layout L = scorer_layout();
    char *b = static_cast<char *>(base);
    Params p;
    float *mst = reinterpret_cast<float *>(b + L.master);
    p.w1 = mst;
    p.b1 = p.w1 + kN1;
    p.w2 = p.b1 + kHid;
    p.b2 = p.w2 + kN2;
    p.w3 = p.b2 + kHid;
    p.b3 = p.w3 + kN3;
    uint16_t *h = reinterpret_cast<uint16_t *>(b + L.bf);
    p.w1h = h;
    p.w2h = h + kN1;
    p.w3h = h + kN1 + kN2;
    p.g = reinterpret_cast<float *>(b + L.grad);
    p.m = reinterpret_cast<float *>(b + L.m);
    p.v = reinterpret_cast<float *>(b + L.v);
    return p;
}

// Work buffer of one batch: activations and their gradients.
struct Work {
    uint16_t *h1, *h2, *dz2, *dz1;  // batch x 256 bf16
    float *logit, *dlogit;          // batch
    float *loss;                    // 1 (sum over the batch)
};

size_t work_bytes(uint32_t batch) {
    return up256(2 * (size_t)batch * kHid) * 4 + up256(4 * (size_t)batch) * 2 + 256;
}

Work work_at(void *base, uint32_t batch) {
    char *b = static_cast<char *>(base);
    const size_t a = up256(2 * (size_t)batch * kHid), f = up256(4 * (size_t)batch);
    Work w;
    w.h1 = reinterpret_cast<uint16_t *>(b);
    w.h2 = reinterpret_cast<uint16_t *>(b + a);
    w.dz2 = reinterpret_cast<uint16_t *>(b + 2 * a);
    w.dz1 = reinterpret_cast<uint16_t *>(b + 3 * a);
    w.logit = reinterpret_cast<float *>(b + 4 * a);
    w.dlogit = reinterpret_cast<float *>(b + 4 * a + f);
    w.loss = reinterpret_cast<float *>(b + 4 * a + 2 * f);
    return w;
}

// ---------------------------------------------------------------- MFMA GEMM
//
// C (M x N) = A (M x K) * B (K x N), BF16 in, FP32 accumulate.  A(i, k) is
// at A[i * lda + k] (TA = 0) or A[k * lda + i] (TA = 1); B(k, j) is at
// B[k * ldb + j] (TB = 0) or B[j * ldb + k] (TB = 1).  One wave computes one
// 32 x 32 tile of C with v_mfma_f32_32x32x16_bf16: lane l supplies A(i, k)
// for i = l % 32 and k = 8 (l / 32) + 0..7 of each 16-wide K step, and
// B(k, j) for j = l % 32 and the same k; it receives C(i, j) for j = l % 32
// and i = 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15.  Out-of-range rows,
// columns and K positions load as zero and are not stored.  A workgroup of
// four waves covers a 64 x 64 block.
enum { kEpiBiasReluBf16 = 0, kEpiStoreF32 = 1, kEpiReluMaskBf16 = 2 };

template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const uint16_t *__restrict__ A, int lda,
                                              const uint16_t *__restrict__ B, int ldb, int M, int N, int K,
                                              const float *__restrict__ bias,      // EPI 0: per column
                                              const uint16_t *__restrict__ mask,   // EPI 2: keep where mask > 0
                                              int ldm, float *__restrict__ Cf, uint16_t *__restrict__ Ch, int ldc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int j0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int ai = i0 + (lane & 31), bj = j0 + (lane & 31), kq = 8 * (lane >> 5);
    floatx16 acc = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        u16x8 a, b;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = k0 + kq + t;
            uint16_t av = 0, bv = 0;
            if (ai < M && k < K) av = TA ? A[(size_t)k * lda + ai] : A[(size_t)ai * lda + k];
            if (bj < N && k < K) bv = TB ? B[(size_t)bj * ldb + k] : B[(size_t)k * ldb + bj];
            a[t] = av;
            b[t] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = bj;
        if (i >= M || j >= N) continue;
        const float c = acc[r];
        if (EPI == kEpiBiasReluBf16) {
            const float z = c + bias[j];
            Ch[(size_t)i * ldc + j] = f2bf(z > 0.f ? z : 0.f);
        } else if (EPI == kEpiStoreF32) {
            Cf[(size_t)i * ldc + j] = c;
        } else {
            Ch[(size_t)i * ldc + j] = mask[(size_t)i * ldm + j] != 0 ? f2bf(c) : (uint16_t)0;
        }
    }
}

template <int TA, int TB, int EPI>
hipError_t gemm(hipStream_t s, const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K,
                const float *bias, const uint16_t *mask, int ldm, float *Cf, uint16_t *Ch, int ldc) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 grid((N + 63) / 64, (M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, bias, mask, ldm, Cf, Ch,
                       ldc);
    return hipGetLastError();
}

// ---------------------------------------------------------------- vector kernels

__global__ void k_zero1(float *x) { x[0] = 0.f; }

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// logit_i = sum_j h2[i][j] * w3[j] (j ascending, FP32) + b3
__global__ void k_head(const uint16_t *__restrict__ h2, const uint16_t *__restrict__ w3h, const float *__restrict__ b3,
                       float *__restrict__ logit, uint32_t batch) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    float acc = 0.f;
    for (int j = 0; j < kHid; ++j) acc += bf2f(h2[(size_t)i * kHid + j]) * bf2f(w3h[j]);
    logit[i] = acc + b3[0];
}

// Mean binary cross-entropy with logits: dlogit_i = (sigmoid(logit_i) - y_i) / batch;
// loss accumulates max(l, 0) - l y + log1p(exp(-|l|)) over the batch.
__global__ void k_loss(const float *__restrict__ logit, const float *__restrict__ y, float *__restrict__ dlogit,
                       float *__restrict__ loss, uint32_t batch) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    float li = 0.f;
    if (i < batch) {
        const float l = logit[i], t = y[i];
        const float p = 1.f / (1.f + expf(-l));
        dlogit[i] = (p - t) / (float)batch;
        li = fmaxf(l, 0.f) - l * t + log1pf(expf(-fabsf(l)));
    }
    for (int off = 32; off >= 1; off >>= 1) li += __shfl_xor(li, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, li);
}

// dz2[i][j] = bf16(h2[i][j] > 0 ? dlogit_i * w3[j] : 0)
__global__ void k_dz2(const uint16_t *__restrict__ h2, const float *__restrict__ dlogit,
                      const uint16_t *__restrict__ w3h, uint16_t *__restrict__ dz2, uint32_t batch) {
    const size_t n = (size_t)batch * kHid;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const size_t i = t / kHid;
        const int j = (int)(t % kHid);
        dz2[t] = h2[t] != 0 ? f2bf(dlogit[i] * bf2f(w3h[j])) : (uint16_t)0;
    }
}

// Column sums over the batch (i ascending, FP32): bias gradients, and the
// head's weight gradient dw3[j] = sum_i h2[i][j] dlogit_i, db3 = sum_i dlogit_i.
__global__ void k_colsum(const uint16_t *__restrict__ d, uint32_t batch, float *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kHid) return;
    float acc = 0.f;
    for (uint32_t i = 0; i < batch; ++i) acc += bf2f(d[(size_t)i * kHid + j]);
    out[j] = acc;
}

__global__ void k_head_grad(const uint16_t *__restrict__ h2, const float *__restrict__ dlogit, uint32_t batch,
                            float *__restrict__ dw3, float *__restrict__ db3) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kHid) {
        float acc = 0.f;
        for (uint32_t i = 0; i < batch; ++i) acc += bf2f(h2[(size_t)i * kHid + j]) * dlogit[i];
        dw3[j] = acc;
    } else if (j == kHid) {
        float acc = 0.f;
        for (uint32_t i = 0; i < batch; ++i) acc += dlogit[i];
        db3[0] = acc;
    }
}

// Adam (Kingma & Ba): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); then the BF16 copies.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       size_t n, float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

#define HIPCHK(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return MPDP_EDEVICE; \
    } while (0)

hipError_t refresh_bf16(const Params &p, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(64), dim3(256), 0, s, p.w1, p.w1h, kN1);
    hipLaunchKernelGGL(k_to_bf16, dim3(256), dim3(256), 0, s, p.w2, p.w2h, kN2);
    hipLaunchKernelGGL(k_to_bf16, dim3(1), dim3(256), 0, s, p.w3, p.w3h, kN3);
    return hipGetLastError();
}

hipError_t forward(const Params &p, const uint16_t *x, uint32_t batch, const Work &w, float *logits, hipStream_t s) {
    hipError_t e = gemm<0, 0, kEpiBiasReluBf16>(s, x, kIn, p.w1h, kHid, (int)batch, kHid, kIn, p.b1, nullptr, 0,
                                                nullptr, w.h1, kHid);
    if (e != hipSuccess) return e;
    e = gemm<0, 0, kEpiBiasReluBf16>(s, w.h1, kHid, p.w2h, kHid, (int)batch, kHid, kHid, p.b2, nullptr, 0, nullptr,
                                     w.h2, kHid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_head, dim3((batch + 255) / 256), dim3(256), 0, s, w.h2, p.w3h, p.b3, logits, batch);
    return hipGetLastError();
}

// Loss and all gradients into p.g (same order as the master values).
hipError_t backward(const Params &p, const uint16_t *x, const float *y, uint32_t batch, const Work &w, hipStream_t s) {
    float *g1 = p.g, *gb1 = g1 + kN1, *g2 = gb1 + kHid, *gb2 = g2 + kN2, *g3 = gb2 + kHid, *gb3 = g3 + kN3;
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, w.loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss, dim3((batch + 255) / 256), dim3(256), 0, s, w.logit, y, w.dlogit, w.loss, batch);
    hipLaunchKernelGGL(k_head_grad, dim3((kHid + 1 + 255) / 256), dim3(256), 0, s, w.h2, w.dlogit, batch, g3, gb3);
    hipLaunchKernelGGL(k_dz2, dim3(256), dim3(256), 0, s, w.h2, w.dlogit, p.w3h, w.dz2, batch);
    // dW2 = H1^T dZ2 (256 x 256, K = batch); db2 = column sums of dZ2
    e = gemm<1, 0, kEpiStoreF32>(s, w.h1, kHid, w.dz2, kHid, kHid, kHid, (int)batch, nullptr, nullptr, 0, g2,
                                 nullptr, kHid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kHid), 0, s, w.dz2, batch, gb2);
    // dZ1 = (dZ2 W2^T) masked by H1 > 0
    e = gemm<0, 1, kEpiReluMaskBf16>(s, w.dz2, kHid, p.w2h, kHid, (int)batch, kHid, kHid, nullptr, w.h1, kHid,
                                     nullptr, w.dz1, kHid);
    if (e != hipSuccess) return e;
    // dW1 = X^T dZ1 (kIn x 256, K = batch); db1
    e = gemm<1, 0, kEpiStoreF32>(s, x, kIn, w.dz1, kHid, kIn, kHid, (int)batch, nullptr, nullptr, 0, g1, nullptr,
                                 kHid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kHid), 0, s, w.dz1, batch, gb1);
    return hipGetLastError();
}

}  // namespace

extern "C" {

size_t mpdp_scorer_param_bytes(void) { return scorer_layout().total; }

size_t mpdp_scorer_work_bytes(uint32_t batch) { return batch ? work_bytes(batch) : 0; }

mpdp_status mpdp_scorer_load(void *d_params, const float *w1, const float *b1, const float *w2, const float *b2,
                             const float *w3, const float *b3, void *hip_stream) {
    if (!d_params || !w1 || !b1 || !w2 || !b2 || !w3 || !b3) return MPDP_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_params) % 256) return MPDP_EINVAL;
    std::vector<float> host(kNParams);
    size_t o = 0;
    auto put = [&](const float *src, size_t n) {
        std::memcpy(host.data() + o, src, 4 * n);
        o += n;
    };
    put(w1, kN1); put(b1, kHid); put(w2, kN2); put(b2, kHid); put(w3, kN3); put(b3, 1);
    for (float x : host)
        if (!std::isfinite(x)) return MPDP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Layout L = scorer_layout();
    const Params p = params_at(d_params);
    char *base = static_cast<char *>(d_params);
    HIPCHK(hipMemcpyAsync(base + L.master, host.data(), 4 * kNParams, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(base + L.m, 0, 4 * kNParams, s));
    HIPCHK(hipMemsetAsync(base + L.v, 0, 4 * kNParams, s));
    HIPCHK(hipMemsetAsync(base + L.grad, 0, 4 * kNParams, s));
    HIPCHK(refresh_bf16(p, s));
    HIPCHK(hipStreamSynchronize(s));
    return MPDP_OK;
}

mpdp_status mpdp_scorer_layout(size_t *off_master, size_t *off_bf16, size_t *off_grad) {
    if (!off_master || !off_bf16 || !off_grad) return MPDP_EINVAL;
    const Layout L = scorer_layout();
    *off_master = L.master;
    *off_bf16 = L.bf;
    *off_grad = L.grad;
    return MPDP_OK;
}

mpdp_status mpdp_scorer_forward(const void *d_params, const uint16_t *d_x, uint32_t batch, float *d_logits,
                                void *d_work, size_t work_size, void *hip_stream) {
    if (!d_params || !d_x || !d_logits || !d_work || batch == 0) return MPDP_EINVAL;
    if (work_size < work_bytes(batch)) return MPDP_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Params p = params_at(const_cast<void *>(d_params));
    const Work w = work_at(d_work, batch);
    HIPCHK(forward(p, d_x, batch, w, d_logits, s));
    return MPDP_OK;
}

mpdp_status mpdp_scorer_grad(void *d_params, const uint16_t *d_x, const float *d_y, uint32_t batch, void *d_work,
                             size_t work_size, void *hip_stream, float *loss_out) {
    if (!d_params || !d_x || !d_y || !d_work || batch == 0) return MPDP_EINVAL;
    if (work_size < work_bytes(batch)) return MPDP_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Params p = params_at(d_params);
    const Work w = work_at(d_work, batch);
    HIPCHK(forward(p, d_x, batch, w, w.logit, s));
    HIPCHK(backward(p, d_x, d_y, batch, w, s));
    if (loss_out) {
        float l = 0.f;
        HIPCHK(hipMemcpyAsync(&l, w.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *loss_out = l / (float)batch;
    }
    return MPDP_OK;
}

mpdp_status mpdp_scorer_train_step(void *d_params, const uint16_t *d_x, const float *d_y, uint32_t batch, float lr,
                                   uint32_t step, void *d_work, size_t work_size, void *hip_stream, float *loss_out) {
    if (step == 0 || !(lr > 0.f)) return MPDP_EINVAL;
    mpdp_status st = mpdp_scorer_grad(d_params, d_x, d_y, batch, d_work, work_size, hip_stream, loss_out);
    if (st != MPDP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const Params p = params_at(d_params);
    const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, s, p.w1, p.g, p.m, p.v, kNParams, lr, c1, c2);
    HIPCHK(hipGetLastError());
    HIPCHK(refresh_bf16(p, s));
    return MPDP_OK;
}

}  // extern "C"
