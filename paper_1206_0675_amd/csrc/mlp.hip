// Training and inference of the learned-step network (16 -> 64 -> 64 -> 16,
// ReLU) on the GPU: lgf_mlp_train, lgf_mlp_grad, lgf_mlp_eval.
//
// The forward pass uses bfloat16-rounded weights with float32 accumulation;
// Adam updates float32 master weights and re-rounds the working copy after
// every step (the model blob stores the rounded weights and float32
// biases).  Forward and backward of a minibatch run in one workgroup; every
// sum over samples is taken in a fixed order, so training is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "runtime.hpp"

using namespace lgf;
using namespace lgf::rt;

namespace {

constexpr int NB = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NB * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NB, NPARAM = OFF_B3 + NB;   // 6288
constexpr int32_t kMagic = kModelMagic;
constexpr size_t kBlobBytes = kModelBytes;
constexpr int kMaxBatch = 1024;

__device__ __forceinline__ float bf16_round(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    float r;
    __builtin_memcpy(&r, &u, 4);
    return r;
}

// scratch per sample: h1[64], h2[64], d2[64], d1[64], d3[16]
constexpr int kAct = 4 * NH + NB;

// Loss sum(m (y - t)^2) / msum and its gradient for the samples idx[0..B).
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_mlp_fwd_bwd(const float* __restrict__ w, const float* __restrict__ X,
                                                     const float* __restrict__ Y, const float* __restrict__ M,
                                                     const int* __restrict__ idx, int B, float* __restrict__ act,
                                                     float* __restrict__ grad, float* __restrict__ loss_out)
{
    __shared__ float red[256];
    __shared__ float msum_s;
    const int tid = threadIdx.x, nth = blockDim.x;
    // sum of the mask over the minibatch (fixed order)
    float ms = 0.f;
    for (int i = tid; i < B * NB; i += nth) ms += M[(int64_t)idx[i / NB] * NB + i % NB];
    red[tid] = ms;
    __syncthreads();
    for (int h = nth >> 1; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) msum_s = red[0] > 0.f ? red[0] : 1.f;
    __syncthreads();
    const float inv = 1.f / msum_s;
    float lp = 0.f;
    for (int n = tid; n < B; n += nth) {
        const int64_t s = idx[n];
        float* a = act + (int64_t)n * kAct;
        float x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = X[s * NB + i];
        for (int j = 0; j < NH; ++j) {
            float z = w[OFF_B1 + j];
#pragma unroll
            for (int i = 0; i < NB; ++i) z = fmaf(x[i], w[OFF_W1 + i * NH + j], z);
            a[j] = z > 0.f ? z : 0.f;
        }
        for (int j = 0; j < NH; ++j) {
            float z = w[OFF_B2 + j];
            for (int i = 0; i < NH; ++i) z = fmaf(a[i], w[OFF_W2 + i * NH + j], z);
            a[NH + j] = z > 0.f ? z : 0.f;
        }
        for (int k = 0; k < NB; ++k) {
            float y = w[OFF_B3 + k];
            for (int i = 0; i < NH; ++i) y = fmaf(a[NH + i], w[OFF_W3 + i * NB + k], y);
            const float m = M[s * NB + k], r = (y - Y[s * NB + k]) * m;
            lp += r * (y - Y[s * NB + k]);
            a[4 * NH + k] = 2.f * r * inv;
        }
    }
    __syncthreads();
    // d2 = (d3 W3^T) * [h2 > 0]
    for (int e = tid; e < B * NH; e += nth) {
        const int n = e / NH, j = e % NH;
        float* a = act + (int64_t)n * kAct;
        float v = 0.f;
        for (int k = 0; k < NB; ++k) v = fmaf(a[4 * NH + k], w[OFF_W3 + j * NB + k], v);
        a[2 * NH + j] = a[NH + j] > 0.f ? v : 0.f;
    }
    __syncthreads();
    // d1 = (d2 W2^T) * [h1 > 0]
    for (int e = tid; e < B * NH; e += nth) {
        const int n = e / NH, i = e % NH;
        float* a = act + (int64_t)n * kAct;
        float v = 0.f;
        for (int j = 0; j < NH; ++j) v = fmaf(a[2 * NH + j], w[OFF_W2 + i * NH + j], v);
        a[3 * NH + i] = a[i] > 0.f ? v : 0.f;
    }
    __syncthreads();
    // parameter gradients, summed over the minibatch in sample order
    for (int e = tid; e < NPARAM; e += nth) {
        float g = 0.f;
        if (e < OFF_B1) {                       // W1[a][i] = sum x[a] d1[i]
            const int ai = e - OFF_W1, ia = ai / NH, ii = ai % NH;
            for (int n = 0; n < B; ++n) g = fmaf(X[(int64_t)idx[n] * NB + ia], act[(int64_t)n * kAct + 3 * NH + ii], g);
        } else if (e < OFF_W2) {
            const int ii = e - OFF_B1;
            for (int n = 0; n < B; ++n) g += act[(int64_t)n * kAct + 3 * NH + ii];
        } else if (e < OFF_B2) {                // W2[i][j] = sum h1[i] d2[j]
            const int ij = e - OFF_W2, ii = ij / NH, jj = ij % NH;
            for (int n = 0; n < B; ++n) g = fmaf(act[(int64_t)n * kAct + ii], act[(int64_t)n * kAct + 2 * NH + jj], g);
        } else if (e < OFF_W3) {
            const int jj = e - OFF_B2;
            for (int n = 0; n < B; ++n) g += act[(int64_t)n * kAct + 2 * NH + jj];
        } else if (e < OFF_B3) {                // W3[j][k] = sum h2[j] d3[k]
            const int jk = e - OFF_W3, jj = jk / NB, kk = jk % NB;
            for (int n = 0; n < B; ++n) g = fmaf(act[(int64_t)n * kAct + NH + jj], act[(int64_t)n * kAct + 4 * NH + kk], g);
        } else {
            const int kk = e - OFF_B3;
            for (int n = 0; n < B; ++n) g += act[(int64_t)n * kAct + 4 * NH + kk];
        }
        grad[e] = g;
    }
    red[tid] = lp;
    __syncthreads();
    for (int h = nth >> 1; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0 && loss_out) *loss_out = red[0] * inv;
}

// Adam on the float32 master weights; working copy = bf16-rounded weights,
// float32 biases.
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ master, const float* __restrict__ g,
                                              float* __restrict__ m1, float* __restrict__ m2, float* __restrict__ work,
                                              float lr, float beta1, float beta2, float eps, float corr1, float corr2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPARAM) return;
    const float gi = g[e];
    const float a = beta1 * m1[e] + (1.f - beta1) * gi;
    const float b = beta2 * m2[e] + (1.f - beta2) * gi * gi;
    m1[e] = a;
    m2[e] = b;
    const float w = master[e] - lr * (a / corr1) / (sqrtf(b / corr2) + eps);
    master[e] = w;
    const bool is_bias = (e >= OFF_B1 && e < OFF_W2) || (e >= OFF_B2 && e < OFF_W3) || e >= OFF_B3;
    work[e] = is_bias ? w : bf16_round(w);
}

template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ w, const float* __restrict__ X, int64_t n,
                                                     float* __restrict__ Y)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[NB], h1[NH];
#pragma unroll
    for (int i = 0; i < NB; ++i) x[i] = X[s * NB + i];
    for (int j = 0; j < NH; ++j) {
        float z = w[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NB; ++i) z = fmaf(x[i], w[OFF_W1 + i * NH + j], z);
        h1[j] = z > 0.f ? z : 0.f;
    }
    float y[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) y[k] = w[OFF_B3 + k];
    for (int j = 0; j < NH; ++j) {
        float z = w[OFF_B2 + j];
        for (int i = 0; i < NH; ++i) z = fmaf(h1[i], w[OFF_W2 + i * NH + j], z);
        const float h = z > 0.f ? z : 0.f;
#pragma unroll
        for (int k = 0; k < NB; ++k) y[k] = fmaf(h, w[OFF_W3 + j * NB + k], y[k]);
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) Y[s * NB + k] = y[k];
}

uint16_t host_bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

float host_bf16_value(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// blob <-> flat float parameters (weights as their bf16 values)
bool blob_to_flat(const void* blob, size_t bytes, std::vector<float>& w)
{
    if (!blob || bytes != kBlobBytes) return false;
    const int32_t* h = static_cast<const int32_t*>(blob);
    if (h[0] != kMagic || h[1] != 1 || h[2] != NB || h[3] != NH || h[4] != NH || h[5] != NB) return false;
    w.assign(NPARAM, 0.f);
    const uint16_t* wb = reinterpret_cast<const uint16_t*>(static_cast<const char*>(blob) + 32);
    const float* bb = reinterpret_cast<const float*>(static_cast<const char*>(blob) + 32 + 2 * (NB * NH + NH * NH + NH * NB));
    for (int i = 0; i < NB * NH; ++i) w[OFF_W1 + i] = host_bf16_value(wb[i]);
    for (int i = 0; i < NH * NH; ++i) w[OFF_W2 + i] = host_bf16_value(wb[NB * NH + i]);
    for (int i = 0; i < NH * NB; ++i) w[OFF_W3 + i] = host_bf16_value(wb[NB * NH + NH * NH + i]);
    for (int i = 0; i < NH; ++i) w[OFF_B1 + i] = bb[i];
    for (int i = 0; i < NH; ++i) w[OFF_B2 + i] = bb[NH + i];
    for (int i = 0; i < NB; ++i) w[OFF_B3 + i] = bb[2 * NH + i];
    return true;
}

void flat_to_blob(const std::vector<float>& w, void* blob)
{
    int32_t* h = static_cast<int32_t*>(blob);
    const int32_t head[8] = {kMagic, 1, NB, NH, NH, NB, 0, 0};
    std::memcpy(h, head, sizeof head);
    uint16_t* wb = reinterpret_cast<uint16_t*>(static_cast<char*>(blob) + 32);
    float* bb = reinterpret_cast<float*>(static_cast<char*>(blob) + 32 + 2 * (NB * NH + NH * NH + NH * NB));
    for (int i = 0; i < NB * NH; ++i) wb[i] = host_bf16_bits(w[OFF_W1 + i]);
    for (int i = 0; i < NH * NH; ++i) wb[NB * NH + i] = host_bf16_bits(w[OFF_W2 + i]);
    for (int i = 0; i < NH * NB; ++i) wb[NB * NH + NH * NH + i] = host_bf16_bits(w[OFF_W3 + i]);
    for (int i = 0; i < NH; ++i) bb[i] = w[OFF_B1 + i];
    for (int i = 0; i < NH; ++i) bb[NH + i] = w[OFF_B2 + i];
    for (int i = 0; i < NB; ++i) bb[2 * NH + i] = w[OFF_B3 + i];
}

// Device buffers of one training or evaluation call.
struct MlpRun : Runner {
    float *w = nullptr, *master = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr, *act = nullptr;
    float *X = nullptr, *Y = nullptr, *M = nullptr, *loss = nullptr;
    int* idx = nullptr;
    ~MlpRun()
    {
        for (void* p : {(void*)w, (void*)master, (void*)g, (void*)m1, (void*)m2, (void*)act, (void*)X, (void*)Y,
                        (void*)M, (void*)loss, (void*)idx})
            (void)hipFree(p);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

int32_t upload(MlpRun& r, float** dst, const void* src, size_t bytes)
{
    HIPCHK(&r, hipMalloc(dst, bytes ? bytes : 4));
    if (bytes && src) HIPCHK(&r, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return LGF_OK;
}

}  // namespace

extern "C" {

size_t lgf_model_bytes(void) { return kBlobBytes; }

int32_t lgf_mlp_eval(const void* blob, size_t bytes, const float* X, int64_t n, float* Y)
{
    std::vector<float> w;
    if (!blob_to_flat(blob, bytes, w)) return fail(nullptr, LGF_E_MODEL, "malformed model blob");
    if (!X || !Y || n < 1) return fail(nullptr, LGF_E_INVALID_ARG, "bad arrays");
    MlpRun r;
    HIPCHK(&r, hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
    TRY(upload(r, &r.w, w.data(), sizeof(float) * NPARAM));
    TRY(upload(r, &r.X, X, sizeof(float) * NB * n));
    TRY(upload(r, &r.Y, nullptr, sizeof(float) * NB * n));
    TRY(launch(&r, K_MLP, k_mlp_forward<>, dim3((unsigned)blocks_for(n, 256)), dim3(256), 0, (const float*)r.w,
               (const float*)r.X, n, r.Y));
    HIPCHK(&r, hipStreamSynchronize(r.stream));
    HIPCHK(&r, hipMemcpy(Y, r.Y, sizeof(float) * NB * n, hipMemcpyDeviceToHost));
    return LGF_OK;
}

int32_t lgf_mlp_grad(const void* blob, size_t bytes, const float* X, const float* Y, const float* M, int64_t n,
                     float* grad, double* loss)
{
    std::vector<float> w;
    if (!blob_to_flat(blob, bytes, w)) return fail(nullptr, LGF_E_MODEL, "malformed model blob");
    if (!X || !Y || !M || !grad || n < 1 || n > kMaxBatch) return fail(nullptr, LGF_E_INVALID_ARG, "bad arrays");
    MlpRun r;
    HIPCHK(&r, hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
    std::vector<int> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
    TRY(upload(r, &r.w, w.data(), sizeof(float) * NPARAM));
    TRY(upload(r, &r.X, X, sizeof(float) * NB * n));
    TRY(upload(r, &r.Y, Y, sizeof(float) * NB * n));
    TRY(upload(r, &r.M, M, sizeof(float) * NB * n));
    TRY(upload(r, &r.g, nullptr, sizeof(float) * NPARAM));
    TRY(upload(r, &r.act, nullptr, sizeof(float) * kAct * n));
    TRY(upload(r, &r.loss, nullptr, sizeof(float)));
    HIPCHK(&r, hipMalloc(&r.idx, sizeof(int) * n));
    HIPCHK(&r, hipMemcpy(r.idx, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    TRY(launch(&r, K_MLP, k_mlp_fwd_bwd<>, dim3(1), dim3(256), 0, (const float*)r.w, (const float*)r.X,
               (const float*)r.Y, (const float*)r.M, (const int*)r.idx, (int)n, r.act, r.g, r.loss));
    HIPCHK(&r, hipStreamSynchronize(r.stream));
    HIPCHK(&r, hipMemcpy(grad, r.g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    float l = 0.f;
    HIPCHK(&r, hipMemcpy(&l, r.loss, sizeof(float), hipMemcpyDeviceToHost));
    if (loss) *loss = l;
    return LGF_OK;
}

int32_t lgf_mlp_train(const float* X, const float* Y, const float* M, int64_t n, const lgf_train_params* tp,
                      void* blob_out, size_t* bytes, float* loss_trace)
{
    if (!X || !Y || !M || !tp || !blob_out || !bytes || n < 1) return fail(nullptr, LGF_E_INVALID_ARG, "bad arguments");
    if (*bytes < kBlobBytes) {
        *bytes = kBlobBytes;
        return fail(nullptr, LGF_E_INVALID_ARG, "blob buffer too small");
    }
    const int B = (int)std::min<int64_t>(std::max(1, tp->batch), std::min<int64_t>(n, kMaxBatch));
    if (tp->steps < 0 || !(tp->lr > 0.f)) return fail(nullptr, LGF_E_INVALID_ARG, "steps >= 0 and lr > 0");
    // He-normal weights, zero biases: the untrained network outputs ~0, i.e.
    // factors ~1 (the plain step)
    std::vector<float> w(NPARAM, 0.f);
    std::mt19937_64 rng((uint64_t)tp->seed);
    auto init = [&](int off, int fan_in, int count, float gain) {
        std::normal_distribution<float> nd(0.f, gain * std::sqrt(2.f / (float)fan_in));
        for (int i = 0; i < count; ++i) w[off + i] = nd(rng);
    };
    init(OFF_W1, NB, NB * NH, 1.f);
    init(OFF_W2, NH, NH * NH, 1.f);
    init(OFF_W3, NH, NH * NB, 0.1f);
    std::vector<float> work(w);
    for (int i = OFF_W1; i < OFF_B1; ++i) work[i] = host_bf16_value(host_bf16_bits(w[i]));
    for (int i = OFF_W2; i < OFF_B2; ++i) work[i] = host_bf16_value(host_bf16_bits(w[i]));
    for (int i = OFF_W3; i < OFF_B3; ++i) work[i] = host_bf16_value(host_bf16_bits(w[i]));
    MlpRun r;
    HIPCHK(&r, hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
    TRY(upload(r, &r.master, w.data(), sizeof(float) * NPARAM));
    TRY(upload(r, &r.w, work.data(), sizeof(float) * NPARAM));
    std::vector<float> zeros(NPARAM, 0.f);
    TRY(upload(r, &r.m1, zeros.data(), sizeof(float) * NPARAM));
    TRY(upload(r, &r.m2, zeros.data(), sizeof(float) * NPARAM));
    TRY(upload(r, &r.g, nullptr, sizeof(float) * NPARAM));
    TRY(upload(r, &r.X, X, sizeof(float) * NB * n));
    TRY(upload(r, &r.Y, Y, sizeof(float) * NB * n));
    TRY(upload(r, &r.M, M, sizeof(float) * NB * n));
    TRY(upload(r, &r.act, nullptr, sizeof(float) * kAct * B));
    TRY(upload(r, &r.loss, nullptr, sizeof(float) * (tp->steps > 0 ? tp->steps : 1)));
    HIPCHK(&r, hipMalloc(&r.idx, sizeof(int) * n));
    std::vector<int> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
    const float b1 = 0.9f, b2 = 0.999f;
    int64_t pos = n;   // forces a shuffle before the first minibatch
    for (int64_t t = 1; t <= tp->steps; ++t) {
        if (pos + B > n) {
            std::shuffle(perm.begin(), perm.end(), rng);
            HIPCHK(&r, hipMemcpyAsync(r.idx, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, r.stream));
            HIPCHK(&r, hipStreamSynchronize(r.stream));
            pos = 0;
        }
        TRY(launch(&r, K_MLP, k_mlp_fwd_bwd<>, dim3(1), dim3(256), 0, (const float*)r.w, (const float*)r.X,
                   (const float*)r.Y, (const float*)r.M, (const int*)(r.idx + pos), B, r.act, r.g, r.loss + (t - 1)));
        const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
        TRY(launch(&r, K_MLP, k_adam<>, dim3((unsigned)blocks_for(NPARAM, 256)), dim3(256), 0, r.master,
                   (const float*)r.g, r.m1, r.m2, r.w, tp->lr, b1, b2, 1e-8f, c1, c2));
        pos += B;
    }
    HIPCHK(&r, hipStreamSynchronize(r.stream));
    HIPCHK(&r, hipMemcpy(w.data(), r.master, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    if (loss_trace && tp->steps > 0)
        HIPCHK(&r, hipMemcpy(loss_trace, r.loss, sizeof(float) * tp->steps, hipMemcpyDeviceToHost));
    flat_to_blob(w, blob_out);
    *bytes = kBlobBytes;
    return LGF_OK;
}

}  // extern "C"
