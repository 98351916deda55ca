// Training kernels for the beam-width predictor (not part of the paper):
// a 16 -> 64 -> 64 -> 1 ReLU network fitted by minibatch Adam to the mean
// squared error.  Parameters are FP32 masters in the layout
// W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3 (5313 values).
//
// Per minibatch:
//   block_grad_kernel : one 64-lane wavefront per tile of samples; lane j owns
//                       hidden unit j of both layers.  For each sample of its
//                       tile (in order) it runs the forward pass, the output
//                       residual and the backward pass, accumulating the
//                       gradient rows of its units in registers; the tile's
//                       partial gradient (and squared-residual sum) goes to
//                       scratch
//   reduce_kernel     : one thread per parameter sums the tiles' partials in
//                       tile order (deterministic, no atomics)
//   adam_kernel       : one thread per parameter
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "jag_internal.h"

namespace jag {
namespace {

constexpr int NP = kPredParams;
constexpr int NPP = NP + 1;  // parameters + the squared-residual sum
constexpr int OFF_B1 = 1024, OFF_W2 = 1088, OFF_B2 = 5184, OFF_W3 = 5248, OFF_B3 = 5312;
constexpr int TILE = 64;     // samples per wavefront

__global__ __launch_bounds__(64) void block_grad_kernel(const float *__restrict P, const float *__restrict X,
                                                        const float *__restrict T,
                                                        const int32_t *__restrict idx, int B,
                                                        float inv_total, float *__restrict partial)
{
    __shared__ float W2s[64 * 64];
    __shared__ float h1s[64];
    __shared__ float dz2s[64];
    __shared__ float xs[16];
    const int j = threadIdx.x;
    for (int t = j; t < 64 * 64; t += 64) W2s[t] = P[OFF_W2 + t];
    float w1[16], gw1[16], w2[64], gw2[64];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        w1[i] = P[j * 16 + i];
        gw1[i] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < 64; i++) {
        w2[i] = P[OFF_W2 + j * 64 + i];
        gw2[i] = 0.f;
    }
    const float b1 = P[OFF_B1 + j], b2 = P[OFF_B2 + j], w3 = P[OFF_W3 + j], b3 = P[OFF_B3];
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, sq = 0.f;
    __syncthreads();
    const int s0 = blockIdx.x * TILE, s1 = min(B, s0 + TILE);
    for (int b = s0; b < s1; b++) {
        const int r = idx ? idx[b] : b;
        if (j < 16) xs[j] = X[(int64_t)r * 16 + j];
        __syncthreads();
        float z1 = b1;
#pragma unroll
        for (int i = 0; i < 16; i++) z1 = __builtin_fmaf(w1[i], xs[i], z1);
        float h1 = z1 > 0.f ? z1 : 0.f;
        h1s[j] = h1;
        __syncthreads();
        float z2 = b2;
#pragma unroll
        for (int i = 0; i < 64; i++) z2 = __builtin_fmaf(w2[i], h1s[i], z2);
        float h2 = z2 > 0.f ? z2 : 0.f;
        float y = w3 * h2;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) y += __shfl_xor(y, m, 64);
        y += b3;
        float res = y - T[r];
        sq += res * res;
        float dy = 2.f * res * inv_total;
        float dz2 = z2 > 0.f ? dy * w3 : 0.f;
        dz2s[j] = dz2;
        __syncthreads();
        // lane j doubles as input unit j of layer 2: dh1_j = sum_u dz2_u W2[u][j]
        float dh1 = 0.f;
#pragma unroll
        for (int u = 0; u < 64; u++) dh1 = __builtin_fmaf(dz2s[u], W2s[u * 64 + j], dh1);
        float dz1 = z1 > 0.f ? dh1 : 0.f;
#pragma unroll
        for (int i = 0; i < 16; i++) gw1[i] = __builtin_fmaf(dz1, xs[i], gw1[i]);
        gb1 += dz1;
#pragma unroll
        for (int i = 0; i < 64; i++) gw2[i] = __builtin_fmaf(dz2, h1s[i], gw2[i]);
        gb2 += dz2;
        gw3 = __builtin_fmaf(dy, h2, gw3);
        gb3 += dy;
        __syncthreads();
    }
    float *o = partial + (int64_t)blockIdx.x * NPP;
#pragma unroll
    for (int i = 0; i < 16; i++) o[j * 16 + i] = gw1[i];
    o[OFF_B1 + j] = gb1;
#pragma unroll
    for (int i = 0; i < 64; i++) o[OFF_W2 + j * 64 + i] = gw2[i];
    o[OFF_B2 + j] = gb2;
    o[OFF_W3 + j] = gw3;
    if (j == 0) {
        o[OFF_B3] = gb3;
        o[NP] = sq;
    }
}

// G[t] = sum over tiles in order; the last slot becomes the mean squared residual
__global__ void reduce_kernel(const float *__restrict partial, int ntiles, int B, float *__restrict G,
                              float *__restrict loss)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPP) return;
    float acc = 0.f;
    for (int b = 0; b < ntiles; b++) acc += partial[(int64_t)b * NPP + t];
    if (t == NP) *loss = acc / (float)B;
    else G[t] = acc;
}

__global__ void adam_kernel(float *__restrict P, const float *__restrict G, float *__restrict M,
                            float *__restrict V, float lr, float b1, float b2, float c1, float c2,
                            float eps)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NP) return;
    float g = G[t];
    float m = b1 * M[t] + (1.f - b1) * g;
    float v = b2 * V[t] + (1.f - b2) * g * g;
    M[t] = m;
    V[t] = v;
    P[t] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

#define HIPCHK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));             \
            return e_ == hipErrorOutOfMemory ? JAG_ENOMEM : JAG_EDEVICE;           \
        }                                                                          \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

jag_status predictor_grad(const float *features, const float *targets, int64_t m,
                          const float *params, float *loss_out, float *grad_out, void *stream)
{
    if (m > (1 << 24)) {
        set_error("at most 2^24 samples");
        return JAG_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    int B = (int)m;
    int ntiles = (B + TILE - 1) / TILE;
    DevBuf scratch, pbuf;
    HIPCHK(hipMalloc(&scratch.p, sizeof(float) * (size_t)ntiles * NPP));
    HIPCHK(hipMalloc(&pbuf.p, sizeof(float) * (2 * NP + 2)));
    float *dP = static_cast<float *>(pbuf.p), *dG = dP + NP, *dL = dG + NP;
    float *part = static_cast<float *>(scratch.p);
    HIPCHK(hipMemcpyAsync(dP, params, sizeof(float) * NP, hipMemcpyHostToDevice, st));
    block_grad_kernel<<<ntiles, 64, 0, st>>>(dP, features, targets, nullptr, B, 1.f / (float)B, part);
    reduce_kernel<<<(NPP + 127) / 128, 128, 0, st>>>(part, ntiles, B, dG, dL);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(grad_out, dG, sizeof(float) * NP, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(loss_out, dL, sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return JAG_OK;
}

jag_status train_predictor(const float *features, const float *targets, int64_t m,
                           float *params_inout, int32_t epochs, int32_t batch, float lr,
                           uint64_t seed, float *loss_out, void *stream)
{
    if (m > (1 << 24)) {
        set_error("at most 2^24 samples");
        return JAG_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    int B = (int)std::min<int64_t>(batch, m);
    int maxtiles = (B + TILE - 1) / TILE;
    DevBuf scratch, pbuf, ibuf;
    HIPCHK(hipMalloc(&scratch.p, sizeof(float) * (size_t)maxtiles * NPP));
    float *part = static_cast<float *>(scratch.p);
    HIPCHK(hipMalloc(&pbuf.p, sizeof(float) * (4 * NP + 2)));
    float *dP = static_cast<float *>(pbuf.p), *dG = dP + NP, *dM = dG + NP, *dV = dM + NP,
          *dL = dV + NP;
    HIPCHK(hipMalloc(&ibuf.p, sizeof(int32_t) * m));
    int32_t *dIdx = static_cast<int32_t *>(ibuf.p);
    HIPCHK(hipMemcpyAsync(dP, params_inout, sizeof(float) * NP, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(dM, 0, sizeof(float) * 2 * NP, st));
    std::vector<int32_t> perm(m);
    std::iota(perm.begin(), perm.end(), 0);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int64_t step = 0;
    int nb = (int)((m + B - 1) / B);
    std::vector<float> batch_loss(nb);
    for (int ep = 0; ep < epochs; ep++) {
        uint64_t z = mix64(seed + 0x51ED27ull * (uint64_t)(ep + 1));
        for (int64_t i = m - 1; i > 0; i--) {
            z = mix64(z);
            std::swap(perm[i], perm[(int64_t)(z % (uint64_t)(i + 1))]);
        }
        HIPCHK(hipMemcpyAsync(dIdx, perm.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        double ep_loss = 0.0;
        for (int bi = 0; bi < nb; bi++) {
            int b0 = bi * B;
            int bs = (int)std::min<int64_t>(B, m - b0);
            step++;
            float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
            int nt = (bs + TILE - 1) / TILE;
            block_grad_kernel<<<nt, 64, 0, st>>>(dP, features, targets, dIdx + b0, bs,
                                                 1.f / (float)bs, part);
            reduce_kernel<<<(NPP + 127) / 128, 128, 0, st>>>(part, nt, bs, dG, dL);
            adam_kernel<<<(NP + 127) / 128, 128, 0, st>>>(dP, dG, dM, dV, lr, b1, b2, c1, c2, eps);
            HIPCHK(hipGetLastError());
            if (loss_out) {
                HIPCHK(hipMemcpyAsync(&batch_loss[bi], dL, sizeof(float), hipMemcpyDeviceToHost, st));
            }
        }
        if (loss_out) {
            HIPCHK(hipStreamSynchronize(st));
            for (int bi = 0; bi < nb; bi++) ep_loss += batch_loss[bi];
            loss_out[ep] = (float)(ep_loss / nb);
        }
    }
    HIPCHK(hipMemcpyAsync(params_inout, dP, sizeof(float) * NP, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return JAG_OK;
}

}  // namespace jag
