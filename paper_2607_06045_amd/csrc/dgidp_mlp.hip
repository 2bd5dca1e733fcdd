// Learned troubled-cell / AMR indicator for gfx950: a 16 -> 64 -> 64 -> 1 ReLU
// network with BF16 weights, MSE loss and Adam on FP32 master weights.
// Inference multiplies BF16 operands (weights, inputs, first hidden layer) on
// the matrix cores with FP32 accumulation; training runs in FP32 arithmetic on
// the BF16 weights.
//
// Parameter vector (5313 floats): W1[64][16], b1[64], W2[64][64], b2[64],
// W3[64], b3 (W[j][k]: output unit j, input k).  The device keeps the FP32
// masters, Adam's moments and a BF16 copy (round to nearest even) that the
// forward and backward passes read; the gradient is taken at the BF16 weights
// and applied to the masters.
//
//  k_mlp_forward   inference on the matrix cores (BF16 products, FP32
//                  accumulation), 32 samples per wave
//  k_mlp_grad      64 samples per pass, 256 threads: forward and backward
//                  vectors of the samples in LDS (four threads per sample, 16
//                  hidden units each), then each thread owns every 256th
//                  parameter and accumulates its gradient over the block's
//                  passes in LDS; one partial row per block
//  k_mlp_update    one thread per parameter: sums the block partials in a fixed
//                  order (deterministic), Adam step, new BF16 copy
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "dgidp_internal.h"
#include "dgidp_mlp_dev.h"

namespace dgidp {

namespace {

using namespace mlp;

constexpr int kRow = kNP + 1;   // partial row: gradient, then the loss sum
constexpr int kGS = 64;         // samples per pass of the gradient kernel
constexpr int kMaxGradBlocks = 1024;

__global__ __launch_bounds__(256) void k_mlp_round(const float* __restrict__ master,
                                                   uint16_t* __restrict__ wb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNP) wb[p] = bf16_rne(master[p]);
}

// inference: 32 samples per wave (the matrix-core pass of forward32), four
// waves per block sharing one LDS copy of the weights; each wave loops over
// its tiles
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ x, int B,
                                                     const uint16_t* __restrict__ wb,
                                                     float* __restrict__ y)
{
    __shared__ __align__(16) LdsWeights sW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = lane & 31, hf = lane >> 5;
    stage_weights(sW, wb, threadIdx.x, 256);
    __syncthreads();
    const int ntiles = (B + 31) / 32;
#pragma unroll 1
    for (int tile = blockIdx.x * 4 + wv; tile < ntiles; tile += gridDim.x * 4) {
        const int s = tile * 32 + c;
        float v[8];
        if (s < B) {
            const float4 p0 = *(const float4*)(x + (size_t)s * kNin + hf * 8);
            const float4 p1 = *(const float4*)(x + (size_t)s * kNin + hf * 8 + 4);
            v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
            v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = 0.0f;
        }
        // an opaque zero offset keeps the weight reads inside the loop (hoisted,
        // they would hold some 140 registers)
        int z = 0;
        asm volatile("" : "+v"(z));
        const LdsWeights& L = *reinterpret_cast<const LdsWeights*>(reinterpret_cast<const char*>(&sW) + z);
        const float o = forward32(L, pack_bf16x8(v), lane);
        if (hf == 0 && s < B) y[s] = o;
    }
}

// gradient of loss = (1/B) sum (y - t)^2 at the BF16 weights; block b handles
// the passes b, b + gridDim.x, ... of kGS samples and writes one partial row
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ x,
                                                  const float* __restrict__ t, int B,
                                                  const uint16_t* __restrict__ wb,
                                                  float* __restrict__ partial)
{
    __shared__ float sw[kNP];
    __shared__ float sX[kGS][kNin + 1];
    __shared__ float sH1[kGS][kNh + 1];
    __shared__ float sH2[kGS][kNh + 1];
    __shared__ float sD1[kGS][kNh + 1];
    __shared__ float sD2[kGS][kNh + 1];
    __shared__ float sDY[kGS];
    __shared__ float sL[kGS];
    __shared__ float sAcc[kNP];  // this block's gradient; entry p belongs to thread p % 256
    const int tid = threadIdx.x;
    for (int p = tid; p < kNP; p += 256) {
        sw[p] = bf16_f(wb[p]);
        sAcc[p] = 0.0f;
    }
    const int s = tid & (kGS - 1), part = tid >> 6;  // sample, quarter of the hidden units
    float lsum = 0.0f;
    const float invB = 1.0f / (float)B;
    const int npass = (B + kGS - 1) / kGS;
    for (int pass = blockIdx.x; pass < npass; pass += gridDim.x) {
        const int gs = pass * kGS + s;
        const bool valid = gs < B;
        __syncthreads();  // previous pass done with the sample arrays; weights staged
        if (part == 0)
            for (int k = 0; k < kNin; ++k) sX[s][k] = valid ? x[(size_t)gs * kNin + k] : 0.0f;
        __syncthreads();
        for (int jj = 0; jj < 16; ++jj) {
            const int j = part * 16 + jj;
            float z = sw[kOffB1 + j];
#pragma unroll
            for (int k = 0; k < kNin; ++k) z = fmaf(sw[kOffW1 + j * kNin + k], sX[s][k], z);
            sH1[s][j] = fmaxf(z, 0.0f);
        }
        __syncthreads();
        for (int jj = 0; jj < 16; ++jj) {
            const int j = part * 16 + jj;
            float z = sw[kOffB2 + j];
#pragma unroll 16
            for (int k = 0; k < kNh; ++k) z = fmaf(sw[kOffW2 + j * kNh + k], sH1[s][k], z);
            sH2[s][j] = fmaxf(z, 0.0f);
        }
        __syncthreads();
        if (part == 0) {
            float yv = sw[kOffB3];
            for (int j = 0; j < kNh; ++j) yv = fmaf(sw[kOffW3 + j], sH2[s][j], yv);
            const float r = valid ? yv - t[gs] : 0.0f;
            sDY[s] = 2.0f * r * invB;
            sL[s] = r * r;
        }
        __syncthreads();
        for (int jj = 0; jj < 16; ++jj) {
            const int j = part * 16 + jj;
            sD2[s][j] = sH2[s][j] > 0.0f ? sDY[s] * sw[kOffW3 + j] : 0.0f;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) {
            const int k = part * 16 + kk;
            float d = 0.0f;
            if (sH1[s][k] > 0.0f)
#pragma unroll 16
                for (int j = 0; j < kNh; ++j) d = fmaf(sw[kOffW2 + j * kNh + k], sD2[s][j], d);
            sD1[s][k] = d;
        }
        __syncthreads();
        // parameter gradients of this pass
#pragma unroll 1
        for (int p = tid; p < kNP; p += 256) {
            float g = 0.0f;
            if (p < kOffB1) {
                const int j = p / kNin, k = p - j * kNin;
                for (int q = 0; q < kGS; ++q) g = fmaf(sD1[q][j], sX[q][k], g);
            } else if (p < kOffW2) {
                const int j = p - kOffB1;
                for (int q = 0; q < kGS; ++q) g += sD1[q][j];
            } else if (p < kOffB2) {
                const int j = (p - kOffW2) / kNh, k = (p - kOffW2) - j * kNh;
                for (int q = 0; q < kGS; ++q) g = fmaf(sD2[q][j], sH1[q][k], g);
            } else if (p < kOffW3) {
                const int j = p - kOffB2;
                for (int q = 0; q < kGS; ++q) g += sD2[q][j];
            } else if (p < kOffB3) {
                const int j = p - kOffW3;
                for (int q = 0; q < kGS; ++q) g = fmaf(sDY[q], sH2[q][j], g);
            } else {
                for (int q = 0; q < kGS; ++q) g += sDY[q];
            }
            sAcc[p] += g;
        }
        if (tid == 0)
            for (int q = 0; q < kGS; ++q) lsum += sL[q];
    }
    float* row = partial + (size_t)blockIdx.x * kRow;
    for (int p = tid; p < kNP; p += 256) row[p] = sAcc[p];
    if (tid == 0) row[kNP] = lsum;
}

// sum of the block partials in block order; Adam when lr > 0
__global__ __launch_bounds__(256) void k_mlp_update(const float* __restrict__ partial, int nblk,
                                                    float* master, float* m, float* v,
                                                    uint16_t* wb, float lr, float bc1, float bc2,
                                                    float* grad_out, float* loss_out, int B)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNP) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += partial[(size_t)b * kRow + p];
    if (p == kNP) {
        if (loss_out) *loss_out = g / (float)B;
        return;
    }
    if (grad_out) grad_out[p] = g;
    if (lr > 0.0f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mn = b1 * m[p] + (1.0f - b1) * g;
        const float vn = b2 * v[p] + (1.0f - b2) * g * g;
        m[p] = mn;
        v[p] = vn;
        const float w = master[p] - lr * (mn / bc1) / (sqrtf(vn / bc2) + eps);
        master[p] = w;
        wb[p] = bf16_rne(w);
    }
}

}  // namespace

struct MlpState {
    float* master = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    uint16_t* wb = nullptr;
    float* partial = nullptr;
    float* loss = nullptr;
    float* scratch[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t scratch_cap[4] = {0, 0, 0, 0};
    int t = 0;
    bool has_weights = false;
};

int mlp_num_params() { return kNP; }

MlpState* mlp_create()
{
    MlpState* s = new MlpState();
    if (hipMalloc((void**)&s->master, kNP * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&s->m, kNP * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&s->v, kNP * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&s->wb, kNPpad * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void**)&s->partial, (size_t)kMaxGradBlocks * kRow * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&s->loss, sizeof(float)) != hipSuccess ||
        hipMemset(s->wb, 0, kNPpad * sizeof(uint16_t)) != hipSuccess) {
        mlp_destroy(s);
        return nullptr;
    }
    return s;
}

void mlp_destroy(MlpState* s)
{
    if (!s) return;
    for (void* p : {(void*)s->master, (void*)s->m, (void*)s->v, (void*)s->wb, (void*)s->partial,
                    (void*)s->loss})
        if (p) (void)hipFree(p);
    for (int i = 0; i < 4; ++i)
        if (s->scratch[i]) (void)hipFree(s->scratch[i]);
    delete s;
}

bool mlp_has_weights(const MlpState* s) { return s && s->has_weights; }

float* mlp_scratch(MlpState* s, int which, size_t floats)
{
    if (which < 0 || which >= 4) return nullptr;
    if (s->scratch_cap[which] < floats) {
        if (s->scratch[which]) (void)hipFree(s->scratch[which]);
        s->scratch[which] = nullptr;
        s->scratch_cap[which] = 0;
        if (hipMalloc((void**)&s->scratch[which], std::max<size_t>(floats, 1) * sizeof(float)) != hipSuccess)
            return nullptr;
        s->scratch_cap[which] = floats;
    }
    return s->scratch[which];
}

int mlp_set_weights(MlpState* s, const float* host_w, hipStream_t st)
{
    if (hipMemcpyAsync(s->master, host_w, kNP * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(s->m, 0, kNP * sizeof(float), st) != hipSuccess ||
        hipMemsetAsync(s->v, 0, kNP * sizeof(float), st) != hipSuccess)
        return -1;
    hipLaunchKernelGGL(k_mlp_round, dim3((kNP + 255) / 256), dim3(256), 0, st, s->master, s->wb);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return -1;
    s->t = 0;
    s->has_weights = true;
    return 0;
}

int mlp_get_weights(MlpState* s, float* host_w, hipStream_t st)
{
    if (hipMemcpyAsync(host_w, s->master, kNP * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    return 0;
}

const uint16_t* mlp_weights_bf16(const MlpState* s) { return s->wb; }  // kNPpad values, 16-B aligned

int mlp_forward(MlpState* s, const float* x, int64_t B, float* y, hipStream_t st)
{
    if (B <= 0) return 0;
    // four waves (128 samples) per block and round; at most 1,024 blocks
    const int64_t tiles = (B + 31) / 32;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + 3) / 4, 1024);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, st, x, (int)B, s->wb, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int mlp_grad_step(MlpState* s, const float* x, const float* t, int64_t B, float lr, float* grad,
                  float* loss_host, hipStream_t st)
{
    const int npass = (int)((B + kGS - 1) / kGS);
    const int nblk = std::min(npass, kMaxGradBlocks);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, st, x, t, (int)B, s->wb, s->partial);
    if (hipGetLastError() != hipSuccess) return -1;
    float bc1 = 1.0f, bc2 = 1.0f;
    if (lr > 0.0f) {
        s->t += 1;
        bc1 = (float)(1.0 - std::pow(0.9, (double)s->t));
        bc2 = (float)(1.0 - std::pow(0.999, (double)s->t));
    }
    hipLaunchKernelGGL(k_mlp_update, dim3((kNP + 1 + 255) / 256), dim3(256), 0, st, s->partial, nblk,
                       s->master, s->m, s->v, s->wb, lr, bc1, bc2, grad, s->loss, (int)B);
    if (hipGetLastError() != hipSuccess) return -1;
    if (loss_host) {
        if (hipMemcpyAsync(loss_host, s->loss, sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return -1;
    }
    return 0;
}

}  // namespace dgidp
