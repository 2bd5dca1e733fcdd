// Device-side pieces of the learned-indicator network (16 -> 64 -> 64 -> 1,
// ReLU, BF16 weights) shared by the stand-alone inference kernel and the fused
// features-and-network kernel: parameter offsets, BF16 rounding, and the
// matrix-core forward pass of 32 samples by one wave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgidp {
namespace mlp {

constexpr int kNin = 16, kNh = 64;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5312;
constexpr int kNP = 5313;
constexpr int kNPpad = 5320;  // BF16 copy on the device, padded to 16-B chunks (tail zero)

// round to nearest even; the inputs here are finite
__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p)
{
    bf16x8 v;
    __builtin_memcpy(&v, p, sizeof(v));  // 16 B, 16-B aligned
    return v;
}

__device__ __forceinline__ bf16x8 pack_bf16x8(const float* v)
{
    uint16_t hb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) hb[t] = bf16_rne(v[t]);
    bf16x8 a;
    __builtin_memcpy(&a, hb, sizeof(a));
    return a;
}

// Inference on the matrix cores with v_mfma_f32_32x32x16_bf16 (BF16 operands,
// FP32 accumulation).  A wave takes 32 samples; the inputs and the first
// hidden layer enter the products rounded to BF16 (nearest even), like the
// weights; biases, ReLU and the output layer stay FP32.  The layers are
// computed transposed, units by samples, so that every lane keeps its own
// sample's hidden units:
//   layer 1: Z1^T = W1 X^T      [64 x 16] x [16 x 32]  two products
//   layer 2: Z2^T = W2 H1^T     [64 x 64] x [64 x 32]  eight products
//   output : y = w3 . relu(Z2 + b2) + b3, each lane's 32 units, then its partner's
// Operand layout (gfx950, checked on the device): lane l holds row (A) or
// column (B) l % 32 and K entries 8 (l / 32) .. 8 (l / 32) + 7; the result
// holds column l % 32 and rows 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15.  So
// lane (s, h) = (l % 32, l / 32) holds units 8 q + 4 h + 0..3 (q = 0..3) of
// each 32-unit tile of sample s; a K step of layer 2 needs units 8 k' .. + 7
// (k' = 2 (K step) + h), half of which the lane's partner l ^ 32 holds: one
// exchange of two packed words per K step.
//
// The weights sit in LDS (one copy per block, staged by stage_weights); the
// weight operands are read from there just before their product.  Rows of W1
// and W2 keep their 16-B chunks, placed by an XOR swizzle so that the 16 lanes
// of a read phase (16 rows, one chunk each) meet 16 different bank groups.
struct LdsWeights {
    uint16_t w1[kNh * kNin];  // row j: 2 chunks
    uint16_t w2[kNh * kNh];   // row j: 8 chunks
    float b1[kNh], b2[kNh], w3[kNh];
    float b3;
};

__device__ __forceinline__ int w1_pos(int j, int ch) { return j * kNin + ((ch ^ ((j >> 3) & 1)) << 3); }
__device__ __forceinline__ int w2_pos(int j, int ch) { return j * kNh + ((ch ^ ((j >> 1) & 7)) << 3); }

// 16-B chunk g (BF16 values 8 g .. 8 g + 7 of the parameter vector) into L
__device__ __forceinline__ void stage_chunk(LdsWeights& L, int g, uint4 v)
{
    uint16_t h[8];
    __builtin_memcpy(h, &v, sizeof(h));
    if (g < kOffB1 / 8) {
        *reinterpret_cast<uint4*>(&L.w1[w1_pos(g >> 1, g & 1)]) = v;
    } else if (g < kOffW2 / 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) L.b1[(g - kOffB1 / 8) * 8 + t] = bf16_f(h[t]);
    } else if (g < kOffB2 / 8) {
        const int k = g - kOffW2 / 8;
        *reinterpret_cast<uint4*>(&L.w2[w2_pos(k >> 3, k & 7)]) = v;
    } else if (g < kOffW3 / 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) L.b2[(g - kOffB2 / 8) * 8 + t] = bf16_f(h[t]);
    } else if (g < kOffB3 / 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t) L.w3[(g - kOffW3 / 8) * 8 + t] = bf16_f(h[t]);
    } else if (g == kOffB3 / 8) {
        L.b3 = bf16_f(h[0]);
    }
}

// the 665 chunks of the padded BF16 vector wb by a block of nthr threads; the
// caller places a barrier before the first read
__device__ __forceinline__ void stage_weights(LdsWeights& L, const uint16_t* __restrict__ wb, int tid, int nthr)
{
    const uint4* w4 = reinterpret_cast<const uint4*>(wb);
    for (int g = tid; g < kNPpad / 8; g += nthr) stage_chunk(L, g, w4[g]);
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    return (uint32_t)bf16_rne(lo) | ((uint32_t)bf16_rne(hi) << 16);
}

// Network output of sample lane % 32 of the wave (both lanes of the sample
// return it).  x: this lane's inputs 8 (lane / 32) .. + 7 of its sample, BF16.
// All 64 lanes of the wave call it together.
__device__ __forceinline__ float forward32(const LdsWeights& L, bf16x8 x, int lane)
{
    const int c = lane & 31, hf = lane >> 5;
    const f32x16 zero = {};
    // layer 1: lane holds units 32 nt + 8 q + 4 hf + (0..3) of sample c,
    // packed two BF16 per word: P[nt][q][0] units +0, +1; P[nt][q][1] units +2, +3
    uint32_t P[2][4][2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const f32x16 d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(&L.w1[w1_pos(nt * 32 + c, hf)]), x,
                                                                 zero, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 b1 = *reinterpret_cast<const float4*>(&L.b1[nt * 32 + q * 8 + hf * 4]);
            P[nt][q][0] = pack_bf16x2(fmaxf(d[4 * q] + b1.x, 0.0f), fmaxf(d[4 * q + 1] + b1.y, 0.0f));
            P[nt][q][1] = pack_bf16x2(fmaxf(d[4 * q + 2] + b1.z, 0.0f), fmaxf(d[4 * q + 3] + b1.w, 0.0f));
        }
    }
    // layer 2 operands: K step kc takes units 16 kc + 8 hf + 0..7 (tile kc / 2,
    // q = 2 (kc % 2) + hf); the lane holds their half 4 hf .. 4 hf + 3 and its
    // partner the other half
    uint32_t Bk[4][4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        const int nt = kc >> 1, q0 = 2 * (kc & 1);
        // hf = 0 keeps q0 and sends q0 + 1; hf = 1 keeps q0 + 1 and sends q0
        const uint32_t s0 = hf ? P[nt][q0][0] : P[nt][q0 + 1][0];
        const uint32_t s1 = hf ? P[nt][q0][1] : P[nt][q0 + 1][1];
        const uint32_t r0 = (uint32_t)__shfl_xor((int)s0, 32, 64);
        const uint32_t r1 = (uint32_t)__shfl_xor((int)s1, 32, 64);
        const uint32_t k0 = hf ? P[nt][q0 + 1][0] : P[nt][q0][0];
        const uint32_t k1 = hf ? P[nt][q0 + 1][1] : P[nt][q0][1];
        // K order: units 8 (2 kc + hf) + 0..3 are the partner's for hf = 1
        Bk[kc][0] = hf ? r0 : k0;
        Bk[kc][1] = hf ? r1 : k1;
        Bk[kc][2] = hf ? k0 : r0;
        Bk[kc][3] = hf ? k1 : r1;
    }
    float y = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        f32x16 d2 = zero;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            bf16x8 bop;
            __builtin_memcpy(&bop, Bk[kc], sizeof(bop));
            d2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf16x8(&L.w2[w2_pos(nt * 32 + c, 2 * kc + hf)]), bop,
                                                        d2, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = nt * 32 + q * 8 + hf * 4;
            const float4 b2 = *reinterpret_cast<const float4*>(&L.b2[j]);
            const float4 w3 = *reinterpret_cast<const float4*>(&L.w3[j]);
            y += w3.x * fmaxf(d2[4 * q] + b2.x, 0.0f);
            y += w3.y * fmaxf(d2[4 * q + 1] + b2.y, 0.0f);
            y += w3.z * fmaxf(d2[4 * q + 2] + b2.z, 0.0f);
            y += w3.w * fmaxf(d2[4 * q + 3] + b2.w, 0.0f);
        }
    }
    // the partner's 32 units; the same sum order in both lanes of the sample
    const float yp = __shfl_xor(y, 32, 64);
    return (hf ? yp + y : y + yp) + L.b3;
}

}  // namespace mlp
}  // namespace dgidp
