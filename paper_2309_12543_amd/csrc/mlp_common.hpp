// Learned per-link SDF surrogate: shared device code.
//
// Network (per link): m(x) = w4 . h3 + b4, h_k = SiLU(W_k h_{k-1} + b_k),
// widths 3 -> 128 -> 128 -> 128 -> 1, SiLU(z) = z / (1 + exp(-z)), input the
// link-frame point normalised to the link's domain.  FP32 master parameters,
// [W1 128x3 | b1 | W2 128x128 | b2 | W3 128x128 | b3 | w4 | b4] (33665).
// The estimate of the link's signed distance is the network's share
// (bounded_share: m, or B tanh(m / B) with the link's remainder bound B) plus
// the distance from the point to the link's core box (its mesh's bounding
// box, core_distance).
//
// Precision: W1, W2, W3, w4 are used as bfloat16 (round to nearest even);
// the input layer runs on the VALU in FP32 (bfloat16 coordinates would be
// millimetres coarse); the two 128x128 layers run on bf16 MFMA with FP32
// accumulation; activations are rounded to bfloat16 before every product.
//
// MFMA layout (v_mfma_f32_16x16x32_bf16, lane l, g = l / 16):
//   A 16x32: row l % 16, k = 8g + e       B 32x16: column l % 16, k = 8g + e
//   D 16x16: column l % 16, rows 4g + r (r < 4)
// Layers are evaluated transposed (pairs along N) so that a layer's result
// tile stays in registers and becomes the next layer's B operand: K-step s
// takes slot e < 4 from result tile 2s (rows 4g + e) and slot e >= 4 from
// tile 2s + 1 (rows 4g + e - 4), i.e. unit u(s, 8g + e) below, and the
// weights are staged into LDS with the same permutation of their K index.
#pragma once

#include "lsdf_internal.hpp"

namespace lsdf {
namespace mlp {

constexpr int H = 128;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * 3;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H * H;
constexpr int OFF_W4 = OFF_B3 + H;
constexpr int OFF_B4 = OFF_W4 + H;
constexpr int NPARAM = OFF_B4 + 1;
static_assert(NPARAM == LSDF_MLP_PARAMS, "parameter layout");

constexpr int NT = 2;                   // 16-pair column tiles per wave tile (evaluation, query)
constexpr int TILE = 16 * NT;           // pairs per wave tile
// Training takes one column tile per wave: twice the waves for the same
// batch, which hides more latency (the evaluation keeps two, which reuse
// each weight tile read from LDS twice)
constexpr int NT_TRAIN = 1;
constexpr int TILE_TRAIN = 16 * NT_TRAIN;
constexpr int WTILE_ELEMS = H * H;      // bf16 elements of one staged 128x128 layer

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Small FP32 parameters kept in LDS (W1 and w4 already rounded to bf16).
struct SmallParams {
    float w1[H][3];
    float b1[H];
    float b2[H];
    float b3[H];
    float w4[H];
    __bf16 w4b[H];   // w4 as bfloat16 pairs for the output layer's dot products
    float b4;
};

__device__ inline int perm_unit(int s, int kappa) {
    const int g = kappa >> 3, e = kappa & 7;
    return 32 * s + (e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4));
}

__device__ inline float bf16_round(float x) { return (float)(__bf16)x; }

// Core term of the estimate: the distance from a link-frame point to the
// link's core box, given u = l - centre and the box's half extents k:
// || max(|u| - k, 0) ||, the square root correctly rounded.
__device__ inline float core_distance(float ux, float uy, float uz, const float (&k)[3]) {
    const float qx = fmaxf(fabsf(ux) - k[0], 0.0f);
    const float qy = fmaxf(fabsf(uy) - k[1], 0.0f);
    const float qz = fmaxf(fabsf(uz) - k[2], 0.0f);
    return __builtin_sqrtf(fmaf(qx, qx, fmaf(qy, qy, qz * qz)));
}

// sigmoid(z) = 1 / (1 + exp(-z)); SiLU(z) = z sigmoid(z) and
// SiLU'(z) = s (1 + z (1 - s)) with s = sigmoid(z)
__device__ inline float sigmoid(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z * 1.44269504088896340736f));
}

__device__ inline float silu(float z) { return z * sigmoid(z); }

// The network's share of the estimate: b t with t = tanh(m / b), evaluated
// as clamp(1 - 2 / (1 + exp(2 m inv_b)), -1, 1) (so |share| <= b exactly),
// inv_b = 1 / b; inv_b = 0 stands for b = +inf: the share is m, t = 0.
__device__ inline float bounded_share(float m, float b, float inv_b, float& t) {
    if (inv_b == 0.0f) {
        t = 0.0f;
        return m;
    }
    const float e = __builtin_amdgcn_exp2f((m * inv_b) * 2.88539008177792681472f);
    t = fminf(fmaxf(1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e), -1.0f), 1.0f);
    return b * t;
}

__device__ inline float silu_grad_of(float z, float s) { return s * (1.0f + z * (1.0f - s)); }

// Stages one 128x128 weight matrix W (row-major [out][in], FP32) into LDS as
// bf16 A-operand tiles [mt][s][lane][8].  transpose = false: rows are output
// units and K runs over input units (forward); transpose = true: rows are
// input units and K runs over output units (backward, W^T).
__device__ inline void stage_weights(__bf16* dst, const float* __restrict__ W, bool transpose) {
    for (int idx = threadIdx.x; idx < WTILE_ELEMS; idx += blockDim.x) {
        const int e = idx & 7;
        const int lane = (idx >> 3) & 63;
        const int s = (idx >> 9) & 3;
        const int mt = idx >> 11;
        const int row = 16 * mt + (lane & 15);
        const int k = perm_unit(s, 8 * (lane >> 4) + e);
        const float v = transpose ? W[k * H + row] : W[row * H + k];
        dst[idx] = (__bf16)v;
    }
}

__device__ inline void stage_small(SmallParams* sp, const float* __restrict__ P) {
    for (int u = threadIdx.x; u < H; u += blockDim.x) {
        for (int k = 0; k < 3; ++k) sp->w1[u][k] = bf16_round(P[OFF_W1 + 3 * u + k]);
        sp->b1[u] = P[OFF_B1 + u];
        sp->b2[u] = P[OFF_B2 + u];
        sp->b3[u] = P[OFF_B3 + u];
        sp->w4[u] = bf16_round(P[OFF_W4 + u]);
        sp->w4b[u] = (__bf16)P[OFF_W4 + u];
    }
    if (threadIdx.x == 0) sp->b4 = P[OFF_B4];
}

__device__ inline bf16x8 lds_a(const __bf16* tiles, int mt, int s, int lane) {
    return *reinterpret_cast<const bf16x8*>(tiles + ((mt * 4 + s) * 64 + lane) * 8);
}

// Forward pass of one wave tile (16 NT_ pairs).  xh[nt] is this lane's input
// for pair 16 nt + lane % 16 (all four lane groups hold the same pairs).
// Returns the output for pair 16 nt + lane % 16 in m[nt] (every lane).
template <int NT_>
__device__ inline void forward_tile(const __bf16* sW2, const __bf16* sW3, const SmallParams* sp,
                                    const float (&xh)[NT_][3], float (&m)[NT_]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    // keeps the weight reads from LDS inside the tile: hoisted out of a tile
    // loop they would need 256 VGPRs
    asm volatile("" ::: "memory");

    // input layer (FP32 VALU) straight into layer 2's B operands
    bf16x8 b[4][NT_];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int u = perm_unit(s, 8 * g + e);
#pragma unroll
            for (int nt = 0; nt < NT_; ++nt) {
                const float z = fmaf(sp->w1[u][0], xh[nt][0],
                                     fmaf(sp->w1[u][1], xh[nt][1], fmaf(sp->w1[u][2], xh[nt][2], sp->b1[u])));
                const __bf16 h = (__bf16)silu(z);
                b[s][nt][e] = h;
            }
        }
    }

    // two 128x128 layers on MFMA
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16* sW = layer == 0 ? sW2 : sW3;
        const float* bias = layer == 0 ? sp->b2 : sp->b3;
        // the accumulators start at the bias: z = b + W h
        f32x4 acc[8][NT_];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const f32x4 b0 = f32x4{bias[16 * mt + 4 * g], bias[16 * mt + 4 * g + 1], bias[16 * mt + 4 * g + 2],
                                   bias[16 * mt + 4 * g + 3]};
#pragma unroll
            for (int nt = 0; nt < NT_; ++nt) acc[mt][nt] = b0;
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bf16x8 a = lds_a(sW, mt, s, lane);
#pragma unroll
                for (int nt = 0; nt < NT_; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[s][nt], acc[mt][nt], 0, 0, 0);
            }
        }
        if (layer == 0) {
            // bias + SiLU, rounded, rearranged into layer 3's B operands
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT_; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float z = acc[mt][nt][r];
                        const __bf16 h = (__bf16)silu(z);
                        b[mt >> 1][nt][(mt & 1) * 4 + r] = h;
                    }
        } else {
            // SiLU, rounded, and this lane's part of w4 . h3 (bfloat16
            // pairs, products exact, FP32 sums)
#pragma unroll
            for (int nt = 0; nt < NT_; ++nt) {
                float part = 0.0f;
#pragma unroll
                for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                    for (int r = 0; r < 4; r += 2) {
                        const int u = 16 * mt + 4 * g + r;
                        const float z0 = acc[mt][nt][r], z1 = acc[mt][nt][r + 1];
                        const __bf16 h0 = (__bf16)silu(z0), h1 = (__bf16)silu(z1);
                        const bf16x2 hp = {h0, h1};
                        const bf16x2 wp = {sp->w4b[u], sp->w4b[u + 1]};
                        part = __builtin_amdgcn_fdot2_f32_bf16(hp, wp, part, false);
                    }
                part += __shfl_xor(part, 16, 64);
                part += __shfl_xor(part, 32, 64);
                m[nt] = part + sp->b4;
            }
        }
    }
}

}  // namespace mlp
}  // namespace lsdf
