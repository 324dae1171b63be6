// The paper's tiny network for the Euclidean grid transformation
// (Sec. III-B-1, Eq. 4-5): f(R) ~ R^T P, the rotated normalised centres of
// the (2m)^3 voxels of a transformed Link SDF block, from the 9 entries of
// the rotation; two fully connected layers with a ReLU between them,
// trained with an L1 loss and Adam (Sec. IV-B).
//
//   x = R row-major (9), h = ReLU(W1 x + b1) (32), out = W2 h + b2 (3 V),
//   V = (2m)^3, output o = 3 j + a, voxel j = (j_z 2m + j_y) 2m + j_x,
//   target_o = sum_b R[b][a] P_j[b],  P_j = (j + 1/2) / m - 1 per axis.
//   Parameters: W1[32][9], b1[32], W2[3V][32], b2[3V] (FP32).
//
// Training step (all FP32, deterministic: no floating-point atomics):
//   hidden kernel  z, h for the B rotations of the batch;
//   output kernel  one thread per output row o, 128 rows per workgroup:
//                  the B outputs of row o, their errors against the exact
//                  target, dW2[o] and db2[o] (each row owned by one thread),
//                  the workgroup's partial loss and its partial of
//                  dh = sum_o g_o W2[o] (g_o = sign(error) / (B 3V)), with
//                  the signs and the rows staged in LDS;
//   reduce kernels sum the partials in two levels (64 slices, then one
//                  workgroup): loss, dh; then dW1, db1 through the ReLU;
//   Adam kernel    one thread per parameter.
// Max-error kernel: max |f(R) - R^T P| over rotations and outputs (the
// paper's 10^7-transformation test), one thread per output row, rotations
// in tiles of 64 whose hidden layers are computed once per workgroup.
#include <algorithm>

#include "lsdf_internal.hpp"

namespace {

constexpr int kH = LSDF_FRNN_HIDDEN;
constexpr int kRows = 128;          // output rows per workgroup
constexpr int kMaxB = 64;           // rotations per training step
constexpr int kTile = 64;           // rotations per tile in the max-error kernel
constexpr int kReduceThreads = 1024;   // the single workgroup of the last reduction
constexpr int kSlices = 64;         // first level of the partial-sum reduction

struct Layout {
    int64_t V, O;                   // voxels, outputs (3 V)
    int64_t w1, b1, w2, b2, n;      // offsets into the parameter vector, count
};

Layout layout(int32_t m) {
    Layout l{};
    l.V = (int64_t)(2 * m) * (2 * m) * (2 * m);
    l.O = 3 * l.V;
    l.w1 = 0;
    l.b1 = l.w1 + kH * 9;
    l.w2 = l.b1 + kH;
    l.b2 = l.w2 + l.O * kH;
    l.n = l.b2 + l.O;
    return l;
}

// Target of output o for rotation r (row-major 3x3).
__device__ inline float frnn_target(const float* r, int64_t o, int m) {
    const int64_t j = o / 3;
    const int a = (int)(o - 3 * j);
    const int w = 2 * m;
    const int jx = (int)(j % w), jy = (int)((j / w) % w), jz = (int)(j / ((int64_t)w * w));
    const float inv = 1.0f / (float)m;
    const float px = fmaf((float)jx + 0.5f, inv, -1.0f);
    const float py = fmaf((float)jy + 0.5f, inv, -1.0f);
    const float pz = fmaf((float)jz + 0.5f, inv, -1.0f);
    return fmaf(r[0 * 3 + a], px, fmaf(r[1 * 3 + a], py, r[2 * 3 + a] * pz));
}

struct TrainArgs {
    const float* params;
    const float* R;          // [B][9]
    float* z;                // [B][kH]
    float* h;                // [B][kH]
    float* grad;             // [n]
    float* part_dh;          // [blocks][B][kH]
    float* part_loss;        // [blocks]
    float* part2_dh;         // [kSlices][B][kH]
    float* part2_loss;       // [kSlices]
    float* loss_out;         // [1] or NULL
    Layout lay;
    int32_t m;
    int32_t B;
    int32_t blocks;
};

__global__ __launch_bounds__(256) void frnn_hidden_kernel(TrainArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= a.B * kH) return;
    const int b = t / kH, u = t - b * kH;
    const float* W1 = a.params + a.lay.w1;
    float acc = a.params[a.lay.b1 + u];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc = fmaf(W1[u * 9 + k], a.R[b * 9 + k], acc);
    a.z[t] = acc;
    a.h[t] = fmaxf(acc, 0.0f);
}

__global__ __launch_bounds__(kRows) void frnn_output_kernel(TrainArgs a) {
    static_assert(kRows == (kMaxB / 4) * (kH / 4), "one 4 x 4 tile of dh per thread");
    __shared__ float hs[kMaxB][kH];
    __shared__ float rs[kMaxB][9];
    // sign of g[row][b] (g is +scale, -scale or 0), transposed: rows contiguous,
    // the pad staggers the rotations over the banks
    __shared__ __align__(16) int8_t sgT[kMaxB][kRows + 4];
    __shared__ float4 ws4[kRows][kH / 4];       // W2 rows in 16 B chunks, chunk c stored at c ^ (row mod 8)
    __shared__ float ls[kRows];
    const int tid = threadIdx.x;
    const int B = a.B;
    for (int k = tid; k < B * kH; k += kRows) hs[k / kH][k % kH] = a.h[k];
    for (int k = tid; k < B * 9; k += kRows) rs[k / 9][k % 9] = a.R[k];
    const int64_t o = (int64_t)blockIdx.x * kRows + tid;
    const bool live = o < a.lay.O;
    float wrow[kH];
    const float* W2 = a.params + a.lay.w2;
#pragma unroll
    for (int u = 0; u < kH; ++u) wrow[u] = live ? W2[o * kH + u] : 0.0f;
#pragma unroll
    for (int c = 0; c < kH / 4; ++c)
        ws4[tid][c ^ (tid & 7)] = make_float4(wrow[4 * c], wrow[4 * c + 1], wrow[4 * c + 2], wrow[4 * c + 3]);
    const float bias = live ? a.params[a.lay.b2 + o] : 0.0f;
    // this row's block voxel and component (the target is R^T P_j, component a)
    int comp = 0;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (live) {
        const int64_t j = o / 3;
        comp = (int)(o - 3 * j);
        const int w = 2 * a.m;
        const int jx = (int)(j % w), jy = (int)((j / w) % w), jz = (int)(j / ((int64_t)w * w));
        const float inv = 1.0f / (float)a.m;
        px = fmaf((float)jx + 0.5f, inv, -1.0f);
        py = fmaf((float)jy + 0.5f, inv, -1.0f);
        pz = fmaf((float)jz + 0.5f, inv, -1.0f);
    }
    __syncthreads();
    const float scale = 1.0f / ((float)B * (float)a.lay.O);
    float dw[kH];
#pragma unroll
    for (int u = 0; u < kH; ++u) dw[u] = 0.0f;
    float db = 0.0f, loss = 0.0f;
    for (int b = 0; b < B; ++b) {
        float y = bias;
#pragma unroll
        for (int u = 0; u < kH; ++u) y = fmaf(wrow[u], hs[b][u], y);
        float g = 0.0f;
        int8_t sg = 0;
        if (live) {
            const float* r = rs[b];
            const float t = fmaf(r[comp], px, fmaf(r[3 + comp], py, r[6 + comp] * pz));
            const float e = y - t;
            loss += fabsf(e);
            sg = e > 0.0f ? 1 : (e < 0.0f ? -1 : 0);
            g = e > 0.0f ? scale : (e < 0.0f ? -scale : 0.0f);
        }
        sgT[b][tid] = sg;
#pragma unroll
        for (int u = 0; u < kH; ++u) dw[u] = fmaf(g, hs[b][u], dw[u]);
        db += g;
    }
    if (live) {
        float* gW2 = a.grad + a.lay.w2 + o * kH;
#pragma unroll
        for (int u = 0; u < kH; ++u) gW2[u] = dw[u];
        a.grad[a.lay.b2 + o] = db;
    }
    ls[tid] = loss;
    __syncthreads();
    // this workgroup's share of dh[b][u] = sum over its rows of g W2[o][u],
    // rows in order; thread t holds b = 4 (t / 8) + i, u = 4 (t mod 8) + k
    const int bt = tid >> 3, ut = tid & 7;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[i][k] = 0.0f;
    for (int r0 = 0; r0 < kRows; r0 += 4) {
        uint32_t sg4[4];   // the signs of rows r0 .. r0 + 3, one byte each
#pragma unroll
        for (int i = 0; i < 4; ++i) sg4[i] = *reinterpret_cast<const uint32_t*>(&sgT[4 * bt + i][r0]);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const float4 wv = ws4[r0 + rr][ut ^ ((r0 + rr) & 7)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // g itself, rebuilt exactly from its sign
                const float gi = (float)(int8_t)(sg4[i] >> (8 * rr)) * scale;
                acc[i][0] = fmaf(gi, wv.x, acc[i][0]);
                acc[i][1] = fmaf(gi, wv.y, acc[i][1]);
                acc[i][2] = fmaf(gi, wv.z, acc[i][2]);
                acc[i][3] = fmaf(gi, wv.w, acc[i][3]);
            }
        }
    }
    float* pd = a.part_dh + (int64_t)blockIdx.x * B * kH;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int b = 4 * bt + i;
        if (b < B) *reinterpret_cast<float4*>(&pd[b * kH + 4 * ut]) = make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
    }
    if (tid == 0) {
        float s = 0.0f;
        for (int r = 0; r < kRows; ++r) s += ls[r];
        a.part_loss[blockIdx.x] = s;
    }
}

// First level of the reduction: slice s sums the output kernel's partials
// of workgroups s, s + kSlices, ... (in that fixed order).
__global__ __launch_bounds__(256) void frnn_slice_kernel(TrainArgs a) {
    const int sl = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int BH = a.B * kH;
    // the sums run in the fixed order; their loads are issued kBatch at a time
    constexpr int kBatch = 8;
    if (p < BH) {
        float s = 0.0f;
        for (int blk0 = sl; blk0 < a.blocks; blk0 += kBatch * kSlices) {
            float v[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int blk = blk0 + k * kSlices;
                v[k] = blk < a.blocks ? a.part_dh[(int64_t)blk * BH + p] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                if (blk0 + k * kSlices < a.blocks) s += v[k];
        }
        a.part2_dh[(int64_t)sl * BH + p] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int blk0 = sl; blk0 < a.blocks; blk0 += kBatch * kSlices) {
            float v[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int blk = blk0 + k * kSlices;
                v[k] = blk < a.blocks ? a.part_loss[blk] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                if (blk0 + k * kSlices < a.blocks) s += v[k];
        }
        a.part2_loss[sl] = s;
    }
}

// One workgroup: sums the slices, then the first layer's gradient through
// the ReLU.
__global__ __launch_bounds__(kReduceThreads) void frnn_reduce_kernel(TrainArgs a) {
    __shared__ float dz[kMaxB][kH];
    __shared__ float rs[kMaxB * 9];
    const int tid = threadIdx.x;
    const int B = a.B;
    for (int k = tid; k < B * 9; k += kReduceThreads) rs[k] = a.R[k];
    // the slices are summed in order, with 16 loads in flight per thread
    for (int p = tid; p < B * kH; p += kReduceThreads) {
        float s = 0.0f;
#pragma unroll
        for (int sl0 = 0; sl0 < kSlices; sl0 += 16) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = a.part2_dh[(int64_t)(sl0 + k) * B * kH + p];
#pragma unroll
            for (int k = 0; k < 16; ++k) s += v[k];
        }
        dz[p / kH][p % kH] = a.z[p] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    for (int p = tid; p < kH * 10; p += kReduceThreads) {
        if (p < kH * 9) {
            const int u = p / 9, k = p - u * 9;
            float s = 0.0f;
            for (int b = 0; b < B; ++b) s = fmaf(dz[b][u], rs[b * 9 + k], s);
            a.grad[a.lay.w1 + p] = s;
        } else {
            const int u = p - kH * 9;
            float s = 0.0f;
            for (int b = 0; b < B; ++b) s += dz[b][u];
            a.grad[a.lay.b1 + u] = s;
        }
    }
    if (tid == 0 && a.loss_out) {
        float v[kSlices];
#pragma unroll
        for (int sl = 0; sl < kSlices; ++sl) v[sl] = a.part2_loss[sl];
        float s = 0.0f;
#pragma unroll
        for (int sl = 0; sl < kSlices; ++sl) s += v[sl];
        a.loss_out[0] = s / ((float)B * (float)a.lay.O);
    }
}

struct AdamArgs {
    float* p;
    float* m;
    float* v;
    const float* g;
    int64_t n;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__global__ __launch_bounds__(256) void frnn_adam_kernel(AdamArgs a) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n) return;
    const float g = a.g[k];
    const float m = fmaf(a.b1, a.m[k], (1.0f - a.b1) * g);
    const float v = fmaf(a.b2, a.v[k], (1.0f - a.b2) * g * g);
    a.m[k] = m;
    a.v[k] = v;
    a.p[k] -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
}

struct EvalArgs {
    const float* params;
    const float* R;          // [N][9]
    int64_t N;
    Layout lay;
    int32_t m;
    uint32_t* out_max;       // float bits of a non-negative maximum
};

__global__ __launch_bounds__(kRows) void frnn_max_error_kernel(EvalArgs a) {
    __shared__ float hs[kTile][kH];
    __shared__ float rs[kTile][9];
    __shared__ float red[kRows];
    const int tid = threadIdx.x;
    const int64_t o = (int64_t)blockIdx.x * kRows + tid;
    const bool live = o < a.lay.O;
    float wrow[kH];
#pragma unroll
    for (int u = 0; u < kH; ++u) wrow[u] = live ? a.params[a.lay.w2 + o * kH + u] : 0.0f;
    const float bias = live ? a.params[a.lay.b2 + o] : 0.0f;
    const float* W1 = a.params + a.lay.w1;
    float worst = 0.0f;
    for (int64_t t0 = (int64_t)blockIdx.y * kTile; t0 < a.N; t0 += (int64_t)gridDim.y * kTile) {
        const int nt = (int)min<int64_t>(kTile, a.N - t0);
        __syncthreads();
        for (int k = tid; k < nt * 9; k += kRows) rs[k / 9][k % 9] = a.R[t0 * 9 + k];
        __syncthreads();
        for (int p = tid; p < nt * kH; p += kRows) {
            const int b = p / kH, u = p - b * kH;
            float acc = a.params[a.lay.b1 + u];
#pragma unroll
            for (int k = 0; k < 9; ++k) acc = fmaf(W1[u * 9 + k], rs[b][k], acc);
            hs[b][u] = fmaxf(acc, 0.0f);
        }
        __syncthreads();
        if (live) {
            for (int b = 0; b < nt; ++b) {
                float y = bias;
#pragma unroll
                for (int u = 0; u < kH; ++u) y = fmaf(wrow[u], hs[b][u], y);
                worst = fmaxf(worst, fabsf(y - frnn_target(rs[b], o, a.m)));
            }
        }
    }
    red[tid] = worst;
    __syncthreads();
    if (tid == 0) {
        float mx = 0.0f;
        for (int r = 0; r < kRows; ++r) mx = fmaxf(mx, red[r]);
        atomicMax(a.out_max, __float_as_uint(mx));   // non-negative: bit order = value order
    }
}

__global__ void frnn_zero_kernel(uint32_t* w) { *w = 0u; }

int check_m(const char* who, int32_t m) {
    if (m < 1 || m > LSDF_FRNN_MAX_HALF)
        return lsdf::fail(LSDF_E_SHAPE, "%s: m = %d out of [1, %d]", who, (int)m, LSDF_FRNN_MAX_HALF);
    return LSDF_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

LSDF_API int lsdf_frnn_nparam(int32_t m, int64_t* n) {
    using namespace lsdf;
    clear_error();
    int rc = check_m("frnn_nparam", m);
    if (rc != LSDF_OK) return rc;
    if (!n) return fail(LSDF_E_INVALID_ARG, "frnn_nparam: n is NULL");
    *n = layout(m).n;
    return LSDF_OK;
}

LSDF_API int lsdf_frnn_train_workspace_size(int32_t m, int32_t B, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    int rc = check_m("frnn_train_workspace_size", m);
    if (rc != LSDF_OK) return rc;
    if (B < 1 || B > kMaxB) return fail(LSDF_E_SHAPE, "frnn_train_workspace_size: B = %d out of [1, %d]", (int)B, kMaxB);
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "frnn_train_workspace_size: bytes is NULL");
    const Layout l = layout(m);
    const int64_t blocks = (l.O + kRows - 1) / kRows;
    *bytes = 2 * align256((size_t)B * kH * 4) + align256((size_t)blocks * B * kH * 4) + align256((size_t)blocks * 4) +
             align256((size_t)kSlices * B * kH * 4) + align256((size_t)kSlices * 4);
    return LSDF_OK;
}

LSDF_API int lsdf_frnn_train_step(float* params, float* adam_m, float* adam_v, int64_t t, float lr, float beta1,
                                  float beta2, float eps, int32_t m, const float* R, int32_t B, float* loss_out,
                                  float* grad, void* workspace, size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    size_t need = 0;
    int rc = lsdf_frnn_train_workspace_size(m, B, &need);
    if (rc != LSDF_OK) return rc;
    if (!params || !R || !grad || !workspace) return fail(LSDF_E_INVALID_ARG, "frnn_train_step: NULL device pointer");
    if ((adam_m == nullptr) != (adam_v == nullptr))
        return fail(LSDF_E_INVALID_ARG, "frnn_train_step: give both Adam moments or neither");
    if (adam_m && t < 1) return fail(LSDF_E_INVALID_ARG, "frnn_train_step: step t must be >= 1");
    if (adam_m && !(std::isfinite(lr) && lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f &&
                    beta2 < 1.0f && eps > 0.0f))
        return fail(LSDF_E_INVALID_ARG, "frnn_train_step: bad Adam hyper-parameters");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "frnn_train_step: workspace is not 256-byte aligned");
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "frnn_train_step: workspace has %zu bytes, needs %zu", ws_bytes, need);
    TrainArgs a{};
    a.lay = layout(m);
    a.params = params;
    a.R = R;
    a.m = m;
    a.B = B;
    a.blocks = (int32_t)((a.lay.O + kRows - 1) / kRows);
    char* ws = static_cast<char*>(workspace);
    a.z = reinterpret_cast<float*>(ws);
    a.h = reinterpret_cast<float*>(ws + align256((size_t)B * kH * 4));
    a.part_dh = reinterpret_cast<float*>(ws + 2 * align256((size_t)B * kH * 4));
    const size_t off_loss = 2 * align256((size_t)B * kH * 4) + align256((size_t)a.blocks * B * kH * 4);
    a.part_loss = reinterpret_cast<float*>(ws + off_loss);
    const size_t off2 = off_loss + align256((size_t)a.blocks * 4);
    a.part2_dh = reinterpret_cast<float*>(ws + off2);
    a.part2_loss = reinterpret_cast<float*>(ws + off2 + align256((size_t)kSlices * B * kH * 4));
    a.grad = grad;
    a.loss_out = loss_out;
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(frnn_hidden_kernel, dim3((B * kH + 255) / 256), dim3(256), 0, s, a);
    if ((rc = check_launch("frnn_train_step (hidden)")) != LSDF_OK) return rc;
    hipLaunchKernelGGL(frnn_output_kernel, dim3((unsigned)a.blocks), dim3(kRows), 0, s, a);
    if ((rc = check_launch("frnn_train_step (output)")) != LSDF_OK) return rc;
    hipLaunchKernelGGL(frnn_slice_kernel, dim3((B * kH + 255) / 256, kSlices), dim3(256), 0, s, a);
    if ((rc = check_launch("frnn_train_step (slices)")) != LSDF_OK) return rc;
    hipLaunchKernelGGL(frnn_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, a);
    if ((rc = check_launch("frnn_train_step (reduce)")) != LSDF_OK) return rc;
    if (!adam_m) return LSDF_OK;   // gradient only
    AdamArgs d{params, adam_m, adam_v, grad, a.lay.n, lr, beta1, beta2, eps,
               (float)(1.0 - std::pow((double)beta1, (double)t)), (float)(1.0 - std::pow((double)beta2, (double)t))};
    hipLaunchKernelGGL(frnn_adam_kernel, dim3((unsigned)((a.lay.n + 255) / 256)), dim3(256), 0, s, d);
    return check_launch("frnn_train_step (adam)");
}

LSDF_API int lsdf_frnn_max_error(const float* params, int32_t m, const float* R, int64_t N, float* out_max,
                                 void* stream) {
    using namespace lsdf;
    clear_error();
    int rc = check_m("frnn_max_error", m);
    if (rc != LSDF_OK) return rc;
    if (N < 0) return fail(LSDF_E_SHAPE, "frnn_max_error: N < 0");
    if (!params || !out_max || (N > 0 && !R)) return fail(LSDF_E_INVALID_ARG, "frnn_max_error: NULL device pointer");
    EvalArgs a{};
    a.params = params;
    a.R = R;
    a.N = N;
    a.lay = layout(m);
    a.m = m;
    a.out_max = reinterpret_cast<uint32_t*>(out_max);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(frnn_zero_kernel, dim3(1), dim3(1), 0, s, a.out_max);
    if ((rc = check_launch("frnn_max_error (zero)")) != LSDF_OK) return rc;
    if (N == 0) return LSDF_OK;
    // rows across x, rotation tiles dealt over y: about 8192 workgroups
    const int64_t xb = (a.lay.O + kRows - 1) / kRows;
    const int64_t tiles = (N + kTile - 1) / kTile;
    const int64_t yb = std::max<int64_t>(1, std::min<int64_t>({tiles, 8192 / xb, 65535}));
    hipLaunchKernelGGL(frnn_max_error_kernel, dim3((unsigned)xb, (unsigned)yb), dim3(kRows), 0, s, a);
    return check_launch("frnn_max_error");
}
