// Batched clearance query (Sec. III-A): per configuration c, the minimum over
// obstacle points and links of link i's grid SDF read at the point moved into
// link i's frame.
//
// One launch does the whole query:
//   * a block owns a tile of CT configurations (all L links) and a tile of
//     256*K points; each lane keeps its K points in registers;
//   * the block forms the world-to-grid affine map of each of its
//     (configuration, link) pairs once, in LDS (the inverse pose of Eq. 4 with
//     the grid scaling folded in);
//   * for every pair a lane maps its points (9 FMAs each), tests the box and
//     gathers + interpolates only inside it; a wave-wide min and an LDS
//     combine across the 4 waves leave one value per pair and block;
//   * blocks merge per-pair minima with one unsigned atomic max on a
//     complemented order-preserving key in the workspace;
//   * the last block to finish (atomic ticket) turns the keys into the
//     outputs and clears them, leaving the workspace all-zero again.
#include "lsdf_internal.hpp"

namespace {

using lsdf::LinkGrid;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr size_t kWsHeader = 256;   // ticket counter lives in the first bytes

struct QueryArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    const float* link_T;
    const float* grid;
    const float* points;
    float* out_dist;
    int32_t* out_link;
    float* out_link_dist;
    uint32_t* keys;      // [C][L] complemented ordered keys, 0 = empty
    uint32_t* ticket;
    int64_t M;
    int32_t C;
    int32_t L;
    int32_t point_tiles;
};

__device__ inline float lerp_exact_ends(float a, float b, float t) {
    return fmaf(t, b, fmaf(-t, a, a));
}

__device__ inline float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

template <int K, int CT>
__global__ __launch_bounds__(kBlock) void query_kernel(QueryArgs p) {
    __shared__ float s_aff[CT * LSDF_MAX_LINKS][12];
    __shared__ float s_part[kWaves][CT * LSDF_MAX_LINKS];
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ptile = blockIdx.x % p.point_tiles;
    const int c0 = (blockIdx.x / p.point_tiles) * CT;
    const int L = p.L;
    const int nc = min(CT, p.C - c0);
    const int npairs = nc * L;

    // 1. affine maps u = A [x; 1] of this block's (configuration, link) pairs
    if (tid < npairs) {
        const int c = c0 + tid / L;
        const int i = tid - (tid / L) * L;
        const float* T = p.link_T + ((int64_t)c * L + i) * 12;
        const LinkGrid& g = p.link[i];
        float Tv[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) Tv[k] = T[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // row a of R^T scaled by invh_a; offset -invh_a (R^T t)_a + nlo_a
            s_aff[tid][4 * a + 0] = g.invh[a] * Tv[0 + a];
            s_aff[tid][4 * a + 1] = g.invh[a] * Tv[4 + a];
            s_aff[tid][4 * a + 2] = g.invh[a] * Tv[8 + a];
            const float rt = fmaf(Tv[0 + a], Tv[3], fmaf(Tv[4 + a], Tv[7], Tv[8 + a] * Tv[11]));
            s_aff[tid][4 * a + 3] = fmaf(-g.invh[a], rt, g.nlo[a]);
        }
    }

    // 2. this lane's points; NaN past the end is never inside a box
    float px[K], py[K], pz[K];
    const int64_t pbase = (int64_t)ptile * (kBlock * K);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t j = pbase + (int64_t)k * kBlock + tid;
        if (j < p.M) {
            px[k] = p.points[3 * j + 0];
            py[k] = p.points[3 * j + 1];
            pz[k] = p.points[3 * j + 2];
        } else {
            px[k] = py[k] = pz[k] = __builtin_nanf("");
        }
    }
    __syncthreads();

    // 3. sweep the pairs
    for (int q = 0; q < npairs; ++q) {
        const int i = q % L;
        const LinkGrid& g = p.link[i];
        const float* G = p.grid + g.offset;
        const int nx = g.n[0];
        const int nxy = g.n[0] * g.n[1];
        float A[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) A[k] = s_aff[q][k];
        float best = INFINITY;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float u0 = fmaf(A[0], px[k], fmaf(A[1], py[k], fmaf(A[2], pz[k], A[3])));
            const float u1 = fmaf(A[4], px[k], fmaf(A[5], py[k], fmaf(A[6], pz[k], A[7])));
            const float u2 = fmaf(A[8], px[k], fmaf(A[9], py[k], fmaf(A[10], pz[k], A[11])));
            const bool inside = (u0 >= 0.0f) & (u0 <= g.umax[0]) & (u1 >= 0.0f) & (u1 <= g.umax[1]) &
                                (u2 >= 0.0f) & (u2 <= g.umax[2]);
            if (inside) {
                // u >= 0 here, so truncation is the floor
                const int ix = min((int)u0, g.n[0] - 2);
                const int iy = min((int)u1, g.n[1] - 2);
                const int iz = min((int)u2, g.n[2] - 2);
                const float fx = u0 - (float)ix;
                const float fy = u1 - (float)iy;
                const float fz = u2 - (float)iz;
                const float* c = G + (iz * nxy + iy * nx + ix);
                const float c000 = c[0], c100 = c[1];
                const float c010 = c[nx], c110 = c[nx + 1];
                const float c001 = c[nxy], c101 = c[nxy + 1];
                const float c011 = c[nxy + nx], c111 = c[nxy + nx + 1];
                const float e00 = lerp_exact_ends(c000, c100, fx);
                const float e10 = lerp_exact_ends(c010, c110, fx);
                const float e01 = lerp_exact_ends(c001, c101, fx);
                const float e11 = lerp_exact_ends(c011, c111, fx);
                const float e0 = lerp_exact_ends(e00, e10, fy);
                const float e1 = lerp_exact_ends(e01, e11, fy);
                const float v = lerp_exact_ends(e0, e1, fz) + 0.0f;   // -0 -> +0
                best = fminf(best, v);
            }
        }
        float m = INFINITY;
        if (__ballot(best < INFINITY)) m = wave_min(best);
        if (lane == 0) s_part[wave][q] = m;
    }
    __syncthreads();

    // 4. merge across waves, then across blocks
    if (tid < npairs) {
        float m = s_part[0][tid];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) m = fminf(m, s_part[w][tid]);
        if (m < INFINITY) {
            const int c = c0 + tid / L;
            const int i = tid - (tid / L) * L;
            atomicMax(&p.keys[(int64_t)c * L + i], ~lsdf::ordered_bits(m));
        }
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned total = gridDim.x;
        s_last = (atomicInc(p.ticket, total - 1) == total - 1);
    }
    __syncthreads();
    if (!s_last) return;

    // 5. last block: outputs, and the workspace back to zero
    __threadfence();
    for (int c = tid; c < p.C; c += kBlock) {
        uint32_t bestk = 0;
        int arg = -1;
        for (int i = 0; i < L; ++i) {
            const uint32_t k = atomicExch(&p.keys[(int64_t)c * L + i], 0u);
            if (p.out_link_dist) p.out_link_dist[(int64_t)c * L + i] = k ? lsdf::from_ordered_bits(~k) : INFINITY;
            if (k > bestk) {
                bestk = k;
                arg = i;
            }
        }
        p.out_dist[c] = bestk ? lsdf::from_ordered_bits(~bestk) : INFINITY;
        p.out_link[c] = arg;
    }
}

size_t keys_bytes(int64_t C, int64_t L) { return ((size_t)(C * L) * 4 + 255) / 256 * 256; }

}  // namespace

LSDF_API int lsdf_query_workspace_size(int32_t C, int32_t L, int64_t M, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "query_workspace_size: bytes is NULL");
    if (C < 0 || M < 0) return fail(LSDF_E_SHAPE, "query_workspace_size: negative size");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "query_workspace_size: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    *bytes = kWsHeader + keys_bytes(C, L);
    return LSDF_OK;
}

LSDF_API int lsdf_query_min_distance(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                     const void* grid_buf, const float* points, int64_t M, float* out_dist,
                                     int32_t* out_link, float* out_link_dist, uint32_t flags, void* workspace,
                                     size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    if (flags != 0) return fail(LSDF_E_UNSUPPORTED, "query: unsupported flags 0x%x", flags);
    if (C < 0 || M < 0) return fail(LSDF_E_SHAPE, "query: negative size (C = %d, M = %lld)", (int)C, (long long)M);
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "query: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (!grids) return fail(LSDF_E_INVALID_ARG, "query: grids is NULL");
    if (C == 0) return LSDF_OK;
    if (!link_T || !grid_buf || !out_dist || !out_link || !workspace)
        return fail(LSDF_E_INVALID_ARG, "query: NULL device pointer");
    if (M > 0 && !points) return fail(LSDF_E_INVALID_ARG, "query: points is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "query: workspace is not 256-byte aligned");
    const size_t need = kWsHeader + keys_bytes(C, L);
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "query: workspace has %zu bytes, needs %zu", ws_bytes, need);

    constexpr int K = 8;
    constexpr int CT = 2;
    const int64_t point_tiles = M > 0 ? (M + kBlock * K - 1) / (kBlock * K) : 1;
    const int64_t conf_tiles = (C + CT - 1) / CT;
    if (point_tiles * conf_tiles > INT32_MAX) return fail(LSDF_E_SHAPE, "query: problem too large for one launch");

    QueryArgs p{};
    for (int i = 0; i < L; ++i) {
        int rc = prepare_link_grid(grids[i], i, &p.link[i]);
        if (rc != LSDF_OK) return rc;
    }
    p.link_T = link_T;
    p.grid = static_cast<const float*>(grid_buf);
    p.points = points;
    p.out_dist = out_dist;
    p.out_link = out_link;
    p.out_link_dist = out_link_dist;
    p.ticket = static_cast<uint32_t*>(workspace);
    p.keys = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + kWsHeader);
    p.M = M;
    p.C = C;
    p.L = L;
    p.point_tiles = (int32_t)point_tiles;
    hipLaunchKernelGGL((query_kernel<K, CT>), dim3((unsigned)(point_tiles * conf_tiles)), dim3(kBlock), 0,
                       as_stream(stream), p);
    return check_launch("query_min_distance");
}
