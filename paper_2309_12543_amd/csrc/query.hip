// Batched clearance query (Sec. III-A): per configuration c, the minimum over
// obstacle points and links of link i's grid SDF read at the point moved into
// link i's frame.
//
// Work layout:
//   * a wave owns one link i and 64 consecutive configurations (one per
//     lane); each lane holds the world-to-grid affine map of its pose (the
//     inverse pose of Eq. 4 with the grid scaling folded in) in 12 VGPRs;
//   * obstacle points are wave-uniform: they stream through scalar loads into
//     SGPRs, so mapping a point is 9 FMAs with no cross-lane traffic, and the
//     per-pair minimum stays in one register per lane;
//   * the box test is one max3 of absolute centred coordinates; lanes inside
//     their box gather 8 corners and interpolate, with the loads of a batch
//     of points issued together so that one wait covers them all;
//   * points are culled 8 at a time: a first small kernel bounds every block
//     of 8 consecutive points by a sphere, and a wave skips a block when no
//     lane's box can hold any of its points (the sphere centre is mapped with
//     the lane's own map; the test widens the box by the radius times the
//     map's row norms plus a bound on FP32 rounding, so the skip is exact);
//   * the iteration space (link, 64-configuration group, point) is cut into
//     chunks of 64 points; each XCD (blocks b = x mod 8) takes a contiguous
//     slice of chunks, which keeps it on one or two links' grids in its L2,
//     and deals its slice round-robin to its waves, which spreads dense
//     regions of the cloud over many waves;
//   * per-pair minima merge across waves with one unsigned atomic max on a
//     complemented order-preserving key; a second small kernel turns the
//     keys into the outputs and clears them, leaving the workspace zero (the
//     kernel boundary orders it after every atomic, with no device fence).
#include <algorithm>

#include "grid_sample.hpp"

namespace {

using lsdf::GridT;
using lsdf::LinkGrid;
using lsdf::Cell;
using lsdf::inside;
using lsdf::interpolate;
using lsdf::locate;

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kXcds = 8;
constexpr float kFar = 1e30f;       // centred coordinate of unused lanes: never inside
constexpr int kBlocksPerCu = 8;

#ifndef LSDF_QUERY_UNROLL
#define LSDF_QUERY_UNROLL 8         // points per any-inside test
#endif
#ifndef LSDF_QUERY_GATHER
#define LSDF_QUERY_GATHER 4         // points whose gathers are in flight together
#endif
#ifndef LSDF_QUERY_CHUNK
#define LSDF_QUERY_CHUNK 32         // points per work chunk
#endif
constexpr int kBlockPts = 8;        // points per culling sphere
constexpr int kUnroll = LSDF_QUERY_UNROLL;
constexpr int kGather = LSDF_QUERY_GATHER;
constexpr int kChunk = LSDF_QUERY_CHUNK;
static_assert(kUnroll % kGather == 0, "gather batch must divide the unroll");
static_assert(kUnroll == kBlockPts && kChunk % kBlockPts == 0, "blocks of 8 points");

struct QueryArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    const float* link_T;
    uint32_t* keys;      // [C][L] complemented ordered keys, 0 = empty
    int64_t M;
    int64_t chunks;      // L * cgroups * chunks_per_group
    int32_t chunks_per_group;
    int32_t C;
    int32_t L;
    int32_t cgroups;     // ceil(C / 64)
    int32_t blocks_per_xcd;
};

struct FinalizeArgs {
    uint32_t* keys;
    float* out_dist;
    int32_t* out_link;
    float* out_link_dist;
    uint32_t* scratch;       // other scratch words to clear (culling spheres), or NULL
    int64_t scratch_words;
    int32_t C;
    int32_t L;
};

template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void query_kernel(QueryArgs p, const float* __restrict__ points,
                                                       const typename GridT<DT>::T* __restrict__ grid,
                                                       const float4* __restrict__ spheres) {
    using E = GridT<DT>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int slot = blockIdx.x / kXcds;
    const int waves_per_xcd = p.blocks_per_xcd * kWavesPerBlock;
    const int wx = slot * kWavesPerBlock + wave;                 // wave index inside the XCD
    const int64_t q_lo = p.chunks * xcd / kXcds;                // this XCD's slice of chunks
    const int64_t q_hi = p.chunks * (xcd + 1) / kXcds;

    for (int64_t q = q_lo + wx; q < q_hi; q += waves_per_xcd) {
        const int64_t g = q / p.chunks_per_group;
        const int64_t j0 = (q - g * p.chunks_per_group) * kChunk;
        const int64_t j1 = min(p.M, j0 + kChunk);
        const int i = (int)(g / p.cgroups);
        const int cb = (int)(g - (int64_t)i * p.cgroups);
        const int c = cb * 64 + lane;
        const LinkGrid& lg = p.link[i];
        const typename E::T* __restrict__ G = grid + lg.offset;

        // this lane's map: v = M [x; y; z] + w (centred grid coordinates)
        float m00 = 0.f, m01 = 0.f, m02 = 0.f, w0 = kFar;
        float m10 = 0.f, m11 = 0.f, m12 = 0.f, w1 = kFar;
        float m20 = 0.f, m21 = 0.f, m22 = 0.f, w2 = kFar;
        if (c < p.C) {
            const float* T = p.link_T + ((int64_t)c * p.L + i) * 12;
            const float r00 = T[0], r01 = T[1], r02 = T[2], t0 = T[3];
            const float r10 = T[4], r11 = T[5], r12 = T[6], t1 = T[7];
            const float r20 = T[8], r21 = T[9], r22 = T[10], t2 = T[11];
            // row a of R^T scaled by invh_a; offset -invh_a (R^T t)_a + cen_a
            m00 = lg.invh[0] * r00; m01 = lg.invh[0] * r10; m02 = lg.invh[0] * r20;
            m10 = lg.invh[1] * r01; m11 = lg.invh[1] * r11; m12 = lg.invh[1] * r21;
            m20 = lg.invh[2] * r02; m21 = lg.invh[2] * r12; m22 = lg.invh[2] * r22;
            w0 = fmaf(-lg.invh[0], fmaf(r00, t0, fmaf(r10, t1, r20 * t2)), lg.cen[0]);
            w1 = fmaf(-lg.invh[1], fmaf(r01, t0, fmaf(r11, t1, r21 * t2)), lg.cen[1]);
            w2 = fmaf(-lg.invh[2], fmaf(r02, t0, fmaf(r12, t1, r22 * t2)), lg.cen[2]);
        }
        const int nx = lg.n[0];
        const int nxy = lg.n[0] * lg.n[1];

        // culling threshold of this lane per axis: half_a + ||M_a|| rho + slack,
        // where rho (per block) already holds the radius and the rounding bound
        // that scales with the coordinates; ||M_a|| is the row's own norm
        const float nr0 = sqrtf(fmaf(m00, m00, fmaf(m01, m01, m02 * m02))) * 1.000001f;
        const float nr1 = sqrtf(fmaf(m10, m10, fmaf(m11, m11, m12 * m12))) * 1.000001f;
        const float nr2 = sqrtf(fmaf(m20, m20, fmaf(m21, m21, m22 * m22))) * 1.000001f;
        const float k0 = lg.half[0] + fmaf(1e-4f, fabsf(w0), 1e-3f);
        const float k1 = lg.half[1] + fmaf(1e-4f, fabsf(w1), 1e-3f);
        const float k2 = lg.half[2] + fmaf(1e-4f, fabsf(w2), 1e-3f);

        float best = INFINITY;
        for (int64_t j = j0; j < j1; j += kBlockPts) {
            const float4 sph = spheres[j / kBlockPts];
            const float s0 = fmaf(m00, sph.x, fmaf(m01, sph.y, fmaf(m02, sph.z, w0)));
            const float s1 = fmaf(m10, sph.x, fmaf(m11, sph.y, fmaf(m12, sph.z, w1)));
            const float s2 = fmaf(m20, sph.x, fmaf(m21, sph.y, fmaf(m22, sph.z, w2)));
            const bool near = (fabsf(s0) <= fmaf(nr0, sph.w, k0)) & (fabsf(s1) <= fmaf(nr1, sph.w, k1)) &
                              (fabsf(s2) <= fmaf(nr2, sph.w, k2));
            if (!__ballot(near)) continue;   // no point of the block is in any lane's box
            if (j + kUnroll <= j1) {
                float v0[kUnroll], v1[kUnroll], v2[kUnroll];
                bool in[kUnroll];
                bool any = false;
#pragma unroll
                for (int k = 0; k < kUnroll; ++k) {
                    const float x = points[3 * j + 3 * k + 0];
                    const float y = points[3 * j + 3 * k + 1];
                    const float z = points[3 * j + 3 * k + 2];
                    v0[k] = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
                    v1[k] = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
                    v2[k] = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
                    in[k] = inside<CUBIC>(lg, v0[k], v1[k], v2[k]);
                    any |= in[k];
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int b = 0; b < kUnroll; b += kGather) {
                        // issue every corner load of the batch, then interpolate
                        float c00[kGather], c10[kGather], c01[kGather], c11[kGather];
                        float d00[kGather], d10[kGather], d01[kGather], d11[kGather];
                        Cell cell[kGather];
#pragma unroll
                        for (int k = 0; k < kGather; ++k) {
                            cell[k] = locate(lg, v0[b + k], v1[b + k], v2[b + k]);
                            // lanes outside the box read the first cell (discarded)
                            const typename E::T* cp = G + (in[b + k] ? cell[k].idx : 0);
                            c00[k] = E::get(cp, 0);        d00[k] = E::get(cp, 1);
                            c10[k] = E::get(cp, nx);       d10[k] = E::get(cp, nx + 1);
                            c01[k] = E::get(cp, nxy);      d01[k] = E::get(cp, nxy + 1);
                            c11[k] = E::get(cp, nxy + nx); d11[k] = E::get(cp, nxy + nx + 1);
                        }
#pragma unroll
                        for (int k = 0; k < kGather; ++k) {
                            const float val = interpolate(c00[k], d00[k], c10[k], d10[k], c01[k], d01[k], c11[k],
                                                          d11[k], cell[k]);
                            if (in[b + k]) best = fminf(best, val);
                        }
                    }
                }
            } else {
                for (int64_t jj = j; jj < j1; ++jj) {   // the cloud's last, partial block
                    const float x = points[3 * jj + 0], y = points[3 * jj + 1], z = points[3 * jj + 2];
                    const float v0 = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
                    const float v1 = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
                    const float v2 = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
                    if (inside<CUBIC>(lg, v0, v1, v2)) {
                        const Cell cl = locate(lg, v0, v1, v2);
                        const typename E::T* cp = G + cl.idx;
                        best = fminf(best, interpolate(E::get(cp, 0), E::get(cp, 1), E::get(cp, nx), E::get(cp, nx + 1),
                                                       E::get(cp, nxy), E::get(cp, nxy + 1), E::get(cp, nxy + nx),
                                                       E::get(cp, nxy + nx + 1), cl));
                    }
                }
            }
        }
        if (c < p.C && best < INFINITY) atomicMax(&p.keys[(int64_t)c * p.L + i], ~lsdf::ordered_bits(best));
    }
}

// Bounding sphere of each block of 8 consecutive points: centre of the
// block's box and a radius widened by a relative 1e-5, by 1e-4 of the sum
// of the coordinates' magnitudes (which bounds FP32 rounding of the mapped
// coordinates) and by 1e-6 m.
__global__ __launch_bounds__(256) void bounds_kernel(const float* __restrict__ points, int64_t M,
                                                     float4* __restrict__ spheres) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = b * kBlockPts;
    if (j0 >= M) return;
    const int64_t j1 = min(M, j0 + kBlockPts);
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    for (int64_t j = j0; j < j1; ++j) {
        lo0 = fminf(lo0, points[3 * j + 0]); hi0 = fmaxf(hi0, points[3 * j + 0]);
        lo1 = fminf(lo1, points[3 * j + 1]); hi1 = fmaxf(hi1, points[3 * j + 1]);
        lo2 = fminf(lo2, points[3 * j + 2]); hi2 = fmaxf(hi2, points[3 * j + 2]);
    }
    const float cx = 0.5f * (lo0 + hi0), cy = 0.5f * (lo1 + hi1), cz = 0.5f * (lo2 + hi2);
    float r2 = 0.0f;
    for (int64_t j = j0; j < j1; ++j) {
        const float dx = points[3 * j + 0] - cx, dy = points[3 * j + 1] - cy, dz = points[3 * j + 2] - cz;
        r2 = fmaxf(r2, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    }
    const float r = sqrtf(r2);
    const float e = fabsf(cx) + fabsf(cy) + fabsf(cz) + 3.0f * r;
    spheres[b] = make_float4(cx, cy, cz, fmaf(r, 1.00001f, fmaf(1e-4f, e, 1e-6f)));
}

// Keys -> outputs, one lane per configuration; clears the keys and the
// rest of the scratch, so that the whole workspace is zero again.
__global__ __launch_bounds__(kBlock) void finalize_kernel(FinalizeArgs p) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    for (int64_t k = c; k < p.scratch_words; k += (int64_t)gridDim.x * kBlock) p.scratch[k] = 0u;
    if (c >= p.C) return;
    uint32_t* row = p.keys + (int64_t)c * p.L;
    uint32_t k[LSDF_MAX_LINKS];
#pragma unroll
    for (int i = 0; i < LSDF_MAX_LINKS; ++i)
        if (i < p.L) k[i] = row[i];
    uint32_t bestk = 0;
    int arg = -1;
#pragma unroll
    for (int i = 0; i < LSDF_MAX_LINKS; ++i) {
        if (i < p.L) {
            row[i] = 0u;
            if (p.out_link_dist) p.out_link_dist[(int64_t)c * p.L + i] = k[i] ? lsdf::from_ordered_bits(~k[i]) : INFINITY;
            if (k[i] > bestk) {   // strict: ties keep the lowest link
                bestk = k[i];
                arg = i;
            }
        }
    }
    p.out_dist[c] = bestk ? lsdf::from_ordered_bits(~bestk) : INFINITY;
    p.out_link[c] = arg;
}

}  // namespace

int lsdf::launch_query_finalize(uint32_t* keys, float* out_dist, int32_t* out_link, float* out_link_dist, int32_t C,
                                int32_t L, hipStream_t s, uint32_t* scratch, int64_t scratch_words) {
    FinalizeArgs f{keys, out_dist, out_link, out_link_dist, scratch, scratch_words, C, L};
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((C + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, f);
    return check_launch("query finalize");
}

namespace {

size_t keys_bytes(int64_t C, int64_t L) { return ((size_t)(C * L) * 4 + 255) / 256 * 256; }
size_t sphere_bytes(int64_t M) { return ((size_t)((M + kBlockPts - 1) / kBlockPts) * 16 + 255) / 256 * 256; }

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace

LSDF_API int lsdf_query_workspace_size(int32_t C, int32_t L, int64_t M, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "query_workspace_size: bytes is NULL");
    if (C < 0 || M < 0) return fail(LSDF_E_SHAPE, "query_workspace_size: negative size");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "query_workspace_size: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    *bytes = keys_bytes(C, L) + sphere_bytes(M);
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
    const size_t need = keys_bytes(C, L) + sphere_bytes(M);
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "query: workspace has %zu bytes, needs %zu", ws_bytes, need);

    QueryArgs p{};
    bool cubic = true;
    const int dtype = grids[0].dtype;
    for (int i = 0; i < L; ++i) {
        int rc = prepare_link_grid(grids[i], i, &p.link[i]);
        if (rc != LSDF_OK) return rc;
        if (grids[i].dtype != dtype) return fail(LSDF_E_UNSUPPORTED, "query: grids of one query must share a dtype");
        cubic = cubic && p.link[i].cubic;
    }
    hipStream_t s = as_stream(stream);
    p.link_T = link_T;
    p.keys = static_cast<uint32_t*>(workspace);
    p.M = M;
    p.C = C;
    p.L = L;
    p.cgroups = (C + 63) / 64;
    p.chunks_per_group = (int32_t)((M + kChunk - 1) / kChunk);
    p.chunks = (int64_t)L * p.cgroups * p.chunks_per_group;
    if (p.chunks > 0) {
        const int cus = device_cus();
        if (cus <= 0) return fail(LSDF_E_DEVICE, "query: cannot read the device's compute-unit count");
        // persistent grid: at most kBlocksPerCu blocks per CU, a multiple of
        // the XCD count, and no more waves than chunks
        int64_t blocks = std::min<int64_t>((int64_t)cus * kBlocksPerCu,
                                           (p.chunks + kWavesPerBlock - 1) / kWavesPerBlock);
        blocks = (blocks + kXcds - 1) / kXcds * kXcds;
        p.blocks_per_xcd = (int32_t)(blocks / kXcds);
        float4* spheres = reinterpret_cast<float4*>(static_cast<char*>(workspace) + keys_bytes(C, L));
        const int64_t nsph = (M + kBlockPts - 1) / kBlockPts;
        hipLaunchKernelGGL(bounds_kernel, dim3((unsigned)((nsph + 255) / 256)), dim3(256), 0, s, points, M, spheres);
        int rc = check_launch("query_min_distance (bounds)");
        if (rc != LSDF_OK) return rc;
        const float4* sph = spheres;
        const dim3 gd((unsigned)blocks), bd(kBlock);
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph); break;
            default: hipLaunchKernelGGL((query_kernel<false, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph); break;
        }
        rc = check_launch("query_min_distance");
        if (rc != LSDF_OK) return rc;
    }
    uint32_t* sph_words = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + keys_bytes(C, L));
    const int64_t nsph_words = ((M + kBlockPts - 1) / kBlockPts) * 4;
    return launch_query_finalize(p.keys, out_dist, out_link, out_link_dist, C, L, s, sph_words, nsph_words);
}
