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
//   * a call may hold many trajectories, each a range of configurations
//     checked against its own range of points (a re-planned path against
//     its latest cloud); a plain query is the one-trajectory case.  The
//     ranges come from device arrays, and the plan that turns them into
//     work (chunk counts and their prefix sums) is built on the device by
//     the first kernel, so that no call reads anything back to the host and
//     a whole step can be captured once in a graph and replayed with new
//     ranges;
//   * the iteration space (trajectory, link, 64-configuration group, point)
//     is cut into chunks of a tunable number of 8-point blocks; each XCD
//     (blocks b = x mod 8) takes a contiguous slice of chunks, which keeps
//     it on one or two links' grids in its L2, and deals its slice
//     round-robin to its waves, which spreads dense regions of a cloud over
//     many waves;
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

#ifndef LSDF_QUERY_UNROLL
#define LSDF_QUERY_UNROLL 8         // points per any-inside test
#endif
#ifndef LSDF_QUERY_GATHER
#define LSDF_QUERY_GATHER 4         // points whose gathers are in flight together
#endif
constexpr int kBlockPts = 8;        // points per culling sphere
constexpr int kUnroll = LSDF_QUERY_UNROLL;
constexpr int kGather = LSDF_QUERY_GATHER;
static_assert(kUnroll % kGather == 0, "gather batch must divide the unroll");
static_assert(kUnroll == kBlockPts, "blocks of 8 points");

// Default tiling: 4 blocks (32 points) per chunk, 8 workgroups per CU.
constexpr int kDefaultChunkPoints = 32;
constexpr int kDefaultBlocksPerCu = 8;
constexpr int kMaxChunkPoints = 8192;
constexpr int kMaxBlocksPerCu = 16;

// Work plan of one trajectory, built on the device.  Entry K (one past the
// last trajectory) holds only chunk_start = the total chunk count.
struct TrajPlan {
    int64_t chunk_start;       // first chunk of this trajectory
    int64_t m_lo, m_hi;        // points [m_lo, m_hi) of the concatenated cloud
    int32_t c_lo, c_n;         // configurations [c_lo, c_lo + c_n)
    int32_t cgroups;           // ceil(c_n / 64)
    int32_t chunks_per_group;  // ceil(8-point blocks touched / chunk_blocks)
    int32_t pad[2];
};
static_assert(sizeof(TrajPlan) == 48, "plan entry layout");

struct QueryArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    const float* link_T;
    uint32_t* keys;          // [C][L] complemented ordered keys, 0 = empty
    int32_t K;               // trajectories
    int32_t L;
    int32_t chunk_blocks;    // 8-point blocks per chunk
    int32_t blocks_per_xcd;
};

struct PrepArgs {
    const float* points;
    float4* spheres;         // [ceil(M / 8)]
    TrajPlan* plan;          // [K + 1]
    const int32_t* c_off;    // device [K + 1] or NULL (one trajectory of all C)
    const int64_t* m_off;    // device [K + 1] or NULL (one trajectory of all M)
    int64_t M;
    int32_t C;
    int32_t K;
    int32_t L;
    int32_t chunk_blocks;
};

struct FinalizeArgs {
    uint32_t* keys;
    float* out_dist;
    int32_t* out_link;
    float* out_link_dist;
    uint32_t* scratch;       // other scratch words to clear (culling spheres, plan), or NULL
    int64_t scratch_words;
    int32_t C;
    int32_t L;
};

template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void query_kernel(QueryArgs p, const float* __restrict__ points,
                                                       const typename GridT<DT>::T* __restrict__ grid,
                                                       const float4* __restrict__ spheres,
                                                       const TrajPlan* __restrict__ plan) {
    using E = GridT<DT>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xcd = blockIdx.x % kXcds;
    const int slot = blockIdx.x / kXcds;
    const int waves_per_xcd = p.blocks_per_xcd * kWavesPerBlock;
    const int wx = slot * kWavesPerBlock + wave;                 // wave index inside the XCD
    const int64_t total = plan[p.K].chunk_start;
    const int64_t q_lo = total * xcd / kXcds;                    // this XCD's slice of chunks
    const int64_t q_hi = total * (xcd + 1) / kXcds;
    if (q_lo + wx >= q_hi) return;

    // trajectory of the first chunk: the last entry whose start is <= q
    int k = 0;
    {
        int hi = p.K - 1;
        const int64_t q0 = q_lo + wx;
        while (k < hi) {
            const int mid = (k + hi + 1) >> 1;
            if (plan[mid].chunk_start <= q0) k = mid; else hi = mid - 1;
        }
    }

    for (int64_t q = q_lo + wx; q < q_hi; q += waves_per_xcd) {
        while (plan[k + 1].chunk_start <= q) ++k;   // stops at k + 1 = K at the latest: q < total
        k = __builtin_amdgcn_readfirstlane(k);
        const int64_t local = q - plan[k].chunk_start;
        const int64_t m_lo = plan[k].m_lo, m_hi = plan[k].m_hi;
        const int c_lo = plan[k].c_lo, c_n = plan[k].c_n;
        const int cgroups = plan[k].cgroups, cpg = plan[k].chunks_per_group;
        int64_t g, mc;
        if (local < ((int64_t)1 << 32)) {
            const uint32_t l32 = (uint32_t)local;
            g = l32 / (uint32_t)cpg;
            mc = l32 - (uint32_t)g * (uint32_t)cpg;
        } else {
            g = local / cpg;
            mc = local - g * cpg;
        }
        const int i = (int)((uint32_t)g / (uint32_t)cgroups);
        const int cb = (int)((uint32_t)g - (uint32_t)i * (uint32_t)cgroups);
        const int cl = cb * 64 + lane;
        const int c = c_lo + cl;
        const LinkGrid& lg = p.link[i];
        const typename E::T* __restrict__ G = grid + lg.offset;
        // the chunk's 8-point blocks (aligned in the concatenated cloud)
        const int64_t jb0 = ((m_lo >> 3) + mc * p.chunk_blocks) * kBlockPts;
        const int64_t jb1 = min(m_hi, jb0 + (int64_t)p.chunk_blocks * kBlockPts);

        // this lane's map: v = M [x; y; z] + w (centred grid coordinates)
        float m00 = 0.f, m01 = 0.f, m02 = 0.f, w0 = kFar;
        float m10 = 0.f, m11 = 0.f, m12 = 0.f, w1 = kFar;
        float m20 = 0.f, m21 = 0.f, m22 = 0.f, w2 = kFar;
        if (cl < c_n) {
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
        for (int64_t j = jb0; j < jb1; j += kBlockPts) {
            // the sphere bounds all 8 points of the block, so also the
            // trajectory's share of a block it shares with its neighbour
            const float4 sph = spheres[j / kBlockPts];
            const float s0 = fmaf(m00, sph.x, fmaf(m01, sph.y, fmaf(m02, sph.z, w0)));
            const float s1 = fmaf(m10, sph.x, fmaf(m11, sph.y, fmaf(m12, sph.z, w1)));
            const float s2 = fmaf(m20, sph.x, fmaf(m21, sph.y, fmaf(m22, sph.z, w2)));
            const bool near = (fabsf(s0) <= fmaf(nr0, sph.w, k0)) & (fabsf(s1) <= fmaf(nr1, sph.w, k1)) &
                              (fabsf(s2) <= fmaf(nr2, sph.w, k2));
            if (!__ballot(near)) continue;   // no point of the block is in any lane's box
            if (j >= m_lo && j + kUnroll <= m_hi) {
                float v0[kUnroll], v1[kUnroll], v2[kUnroll];
                bool in[kUnroll];
                bool any = false;
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const float x = points[3 * j + 3 * u + 0];
                    const float y = points[3 * j + 3 * u + 1];
                    const float z = points[3 * j + 3 * u + 2];
                    v0[u] = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
                    v1[u] = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
                    v2[u] = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
                    in[u] = inside<CUBIC>(lg, v0[u], v1[u], v2[u]);
                    any |= in[u];
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int b = 0; b < kUnroll; b += kGather) {
                        // issue every corner load of the batch, then interpolate
                        float c00[kGather], c10[kGather], c01[kGather], c11[kGather];
                        float d00[kGather], d10[kGather], d01[kGather], d11[kGather];
                        Cell cell[kGather];
#pragma unroll
                        for (int u = 0; u < kGather; ++u) {
                            cell[u] = locate(lg, v0[b + u], v1[b + u], v2[b + u]);
                            // lanes outside the box read the first cell (discarded)
                            const typename E::T* cp = G + (in[b + u] ? cell[u].idx : 0);
                            c00[u] = E::get(cp, 0);        d00[u] = E::get(cp, 1);
                            c10[u] = E::get(cp, nx);       d10[u] = E::get(cp, nx + 1);
                            c01[u] = E::get(cp, nxy);      d01[u] = E::get(cp, nxy + 1);
                            c11[u] = E::get(cp, nxy + nx); d11[u] = E::get(cp, nxy + nx + 1);
                        }
#pragma unroll
                        for (int u = 0; u < kGather; ++u) {
                            const float val = interpolate(c00[u], d00[u], c10[u], d10[u], c01[u], d01[u], c11[u],
                                                          d11[u], cell[u]);
                            if (in[b + u]) best = fminf(best, val);
                        }
                    }
                }
            } else {
                // a block at either end of the trajectory's points
                const int64_t ja = max(j, m_lo), jz = min(j + kBlockPts, m_hi);
                for (int64_t jj = ja; jj < jz; ++jj) {
                    const float x = points[3 * jj + 0], y = points[3 * jj + 1], z = points[3 * jj + 2];
                    const float v0 = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
                    const float v1 = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
                    const float v2 = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
                    if (inside<CUBIC>(lg, v0, v1, v2)) {
                        const Cell ce = locate(lg, v0, v1, v2);
                        const typename E::T* cp = G + ce.idx;
                        best = fminf(best, interpolate(E::get(cp, 0), E::get(cp, 1), E::get(cp, nx), E::get(cp, nx + 1),
                                                       E::get(cp, nxy), E::get(cp, nxy + 1), E::get(cp, nxy + nx),
                                                       E::get(cp, nxy + nx + 1), ce));
                    }
                }
            }
        }
        if (cl < c_n && best < INFINITY) atomicMax(&p.keys[(int64_t)c * p.L + i], ~lsdf::ordered_bits(best));
    }
}

// First kernel of a query.  Every thread bounds one block of 8 consecutive
// points of the concatenated cloud by a sphere: the centre of the block's
// box and a radius widened by a relative 1e-5, by 1e-4 of the sum of the
// coordinates' magnitudes (which bounds FP32 rounding of the mapped
// coordinates) and by 1e-6 m.  Workgroup 0 also builds the plan: each
// trajectory's ranges clamped into [0, C) and [0, M) (so a bad offset table
// gives wrong ranges, never an access out of bounds), its chunk count and
// the exclusive prefix sum of the counts.
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = b * kBlockPts;
    if (j0 < a.M) {
        const float* points = a.points;
        const int64_t j1 = min(a.M, j0 + kBlockPts);
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
        a.spheres[b] = make_float4(cx, cy, cz, fmaf(r, 1.00001f, fmaf(1e-4f, e, 1e-6f)));
    }
    if (blockIdx.x != 0) return;

    __shared__ int64_t scan[256];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int base = 0; base < a.K; base += 256) {
        const int k = base + t;
        TrajPlan e{};
        int64_t n = 0;
        if (k < a.K) {
            const int32_t c0 = a.c_off ? min(max(a.c_off[k], 0), a.C) : 0;
            const int32_t c1 = a.c_off ? min(max(a.c_off[k + 1], c0), a.C) : a.C;
            const int64_t m0 = a.m_off ? min(max(a.m_off[k], (int64_t)0), a.M) : 0;
            const int64_t m1 = a.m_off ? min(max(a.m_off[k + 1], m0), a.M) : a.M;
            e.m_lo = m0;
            e.m_hi = m1;
            e.c_lo = c0;
            e.c_n = c1 - c0;
            e.cgroups = (e.c_n + 63) / 64;
            const int64_t nb = m1 > m0 ? ((m1 + kBlockPts - 1) / kBlockPts) - m0 / kBlockPts : 0;
            e.chunks_per_group = (int32_t)((nb + a.chunk_blocks - 1) / a.chunk_blocks);
            n = (int64_t)a.L * e.cgroups * e.chunks_per_group;
        }
        scan[t] = n;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan
            const int64_t v = t >= off ? scan[t - off] : 0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        if (k < a.K) {
            e.chunk_start = carry + scan[t] - n;
            a.plan[k] = e;
        }
        carry += scan[255];
        __syncthreads();
    }
    if (t == 0) {
        TrajPlan e{};
        e.chunk_start = carry;
        a.plan[a.K] = e;
    }
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
    const int64_t rows = std::max<int64_t>(C, std::min<int64_t>(scratch_words, (int64_t)1 << 20));
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)std::max<int64_t>(1, (rows + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, f);
    return check_launch("query finalize");
}

namespace {

size_t keys_bytes(int64_t C, int64_t L) { return ((size_t)(C * L) * 4 + 255) / 256 * 256; }
size_t sphere_bytes(int64_t M) { return ((size_t)((M + kBlockPts - 1) / kBlockPts) * 16 + 255) / 256 * 256; }
size_t plan_bytes(int64_t K) { return ((size_t)(K + 1) * sizeof(TrajPlan) + 255) / 256 * 256; }

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int check_tuning(const char* who, const lsdf_query_tuning* t, int* chunk_blocks, int* blocks_per_cu) {
    using lsdf::fail;
    *chunk_blocks = kDefaultChunkPoints / kBlockPts;
    *blocks_per_cu = kDefaultBlocksPerCu;
    if (!t) return LSDF_OK;
    if (t->chunk_points != 0) {
        if (t->chunk_points < kBlockPts || t->chunk_points > kMaxChunkPoints || t->chunk_points % kBlockPts != 0)
            return fail(LSDF_E_INVALID_ARG, "%s: chunk_points = %d is not a multiple of 8 in [8, %d]", who,
                        (int)t->chunk_points, kMaxChunkPoints);
        *chunk_blocks = t->chunk_points / kBlockPts;
    }
    if (t->blocks_per_cu != 0) {
        if (t->blocks_per_cu < 1 || t->blocks_per_cu > kMaxBlocksPerCu)
            return fail(LSDF_E_INVALID_ARG, "%s: blocks_per_cu = %d out of [1, %d]", who, (int)t->blocks_per_cu,
                        kMaxBlocksPerCu);
        *blocks_per_cu = t->blocks_per_cu;
    }
    return LSDF_OK;
}

// Shared body of the plain (K = 1, no offset arrays) and batched queries.
int run_query(const char* who, int32_t K, const int32_t* c_off, const int64_t* m_off, const float* link_T, int32_t C,
              int32_t L, const lsdf_grid* grids, const void* grid_buf, const float* points, int64_t M, float* out_dist,
              int32_t* out_link, float* out_link_dist, const lsdf_query_tuning* tuning, uint32_t flags,
              void* workspace, size_t ws_bytes, void* stream) {
    using namespace lsdf;
    if (flags != 0) return fail(LSDF_E_UNSUPPORTED, "%s: unsupported flags 0x%x", who, flags);
    if (C < 0 || M < 0 || M > LSDF_MAX_POINTS)
        return fail(LSDF_E_SHAPE, "%s: size out of range (C = %d, M = %lld)", who, (int)C, (long long)M);
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "%s: L = %d out of [1, %d]", who, (int)L, LSDF_MAX_LINKS);
    if (K < 1 || K > LSDF_MAX_TRAJECTORIES)
        return fail(LSDF_E_SHAPE, "%s: K = %d out of [1, %d]", who, (int)K, LSDF_MAX_TRAJECTORIES);
    if (!grids) return fail(LSDF_E_INVALID_ARG, "%s: grids is NULL", who);
    int chunk_blocks = 0, blocks_per_cu = 0;
    int rc = check_tuning(who, tuning, &chunk_blocks, &blocks_per_cu);
    if (rc != LSDF_OK) return rc;
    if (C == 0) return LSDF_OK;
    if (!link_T || !grid_buf || !out_dist || !out_link || !workspace)
        return fail(LSDF_E_INVALID_ARG, "%s: NULL device pointer", who);
    if (M > 0 && !points) return fail(LSDF_E_INVALID_ARG, "%s: points is NULL", who);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "%s: workspace is not 256-byte aligned", who);
    const size_t need = keys_bytes(C, L) + sphere_bytes(M) + plan_bytes(K);
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "%s: workspace has %zu bytes, needs %zu", who, ws_bytes, need);

    QueryArgs p{};
    bool cubic = true;
    const int dtype = grids[0].dtype;
    for (int i = 0; i < L; ++i) {
        rc = prepare_link_grid(grids[i], i, &p.link[i]);
        if (rc != LSDF_OK) return rc;
        if (grids[i].dtype != dtype) return fail(LSDF_E_UNSUPPORTED, "%s: grids of one query must share a dtype", who);
        cubic = cubic && p.link[i].cubic;
    }
    hipStream_t s = as_stream(stream);
    char* ws = static_cast<char*>(workspace);
    float4* spheres = reinterpret_cast<float4*>(ws + keys_bytes(C, L));
    TrajPlan* plan = reinterpret_cast<TrajPlan*>(ws + keys_bytes(C, L) + sphere_bytes(M));
    p.link_T = link_T;
    p.keys = reinterpret_cast<uint32_t*>(ws);
    p.K = K;
    p.L = L;
    p.chunk_blocks = chunk_blocks;
    if (M > 0) {
        const int cus = device_cus();
        if (cus <= 0) return fail(LSDF_E_DEVICE, "%s: cannot read the device's compute-unit count", who);
        // persistent grid: blocks_per_cu workgroups per CU, a multiple of
        // the XCD count; when the chunk count is known here (one trajectory
        // given by C and M), no more waves than chunks
        int64_t blocks = (int64_t)cus * blocks_per_cu;
        if (!c_off) {
            const int64_t nb = (M + kBlockPts - 1) / kBlockPts;
            const int64_t chunks = (int64_t)L * ((C + 63) / 64) * ((nb + chunk_blocks - 1) / chunk_blocks);
            blocks = std::min<int64_t>(blocks, (chunks + kWavesPerBlock - 1) / kWavesPerBlock);
        }
        blocks = (blocks + kXcds - 1) / kXcds * kXcds;
        p.blocks_per_xcd = (int32_t)(blocks / kXcds);

        PrepArgs a{points, spheres, plan, c_off, m_off, M, C, K, L, chunk_blocks};
        const int64_t nsph = (M + kBlockPts - 1) / kBlockPts;
        hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((nsph + 255) / 256)), dim3(256), 0, s, a);
        rc = check_launch(who);
        if (rc != LSDF_OK) return rc;
        const float4* sph = spheres;
        const TrajPlan* pl = plan;
        const dim3 gd((unsigned)blocks), bd(kBlock);
        hipEvent_t ev0, ev1;
        take_kernel_events(&ev0, &ev1);
        if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return fail(LSDF_E_DEVICE, "%s: event record failed", who);
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph, pl); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph, pl); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph, pl); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph, pl); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph, pl); break;
            default: hipLaunchKernelGGL((query_kernel<false, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph, pl); break;
        }
        rc = check_launch(who);
        if (rc != LSDF_OK) return rc;
        if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return fail(LSDF_E_DEVICE, "%s: event record failed", who);
    }
    // the spheres and the plan are cleared with the keys: the next call may
    // lay its keys over them
    uint32_t* scratch = reinterpret_cast<uint32_t*>(spheres);
    const int64_t scratch_words = M > 0 ? (int64_t)(sphere_bytes(M) + plan_bytes(K)) / 4 : 0;
    return launch_query_finalize(p.keys, out_dist, out_link, out_link_dist, C, L, s, scratch, scratch_words);
}

}  // namespace

LSDF_API int lsdf_query_workspace_size(int32_t C, int32_t L, int64_t M, size_t* bytes) {
    return lsdf_query_batched_workspace_size(1, C, L, M, bytes);
}

LSDF_API int lsdf_query_batched_workspace_size(int32_t K, int32_t C, int32_t L, int64_t M, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "query_workspace_size: bytes is NULL");
    if (C < 0 || M < 0 || M > LSDF_MAX_POINTS) return fail(LSDF_E_SHAPE, "query_workspace_size: size out of range");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "query_workspace_size: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (K < 1 || K > LSDF_MAX_TRAJECTORIES)
        return fail(LSDF_E_SHAPE, "query_workspace_size: K = %d out of [1, %d]", (int)K, LSDF_MAX_TRAJECTORIES);
    *bytes = keys_bytes(C, L) + sphere_bytes(M) + plan_bytes(K);
    return LSDF_OK;
}

LSDF_API int lsdf_query_min_distance(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                     const void* grid_buf, const float* points, int64_t M, float* out_dist,
                                     int32_t* out_link, float* out_link_dist, uint32_t flags, void* workspace,
                                     size_t ws_bytes, void* stream) {
    lsdf::clear_error();
    return run_query("query", 1, nullptr, nullptr, link_T, C, L, grids, grid_buf, points, M, out_dist, out_link,
                     out_link_dist, nullptr, flags, workspace, ws_bytes, stream);
}

LSDF_API int lsdf_query_min_distance_batched(int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                                             const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                             const void* grid_buf, const float* points, int64_t M, float* out_dist,
                                             int32_t* out_link, float* out_link_dist,
                                             const lsdf_query_tuning* tuning, uint32_t flags, void* workspace,
                                             size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    if (!traj_c_offset || !traj_m_offset) return fail(LSDF_E_INVALID_ARG, "query_batched: NULL offset array");
    return run_query("query_batched", K, traj_c_offset, traj_m_offset, link_T, C, L, grids, grid_buf, points, M,
                     out_dist, out_link, out_link_dist, tuning, flags, workspace, ws_bytes, stream);
}

LSDF_API int lsdf_query_autotune(int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                                 const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                 const void* grid_buf, const float* points, int64_t M, float* out_dist,
                                 int32_t* out_link, const lsdf_query_tuning* candidates, int32_t n_candidates,
                                 int32_t reps, void* workspace, size_t ws_bytes, void* stream,
                                 lsdf_query_tuning* best, float* best_ms) {
    using namespace lsdf;
    clear_error();
    if (!traj_c_offset || !traj_m_offset) return fail(LSDF_E_INVALID_ARG, "query_autotune: NULL offset array");
    if (!best) return fail(LSDF_E_INVALID_ARG, "query_autotune: best is NULL");
    if (reps < 1 || reps > 1000) return fail(LSDF_E_INVALID_ARG, "query_autotune: reps = %d out of [1, 1000]", (int)reps);
    static const lsdf_query_tuning kGrid[] = {
        {8, 8},   {16, 8},  {32, 8},  {64, 8},  {128, 8}, {256, 8}, {1024, 8},
        {16, 4},  {32, 4},  {64, 4},  {128, 4}, {32, 2},  {64, 2},  {128, 2},
    };
    if (!candidates) {
        candidates = kGrid;
        n_candidates = (int32_t)(sizeof(kGrid) / sizeof(kGrid[0]));
    }
    if (n_candidates < 1) return fail(LSDF_E_INVALID_ARG, "query_autotune: no candidates");
    for (int32_t c = 0; c < n_candidates; ++c) {
        int cb = 0, bpc = 0;
        int rc = check_tuning("query_autotune", &candidates[c], &cb, &bpc);
        if (rc != LSDF_OK) return rc;
    }
    hipStream_t s = as_stream(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(LSDF_E_DEVICE, "query_autotune: cannot create events");
    }
    int rc = LSDF_OK;
    float best_t = INFINITY;
    int32_t best_i = -1;
    for (int32_t c = 0; c < n_candidates && rc == LSDF_OK; ++c) {
        // one untimed call, then reps timed calls between two events
        rc = run_query("query_autotune", K, traj_c_offset, traj_m_offset, link_T, C, L, grids, grid_buf, points, M,
                       out_dist, out_link, nullptr, &candidates[c], 0, workspace, ws_bytes, stream);
        if (rc != LSDF_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(LSDF_E_DEVICE, "query_autotune: event record failed"); break; }
        for (int32_t r = 0; r < reps && rc == LSDF_OK; ++r)
            rc = run_query("query_autotune", K, traj_c_offset, traj_m_offset, link_T, C, L, grids, grid_buf, points,
                           M, out_dist, out_link, nullptr, &candidates[c], 0, workspace, ws_bytes, stream);
        if (rc != LSDF_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(LSDF_E_DEVICE, "query_autotune: event timing failed");
            break;
        }
        ms /= (float)reps;
        if (ms < best_t) {
            best_t = ms;
            best_i = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LSDF_OK) return rc;
    if (best_i < 0) return fail(LSDF_E_DEVICE, "query_autotune: no candidate could be timed");
    *best = candidates[best_i];
    if (best_ms) *best_ms = best_t;
    return LSDF_OK;
}
