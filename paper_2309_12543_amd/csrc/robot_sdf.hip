// The paper's own pipeline (Sec. III-A, Eq. 1-4): per configuration, a
// "Robot SDF" over the voxels of the environment, the minimum over links of
// each link's SDF transformed by its pose and aligned to the environment
// grid; at run time the distance of a configuration is a pure gather, the
// minimum of its Robot SDF over the voxels the obstacle points occupy.
// It is kept here as the comparator of the per-point query: heavy
// preparation and C x V voxels of memory against a trivial runtime.
//
// Build (one thread per environment voxel column of 32, or of 8 for the
// network build, voxels x fastest,
// so every store is coalesced and each voxel is written exactly once,
// without atomics):
//   * link i's block at configuration c covers voxels k .. k + 2m - 1 per
//     axis, with k from the alignment of Eq. 1-3 (computed in double from
//     the link origin: T_O = t - lo, k = round(T_O / r) - m) and m the
//     block half-width in voxels (the farthest corner of the link's grid box
//     from the link origin, rounded up, plus two voxels, so that the block
//     holds every voxel whose centre can fall in the box);
//   * a voxel's value is the minimum, over the links whose block covers it,
//     of the link grid's interpolant at the voxel centre moved into the link
//     frame (the transformation of Eq. 4), +inf where no such link's box
//     holds the centre.  The centre is lo + (v + 1/2) r (double, rounded
//     once to float) and the interpolant uses the plain query's arithmetic,
//     so each value is bit-identical to the plain query at that point.
// Runtime: zero an occupancy bitmap and a counter; voxelise the points
// (floor((x - lo) / r) in double), keeping the first point of each voxel
// in a list of distinct occupied voxels; one workgroup per configuration
// takes the minimum of its Robot SDF over the list.
#include <algorithm>

#include "grid_sample.hpp"

namespace {

using lsdf::GridT;
using lsdf::LinkGrid;

constexpr int kBlock = 256;

struct LinkBlock {   // per (configuration, link): block corner and grid map
    int32_t k[3];
    int32_t pad;
    lsdf::GridMap gm;
};
static_assert(sizeof(LinkBlock) == 64, "LinkBlock layout");

struct BuildArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    int32_t halfw[LSDF_MAX_LINKS];   // m_i
    double lo[3];
    double r;
    int32_t n[3];
    int32_t C, L;
    const float* link_T;
    LinkBlock* blocks;               // [C][L]
    float* rs;                       // [C][n_z][n_y][n_x]
};

__global__ __launch_bounds__(kBlock) void align_kernel(BuildArgs a) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)a.C * a.L) return;
    const int i = (int)(t % a.L);
    const LinkGrid& lg = a.link[i];
    const float* T = a.link_T + t * 12;
    LinkBlock b{};
    // Eq. 1-2: T_O = t - lo, k = round(T_O / r) - m
    const float tr[3] = {T[3], T[7], T[11]};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) b.k[ax] = (int32_t)rint(((double)tr[ax] - a.lo[ax]) / a.r) - a.halfw[i];
    // the plain query's world-to-grid map of this pose (the transformation
    // of Eq. 4 with the grid scaling folded in)
    b.gm = lsdf::grid_map(lg, T);
    a.blocks[t] = b;
}

// Build tiles: a workgroup covers 64 (x, one per lane) x 4 (y, one per
// wave) x TZ (z, looped) voxels of one configuration, so that each wave
// reads a link's block corner and map once (scalar loads) for TZ x 64
// voxels and skips, with one uniform test, every link whose block misses
// its tile.  The exact build takes TZ = 32: four times fewer workgroups
// than 8, and its stores stream past the caches (non-temporal), since the
// Robot SDFs are read only by a later runtime call (1.62 -> 1.06 ms for 500
// waypoints over 128^3 voxels, against 0.61 ms for a plain fill of the same
// 4.2 GB).  The network build keeps TZ = 8 (its per-voxel work is larger).
constexpr int kTileX = 64, kTileY = kBlock / 64, kTileZ = 8, kBuildTileZ = 32;

struct Tile {
    int vx, vy, z0;
    bool lane_ok;        // this lane's x and the wave's y lie in the environment
};

__device__ inline Tile tile_of(const int32_t n[3], int tz) {
    const int tiles_x = (n[0] + kTileX - 1) / kTileX;
    const int ty = (int)blockIdx.x / tiles_x;
    const int tx = (int)blockIdx.x - ty * tiles_x;
    Tile t;
    t.vx = tx * kTileX + (int)(threadIdx.x & 63);
    t.vy = ty * kTileY + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    t.z0 = (int)blockIdx.y * tz;
    t.lane_ok = t.vx < n[0] && t.vy < n[1];
    return t;
}

// Does the block [k, k + w) per axis meet this wave's tile (x over the
// wave's 64 voxels, its y row, z over tz levels)?  Wave-uniform.
__device__ inline bool tile_meets(const Tile& t, const int32_t k[3], int w, int tz) {
    const int x0 = t.vx - (int)(threadIdx.x & 63);
    return k[0] < x0 + kTileX && k[0] + w > x0 && t.vy >= k[1] && t.vy < k[1] + w && k[2] < t.z0 + tz &&
           k[2] + w > t.z0;
}

template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void build_kernel(BuildArgs a, int32_t c0,
                                                       const typename GridT<DT>::T* __restrict__ grid) {
    const Tile t = tile_of(a.n, kBuildTileZ);
    const int c = c0 + (int)blockIdx.z;
    const float x = (float)(a.lo[0] + ((double)t.vx + 0.5) * a.r);
    const float y = (float)(a.lo[1] + ((double)t.vy + 0.5) * a.r);
    float zc[kBuildTileZ], best[kBuildTileZ];
#pragma unroll
    for (int dz = 0; dz < kBuildTileZ; ++dz) {
        zc[dz] = (float)(a.lo[2] + ((double)(t.z0 + dz) + 0.5) * a.r);
        best[dz] = INFINITY;
    }
    const LinkBlock* bl = a.blocks + (int64_t)c * a.L;
    for (int i = 0; i < a.L; ++i) {
        const LinkBlock b = bl[i];
        const int w = 2 * a.halfw[i];
        if (!tile_meets(t, b.k, w, kBuildTileZ)) continue;
        // only the voxels the link's aligned block covers
        if (!(t.vx >= b.k[0] && t.vx < b.k[0] + w)) continue;
        const LinkGrid& lg = a.link[i];
#pragma unroll
        for (int dz = 0; dz < kBuildTileZ; ++dz) {
            const int vz = t.z0 + dz;
            if (vz >= b.k[2] && vz < b.k[2] + w)
                best[dz] = fminf(best[dz], lsdf::sample_or_inf<CUBIC, DT>(grid + lg.offset, lg, b.gm, x, y, zc[dz]));
        }
    }
    if (!t.lane_ok) return;
    const int64_t V = (int64_t)a.n[0] * a.n[1] * a.n[2];
    float* out = a.rs + (int64_t)c * V + ((int64_t)t.z0 * a.n[1] + t.vy) * a.n[0] + t.vx;
#pragma unroll
    for (int dz = 0; dz < kBuildTileZ; ++dz)
        if (t.z0 + dz < a.n[2]) __builtin_nontemporal_store(best[dz], &out[(int64_t)dz * a.n[0] * a.n[1]]);
}

// The same build with the transformation of Eq. 5: each block voxel's
// link-frame position comes from the grid-transformation network,
// G = f(R) + dt_inv with dt_inv = -R^T dt / e_r, l = e_r G, e_r = m r, for a
// block half-width m shared by all links (the network's).
struct LinkBlockNN {
    int32_t k[3];
    int32_t pad;
    float h[LSDF_FRNN_HIDDEN];       // hidden layer of f at this rotation
    float dtinv[3];
    float pad2;
};
static_assert(sizeof(LinkBlockNN) == 160, "LinkBlockNN layout");

struct BuildNNArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    double lo[3];
    double r;
    int32_t n[3];
    int32_t C, L, m;
    float er;                        // m r
    const float* link_T;
    const float* params;             // W1[32][9], b1[32], W2[3V][32], b2[3V]
    LinkBlockNN* blocks;             // [C][L]
    float* rs;
};

__global__ __launch_bounds__(kBlock) void align_nn_kernel(BuildNNArgs a) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)a.C * a.L) return;
    const float* T = a.link_T + t * 12;
    LinkBlockNN b{};
    double dt[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        // Eq. 1-3: T_O = t - lo, k = round(T_O / r) - m, dt = T_O - (k + m) r
        const double t_o = (double)T[4 * ax + 3] - a.lo[ax];
        b.k[ax] = (int32_t)rint(t_o / a.r) - a.m;
        dt[ax] = t_o - ((double)b.k[ax] + (double)a.m) * a.r;
    }
    // dt_inv = -R^T dt / e_r  (R[row][col] = T[4 row + col])
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
        b.dtinv[ax] = (float)(-((double)T[ax] * dt[0] + (double)T[4 + ax] * dt[1] + (double)T[8 + ax] * dt[2]) /
                              (double)a.er);
    const float x[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
    const float* W1 = a.params;
    const float* b1 = W1 + LSDF_FRNN_HIDDEN * 9;
    for (int u = 0; u < LSDF_FRNN_HIDDEN; ++u) {
        float acc = b1[u];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc = fmaf(W1[u * 9 + k], x[k], acc);
        b.h[u] = fmaxf(acc, 0.0f);
    }
    a.blocks[t] = b;
}

template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void build_nn_kernel(BuildNNArgs a, int32_t c0,
                                                          const typename GridT<DT>::T* __restrict__ grid) {
    const Tile t = tile_of(a.n, kTileZ);
    const int c = c0 + (int)blockIdx.z;
    const int w = 2 * a.m;
    const int64_t O = 3 * (int64_t)w * w * w;
    const float* W2 = a.params + LSDF_FRNN_HIDDEN * 10;
    const float* b2 = W2 + O * LSDF_FRNN_HIDDEN;
    float best[kTileZ];
#pragma unroll
    for (int dz = 0; dz < kTileZ; ++dz) best[dz] = INFINITY;
    const LinkBlockNN* bl = a.blocks + (int64_t)c * a.L;
    for (int i = 0; i < a.L; ++i) {
        const LinkBlockNN& b = bl[i];
        if (!tile_meets(t, b.k, w, kTileZ)) continue;
        const int jx = t.vx - b.k[0], jy = t.vy - b.k[1];
        if (!(jx >= 0 && jx < w)) continue;
        const LinkGrid& lg = a.link[i];
        // link-frame point to centred grid coordinates: v_a = l_a invh_a + cen_a
        lsdf::GridMap id{};
        id.m00 = lg.invh[0]; id.w0 = lg.cen[0];
        id.m11 = lg.invh[1]; id.w1 = lg.cen[1];
        id.m22 = lg.invh[2]; id.w2 = lg.cen[2];
        for (int dz = 0; dz < kTileZ; ++dz) {
            const int jz = t.z0 + dz - b.k[2];
            if (jz < 0 || jz >= w) continue;
            const int64_t o = 3 * (((int64_t)jz * w + jy) * w + jx);
            float l[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float* row = W2 + (o + ax) * LSDF_FRNN_HIDDEN;
                float yv = b2[o + ax];
#pragma unroll
                for (int u = 0; u < LSDF_FRNN_HIDDEN; ++u) yv = fmaf(row[u], b.h[u], yv);
                l[ax] = a.er * (yv + b.dtinv[ax]);
            }
            best[dz] = fminf(best[dz], lsdf::sample_or_inf<CUBIC, DT>(grid + lg.offset, lg, id, l[0], l[1], l[2]));
        }
    }
    if (!t.lane_ok) return;
    const int64_t V = (int64_t)a.n[0] * a.n[1] * a.n[2];
    float* out = a.rs + (int64_t)c * V + ((int64_t)t.z0 * a.n[1] + t.vy) * a.n[0] + t.vx;
#pragma unroll
    for (int dz = 0; dz < kTileZ; ++dz)
        if (t.z0 + dz < a.n[2]) out[(int64_t)dz * a.n[0] * a.n[1]] = best[dz];
}

struct RuntimeArgs {
    double lo[3];
    double r;
    int32_t n[3];
    int32_t C;
    const float* points;
    int64_t M;
    uint32_t* bitmap;    // [ceil(V / 32)]
    uint32_t* count;     // distinct occupied voxels
    uint32_t* list;      // [min(M, V)]
    int64_t bitmap_words;
    const float* rs;
    float* out_dist;
};

__global__ __launch_bounds__(kBlock) void runtime_zero_kernel(RuntimeArgs a) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < a.bitmap_words) a.bitmap[t] = 0u;
    if (t == 0) *a.count = 0u;
}

// Voxels a workgroup's points fall in are first made unique in an LDS hash
// set (open addressing, twice as many slots as points, so every insertion
// ends within the table), and only one point per distinct voxel sets the
// voxel's bit with a device atomic: points of one obstacle lie together in
// the cloud, and their atomics on the same few bitmap words would otherwise
// run one after another.
constexpr int kHashSlots = 2 * kBlock;
constexpr uint32_t kHashEmpty = 0xffffffffu;

__global__ __launch_bounds__(kBlock) void voxelise_kernel(RuntimeArgs a) {
    __shared__ uint32_t s_key[kHashSlots];
    for (int k = threadIdx.x; k < kHashSlots; k += kBlock) s_key[k] = kHashEmpty;
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool inside = j < a.M;
    int64_t q[3] = {0, 0, 0};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double u = inside ? floor(((double)a.points[3 * j + ax] - a.lo[ax]) / a.r) : -1.0;
        inside = inside && u >= 0.0 && u < (double)a.n[ax];   // points outside the environment are dropped
        q[ax] = inside ? (int64_t)u : 0;
    }
    const int64_t v = (q[2] * a.n[1] + q[1]) * (int64_t)a.n[0] + q[0];
    // this point stands for its voxel in the workgroup when it inserts the
    // voxel into the set first (voxel 2^32 - 1, the empty key, always does)
    bool rep = inside && (uint32_t)v == kHashEmpty;
    if (inside && !rep) {
        uint32_t h = ((uint32_t)v * 2654435761u) % (uint32_t)kHashSlots;
        for (int probe = 0; probe < kHashSlots; ++probe) {
            const uint32_t prev = atomicCAS(&s_key[h], kHashEmpty, (uint32_t)v);
            if (prev == kHashEmpty) {
                rep = true;
                break;
            }
            if (prev == (uint32_t)v) break;
            h = (h + 1u) % (uint32_t)kHashSlots;
        }
    }
    const uint32_t bit = 1u << (v & 31);
    const bool first = rep && !(atomicOr(&a.bitmap[v >> 5], bit) & bit);   // first point of this voxel
    // the wave's new voxels take consecutive list slots: one counter atomic per wave
    const uint64_t mask = __ballot(first);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(mask);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(a.count, (uint32_t)__builtin_popcountll(mask));
    base = __shfl(base, leader, 64);
    if (first) a.list[base + (uint32_t)__builtin_popcountll(mask & ((1ull << lane) - 1))] = (uint32_t)v;
}

// One workgroup per configuration: the minimum of its Robot SDF over the
// occupied voxels.
__global__ __launch_bounds__(kBlock) void gather_kernel(RuntimeArgs a) {
    const int c = blockIdx.x;
    const int64_t V = (int64_t)a.n[0] * a.n[1] * a.n[2];
    const float* rs = a.rs + (int64_t)c * V;
    const uint32_t cnt = *a.count;
    // four independent loads in flight per step
    float b0 = INFINITY, b1 = INFINITY, b2 = INFINITY, b3 = INFINITY;
    uint32_t k = threadIdx.x;
    for (; k + 3 * kBlock < cnt; k += 4 * kBlock) {
        const uint32_t v0 = a.list[k], v1 = a.list[k + kBlock], v2 = a.list[k + 2 * kBlock], v3 = a.list[k + 3 * kBlock];
        b0 = fminf(b0, rs[v0]);
        b1 = fminf(b1, rs[v1]);
        b2 = fminf(b2, rs[v2]);
        b3 = fminf(b3, rs[v3]);
    }
    for (; k < cnt; k += kBlock) b0 = fminf(b0, rs[a.list[k]]);
    float best = fminf(fminf(b0, b1), fminf(b2, b3));
    // workgroup minimum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = fminf(best, __shfl_xor(best, off));
    __shared__ float wmin[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = wmin[0];
        for (int w = 1; w < kBlock / 64; ++w) m = fminf(m, wmin[w]);
        a.out_dist[c] = m;
    }
}

// Block half-width of a link: the farthest grid-box corner from the link
// origin, in voxels, rounded up, plus two.
double block_halfwidth(const lsdf_grid& g, float voxel) {
    double far2 = 0.0;
    for (int k = 0; k < 8; ++k) {
        double s = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const double cc = (k >> ax) & 1 ? g.hi[ax] : g.lo[ax];
            s += cc * cc;
        }
        far2 = std::max(far2, s);
    }
    return std::ceil(std::sqrt(far2) / (double)voxel) + 2.0;
}

int check_env(const char* who, const lsdf_env* env, int64_t* V) {
    using lsdf::fail;
    if (!env) return fail(LSDF_E_INVALID_ARG, "%s: env is NULL", who);
    if (!lsdf::finite3(env->lo) || !std::isfinite(env->voxel) || !(env->voxel > 0.0f))
        return fail(LSDF_E_INVALID_ARG, "%s: env needs a finite corner and a positive voxel edge", who);
    for (int a = 0; a < 3; ++a)
        if (env->n[a] < 1 || env->n[a] > 4096)
            return fail(LSDF_E_SHAPE, "%s: env n[%d] = %d out of [1, 4096]", who, a, (int)env->n[a]);
    *V = (int64_t)env->n[0] * env->n[1] * env->n[2];
    if (*V > ((int64_t)1 << 32)) return fail(LSDF_E_SHAPE, "%s: more than 2^32 voxels", who);
    return LSDF_OK;
}

// room for either form's per-(configuration, link) table
size_t blocks_bytes(int64_t C, int64_t L) {
    return ((size_t)(C * L) * std::max(sizeof(LinkBlock), sizeof(LinkBlockNN)) + 255) / 256 * 256;
}

}  // namespace

LSDF_API int lsdf_robot_sdf_size(int32_t C, const lsdf_env* env, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    int64_t V = 0;
    int rc = check_env("robot_sdf_size", env, &V);
    if (rc != LSDF_OK) return rc;
    if (C < 0) return fail(LSDF_E_SHAPE, "robot_sdf_size: C < 0");
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "robot_sdf_size: bytes is NULL");
    *bytes = (size_t)C * (size_t)V * 4;
    return LSDF_OK;
}

LSDF_API int lsdf_robot_sdf_build_workspace_size(int32_t C, int32_t L, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    if (C < 0 || L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "robot_sdf_build_workspace_size: bad C or L");
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "robot_sdf_build_workspace_size: bytes is NULL");
    *bytes = blocks_bytes(C, L);
    return LSDF_OK;
}

LSDF_API int lsdf_robot_sdf_build(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                  const void* grid_buf, const lsdf_env* env, float* robot_sdf, void* workspace,
                                  size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    int64_t V = 0;
    int rc = check_env("robot_sdf_build", env, &V);
    if (rc != LSDF_OK) return rc;
    if (C < 0) return fail(LSDF_E_SHAPE, "robot_sdf_build: C < 0");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "robot_sdf_build: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (!grids) return fail(LSDF_E_INVALID_ARG, "robot_sdf_build: grids is NULL");
    if (C == 0) return LSDF_OK;
    if (!link_T || !grid_buf || !robot_sdf || !workspace)
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_build: NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_build: workspace is not 256-byte aligned");
    if (ws_bytes < blocks_bytes(C, L))
        return fail(LSDF_E_SHAPE, "robot_sdf_build: workspace has %zu bytes, needs %zu", ws_bytes, blocks_bytes(C, L));
    BuildArgs a{};
    bool cubic = true;
    const int dtype = grids[0].dtype;
    for (int i = 0; i < L; ++i) {
        rc = prepare_link_grid(grids[i], i, &a.link[i]);
        if (rc != LSDF_OK) return rc;
        if (grids[i].dtype != dtype) return fail(LSDF_E_UNSUPPORTED, "robot_sdf_build: grids must share a dtype");
        cubic = cubic && a.link[i].cubic;
        const double hw = block_halfwidth(grids[i], env->voxel);
        if (hw > 65536.0) return fail(LSDF_E_SHAPE, "robot_sdf_build: link %d's block is too wide", i);
        a.halfw[i] = (int32_t)hw;
    }
    for (int ax = 0; ax < 3; ++ax) {
        a.lo[ax] = env->lo[ax];
        a.n[ax] = env->n[ax];
    }
    a.r = env->voxel;
    a.C = C;
    a.L = L;
    a.link_T = link_T;
    a.blocks = static_cast<LinkBlock*>(workspace);
    a.rs = robot_sdf;
    hipStream_t s = as_stream(stream);
    const int64_t CL = (int64_t)C * L;
    hipLaunchKernelGGL(align_kernel, dim3((unsigned)((CL + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    if ((rc = check_launch("robot_sdf_build (align)")) != LSDF_OK) return rc;
    // x, y: the tiles of one configuration, z: up to 65535 configurations per launch
    const dim3 bd(kBlock);
    for (int32_t c0 = 0; c0 < C; c0 += 65535) {
        const dim3 gd((unsigned)(((env->n[0] + kTileX - 1) / kTileX) * ((env->n[1] + kTileY - 1) / kTileY)),
                      (unsigned)((env->n[2] + kBuildTileZ - 1) / kBuildTileZ), (unsigned)std::min<int32_t>(65535, C - c0));
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((build_kernel<true, LSDF_F32>), gd, bd, 0, s, a, c0, static_cast<const float*>(grid_buf)); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((build_kernel<false, LSDF_F32>), gd, bd, 0, s, a, c0, static_cast<const float*>(grid_buf)); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((build_kernel<true, LSDF_BF16>), gd, bd, 0, s, a, c0, static_cast<const uint16_t*>(grid_buf)); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((build_kernel<false, LSDF_BF16>), gd, bd, 0, s, a, c0, static_cast<const uint16_t*>(grid_buf)); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((build_kernel<true, LSDF_F16>), gd, bd, 0, s, a, c0, static_cast<const _Float16*>(grid_buf)); break;
            default: hipLaunchKernelGGL((build_kernel<false, LSDF_F16>), gd, bd, 0, s, a, c0, static_cast<const _Float16*>(grid_buf)); break;
        }
        if ((rc = check_launch("robot_sdf_build")) != LSDF_OK) return rc;
    }
    return LSDF_OK;
}

LSDF_API int lsdf_robot_sdf_build_frnn(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                       const void* grid_buf, const lsdf_env* env, const float* frnn_params,
                                       int32_t m, float* robot_sdf, void* workspace, size_t ws_bytes,
                                       void* stream) {
    using namespace lsdf;
    clear_error();
    int64_t V = 0;
    int rc = check_env("robot_sdf_build_frnn", env, &V);
    if (rc != LSDF_OK) return rc;
    if (C < 0) return fail(LSDF_E_SHAPE, "robot_sdf_build_frnn: C < 0");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "robot_sdf_build_frnn: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (m < 1 || m > LSDF_FRNN_MAX_HALF) return fail(LSDF_E_SHAPE, "robot_sdf_build_frnn: m = %d out of [1, %d]", (int)m, LSDF_FRNN_MAX_HALF);
    if (!grids) return fail(LSDF_E_INVALID_ARG, "robot_sdf_build_frnn: grids is NULL");
    if (C == 0) return LSDF_OK;
    if (!link_T || !grid_buf || !robot_sdf || !workspace || !frnn_params)
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_build_frnn: NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_build_frnn: workspace is not 256-byte aligned");
    if (ws_bytes < blocks_bytes(C, L))
        return fail(LSDF_E_SHAPE, "robot_sdf_build_frnn: workspace has %zu bytes, needs %zu", ws_bytes, blocks_bytes(C, L));
    BuildNNArgs a{};
    bool cubic = true;
    const int dtype = grids[0].dtype;
    for (int i = 0; i < L; ++i) {
        rc = prepare_link_grid(grids[i], i, &a.link[i]);
        if (rc != LSDF_OK) return rc;
        if (grids[i].dtype != dtype) return fail(LSDF_E_UNSUPPORTED, "robot_sdf_build_frnn: grids must share a dtype");
        cubic = cubic && a.link[i].cubic;
        if (block_halfwidth(grids[i], env->voxel) > (double)m)
            return fail(LSDF_E_SHAPE, "robot_sdf_build_frnn: the network's block (m = %d) does not hold link %d's box",
                        (int)m, i);
    }
    for (int ax = 0; ax < 3; ++ax) {
        a.lo[ax] = env->lo[ax];
        a.n[ax] = env->n[ax];
    }
    a.r = env->voxel;
    a.C = C;
    a.L = L;
    a.m = m;
    a.er = (float)((double)m * (double)env->voxel);
    a.link_T = link_T;
    a.params = frnn_params;
    a.blocks = static_cast<LinkBlockNN*>(workspace);
    a.rs = robot_sdf;
    hipStream_t s = as_stream(stream);
    const int64_t CL = (int64_t)C * L;
    hipLaunchKernelGGL(align_nn_kernel, dim3((unsigned)((CL + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    if ((rc = check_launch("robot_sdf_build_frnn (align)")) != LSDF_OK) return rc;
    // x, y: the tiles of one configuration, z: up to 65535 configurations per launch
    const dim3 bd(kBlock);
    for (int32_t c0 = 0; c0 < C; c0 += 65535) {
        const dim3 gd((unsigned)(((env->n[0] + kTileX - 1) / kTileX) * ((env->n[1] + kTileY - 1) / kTileY)),
                      (unsigned)((env->n[2] + kTileZ - 1) / kTileZ), (unsigned)std::min<int32_t>(65535, C - c0));
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((build_nn_kernel<true, LSDF_F32>), gd, bd, 0, s, a, c0, static_cast<const float*>(grid_buf)); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((build_nn_kernel<false, LSDF_F32>), gd, bd, 0, s, a, c0, static_cast<const float*>(grid_buf)); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((build_nn_kernel<true, LSDF_BF16>), gd, bd, 0, s, a, c0, static_cast<const uint16_t*>(grid_buf)); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((build_nn_kernel<false, LSDF_BF16>), gd, bd, 0, s, a, c0, static_cast<const uint16_t*>(grid_buf)); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((build_nn_kernel<true, LSDF_F16>), gd, bd, 0, s, a, c0, static_cast<const _Float16*>(grid_buf)); break;
            default: hipLaunchKernelGGL((build_nn_kernel<false, LSDF_F16>), gd, bd, 0, s, a, c0, static_cast<const _Float16*>(grid_buf)); break;
        }
        if ((rc = check_launch("robot_sdf_build_frnn")) != LSDF_OK) return rc;
    }
    return LSDF_OK;
}

namespace {

size_t words256(int64_t words) { return ((size_t)words * 4 + 255) / 256 * 256; }

void runtime_layout(int64_t V, int64_t M, int64_t* bitmap_words, size_t* list_off, size_t* total) {
    *bitmap_words = (V + 31) / 32;
    const size_t count_off = words256(*bitmap_words);
    *list_off = count_off + 256;
    *total = *list_off + words256(std::min<int64_t>(M, V));
}

}  // namespace

LSDF_API int lsdf_robot_sdf_query_workspace_size(const lsdf_env* env, int64_t M, size_t* bytes) {
    using namespace lsdf;
    clear_error();
    int64_t V = 0;
    int rc = check_env("robot_sdf_query_workspace_size", env, &V);
    if (rc != LSDF_OK) return rc;
    if (M < 0) return fail(LSDF_E_SHAPE, "robot_sdf_query_workspace_size: M < 0");
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "robot_sdf_query_workspace_size: bytes is NULL");
    int64_t bw = 0;
    size_t lo = 0;
    runtime_layout(V, M, &bw, &lo, bytes);
    return LSDF_OK;
}

LSDF_API int lsdf_robot_sdf_query(const float* robot_sdf, int32_t C, const lsdf_env* env, const float* points,
                                  int64_t M, float* out_dist, void* workspace, size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    int64_t V = 0;
    int rc = check_env("robot_sdf_query", env, &V);
    if (rc != LSDF_OK) return rc;
    if (C < 0 || M < 0 || M > LSDF_MAX_POINTS) return fail(LSDF_E_SHAPE, "robot_sdf_query: size out of range");
    if (C == 0) return LSDF_OK;
    if (!robot_sdf || !out_dist || !workspace || (M > 0 && !points))
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_query: NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "robot_sdf_query: workspace is not 256-byte aligned");
    RuntimeArgs a{};
    size_t list_off = 0, need = 0;
    runtime_layout(V, M, &a.bitmap_words, &list_off, &need);
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "robot_sdf_query: workspace has %zu bytes, needs %zu", ws_bytes, need);
    for (int ax = 0; ax < 3; ++ax) {
        a.lo[ax] = env->lo[ax];
        a.n[ax] = env->n[ax];
    }
    a.r = env->voxel;
    a.C = C;
    a.points = points;
    a.M = M;
    char* ws = static_cast<char*>(workspace);
    a.bitmap = reinterpret_cast<uint32_t*>(ws);
    a.count = reinterpret_cast<uint32_t*>(ws + words256(a.bitmap_words));
    a.list = reinterpret_cast<uint32_t*>(ws + list_off);
    a.rs = robot_sdf;
    a.out_dist = out_dist;
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(runtime_zero_kernel, dim3((unsigned)((a.bitmap_words + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       a);
    if ((rc = check_launch("robot_sdf_query (zero)")) != LSDF_OK) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(voxelise_kernel, dim3((unsigned)((M + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
        if ((rc = check_launch("robot_sdf_query (voxelise)")) != LSDF_OK) return rc;
    }
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)C), dim3(kBlock), 0, s, a);
    return check_launch("robot_sdf_query (gather)");
}
