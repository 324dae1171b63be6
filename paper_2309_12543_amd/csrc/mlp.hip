// Learned per-link SDF surrogate: evaluation, clearance with exact-grid
// fallback, training (forward, backward, weight gradients, Adam) and labels.
#include <algorithm>
#include <cmath>

#include "grid_sample.hpp"
#include "mlp_common.hpp"

namespace {

using namespace lsdf;
using namespace lsdf::mlp;

constexpr int kBlock = 512;                 // 8 waves
constexpr int kWaves = kBlock / 64;
constexpr int kSplit = 512;                 // samples per weight-gradient split
constexpr int kSmallGradBlocks = 16;         // workgroups per split for the small gradients
constexpr int kBlocksPerCu = 2;             // 69 KB of LDS per block
// The clearance query: 12 waves share one copy of the staged weights, the 3
// waves per SIMD that its register budget (168 VGPRs) allows; one workgroup
// per CU
constexpr int kQueryBlock = 768;
constexpr int kQueryWaves = kQueryBlock / 64;
constexpr int kTileChunk = 8;               // 32-pair tiles a wave takes at a time: 256 points of one configuration
constexpr int kChunkPts = kTileChunk * TILE;

struct Domain {
    float cen[3];
    float inv[3];    // 1 / half
    float core[3];   // half extents of the core box
    float bound;     // remainder bound B (+inf: unbounded)
    float inv_bound; // 1 / B, 0 when B = +inf
};

// A pair's link-frame point relative to the domain centre (u), its
// normalised network input (xh) and whether it lies in the domain, from the
// pose (R, t) and the world point: the same operations in every kernel that
// decides or evaluates pairs, so that they agree bit for bit.
__device__ inline bool pair_frame(const float (&R)[9], const float (&tr)[3], const Domain& dm, float x, float y,
                                  float z, float (&u)[3], float (&xh)[3]) {
    const float dx = x - tr[0], dy = y - tr[1], dz = z - tr[2];
    float mx = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float l = fmaf(R[a], dx, fmaf(R[3 + a], dy, R[6 + a] * dz));   // (R^T d)_a
        u[a] = l - dm.cen[a];
        xh[a] = u[a] * dm.inv[a];
        mx = fmaxf(mx, fabsf(xh[a]));
    }
    return mx <= 1.0f;
}

// Whether every point of sphere (x, y, z, radius) has E - B above thr at this
// pose: E at the centre (pair_frame's and core_distance's arithmetic) less
// the radius, less B, above thr.
__device__ inline bool sphere_beyond(const float4& sph, const float (&R)[9], const float (&tr)[3], const Domain& dm,
                                     float thr) {
    float u[3], xh[3];
    pair_frame(R, tr, dm, sph.x, sph.y, sph.z, u, xh);
    return (core_distance(u[0], u[1], u[2], dm.core) - sph.w) - dm.bound > thr;
}

__device__ inline float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// evaluation at given link-frame points
// ---------------------------------------------------------------------------

struct EvalArgs {
    Domain d;
    const float* params;
    const float* points;
    float* out;
    int64_t N;
    int64_t tiles;
};

__global__ __launch_bounds__(kBlock) void mlp_eval_kernel(EvalArgs p) {
    __shared__ __bf16 sW2[WTILE_ELEMS];
    __shared__ __bf16 sW3[WTILE_ELEMS];
    __shared__ SmallParams sp;
    stage_weights(sW2, p.params + OFF_W2, false);
    stage_weights(sW3, p.params + OFF_W3, false);
    stage_small(&sp, p.params);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t t = (int64_t)blockIdx.x * kWaves + wave; t < p.tiles; t += (int64_t)gridDim.x * kWaves) {
        float xh[NT][3], e[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t j = min(t * TILE + 16 * nt + (lane & 15), p.N - 1);
            float u[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[a] = p.points[3 * j + a] - p.d.cen[a];
                xh[nt][a] = u[a] * p.d.inv[a];
            }
            e[nt] = core_distance(u[0], u[1], u[2], p.d.core);
        }
        float m[NT];
        forward_tile<NT>(sW2, sW3, &sp, xh, m);
        if (lane < 16) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int64_t j = t * TILE + 16 * nt + lane;
                float t;
                if (j < p.N) p.out[j] = bounded_share(m[nt], p.d.bound, p.d.inv_bound, t) + e[nt];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// clearance: network per pair, exact grid below the margin
// ---------------------------------------------------------------------------

struct QueryMlpArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    Domain dom[LSDF_MAX_LINKS];
    const float* link_T;
    const float* params;
    const void* grid;
    const float* points;
    uint32_t* keys;
    const float* ubound;     // [C][L] upper bounds U of the first kernel, or NULL (no bound: no skipping)
    const float4* tile_sph;  // [ceil(M / 32)] spheres bounding each tile's points (when ubound != NULL)
    const float4* chunk_sph; // [ceil(M / 256)] spheres bounding each chunk's points
    const int32_t* seed;     // [2][C][L] the chunks holding the pair that gave U and the sampled pair
                             // nearest the core box (-1: none), taken first
    int64_t M;
    int64_t tiles_per_link;
    int32_t tiles_per_c;
    int32_t C;
    int32_t L;
    float margin;
};

template <bool CUBIC, int DT>
// The register budget of 3 waves per SIMD (168 VGPRs) also schedules the tile
// loop better than the default 2 (248).
__global__ __launch_bounds__(kQueryBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) void query_mlp_kernel(QueryMlpArgs p) {
    __shared__ __bf16 sW2[WTILE_ELEMS];
    __shared__ __bf16 sW3[WTILE_ELEMS];
    __shared__ SmallParams sp;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // every workgroup takes every link in turn (its weights staged once per
    // link); a link's chunks (kTileChunk tiles, 256 points of one
    // configuration) are dealt round-robin to the workgroups, and a
    // workgroup's waves take its chunks one at a time from a counter in LDS:
    // the tiles a bounded query must evaluate cluster (points near a link, at
    // configurations near the obstacle), so a fixed share per wave would
    // leave the workgroup waiting on its busiest wave at every link
    __shared__ int s_next;
    const int64_t groups = (p.M + kChunkPts - 1) / kChunkPts;   // chunks per configuration
    const int64_t nchunks = (int64_t)p.C * groups;
    // a bounded query first takes, per configuration, the chunk that holds the
    // pair that gave U (slots below C), then the chunk holding the sampled
    // pair nearest the core box (slots C to 2 C: where a minimum that falls
    // back to the grid lies), so that the keys hold a small value early and
    // the other chunks skip against it; every other chunk then follows (the
    // seed slots of (c, i) process their chunks in any case)
    const int64_t nseed = p.seed ? 2 * (int64_t)p.C : 0;
    for (int i = 0; i < p.L; ++i) {
        const float* P = p.params + (int64_t)i * NPARAM;
        __syncthreads();   // every wave is done with the previous link's weights and chunks
        if (threadIdx.x == 0) s_next = 0;
        stage_weights(sW2, P + OFF_W2, false);
        stage_weights(sW3, P + OFF_W3, false);
        stage_small(&sp, P);
        __syncthreads();

        const LinkGrid& lg = p.link[i];
        const Domain& dm = p.dom[i];
        const typename GridT<DT>::T* G = static_cast<const typename GridT<DT>::T*>(p.grid) + lg.offset;
        float best = INFINITY;
        int cur = -1;
        GridMap gm{};
        float R[9] = {}, tr[3] = {};
        float thr = INFINITY;   // tiles whose pairs all have E - B above this are skipped
        float ub_c = INFINITY;  // the current configuration's upper bound U
        int64_t seed_c = -1, near_c = -1;   // and its seed chunks
        auto flush = [&](int c) {
            const float w = wave_min(best);
            if (lane == 0 && w < INFINITY) atomicMax(&p.keys[(int64_t)c * p.L + i], ~lsdf::ordered_bits(w));
            best = INFINITY;
        };
        for (;;) {
            int slot = 0;
            if (lane == 0) slot = atomicAdd(&s_next, 1);
            slot = __builtin_amdgcn_readfirstlane(__shfl(slot, 0, 64));
            const int64_t vs = (int64_t)blockIdx.x + (int64_t)slot * gridDim.x;
            if (vs >= nseed + nchunks) break;
            int c;
            int64_t grp;
            if (vs < nseed) {
                c = (int)(vs < p.C ? vs : vs - p.C);
                grp = p.seed[vs * p.L + i];
                // the near chunk when it is not the first one already
                if (grp < 0 || (vs >= p.C && grp == p.seed[(int64_t)c * p.L + i])) continue;
            } else {
                c = (int)((vs - nseed) / groups);
                grp = (vs - nseed) - (int64_t)c * groups;
            }
            if (c != cur) {
                if (cur >= 0 && !p.ubound) flush(cur);   // (a bounded query flushes every chunk)
                cur = c;
                const float* T = p.link_T + ((int64_t)c * p.L + i) * 12;
                gm = grid_map(lg, T);
                for (int r = 0; r < 3; ++r) {
                    for (int s = 0; s < 3; ++s) R[3 * r + s] = T[4 * r + s];
                    tr[r] = T[4 * r + 3];
                }
                if (p.ubound) ub_c = p.ubound[(int64_t)c * p.L + i];
                if (p.seed) {
                    seed_c = p.seed[(int64_t)c * p.L + i];
                    near_c = p.seed[((int64_t)p.C + c) * p.L + i];
                }
            }
            if (vs >= nseed && (grp == seed_c || grp == near_c)) continue;   // taken in the seed slots
            if (p.ubound) {
                // the threshold also falls to the smallest value found so far
                // for (c, i) by any wave (the key; a stale read is larger, so
                // still a bound of the minimum from above)
                float lim = ub_c;
                const uint32_t kv =
                    __hip_atomic_load(&p.keys[(int64_t)c * p.L + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (kv) lim = fminf(lim, lsdf::from_ordered_bits(~kv));
                thr = fmaxf(lim, p.margin);
            }
            // a chunk (then a tile) whose bounding sphere keeps every pair's
            // E - B above thr is skipped whole: E is 1-Lipschitz in the
            // link-frame point, so E >= E(centre) - radius over the sphere
            // (the radius is widened far beyond the FP32 rounding of E)
            if (p.ubound && sphere_beyond(p.chunk_sph[grp], R, tr, dm, thr)) continue;
            for (int64_t k = grp * kTileChunk; k < min((grp + 1) * kTileChunk, (int64_t)p.tiles_per_c); ++k) {
                if (p.ubound && sphere_beyond(p.tile_sph[k], R, tr, dm, thr)) continue;
                const int64_t j0 = k * TILE;
                float xh[NT][3], px[NT][3], e[NT];
                bool indom[NT];
                bool any[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int64_t j = j0 + 16 * nt + (lane & 15);
                    const int64_t jj = min(j, p.M - 1);
                    px[nt][0] = p.points[3 * jj + 0];
                    px[nt][1] = p.points[3 * jj + 1];
                    px[nt][2] = p.points[3 * jj + 2];
                    float u[3];
                    const bool in = pair_frame(R, tr, dm, px[nt][0], px[nt][1], px[nt][2], u, xh[nt]);
                    e[nt] = core_distance(u[0], u[1], u[2], dm.core);
                    indom[nt] = (j < p.M) && in;
                    // a pair with E - B above thr cannot hold the minimum (its
                    // value exceeds the value of some pair: a found minimum,
                    // or the upper bound U of a pair that cannot fall back)
                    any[nt] = __ballot(indom[nt] && (e[nt] - dm.bound <= thr)) != 0;
                }
                static_assert(NT == 2, "a tile of two 16-pair halves");
                if (!any[0] && !any[1]) continue;
                float m[NT];
                if (any[0] && any[1]) {
                    forward_tile<NT>(sW2, sW3, &sp, xh, m);
                } else {
                    // only one half may hold the minimum: the network runs on
                    // that half alone (each 16-pair half is its own MFMA
                    // column group, so its values are the same bits), and the
                    // other half's pairs are skipped like a whole tile's
                    const bool h0 = any[0];
                    const float xs[1][3] = {{h0 ? xh[0][0] : xh[1][0], h0 ? xh[0][1] : xh[1][1],
                                             h0 ? xh[0][2] : xh[1][2]}};
                    float m1[1];
                    forward_tile<1>(sW2, sW3, &sp, xs, m1);
                    m[0] = m1[0];
                    m[1] = m1[0];
                    if (h0) indom[1] = false; else indom[0] = false;
                }
                if (lane < 16) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        if (!indom[nt]) continue;
                        // below the margin the grid's value replaces the estimate;
                        // a point outside the grid box keeps the estimate, since
                        // the grid has no value there
                        float tb;
                        const float est = bounded_share(m[nt], dm.bound, dm.inv_bound, tb) + e[nt];
                        float v = est;
                        if (est < p.margin) {
                            const float g = sample_or_inf<CUBIC, DT>(G, lg, gm, px[nt][0], px[nt][1], px[nt][2]);
                            if (g < INFINITY) v = g;
                        }
                        best = fminf(best, v);
                    }
                }
            }
            // this chunk's minimum goes to the key at once, so that later
            // chunks of (c, i), on any wave, skip against it
            if (p.ubound) flush(c);
        }
        if (cur >= 0) flush(cur);
    }
}

// Bounding spheres of the learned query's point tiles (32 points) and chunks
// (256 points), one thread per tile: the centre of the points' box and the
// largest distance to it, widened by a relative 1e-5 and by 1e-4 m, which
// covers the FP32 rounding of the pose and of E (about 1e-6 m on clouds a few
// metres across) many times over.  A chunk's sphere bounds its tiles'
// spheres (eight adjacent lanes combine by shuffles).
__global__ __launch_bounds__(256) void mlp_sphere_kernel(const float* __restrict__ points, int64_t M,
                                                         float4* tile_sph, float4* chunk_sph) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nt = (M + TILE - 1) / TILE;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t j0 = k * TILE, j1 = min(j0 + TILE, M);
    for (int64_t j = j0; j < j1; ++j)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], points[3 * j + a]);
            hi[a] = fmaxf(hi[a], points[3 * j + a]);
        }
    float cen[3];
    for (int a = 0; a < 3; ++a) cen[a] = 0.5f * (lo[a] + hi[a]);
    float r2 = 0.0f;
    for (int64_t j = j0; j < j1; ++j) {
        const float dx = points[3 * j] - cen[0], dy = points[3 * j + 1] - cen[1], dz = points[3 * j + 2] - cen[2];
        r2 = fmaxf(r2, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    }
    const float r = fmaf(sqrtf(r2), 1.00001f, 1e-4f);
    if (k < nt) tile_sph[k] = make_float4(cen[0], cen[1], cen[2], r);
    // the chunk: box of the eight tiles' boxes, then the farthest tile sphere
    float clo[3], chi[3];
    for (int a = 0; a < 3; ++a) {
        clo[a] = lo[a];
        chi[a] = hi[a];
        for (int o = 1; o < kTileChunk; o <<= 1) {
            clo[a] = fminf(clo[a], __shfl_xor(clo[a], o, 64));
            chi[a] = fmaxf(chi[a], __shfl_xor(chi[a], o, 64));
        }
    }
    float cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = 0.5f * (clo[a] + chi[a]);
    float rr = 0.0f;
    if (k < nt) {
        const float dx = cen[0] - cc[0], dy = cen[1] - cc[1], dz = cen[2] - cc[2];
        rr = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) + r;
    }
    for (int o = 1; o < kTileChunk; o <<= 1) rr = fmaxf(rr, __shfl_xor(rr, o, 64));
    if (k < nt && k % kTileChunk == 0) chunk_sph[k / kTileChunk] = make_float4(cc[0], cc[1], cc[2], fmaf(rr, 1.00001f, 1e-4f));
}

// First kernel of a bounded learned query: per (configuration c, link i),
// U = the smallest E + B over a sample of the in-domain pairs with
// E - B >= margin (pairs whose estimate, at least E - B, cannot fall below
// the margin and so cannot take the grid's value): the first point of every
// 32-point tile; +inf if none.  Every such pair's value is at most its
// E + B, so U bounds the minimum from above (over any sample of pairs), and a
// pair with E - B > U cannot hold it.  Also the chunk holding the sampled
// pair that gave U (the query takes it first).  A workgroup takes one link
// and kBoundConfigs configurations (their poses in scalar registers) and
// strides over the tiles; the pair arithmetic is pair_frame's and
// core_distance's, as in the query.
constexpr int kBoundBlock = 256;
constexpr int kBoundConfigs = 4;

struct BoundArgs {
    Domain dom[LSDF_MAX_LINKS];
    const float* link_T;
    const float* points;
    float* ubound;           // [C][L]
    int32_t* seed;           // [2][C][L] chunk (256 points) of a pair that gave U, -1 if U = +inf; then
                             // that of the sampled in-domain pair with the smallest E, -1 if none
    int64_t M;
    int32_t C;
    int32_t L;
    float margin;
};

__global__ __launch_bounds__(kBoundBlock) void mlp_bound_kernel(BoundArgs p) {
    const int i = blockIdx.y;
    const int c0 = blockIdx.x * kBoundConfigs;
    const Domain& dm = p.dom[i];
    float R[kBoundConfigs][9], tr[kBoundConfigs][3], ub[kBoundConfigs], en[kBoundConfigs];
    int ag[kBoundConfigs], ng[kBoundConfigs];
#pragma unroll
    for (int k = 0; k < kBoundConfigs; ++k) {
        const int c = min(c0 + k, p.C - 1);
        const float* T = p.link_T + ((int64_t)c * p.L + i) * 12;
        for (int r = 0; r < 3; ++r) {
            for (int s = 0; s < 3; ++s) R[k][3 * r + s] = T[4 * r + s];
            tr[k][r] = T[4 * r + 3];
        }
        ub[k] = INFINITY;
        ag[k] = -1;
        en[k] = INFINITY;
        ng[k] = -1;
    }
    for (int64_t j = (int64_t)threadIdx.x * TILE; j < p.M; j += (int64_t)kBoundBlock * TILE) {
        const float x = p.points[3 * j + 0], y = p.points[3 * j + 1], z = p.points[3 * j + 2];
#pragma unroll
        for (int k = 0; k < kBoundConfigs; ++k) {
            float u[3], xh[3];
            if (!pair_frame(R[k], tr[k], dm, x, y, z, u, xh)) continue;
            const float e = core_distance(u[0], u[1], u[2], dm.core);
            if (e - dm.bound >= p.margin && e + dm.bound < ub[k]) {
                ub[k] = e + dm.bound;
                ag[k] = (int)(j / kChunkPts);
            }
            if (e < en[k]) {
                en[k] = e;
                ng[k] = (int)(j / kChunkPts);
            }
        }
    }
    __shared__ float s_ub[kBoundConfigs][kBoundBlock / 64], s_en[kBoundConfigs][kBoundBlock / 64];
    __shared__ int s_ag[kBoundConfigs], s_ng[kBoundConfigs];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < kBoundConfigs) {
        s_ag[threadIdx.x] = INT32_MAX;
        s_ng[threadIdx.x] = INT32_MAX;
    }
#pragma unroll
    for (int k = 0; k < kBoundConfigs; ++k) {
        const float w = wave_min(ub[k]), we = wave_min(en[k]);
        if (lane == 0) {
            s_ub[k][wave] = w;
            s_en[k][wave] = we;
        }
    }
    __syncthreads();
    // the block minima, and the lowest chunk holding a pair that gives each
#pragma unroll
    for (int k = 0; k < kBoundConfigs; ++k) {
        float v = INFINITY, ve = INFINITY;
        for (int w = 0; w < kBoundBlock / 64; ++w) {
            v = fminf(v, s_ub[k][w]);
            ve = fminf(ve, s_en[k][w]);
        }
        if (v < INFINITY && ub[k] == v) atomicMin(&s_ag[k], ag[k]);
        if (ve < INFINITY && en[k] == ve) atomicMin(&s_ng[k], ng[k]);
    }
    __syncthreads();
    if (threadIdx.x < kBoundConfigs && c0 + (int)threadIdx.x < p.C) {
        float v = INFINITY, ve = INFINITY;
        for (int w = 0; w < kBoundBlock / 64; ++w) {
            v = fminf(v, s_ub[threadIdx.x][w]);
            ve = fminf(ve, s_en[threadIdx.x][w]);
        }
        const int64_t o = (int64_t)(c0 + threadIdx.x) * p.L + i;
        p.ubound[o] = v;
        p.seed[o] = v < INFINITY ? s_ag[threadIdx.x] : -1;
        p.seed[(int64_t)p.C * p.L + o] = ve < INFINITY ? s_ng[threadIdx.x] : -1;
    }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------

// Per-link slices of the training workspace ([L][...] arrays).
struct TrainBufs {
    float* dz1;     // [L][128][B]
    __bf16* h1;     // [L][128][B]
    __bf16* h2;
    __bf16* h3;
    __bf16* dz2;
    __bf16* dz3;
    float* xh;      // [L][B][3]
    float* dm;      // [L][B]
    float* loss;    // [L][B / TILE_TRAIN]
    float* gpart;   // [L][nsplit][NPARAM]
};

struct TrainArgs {
    Domain dom[LSDF_MAX_LINKS];
    TrainBufs w;
    const float* params;
    const float* samples;
    const float* labels;
    const int32_t* bidx;
    int64_t N;
    int32_t B;
    int32_t nsplit;
};

// Forward and backward pass of one wave tile of the batch (16 samples per
// wave), in one kernel: the pre-activations never leave the registers.
// SiLU(z) and SiLU'(z) share one sigmoid, s = 1 / (1 + exp(-z)):
// SiLU = z s, SiLU' = s (1 + z (1 - s)).  SiLU'(z2) and SiLU'(z3) of every
// unit a lane holds are kept for the backward pass; SiLU'(z1), needed last,
// is recomputed from the inputs then (the same bits, three FMA and the
// sigmoid per unit), which keeps the kernel within its registers.  A
// lane's units in a result tile (16 mt + 4 g + r) are the units of its B
// operand slots (perm_unit), so the kept derivatives line up with the
// backward products with no exchange.
// Stored for the weight gradients: the rounded activations h1, h2, h3, the
// rounded deltas dz3, dz2 and the FP32 delta dz1, the normalised inputs and
// dm = d(loss)/dm; the loss per tile.
#ifndef LSDF_TRAIN_BLOCK
#define LSDF_TRAIN_BLOCK 512
#endif
constexpr int kTrainBlock = LSDF_TRAIN_BLOCK;
constexpr int kTrainWaves = kTrainBlock / 64;
static_assert(kSplit % (TILE_TRAIN * kTrainWaves) == 0, "a batch of whole workgroups");

__global__ __launch_bounds__(kTrainBlock) void train_fwdbwd_kernel(TrainArgs p) {
    __shared__ __bf16 sW2[WTILE_ELEMS];
    __shared__ __bf16 sW3[WTILE_ELEMS];
    __shared__ __bf16 sW3t[WTILE_ELEMS];
    __shared__ __bf16 sW2t[WTILE_ELEMS];
    __shared__ SmallParams sp;
    const int l = blockIdx.y;
    const float* P = p.params + (int64_t)l * NPARAM;
    stage_weights(sW2, P + OFF_W2, false);
    stage_weights(sW3, P + OFF_W3, false);
    stage_weights(sW3t, P + OFF_W3, true);
    stage_weights(sW2t, P + OFF_W2, true);
    stage_small(&sp, P);
    __syncthreads();
    static_assert(NT_TRAIN == 1, "one 16-sample column tile per wave");
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int col = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tt = blockIdx.x * kTrainWaves + wave;          // tile of this wave
    const int64_t B = p.B;
    const int64_t lB = (int64_t)l * B;
    const int64_t plane = (int64_t)l * H * B;
    const int64_t s_idx = (int64_t)tt * TILE_TRAIN + col;   // this lane's sample in the batch
    const int64_t c = s_idx;
    int64_t k = p.bidx ? (int64_t)p.bidx[lB + s_idx] : s_idx;
    k = min(max(k, (int64_t)0), p.N - 1);              // a bad index reads a valid sample
    const int64_t idx = (int64_t)l * p.N + k;
    const Domain& d = p.dom[l];
    float xh[3], u3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u3[a] = p.samples[3 * idx + a] - d.cen[a];
        xh[a] = u3[a] * d.inv[a];
    }
    const float e_core = core_distance(u3[0], u3[1], u3[2], d.core);
    if (lane < 16) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p.w.xh[(lB + s_idx) * 3 + a] = xh[a];
    }
    asm volatile("" ::: "memory");

    // ---- forward ----
    float g2[8][4], g3[8][4];   // SiLU' of this lane's units
    bf16x8 b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int u = perm_unit(s, 8 * g + e);
            const float z = fmaf(sp.w1[u][0], xh[0], fmaf(sp.w1[u][1], xh[1], fmaf(sp.w1[u][2], xh[2], sp.b1[u])));
            const __bf16 h = (__bf16)silu(z);
            b[s][e] = h;
            p.w.h1[plane + u * B + c] = h;
        }
    float m = 0.0f;
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16* sW = layer == 0 ? sW2 : sW3;
        const float* bias = layer == 0 ? sp.b2 : sp.b3;
        f32x4 acc[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
            acc[mt] = f32x4{bias[16 * mt + 4 * g], bias[16 * mt + 4 * g + 1], bias[16 * mt + 4 * g + 2],
                            bias[16 * mt + 4 * g + 3]};
        asm volatile("" ::: "memory");   // the layer's weight reads stay inside the layer
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_a(sW, mt, s, lane), b[s], acc[mt], 0, 0, 0);
        if (layer == 0) {
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int u = 16 * mt + 4 * g + r;
                    const float z = acc[mt][r];
                    const float sg = sigmoid(z);
                    const __bf16 h = (__bf16)(z * sg);
                    g2[mt][r] = silu_grad_of(z, sg);
                    b[mt >> 1][(mt & 1) * 4 + r] = h;
                    p.w.h2[plane + u * B + c] = h;
                }
        } else {
            float part = 0.0f;
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                for (int r = 0; r < 4; r += 2) {
                    const int u = 16 * mt + 4 * g + r;
                    __bf16 hh[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const float z = acc[mt][r + q];
                        const float sg = sigmoid(z);
                        hh[q] = (__bf16)(z * sg);
                        g3[mt][r + q] = silu_grad_of(z, sg);
                        p.w.h3[plane + (u + q) * B + c] = hh[q];
                    }
                    const bf16x2 hp = {hh[0], hh[1]};
                    const bf16x2 wp = {sp.w4b[u], sp.w4b[u + 1]};
                    part = __builtin_amdgcn_fdot2_f32_bf16(hp, wp, part, false);
                }
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            m = part + sp.b4;
        }
    }
    // loss of the estimate (bounded network share + core distance) and its
    // derivative with respect to the network's output m
    float tb;
    const float share = bounded_share(m, d.bound, d.inv_bound, tb);
    const float r_ = (share + e_core) - p.labels[idx];
    float dm = (r_ > 0.0f ? 1.0f : (r_ < 0.0f ? -1.0f : 0.0f)) / (float)B;
    if (d.inv_bound != 0.0f) dm *= 1.0f - tb * tb;
    float absr = lane < 16 ? fabsf(r_) : 0.0f;
    if (lane < 16) p.w.dm[lB + s_idx] = dm;
    absr = wave_sum(absr);
    if (lane == 0) p.w.loss[(int64_t)l * (B / TILE_TRAIN) + tt] = absr;

    // ---- backward ----
    // dz3 = dm * w4 * SiLU'(z3), rounded: B operand of dh2 = W3^T dz3
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int u = perm_unit(s, 8 * g + e);
            const __bf16 db = (__bf16)(dm * sp.w4[u] * g3[2 * s + (e >> 2)][e & 3]);
            b[s][e] = db;
            p.w.dz3[plane + u * B + c] = db;
        }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16* sW = layer == 0 ? sW3t : sW2t;
        f32x4 acc[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        asm volatile("" ::: "memory");
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_a(sW, mt, s, lane), b[s], acc[mt], 0, 0, 0);
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = 16 * mt + 4 * g + r;
                if (layer == 0) {
                    // dz2 = (W3^T dz3) * SiLU'(z2), rounded: B operand of dh1 = W2^T dz2
                    const __bf16 db = (__bf16)(acc[mt][r] * g2[mt][r]);
                    b[mt >> 1][(mt & 1) * 4 + r] = db;
                    p.w.dz2[plane + u * B + c] = db;
                } else {
                    // dz1 = (W2^T dz2) * SiLU'(z1), kept in FP32
                    const float z = fmaf(sp.w1[u][0], xh[0], fmaf(sp.w1[u][1], xh[1], fmaf(sp.w1[u][2], xh[2], sp.b1[u])));
                    p.w.dz1[plane + u * B + c] = acc[mt][r] * silu_grad_of(z, sigmoid(z));
                }
            }
    }
}

// Weight gradients over one split of the batch.  Workgroups with z = 0:
// dW3 = dz3^T h2 and dW2 = dz2^T h1 on MFMA (K = samples), a 64 x 64 output
// quarter per wave, the next K step's operands loaded while the current one
// multiplies.  Workgroups with z >= 1: the small gradients (W1 and b1, b2,
// b3, w4, b4), a share of the (kind, unit) items each; a wave takes one item
// at a time, its lanes stride the split's samples (coalesced reads) and a
// butterfly sums the lanes.
__global__ __launch_bounds__(kBlock) void train_wgrad_kernel(TrainArgs p) {
    const int l = blockIdx.y;
    const int split = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int col = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t B = p.B;
    const int64_t plane = (int64_t)l * H * B;
    const int64_t k0 = (int64_t)split * kSplit;
    float* gp = p.w.gpart + ((int64_t)l * p.nsplit + split) * NPARAM;

    if (blockIdx.z == 0) {
        const bool third = wave < 4;
        const int q = wave & 3;
        const __bf16* A = (third ? p.w.dz3 : p.w.dz2) + plane;   // [out][B]
        const __bf16* Bm = (third ? p.w.h2 : p.w.h1) + plane;    // [in][B]
        const int r0 = 64 * (q >> 1), c0 = 64 * (q & 1);
        f32x4 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        bf16x8 a[4], bb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = *reinterpret_cast<const bf16x8*>(A + (r0 + 16 * mt + col) * B + k0 + 8 * g);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) bb[nt] = *reinterpret_cast<const bf16x8*>(Bm + (c0 + 16 * nt + col) * B + k0 + 8 * g);
        for (int64_t k = k0; k < k0 + kSplit; k += 32) {
            bf16x8 an[4], bn[4];
            const int64_t kn = k + 32 < k0 + kSplit ? k + 32 : k;   // the last step reloads its own operands
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                an[mt] = *reinterpret_cast<const bf16x8*>(A + (r0 + 16 * mt + col) * B + kn + 8 * g);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                bn[nt] = *reinterpret_cast<const bf16x8*>(Bm + (c0 + 16 * nt + col) * B + kn + 8 * g);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], bb[nt], acc[mt][nt], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = an[t];
                bb[t] = bn[t];
            }
        }
        const int off = third ? OFF_W3 : OFF_W2;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    gp[off + (r0 + 16 * mt + 4 * g + r) * H + (c0 + 16 * nt + col)] = acc[mt][nt][r];
        return;
    }

    // items 0 .. 4 H: kind = item / H (0: W1 row and b1, 1: b2, 2: b3,
    // 3: w4), unit = item mod H; item 4 H is b4
    constexpr int kItems = 4 * H + 1;
    const int share = (kItems + kSmallGradBlocks - 1) / kSmallGradBlocks;
    const int i0 = (blockIdx.z - 1) * share;
    const int i1 = min(kItems, i0 + share);
    const int64_t lB = (int64_t)l * B;
    static_assert(kSplit % 64 == 0, "split of whole waves");
    for (int item = i0 + wave; item < i1; item += kWaves) {
        const int kind = item / H;
        const int u = item - kind * H;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
        for (int it = 0; it < kSplit / 64; ++it) {
            const int64_t k = k0 + 64 * it + lane;
            if (kind == 0) {
                const float d = p.w.dz1[plane + u * B + k];
                const float* x = p.w.xh + (lB + k) * 3;
                s0 = fmaf(d, x[0], s0);
                s1 = fmaf(d, x[1], s1);
                s2 = fmaf(d, x[2], s2);
                s3 += d;
            } else if (kind == 1) {
                s0 += (float)p.w.dz2[plane + u * B + k];
            } else if (kind == 2) {
                s0 += (float)p.w.dz3[plane + u * B + k];
            } else if (kind == 3) {
                s0 = fmaf(p.w.dm[lB + k], (float)p.w.h3[plane + u * B + k], s0);
            } else {
                s0 += p.w.dm[lB + k];
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            s0 += __shfl_xor(s0, o, 64);
            s1 += __shfl_xor(s1, o, 64);
            s2 += __shfl_xor(s2, o, 64);
            s3 += __shfl_xor(s3, o, 64);
        }
        if (lane == 0) {
            if (kind == 0) {
                gp[OFF_W1 + 3 * u + 0] = s0;
                gp[OFF_W1 + 3 * u + 1] = s1;
                gp[OFF_W1 + 3 * u + 2] = s2;
                gp[OFF_B1 + u] = s3;
            } else if (kind == 1) {
                gp[OFF_B2 + u] = s0;
            } else if (kind == 2) {
                gp[OFF_B3 + u] = s0;
            } else if (kind == 3) {
                gp[OFF_W4 + u] = s0;
            } else {
                gp[OFF_B4] = s0;
            }
        }
    }
}

struct ReduceArgs {
    TrainBufs w;
    float* params;
    float* m;
    float* v;
    float* grad_out;
    float* loss_out;
    int32_t L;
    int32_t B;
    int32_t nsplit;
    int32_t adam;
    float lr;      // step size
    float beta1;
    float beta2;
    float eps;
    float c1;      // 1 - beta1^t
    float c2;      // 1 - beta2^t
};

// Sums the split partials into the gradient; optionally applies Adam.
__global__ __launch_bounds__(256) void train_reduce_kernel(ReduceArgs p) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < (int64_t)p.L * NPARAM) {
        const int l = (int)(k / NPARAM);
        const int pk = (int)(k - (int64_t)l * NPARAM);
        // the split partials in order, their loads issued 8 at a time
        float gsum = 0.f;
        for (int s0 = 0; s0 < p.nsplit; s0 += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = s0 + u < p.nsplit ? p.w.gpart[((int64_t)l * p.nsplit + s0 + u) * NPARAM + pk] : 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (s0 + u < p.nsplit) gsum += v[u];
        }
        if (p.grad_out) p.grad_out[k] = gsum;
        if (p.adam) {
            const float mk = p.beta1 * p.m[k] + (1.0f - p.beta1) * gsum;
            const float vk = p.beta2 * p.v[k] + (1.0f - p.beta2) * gsum * gsum;
            p.m[k] = mk;
            p.v[k] = vk;
            p.params[k] -= p.lr * (mk / p.c1) / (sqrtf(vk / p.c2) + p.eps);
        }
    }
    // mean loss per link: wave l sums link l's tiles (lanes stride them, then a butterfly)
    if (p.loss_out && k < (int64_t)p.L * 64) {
        const int l = (int)(k >> 6), lane = (int)(k & 63);
        const int tiles = p.B / TILE_TRAIN;
        float s = 0.f;
        for (int t = lane; t < tiles; t += 64) s += p.w.loss[(int64_t)l * tiles + t];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) p.loss_out[l] = s / (float)p.B;
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

int make_domain(const lsdf_mlp_domain& d, int index, Domain* out) {
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(d.centre[a]) || !std::isfinite(d.half[a]) || !(d.half[a] > 0.0f))
            return fail(LSDF_E_INVALID_ARG, "mlp domain %d: centre must be finite and half > 0", index);
        if (!std::isfinite(d.core_half[a]) || !(d.core_half[a] >= 0.0f))
            return fail(LSDF_E_INVALID_ARG, "mlp domain %d: core_half must be finite and >= 0", index);
        out->cen[a] = d.centre[a];
        out->inv[a] = (float)(1.0 / (double)d.half[a]);
        out->core[a] = d.core_half[a];
    }
    if (!(d.bound > 0.0f))   // NaN, zero or negative; +inf is allowed
        return fail(LSDF_E_INVALID_ARG, "mlp domain %d: bound must be > 0 (or +inf)", index);
    out->bound = d.bound;
    out->inv_bound = std::isinf(d.bound) ? 0.0f : (float)(1.0 / (double)d.bound);
    return LSDF_OK;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Carves the training workspace; returns the bytes it needs.
size_t train_layout(int32_t L, int32_t B, char* base, TrainBufs* w) {
    const size_t f_plane = align256((size_t)L * H * B * sizeof(float));
    const size_t h_plane = align256((size_t)L * H * B * sizeof(__bf16));
    const int nsplit = B / kSplit;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    TrainBufs t{};
    t.dz1 = (float*)take(f_plane);
    t.h1 = (__bf16*)take(h_plane);
    t.h2 = (__bf16*)take(h_plane);
    t.h3 = (__bf16*)take(h_plane);
    t.dz2 = (__bf16*)take(h_plane);
    t.dz3 = (__bf16*)take(h_plane);
    t.xh = (float*)take((size_t)L * B * 3 * sizeof(float));
    t.dm = (float*)take((size_t)L * B * sizeof(float));
    t.loss = (float*)take((size_t)L * (B / TILE_TRAIN) * sizeof(float));
    t.gpart = (float*)take((size_t)L * nsplit * NPARAM * sizeof(float));
    if (w) *w = t;
    return off;
}

int check_train_sizes(int32_t L, int32_t B, int64_t N) {
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "mlp train: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (B < kSplit || B % kSplit != 0) return fail(LSDF_E_SHAPE, "mlp train: B = %d must be a positive multiple of %d", (int)B, kSplit);
    if (N < 1) return fail(LSDF_E_SHAPE, "mlp train: N = %lld < 1", (long long)N);
    return LSDF_OK;
}

int train_common(const float* params, float* adam_m, float* adam_v, int64_t t, float lr, float beta1, float beta2,
                 float eps, bool adam, const lsdf_mlp_domain* domains, int32_t L, const float* samples,
                 const float* labels, int64_t N, const int32_t* batch_index, int32_t B, float* loss_out,
                 float* grad_out, void* workspace, size_t ws_bytes, void* stream) {
    int rc = check_train_sizes(L, B, N);
    if (rc != LSDF_OK) return rc;
    if (!params || !domains || !samples || !labels || !workspace)
        return fail(LSDF_E_INVALID_ARG, "mlp train: NULL pointer");
    if (adam && (!adam_m || !adam_v)) return fail(LSDF_E_INVALID_ARG, "mlp train: NULL Adam moments");
    if (adam && t < 1) return fail(LSDF_E_INVALID_ARG, "mlp train: step t = %lld < 1", (long long)t);
    if (adam && !(std::isfinite(lr) && std::isfinite(beta1) && std::isfinite(beta2) && std::isfinite(eps) &&
                  beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return fail(LSDF_E_INVALID_ARG, "mlp train: bad Adam hyper-parameters");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "mlp train: workspace is not 256-byte aligned");
    const size_t need = train_layout(L, B, nullptr, nullptr);
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "mlp train: workspace has %zu bytes, needs %zu", ws_bytes, need);
    TrainArgs a{};
    for (int i = 0; i < L; ++i) {
        rc = make_domain(domains[i], i, &a.dom[i]);
        if (rc != LSDF_OK) return rc;
    }
    train_layout(L, B, static_cast<char*>(workspace), &a.w);
    a.params = params;
    a.samples = samples;
    a.labels = labels;
    a.bidx = batch_index;
    a.N = N;
    a.B = B;
    a.nsplit = B / kSplit;
    hipStream_t s = as_stream(stream);
    const dim3 tiles_grid(B / (TILE_TRAIN * kTrainWaves), L);
    hipLaunchKernelGGL(train_fwdbwd_kernel, tiles_grid, dim3(kTrainBlock), 0, s, a);
    if ((rc = check_launch("mlp train forward and backward")) != LSDF_OK) return rc;
    hipLaunchKernelGGL(train_wgrad_kernel, dim3(a.nsplit, L, 1 + kSmallGradBlocks), dim3(kBlock), 0, s, a);
    if ((rc = check_launch("mlp train weight gradients")) != LSDF_OK) return rc;
    ReduceArgs r{};
    r.w = a.w;
    r.params = const_cast<float*>(params);
    r.m = adam_m;
    r.v = adam_v;
    r.grad_out = grad_out;
    r.loss_out = loss_out;
    r.L = L;
    r.B = B;
    r.nsplit = a.nsplit;
    r.adam = adam ? 1 : 0;
    if (adam) {
        r.lr = lr;
        r.beta1 = beta1;
        r.beta2 = beta2;
        r.eps = eps;
        r.c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
        r.c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    }
    const int64_t total = (int64_t)L * NPARAM;
    hipLaunchKernelGGL(train_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, r);
    return check_launch("mlp train reduce");
}

}  // namespace

LSDF_API int lsdf_mlp_eval(const float* params, const lsdf_mlp_domain* domain, const float* points, int64_t N,
                           float* out, void* stream) {
    clear_error();
    if (!domain) return fail(LSDF_E_INVALID_ARG, "mlp_eval: domain is NULL");
    if (N < 0) return fail(LSDF_E_SHAPE, "mlp_eval: N < 0");
    if (N == 0) return LSDF_OK;
    if (!params || !points || !out) return fail(LSDF_E_INVALID_ARG, "mlp_eval: NULL device pointer");
    EvalArgs a{};
    int rc = make_domain(*domain, 0, &a.d);
    if (rc != LSDF_OK) return rc;
    const int cus = device_cus();
    if (cus <= 0) return fail(LSDF_E_DEVICE, "mlp_eval: cannot read the device's compute-unit count");
    a.params = params;
    a.points = points;
    a.out = out;
    a.N = N;
    a.tiles = (N + TILE - 1) / TILE;
    const int64_t blocks = std::min<int64_t>((int64_t)cus * kBlocksPerCu, (a.tiles + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(mlp_eval_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, as_stream(stream), a);
    return check_launch("mlp_eval");
}

LSDF_API int lsdf_query_min_distance_mlp(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                         const void* grid_buf, const float* mlp_params, const lsdf_mlp_domain* domains,
                                         float margin, const float* points, int64_t M, float* out_dist,
                                         int32_t* out_link, float* out_link_dist, uint32_t flags, void* workspace,
                                         size_t ws_bytes, void* stream) {
    clear_error();
    if (flags != 0) return fail(LSDF_E_UNSUPPORTED, "query_mlp: unsupported flags 0x%x", flags);
    if (C < 0 || M < 0) return fail(LSDF_E_SHAPE, "query_mlp: negative size");
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "query_mlp: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (!grids || !domains) return fail(LSDF_E_INVALID_ARG, "query_mlp: grids or domains is NULL");
    if (std::isnan(margin)) return fail(LSDF_E_INVALID_ARG, "query_mlp: margin is NaN");
    if (C == 0) return LSDF_OK;
    if (!link_T || !grid_buf || !mlp_params || !out_dist || !out_link || !workspace)
        return fail(LSDF_E_INVALID_ARG, "query_mlp: NULL device pointer");
    if (M > 0 && !points) return fail(LSDF_E_INVALID_ARG, "query_mlp: points is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "query_mlp: workspace is not 256-byte aligned");
    size_t need = 0;
    int rc = lsdf_query_workspace_size(C, L, M, flags, &need);
    if (rc != LSDF_OK) return rc;
    if (ws_bytes < need) return fail(LSDF_E_SHAPE, "query_mlp: workspace has %zu bytes, needs %zu", ws_bytes, need);
    QueryMlpArgs a{};
    bool cubic = true;
    const int dtype = grids[0].dtype;
    for (int i = 0; i < L; ++i) {
        if ((rc = prepare_link_grid(grids[i], i, &a.link[i])) != LSDF_OK) return rc;
        if ((rc = make_domain(domains[i], i, &a.dom[i])) != LSDF_OK) return rc;
        if (grids[i].dtype != dtype) return fail(LSDF_E_UNSUPPORTED, "query_mlp: grids of one query must share a dtype");
        cubic = cubic && a.link[i].cubic;
    }
    hipStream_t s = as_stream(stream);
    a.link_T = link_T;
    a.params = mlp_params;
    a.grid = grid_buf;
    a.points = points;
    a.keys = static_cast<uint32_t*>(workspace);
    a.M = M;
    a.C = C;
    a.L = L;
    a.margin = margin;
    a.tiles_per_c = (int32_t)((M + TILE - 1) / TILE);
    a.tiles_per_link = (int64_t)C * a.tiles_per_c;
    if (a.tiles_per_link > 0) {
        const int cus = device_cus();
        if (cus <= 0) return fail(LSDF_E_DEVICE, "query_mlp: cannot read the device's compute-unit count");
        // one workgroup per CU (each takes every link in turn), no more than
        // the chunks of one link need
        const int64_t chunks = (a.tiles_per_link + kTileChunk - 1) / kTileChunk;
        const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(cus, (chunks + kQueryWaves - 1) / kQueryWaves)));
        if ((rc = launch_zero_words(a.keys, (int64_t)C * L, s)) != LSDF_OK) return rc;
        bool bounded = false;
        for (int i = 0; i < L; ++i) bounded = bounded || a.dom[i].inv_bound != 0.0f;
        if (bounded) {
            // the upper bounds, after the keys in the workspace (which holds
            // the plain query's tables too, far more than C L words)
            float* ub = reinterpret_cast<float*>(static_cast<char*>(workspace) + ((size_t)C * L * 4 + 255) / 256 * 256);
            // then the tile and chunk spheres and the seed chunks
            const int64_t nt = (M + TILE - 1) / TILE;
            float4* tsph = reinterpret_cast<float4*>(reinterpret_cast<char*>(ub) + ((size_t)C * L * 4 + 255) / 256 * 256);
            float4* csph = tsph + (nt + 15) / 16 * 16;
            int32_t* seed = reinterpret_cast<int32_t*>(csph + (nt + kTileChunk - 1) / kTileChunk);
            const size_t used = static_cast<size_t>(reinterpret_cast<char*>(seed + 2 * (int64_t)C * L) -
                                                    static_cast<char*>(workspace));
            if (used > need) return fail(LSDF_E_SHAPE, "query_mlp: workspace layout exceeds %zu bytes", need);
            BoundArgs b{};
            for (int i = 0; i < L; ++i) b.dom[i] = a.dom[i];
            b.link_T = link_T;
            b.points = points;
            b.ubound = ub;
            b.seed = seed;
            b.M = M;
            b.C = C;
            b.L = L;
            b.margin = margin;
            hipLaunchKernelGGL(mlp_bound_kernel, dim3((unsigned)((C + kBoundConfigs - 1) / kBoundConfigs), L),
                               dim3(kBoundBlock), 0, s, b);
            if ((rc = check_launch("query_min_distance_mlp bounds")) != LSDF_OK) return rc;
            hipLaunchKernelGGL(mlp_sphere_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, points, M, tsph,
                               csph);
            if ((rc = check_launch("query_min_distance_mlp spheres")) != LSDF_OK) return rc;
            a.ubound = ub;
            a.tile_sph = tsph;
            a.chunk_sph = csph;
            a.seed = seed;
        }
        hipEvent_t ev0, ev1;
        take_kernel_events(&ev0, &ev1);
        if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return fail(LSDF_E_DEVICE, "query_mlp: event record failed");
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((query_mlp_kernel<true, LSDF_F32>), grid, dim3(kQueryBlock), 0, s, a); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((query_mlp_kernel<false, LSDF_F32>), grid, dim3(kQueryBlock), 0, s, a); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((query_mlp_kernel<true, LSDF_BF16>), grid, dim3(kQueryBlock), 0, s, a); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((query_mlp_kernel<false, LSDF_BF16>), grid, dim3(kQueryBlock), 0, s, a); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((query_mlp_kernel<true, LSDF_F16>), grid, dim3(kQueryBlock), 0, s, a); break;
            default: hipLaunchKernelGGL((query_mlp_kernel<false, LSDF_F16>), grid, dim3(kQueryBlock), 0, s, a); break;
        }
        if ((rc = check_launch("query_min_distance_mlp")) != LSDF_OK) return rc;
        if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return fail(LSDF_E_DEVICE, "query_mlp: event record failed");
    }
    return lsdf::launch_query_finalize(a.tiles_per_link > 0 ? a.keys : nullptr, out_dist, out_link, out_link_dist, C, L,
                                       s);
}

LSDF_API int lsdf_mlp_train_workspace_size(int32_t L, int32_t B, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(LSDF_E_INVALID_ARG, "mlp_train_workspace_size: bytes is NULL");
    int rc = check_train_sizes(L, B, 1);
    if (rc != LSDF_OK) return rc;
    *bytes = train_layout(L, B, nullptr, nullptr);
    return LSDF_OK;
}

LSDF_API int lsdf_mlp_loss_grad(const float* params, const lsdf_mlp_domain* domains, int32_t L, const float* samples,
                                const float* labels, int64_t N, const int32_t* batch_index, int32_t B, float* loss_out,
                                float* grad_out, void* workspace, size_t ws_bytes, void* stream) {
    clear_error();
    if (!grad_out) return fail(LSDF_E_INVALID_ARG, "mlp_loss_grad: grad_out is NULL");
    return train_common(params, nullptr, nullptr, 0, 0.f, 0.f, 0.f, 0.f, false, domains, L, samples, labels, N,
                        batch_index, B, loss_out, grad_out, workspace, ws_bytes, stream);
}

LSDF_API int lsdf_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t t, float lr, float beta1,
                                 float beta2, float eps, const lsdf_mlp_domain* domains, int32_t L,
                                 const float* samples, const float* labels, int64_t N, const int32_t* batch_index,
                                 int32_t B, float* loss_out, float* grad_out, void* workspace, size_t ws_bytes,
                                 void* stream) {
    clear_error();
    return train_common(params, adam_m, adam_v, t, lr, beta1, beta2, eps, true, domains, L, samples, labels, N,
                        batch_index, B, loss_out, grad_out, workspace, ws_bytes, stream);
}
