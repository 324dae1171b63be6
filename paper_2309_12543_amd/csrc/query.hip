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
//     of 8 consecutive points by a sphere (and every quad of 4 blocks by
//     another), and a wave skips a quad or block when no lane's box can hold
//     any of its points (the sphere centre is mapped with the lane's own map;
//     the test widens the box by the radius times the map's row norms plus a
//     bound on FP32 rounding, so the skip is exact);
//   * a block that survives is recorded in a list in the workgroup's LDS;
//     after a barrier the workgroup's waves share out the recorded blocks,
//     so that a wave that drew many does not hold up the kernel alone;
//   * a call may hold many trajectories, each a range of configurations
//     checked against its own range of points (a re-planned path against
//     its latest cloud); a plain query is the one-trajectory case.  The
//     ranges come from device arrays, and the plan that turns them into
//     work (chunk counts and their prefix sums) is built on the device by
//     the first kernel, so that no call reads anything back to the host and
//     a whole step can be captured once in a graph and replayed with new
//     ranges;
//   * the first kernel also writes, per (link, configuration), the lane's
//     map and culling thresholds into a field-major table (one coalesced
//     load per field per chunk) and zeroes the keys;
//   * the iteration space (trajectory, link, 64-configuration group, point)
//     is cut into chunks of a tunable number of 8-point blocks (a chunk takes
//     every n-th quad of its trajectory's cloud), dealt to the waves
//     round-robin, either over the whole grid or inside per-XCD slices
//     (blocks b = x mod 8 take a contiguous slice, which keeps an XCD on one
//     or two links' grids in its L2); the four waves of a workgroup take
//     chunks from four different parts of the order;
//   * per-pair minima merge across waves with one unsigned atomic max on a
//     complemented order-preserving key; a last small kernel turns the keys
//     into the outputs (the kernel boundary orders it after every atomic,
//     with no device fence).
#include <algorithm>
#include <atomic>
#include <mutex>

#include "fk_chain.hpp"
#include "grid_sample.hpp"

namespace {

using lsdf::GridT;
using lsdf::LinkGrid;
using lsdf::Cell;
using lsdf::inside;
using lsdf::interpolate;
using lsdf::locate;

#ifndef LSDF_QUERY_BLOCK
#define LSDF_QUERY_BLOCK 256         // threads per workgroup of the query kernel
#endif
constexpr int kBlock = LSDF_QUERY_BLOCK;
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
constexpr int kSphereBatch = 4;     // culling spheres tested together: the blocks of a quad
constexpr int kQuadPts = kBlockPts * kSphereBatch;   // points per quad
#ifndef LSDF_QUERY_QUAD_BATCH
#define LSDF_QUERY_QUAD_BATCH 8     // quad spheres of a chunk loaded and tested together
#endif
constexpr int kQuadBatch = LSDF_QUERY_QUAD_BATCH;
constexpr int kUnroll = LSDF_QUERY_UNROLL;
constexpr int kGather = LSDF_QUERY_GATHER;
static_assert(kUnroll % kGather == 0, "gather batch must divide the unroll");
static_assert(kUnroll == kBlockPts, "blocks of 8 points");

// Default tiling: as many workgroups per CU as can be resident at once (so
// that no wave of the persistent grid waits for another to finish; 8 if
// the runtime cannot say), chunks dealt over the whole grid, at most about
// one chunk per wave of the grid for the call's sizes (with offset arrays,
// the capacities C and M): the smallest power of two of blocks of 8 points
// between 4 and 128 that gives no more chunks than waves.
constexpr int kDefaultChunkPoints = 1024;
constexpr int kDefaultBlocksPerCu = 8;
constexpr int kDefaultSchedule = LSDF_SCHED_INTERLEAVED;

int default_chunk_blocks(int64_t C, int64_t L, int64_t M, int64_t waves) {
    const int64_t units = L * ((C + 63) / 64) * ((M + kBlockPts - 1) / kBlockPts);
    int64_t cb = 4;
    while (cb < 128 && cb * waves <= units) cb *= 2;
    return (int)cb;
}
constexpr int kMaxChunkPoints = 8192;
constexpr int kMaxBlocksPerCu = 16;

// Work plan of one trajectory, built on the device.  Entry K (one past the
// last trajectory) holds only chunk_start = the total chunk count.
struct TrajPlan {
    int64_t chunk_start;       // first chunk of this trajectory
    int64_t m_lo, m_hi;        // points [m_lo, m_hi) of the concatenated cloud
    int32_t c_lo, c_n;         // configurations [c_lo, c_lo + c_n)
    int32_t cgroups;           // ceil(c_n / 64)
    int32_t chunks_per_group;  // ceil(quads touched / chunk_quads)
    int32_t pad[2];
};
static_assert(sizeof(TrajPlan) == 48, "plan entry layout");

// A surviving block handed from the wave that found it to whichever wave of
// the workgroup is free once every wave has tested its own chunks.
struct Deferred {
    uint64_t mask;             // lanes (configurations c0 + lane) whose box may reach the block
    int64_t blk;               // block of 8 points in the concatenated cloud
    int64_t m_lo, m_hi;        // the trajectory's points
    int32_t c0;                // configuration of lane 0
    int32_t link;
};
#ifndef LSDF_QUERY_DEFER
#define LSDF_QUERY_DEFER 128       // surviving blocks a workgroup may pass between its waves
#endif
constexpr int kDeferCap = LSDF_QUERY_DEFER;

struct QueryArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    const float* maps;       // [L][kMapFields][C]
    uint32_t* keys;          // [C][L] complemented ordered keys, 0 = empty
    int32_t C;
    int32_t K;               // trajectories
    int32_t L;
    int32_t chunk_quads;     // quads (4 blocks of 8 points) per chunk
    int32_t blocks_per_xcd;
    int32_t schedule;        // LSDF_SCHED_*
};

// Per (link, configuration): the world-to-grid map and the culling
// thresholds, stored field-major ([L][kMapFields][C]) so that a wave's 64
// consecutive configurations read each field with one coalesced load.
constexpr int kMapFields = 18;   // M (9, row-major), w (3), ||M_a|| (3), k_a (3)

struct PrepArgs {
    LinkGrid link[LSDF_MAX_LINKS];
    lsdf::DhTable dh;        // used when q != NULL
    const float* q;          // joint angles [C][dof], or NULL: poses come from link_T
    float* link_T_out;       // poses computed from q are stored here when not NULL
    const float* link_T;
    const float* points;
    float4* spheres;         // [4 ceil(M / 32)] one per 8-point block (the last few unused)
    float4* qspheres;        // [ceil(M / 32)] one per quad of 4 blocks
    TrajPlan* plan;          // [K + 1]
    float* maps;             // [L][kMapFields][C]
    uint32_t* keys;          // [C][L], zeroed here
    const int32_t* c_off;    // device [K + 1] or NULL (one trajectory of all C)
    const int64_t* m_off;    // device [K + 1] or NULL (one trajectory of all M)
    int64_t M;
    int64_t sphere_base;     // first thread of the sphere job: C L rounded up to the wave size
    int32_t C;
    int32_t K;
    int32_t L;
    int32_t chunk_quads;
};

struct FinalizeArgs {
    const uint32_t* keys;    // [C][L], or NULL
    float* out_dist;
    int32_t* out_link;
    float* out_link_dist;
    int32_t C;
    int32_t L;
};

// One 8-point block against every lane's box: the point tests, then the
// corner gathers and interpolation of the points inside some lane's box.
template <bool CUBIC, int DT>
__device__ __forceinline__ void block_min(const float* __restrict__ points, int64_t j, int64_t m_lo, int64_t m_hi,
                                          const LinkGrid& lg, const typename GridT<DT>::T* __restrict__ G,
                                          int nx, int nxy, float m00, float m01, float m02, float w0, float m10,
                                          float m11, float m12, float w1, float m20, float m21, float m22, float w2,
                                          float& best) {
    using E = GridT<DT>;
    if (j >= m_lo && j + kUnroll <= m_hi) {
        // first the box tests of the 8 points (lane masks), then the gathers
        // of the points some lane holds, a batch at a time; the mapped
        // coordinates are recomputed for the gathers rather than kept, which
        // keeps register use (and so the number of resident waves) in check
        bool in[kUnroll];
        bool any = false;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const float x = points[3 * j + 3 * u + 0];
            const float y = points[3 * j + 3 * u + 1];
            const float z = points[3 * j + 3 * u + 2];
            const float v0 = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
            const float v1 = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
            const float v2 = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
            in[u] = inside<CUBIC>(lg, v0, v1, v2);
            any |= in[u];
        }
        if (!__ballot(any)) return;
#pragma unroll
        for (int b = 0; b < kUnroll; b += kGather) {
            // issue every corner load of the batch, then interpolate
            float c00[kGather], c10[kGather], c01[kGather], c11[kGather];
            float d00[kGather], d10[kGather], d01[kGather], d11[kGather];
            Cell cell[kGather];
#pragma unroll
            for (int u = 0; u < kGather; ++u) {
                const float x = points[3 * j + 3 * (b + u) + 0];
                const float y = points[3 * j + 3 * (b + u) + 1];
                const float z = points[3 * j + 3 * (b + u) + 2];
                const float v0 = fmaf(m00, x, fmaf(m01, y, fmaf(m02, z, w0)));
                const float v1 = fmaf(m10, x, fmaf(m11, y, fmaf(m12, z, w1)));
                const float v2 = fmaf(m20, x, fmaf(m21, y, fmaf(m22, z, w2)));
                cell[u] = locate(lg, v0, v1, v2);
                // lanes outside the box read the first cell (discarded)
                const typename E::T* cp = G + (in[b + u] ? cell[u].idx : 0);
                c00[u] = E::get(cp, 0);        d00[u] = E::get(cp, 1);
                c10[u] = E::get(cp, nx);       d10[u] = E::get(cp, nx + 1);
                c01[u] = E::get(cp, nxy);      d01[u] = E::get(cp, nxy + 1);
                c11[u] = E::get(cp, nxy + nx); d11[u] = E::get(cp, nxy + nx + 1);
            }
#pragma unroll
            for (int u = 0; u < kGather; ++u) {
                const float val = interpolate(c00[u], d00[u], c10[u], d10[u], c01[u], d01[u], c11[u], d11[u], cell[u]);
                if (in[b + u]) best = fminf(best, val);
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

// A 64-bit value that every lane holds alike, moved to scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The 12 map entries of (link i, configuration c) from the table the first
// kernel built; a lane with valid = false gets a map that sends every point
// far outside the box.
struct Map {
    float m00, m01, m02, w0, m10, m11, m12, w1, m20, m21, m22, w2;
};
__device__ __forceinline__ void load_map(const QueryArgs& p, int i, int c, bool valid, Map& m) {
    m = Map{0.f, 0.f, 0.f, kFar, 0.f, 0.f, 0.f, kFar, 0.f, 0.f, 0.f, kFar};
    if (valid) {
        const float* mp = p.maps + (int64_t)i * kMapFields * p.C + c;
        const int64_t C = p.C;
        m.m00 = mp[0 * C]; m.m01 = mp[1 * C]; m.m02 = mp[2 * C];
        m.m10 = mp[3 * C]; m.m11 = mp[4 * C]; m.m12 = mp[5 * C];
        m.m20 = mp[6 * C]; m.m21 = mp[7 * C]; m.m22 = mp[8 * C];
        m.w0 = mp[9 * C]; m.w1 = mp[10 * C]; m.w2 = mp[11 * C];
    }
}

// A deferred block as a wave holds it: the record's fields in scalar
// registers, and this lane's bit of the mask.
struct DeferredView {
    int64_t blk, m_lo, m_hi;
    int c0, link;
    bool mine;
};
__device__ __forceinline__ DeferredView read_deferred(const Deferred& d, int lane) {
    DeferredView v;
    const uint64_t mask = (uint64_t)uniform64((int64_t)d.mask);
    v.blk = uniform64(d.blk);
    v.m_lo = uniform64(d.m_lo);
    v.m_hi = uniform64(d.m_hi);
    v.c0 = __builtin_amdgcn_readfirstlane(d.c0);
    v.link = __builtin_amdgcn_readfirstlane(d.link);
    v.mine = (mask >> lane) & 1u;
    return v;
}

// The first pass of a wave: the chunks q_first, q_first + q_step, ... below
// q_end.  A chunk's quads are tested against every lane's box, then their
// blocks; a block some lane's box may reach is appended to the workgroup's
// list s_def while it has room (its points are tested after the workgroup's
// barrier, by whichever wave is free) and tested here once the list is full.
template <bool CUBIC, int DT>
__device__ __forceinline__ void test_chunks(const QueryArgs& p, const float* __restrict__ points,
                                            const typename GridT<DT>::T* __restrict__ grid,
                                            const float4* __restrict__ spheres,
                                            const float4* __restrict__ qspheres,
                                            const TrajPlan* __restrict__ plan, int64_t q_first, int64_t q_end,
                                            int64_t q_step, int lane, Deferred* s_def, int* ndef) {
    using E = GridT<DT>;
    // trajectory of the first chunk: the last entry whose start is <= q
    int k = 0;
    {
        int hi = p.K - 1;
        while (k < hi) {
            const int mid = (k + hi + 1) >> 1;
            if (plan[mid].chunk_start <= q_first) k = mid; else hi = mid - 1;
        }
    }
    // the current trajectory's plan, kept in registers until q passes its end
    int64_t t_start = plan[k].chunk_start, t_next = plan[k + 1].chunk_start;
    int64_t m_lo = plan[k].m_lo, m_hi = plan[k].m_hi;
    int c_lo = plan[k].c_lo, c_n = plan[k].c_n, cgroups = plan[k].cgroups, cpg = plan[k].chunks_per_group;

    for (int64_t q = q_first; q < q_end; q += q_step) {
        if (q >= t_next) {   // stops at k + 1 = K at the latest: q < total
            do {
                ++k;
                t_next = plan[k + 1].chunk_start;
            } while (q >= t_next);
            t_start = plan[k].chunk_start;
            m_lo = plan[k].m_lo;
            m_hi = plan[k].m_hi;
            c_lo = plan[k].c_lo;
            c_n = plan[k].c_n;
            cgroups = plan[k].cgroups;
            cpg = plan[k].chunks_per_group;
        }
        const int64_t local = q - t_start;
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
        // the trajectory's points lie in quads of 4 blocks of 8 (aligned in the
        // concatenated cloud); chunk mc takes every cpg-th quad from the
        // trajectory's quad mc, so that points near a link, which lie together
        // in the cloud, spread over the chunks rather than piling onto a few
        // waves
        const int64_t blk0 = m_lo >> 3, blk1 = (m_hi + kBlockPts - 1) >> 3;   // the trajectory's blocks
        const int64_t quad0 = m_lo / kQuadPts;
        const int64_t nquad = (m_hi + kQuadPts - 1) / kQuadPts - quad0;

        // this lane's map v = M [x; y; z] + w (centred grid coordinates) and
        // its culling thresholds, from the table the first kernel built;
        // lanes past the trajectory's configurations are never near or inside
        float m00 = 0.f, m01 = 0.f, m02 = 0.f, w0 = kFar;
        float m10 = 0.f, m11 = 0.f, m12 = 0.f, w1 = kFar;
        float m20 = 0.f, m21 = 0.f, m22 = 0.f, w2 = kFar;
        float nr0 = 0.f, nr1 = 0.f, nr2 = 0.f, k0 = 0.f, k1 = 0.f, k2 = 0.f;
        if (cl < c_n) {
            const float* mp = p.maps + (int64_t)i * kMapFields * p.C + c;
            const int64_t C = p.C;
            m00 = mp[0 * C]; m01 = mp[1 * C]; m02 = mp[2 * C];
            m10 = mp[3 * C]; m11 = mp[4 * C]; m12 = mp[5 * C];
            m20 = mp[6 * C]; m21 = mp[7 * C]; m22 = mp[8 * C];
            w0 = mp[9 * C]; w1 = mp[10 * C]; w2 = mp[11 * C];
            nr0 = mp[12 * C]; nr1 = mp[13 * C]; nr2 = mp[14 * C];
            k0 = mp[15 * C]; k1 = mp[16 * C]; k2 = mp[17 * C];
        }
        const int nx = lg.n[0];
        const int nxy = lg.n[0] * lg.n[1];

        float best = INFINITY;
        // kQuadBatch quads of the chunk at a time: their spheres are loaded
        // together and tested (one round trip for the batch); only the
        // quads some lane's box may reach go on to their blocks' spheres
        for (int64_t qb = mc; qb < nquad; qb += (int64_t)kQuadBatch * cpg) {
            float4 qs[kQuadBatch];
#pragma unroll
            for (int k = 0; k < kQuadBatch; ++k)   // past the trajectory's quads: its last one, not tested
                qs[k] = qspheres[quad0 + min(qb + (int64_t)k * cpg, nquad - 1)];
            uint32_t qnear = 0;
#pragma unroll
            for (int k = 0; k < kQuadBatch; ++k) {
                const float s0 = fmaf(m00, qs[k].x, fmaf(m01, qs[k].y, fmaf(m02, qs[k].z, w0)));
                const float s1 = fmaf(m10, qs[k].x, fmaf(m11, qs[k].y, fmaf(m12, qs[k].z, w1)));
                const float s2 = fmaf(m20, qs[k].x, fmaf(m21, qs[k].y, fmaf(m22, qs[k].z, w2)));
                const bool near = (fabsf(s0) <= fmaf(nr0, qs[k].w, k0)) & (fabsf(s1) <= fmaf(nr1, qs[k].w, k1)) &
                                  (fabsf(s2) <= fmaf(nr2, qs[k].w, k2));
                if (__ballot(near) && qb + (int64_t)k * cpg < nquad) qnear |= 1u << k;
            }
            while (qnear) {   // wave-uniform
                const int kq = __builtin_ctz(qnear);
                qnear &= qnear - 1;
                // a sphere bounds all points of its quad or block, so also the
                // trajectory's share of one it shares with its neighbour
                const int64_t qg = quad0 + qb + (int64_t)kq * cpg;
                float4 sph[kSphereBatch];
#pragma unroll
                for (int u = 0; u < kSphereBatch; ++u) sph[u] = spheres[kSphereBatch * qg + u];
                const int64_t jb = kQuadPts * qg;
                uint32_t near_mask = 0;
                uint64_t lanes[kSphereBatch];
#pragma unroll
                for (int u = 0; u < kSphereBatch; ++u) {
                    const float s0 = fmaf(m00, sph[u].x, fmaf(m01, sph[u].y, fmaf(m02, sph[u].z, w0)));
                    const float s1 = fmaf(m10, sph[u].x, fmaf(m11, sph[u].y, fmaf(m12, sph[u].z, w1)));
                    const float s2 = fmaf(m20, sph[u].x, fmaf(m21, sph[u].y, fmaf(m22, sph[u].z, w2)));
                    const bool near = (fabsf(s0) <= fmaf(nr0, sph[u].w, k0)) &
                                      (fabsf(s1) <= fmaf(nr1, sph[u].w, k1)) & (fabsf(s2) <= fmaf(nr2, sph[u].w, k2));
                    const int64_t blk = kSphereBatch * qg + u;
                    lanes[u] = __ballot(near);
                    if (lanes[u] && blk >= blk0 && blk < blk1) near_mask |= 1u << u;
                }
                // the blocks some lane's box may reach: handed to the workgroup
                // while it has room, else tested here
                int slot = kDeferCap;
                if (near_mask && lane == 0 && *ndef < kDeferCap) slot = atomicAdd(ndef, __builtin_popcount(near_mask));
                slot = __builtin_amdgcn_readfirstlane(slot);
                while (near_mask) {   // wave-uniform
                    const int u = __builtin_ctz(near_mask);
                    near_mask &= near_mask - 1;
                    if (slot < kDeferCap) {
                        if (lane == 0)
                            s_def[slot] = Deferred{lanes[u], kSphereBatch * qg + u, m_lo, m_hi, c_lo + cb * 64, i};
                        ++slot;
                    } else {
                        block_min<CUBIC, DT>(points, jb + u * kBlockPts, m_lo, m_hi, lg, G, nx, nxy, m00, m01, m02,
                                             w0, m10, m11, m12, w1, m20, m21, m22, w2, best);
                    }
                }
            }
        }
        if (cl < c_n && best < INFINITY) atomicMax(&p.keys[(int64_t)c * p.L + i], ~lsdf::ordered_bits(best));
    }
}


// Slot of workgroup b (of n) for its wave w: waves 2 and 3 shift by half
// the grid and odd waves count from the other end, so that a workgroup's
// four chunks come from four different parts of the chunk order (early and
// late links, early and late configuration groups).  A bijection of [0, n)
// for each w.
__device__ __forceinline__ int mix_slot(int b, int n, int w) {
    int s = (w & 2) ? (b + n / 2) % n : b;
    return (w & 1) ? n - 1 - s : s;
}

template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void query_kernel(QueryArgs p, const float* __restrict__ points,
                                                       const typename GridT<DT>::T* __restrict__ grid,
                                                       const float4* __restrict__ spheres,
                                                       const float4* __restrict__ qspheres,
                                                       const TrajPlan* __restrict__ plan) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = plan[p.K].chunk_start;
    int64_t q_first, q_end, q_step;
    if (p.schedule == LSDF_SCHED_XCD_SLICES) {
        // each XCD (blocks b = x mod 8) takes a contiguous slice of chunks
        // and deals it round-robin to its waves
        const int xcd = blockIdx.x % kXcds;
        const int slot = blockIdx.x / kXcds;
        q_first = total * xcd / kXcds + (int64_t)wave * p.blocks_per_xcd + mix_slot(slot, p.blocks_per_xcd, wave);
        q_end = total * (xcd + 1) / kXcds;
        q_step = (int64_t)p.blocks_per_xcd * kWavesPerBlock;
    } else {
        // every wave of the grid takes every W-th chunk
        q_first = (int64_t)wave * gridDim.x + mix_slot((int)blockIdx.x, (int)gridDim.x, wave);
        q_end = total;
        q_step = (int64_t)gridDim.x * kWavesPerBlock;
    }
    // (the waves of one workgroup start a grid's width apart, on different
    // links or configuration groups, so that their loads differ and the
    // deferred blocks even them out; mix_slot shuffles which workgroup each
    // wave index lands in)
    __shared__ Deferred s_def[kDeferCap];
    __shared__ int s_ndef;
    if (threadIdx.x == 0) s_ndef = 0;
    __syncthreads();
    if (q_first < q_end)
        test_chunks<CUBIC, DT>(p, points, grid, spheres, qspheres, plan, q_first, q_end, q_step, lane, s_def, &s_ndef);
    __syncthreads();

    // the deferred blocks, dealt round-robin to the workgroup's waves
    const int nd = min(s_ndef, kDeferCap);
    for (int it = wave; it < nd; it += kWavesPerBlock) {
        const DeferredView d = read_deferred(s_def[it], lane);
        const int c = d.c0 + lane;
        const LinkGrid& lg = p.link[d.link];
        Map mp;
        load_map(p, d.link, c, d.mine, mp);
        float best = INFINITY;
        block_min<CUBIC, DT>(points, d.blk * kBlockPts, d.m_lo, d.m_hi, lg, grid + lg.offset, lg.n[0],
                             lg.n[0] * lg.n[1], mp.m00, mp.m01, mp.m02, mp.w0, mp.m10, mp.m11, mp.m12, mp.w1, mp.m20,
                             mp.m21, mp.m22, mp.w2, best);
        if (d.mine && best < INFINITY) atomicMax(&p.keys[(int64_t)c * p.L + d.link], ~lsdf::ordered_bits(best));
    }
}

// Culling spheres of block b (8 points from 8 b) and, for b = 4 q, of quad
// q (blocks 4 q to 4 q + 3), from the thread of block b; the four threads of
// a quad are adjacent lanes and combine their boxes and radii by shuffles.
// A sphere's centre is the centre of its points' box and its radius the
// largest distance to it, widened by a relative 1e-5, by 1e-4 of the sum of
// the coordinates' magnitudes (which bounds FP32 rounding of the mapped
// coordinates) and by 1e-6 m.  Past the end of the cloud the last point
// repeats, which changes neither a box nor a radius.  Every lane of a quad
// must call this together.
__device__ __forceinline__ float4 widen(float cx, float cy, float cz, float r2) {
    const float r = sqrtf(r2);
    const float e = fabsf(cx) + fabsf(cy) + fabsf(cz) + 3.0f * r;
    return make_float4(cx, cy, cz, fmaf(r, 1.00001f, fmaf(1e-4f, e, 1e-6f)));
}

__device__ __forceinline__ void block_and_quad_spheres(const float* __restrict__ points, int64_t b, int64_t M,
                                                       float4* block_out, float4* quad_out) {
    float x[kBlockPts], y[kBlockPts], z[kBlockPts];
#pragma unroll
    for (int k = 0; k < kBlockPts; ++k) {
        const int64_t j = min(b * kBlockPts + k, M - 1);
        x[k] = points[3 * j + 0];
        y[k] = points[3 * j + 1];
        z[k] = points[3 * j + 2];
    }
    float lo0 = x[0], lo1 = y[0], lo2 = z[0], hi0 = x[0], hi1 = y[0], hi2 = z[0];
#pragma unroll
    for (int k = 1; k < kBlockPts; ++k) {
        lo0 = fminf(lo0, x[k]); hi0 = fmaxf(hi0, x[k]);
        lo1 = fminf(lo1, y[k]); hi1 = fmaxf(hi1, y[k]);
        lo2 = fminf(lo2, z[k]); hi2 = fmaxf(hi2, z[k]);
    }
    auto radius2 = [&](float cx, float cy, float cz) {
        float r2 = 0.0f;
#pragma unroll
        for (int k = 0; k < kBlockPts; ++k) {
            const float dx = x[k] - cx, dy = y[k] - cy, dz = z[k] - cz;
            r2 = fmaxf(r2, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        }
        return r2;
    };
    {
        const float cx = 0.5f * (lo0 + hi0), cy = 0.5f * (lo1 + hi1), cz = 0.5f * (lo2 + hi2);
        const float4 sb = widen(cx, cy, cz, radius2(cx, cy, cz));
        if (b * kBlockPts < M) *block_out = sb;
    }
#pragma unroll
    for (int o = 1; o < kSphereBatch; o <<= 1) {
        lo0 = fminf(lo0, __shfl_xor(lo0, o, 64)); hi0 = fmaxf(hi0, __shfl_xor(hi0, o, 64));
        lo1 = fminf(lo1, __shfl_xor(lo1, o, 64)); hi1 = fmaxf(hi1, __shfl_xor(hi1, o, 64));
        lo2 = fminf(lo2, __shfl_xor(lo2, o, 64)); hi2 = fmaxf(hi2, __shfl_xor(hi2, o, 64));
    }
    const float cx = 0.5f * (lo0 + hi0), cy = 0.5f * (lo1 + hi1), cz = 0.5f * (lo2 + hi2);
    float r2 = radius2(cx, cy, cz);
#pragma unroll
    for (int o = 1; o < kSphereBatch; o <<= 1) r2 = fmaxf(r2, __shfl_xor(r2, o, 64));
    if ((b & (kSphereBatch - 1)) == 0) *quad_out = widen(cx, cy, cz, r2);
}

// The plan of the batched queries (in one workgroup of 256 threads).
__device__ __forceinline__ void build_plan(const PrepArgs& a) {
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
            // the quads (aligned in the concatenated cloud) that hold a point of [m0, m1)
            const int64_t nq = m1 > m0 ? (m1 + kQuadPts - 1) / kQuadPts - m0 / kQuadPts : 0;
            e.chunks_per_group = (int32_t)((nq + a.chunk_quads - 1) / a.chunk_quads);
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

// First kernel of a query, three independent jobs on separate threads so
// that their latencies overlap.  Thread t < C L zeroes key t and writes the
// map table entry of (link t / C, configuration t mod C), from the given pose
// or, in the fused form, from the pose it computes from the joint angles.
// Thread sphere_base + s bounds block s of 8 consecutive points of the
// concatenated cloud by a sphere, and with its quad's three other lanes quad
// s / 4 (blocks s - s mod 4 to s - s mod 4 + 3) by another (sphere_base is
// a multiple of the wave size, so every wave holds whole quads).  The last
// workgroup builds the plan: each trajectory's ranges clamped into [0, C)
// and [0, M) (so a bad offset table gives wrong ranges, never an access out
// of bounds), its chunk count and the exclusive prefix sum of the counts.
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == gridDim.x - 1) {
        build_plan(a);
        return;
    }
    if (b >= a.sphere_base) {
        const int64_t sb = b - a.sphere_base;
        // uniform over the four lanes of a quad
        if (sb / kSphereBatch * kQuadPts < a.M)
            block_and_quad_spheres(a.points, sb, a.M, &a.spheres[sb], &a.qspheres[sb / kSphereBatch]);
        return;
    }
    if (b < (int64_t)a.C * a.L) {
        a.keys[b] = 0u;
        // map of link i at configuration c: row a of R^T scaled by invh_a,
        // offset -invh_a (R^T t)_a + cen_a (the inverse pose of Eq. 4 with
        // the grid scaling folded in); then the culling thresholds: the
        // row norms (x (1 + 1e-6)) and half_a plus a bound on FP32 rounding
        const int i = (int)(b / a.C);
        const int64_t c = b - (int64_t)i * a.C;
        const LinkGrid& lg = a.link[i];
        float T[12];
        if (a.q) {
            // the pose from the joint angles, with the kinematics kernel's
            // arithmetic (same bits as lsdf_fk_batch)
            lsdf::chain_pose(a.dh, a.q + c * a.dh.dof, i, T);
            if (a.link_T_out) {
                float* o = a.link_T_out + (c * a.L + i) * 12;
#pragma unroll
                for (int k = 0; k < 12; ++k) o[k] = T[k];
            }
        } else {
            const float* src = a.link_T + (c * a.L + i) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) T[k] = src[k];
        }
        const float r00 = T[0], r01 = T[1], r02 = T[2], t0 = T[3];
        const float r10 = T[4], r11 = T[5], r12 = T[6], t1 = T[7];
        const float r20 = T[8], r21 = T[9], r22 = T[10], t2 = T[11];
        float f[kMapFields];
        f[0] = lg.invh[0] * r00; f[1] = lg.invh[0] * r10; f[2] = lg.invh[0] * r20;
        f[3] = lg.invh[1] * r01; f[4] = lg.invh[1] * r11; f[5] = lg.invh[1] * r21;
        f[6] = lg.invh[2] * r02; f[7] = lg.invh[2] * r12; f[8] = lg.invh[2] * r22;
        f[9] = fmaf(-lg.invh[0], fmaf(r00, t0, fmaf(r10, t1, r20 * t2)), lg.cen[0]);
        f[10] = fmaf(-lg.invh[1], fmaf(r01, t0, fmaf(r11, t1, r21 * t2)), lg.cen[1]);
        f[11] = fmaf(-lg.invh[2], fmaf(r02, t0, fmaf(r12, t1, r22 * t2)), lg.cen[2]);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const float* m = f + 3 * ax;
            f[12 + ax] = sqrtf(fmaf(m[0], m[0], fmaf(m[1], m[1], m[2] * m[2]))) * 1.000001f;
            f[15 + ax] = lg.half[ax] + fmaf(1e-4f, fabsf(f[9 + ax]), 1e-3f);
        }
        float* out = a.maps + (int64_t)i * kMapFields * a.C + c;
#pragma unroll
        for (int k = 0; k < kMapFields; ++k) out[(int64_t)k * a.C] = f[k];
    }
}

// Keys -> outputs, one lane per configuration (keys == NULL: no pair was
// evaluated, every configuration gets +inf and -1).
__global__ __launch_bounds__(kBlock) void finalize_kernel(FinalizeArgs p) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= p.C) return;
    uint32_t k[LSDF_MAX_LINKS];
#pragma unroll
    for (int i = 0; i < LSDF_MAX_LINKS; ++i)
        if (i < p.L) k[i] = p.keys ? p.keys[(int64_t)c * p.L + i] : 0u;
    uint32_t bestk = 0;
    int arg = -1;
#pragma unroll
    for (int i = 0; i < LSDF_MAX_LINKS; ++i) {
        if (i < p.L) {
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

// Zeroes n words (the learned query's keys before its main kernel).
__global__ __launch_bounds__(kBlock) void zero_kernel(uint32_t* w, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n) w[t] = 0u;
}

}  // namespace

int lsdf::launch_query_finalize(const uint32_t* keys, float* out_dist, int32_t* out_link, float* out_link_dist, int32_t C,
                                int32_t L, hipStream_t s) {
    FinalizeArgs f{keys, out_dist, out_link, out_link_dist, C, L};
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((C + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, f);
    return check_launch("query finalize");
}

int lsdf::launch_zero_words(uint32_t* w, int64_t n, hipStream_t s) {
    if (n <= 0) return LSDF_OK;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, w, n);
    return check_launch("zero words");
}

namespace {

size_t keys_bytes(int64_t C, int64_t L) { return ((size_t)(C * L) * 4 + 255) / 256 * 256; }
// Block spheres for whole quads (the query loads a quad's four together and
// ignores those past the cloud's last block), then the quad spheres.
int64_t quad_count(int64_t M) { return (M + kQuadPts - 1) / kQuadPts; }
size_t sphere_bytes(int64_t M) { return ((size_t)quad_count(M) * (kSphereBatch + 1) * 16 + 255) / 256 * 256; }
size_t plan_bytes(int64_t K) { return ((size_t)(K + 1) * sizeof(TrajPlan) + 255) / 256 * 256; }
size_t map_bytes(int64_t C, int64_t L) { return ((size_t)(C * L) * kMapFields * 4 + 255) / 256 * 256; }

// Workspace: keys | block and quad spheres | plan | maps, each 256-byte aligned.
size_t workspace_bytes(int64_t K, int64_t C, int64_t L, int64_t M) {
    return keys_bytes(C, L) + sphere_bytes(M) + plan_bytes(K) + map_bytes(C, L);
}

// Workgroups of the query kernel variant that fit on one CU at once.
template <bool CUBIC, int DT>
int resident_blocks_of() {
    static std::atomic<int> cached{0};
    int v = cached.load(std::memory_order_relaxed);
    if (v > 0) return v;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, query_kernel<CUBIC, DT>, kBlock, 0) != hipSuccess || n < 1)
        n = kDefaultBlocksPerCu;
    n = std::min(n, kMaxBlocksPerCu);
    cached.store(n, std::memory_order_relaxed);
    return n;
}

int resident_blocks(int dtype, bool cubic) {
    switch (dtype * 2 + (cubic ? 1 : 0)) {
        case LSDF_F32 * 2 + 1: return resident_blocks_of<true, LSDF_F32>();
        case LSDF_F32 * 2: return resident_blocks_of<false, LSDF_F32>();
        case LSDF_BF16 * 2 + 1: return resident_blocks_of<true, LSDF_BF16>();
        case LSDF_BF16 * 2: return resident_blocks_of<false, LSDF_BF16>();
        case LSDF_F16 * 2 + 1: return resident_blocks_of<true, LSDF_F16>();
        default: return resident_blocks_of<false, LSDF_F16>();
    }
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

int check_tuning(const char* who, const lsdf_query_tuning* t, int* chunk_blocks, int* blocks_per_cu,
                 int* schedule) {
    using lsdf::fail;
    *chunk_blocks = kDefaultChunkPoints / kBlockPts;
    *blocks_per_cu = kDefaultBlocksPerCu;
    *schedule = kDefaultSchedule;
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
    if (t->schedule != LSDF_SCHED_DEFAULT) {
        if (t->schedule != LSDF_SCHED_XCD_SLICES && t->schedule != LSDF_SCHED_INTERLEAVED)
            return fail(LSDF_E_INVALID_ARG, "%s: unknown schedule %d", who, (int)t->schedule);
        *schedule = t->schedule;
    }
    if (t->reserved != 0) return fail(LSDF_E_INVALID_ARG, "%s: tuning.reserved must be 0", who);
    return LSDF_OK;
}

// Shared body of the plain (K = 1, no offset arrays) and batched queries.
// With dh != NULL the poses are computed from the joint angles q in the
// first kernel (and stored in link_T when it is not NULL).
int run_query(const char* who, int32_t K, const int32_t* c_off, const int64_t* m_off, const float* link_T, int32_t C,
              int32_t L, const lsdf_grid* grids, const void* grid_buf, const float* points, int64_t M, float* out_dist,
              int32_t* out_link, float* out_link_dist, const lsdf_query_tuning* tuning, uint32_t flags,
              void* workspace, size_t ws_bytes, void* stream, const lsdf::DhTable* dh = nullptr,
              const float* q = nullptr) {
    using namespace lsdf;
    if (flags != 0) return fail(LSDF_E_UNSUPPORTED, "%s: unsupported flags 0x%x", who, flags);
    if (C < 0 || M < 0 || M > LSDF_MAX_POINTS)
        return fail(LSDF_E_SHAPE, "%s: size out of range (C = %d, M = %lld)", who, (int)C, (long long)M);
    if (L < 1 || L > LSDF_MAX_LINKS) return fail(LSDF_E_SHAPE, "%s: L = %d out of [1, %d]", who, (int)L, LSDF_MAX_LINKS);
    if (K < 1 || K > LSDF_MAX_TRAJECTORIES)
        return fail(LSDF_E_SHAPE, "%s: K = %d out of [1, %d]", who, (int)K, LSDF_MAX_TRAJECTORIES);
    if (!grids) return fail(LSDF_E_INVALID_ARG, "%s: grids is NULL", who);
    int chunk_blocks = 0, blocks_per_cu = 0, schedule = 0;
    int rc = check_tuning(who, tuning, &chunk_blocks, &blocks_per_cu, &schedule);
    if (rc != LSDF_OK) return rc;
    if (C == 0) return LSDF_OK;
    if ((!dh && !link_T) || (dh && !q) || !grid_buf || !out_dist || !out_link || !workspace)
        return fail(LSDF_E_INVALID_ARG, "%s: NULL device pointer", who);
    if (dh && L != dh->dof + 1)
        return fail(LSDF_E_SHAPE, "%s: %d grids for a %d-joint arm (needs dof + 1)", who, (int)L, (int)dh->dof);
    if (M > 0 && !points) return fail(LSDF_E_INVALID_ARG, "%s: points is NULL", who);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(LSDF_E_INVALID_ARG, "%s: workspace is not 256-byte aligned", who);
    const size_t need = workspace_bytes(K, C, L, M);
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
    const int cus = device_cus();
    if (cus <= 0) return fail(LSDF_E_DEVICE, "%s: cannot read the device's compute-unit count", who);
    if (!(tuning && tuning->blocks_per_cu != 0)) blocks_per_cu = resident_blocks(dtype, cubic);
    if (!(tuning && tuning->chunk_points != 0))   // from the capacities C and M when offsets are given
        chunk_blocks = default_chunk_blocks(C, L, M, (int64_t)cus * blocks_per_cu * kWavesPerBlock);
    hipStream_t s = as_stream(stream);
    char* ws = static_cast<char*>(workspace);
    float4* spheres = reinterpret_cast<float4*>(ws + keys_bytes(C, L));
    float4* qspheres = spheres + kSphereBatch * quad_count(M);
    TrajPlan* plan = reinterpret_cast<TrajPlan*>(ws + keys_bytes(C, L) + sphere_bytes(M));
    float* maps = reinterpret_cast<float*>(ws + keys_bytes(C, L) + sphere_bytes(M) + plan_bytes(K));
    p.maps = maps;
    p.keys = reinterpret_cast<uint32_t*>(ws);
    p.C = C;
    p.K = K;
    p.L = L;
    p.chunk_quads = (chunk_blocks + kSphereBatch - 1) / kSphereBatch;
    p.schedule = schedule;
    // the first kernel runs when there are points to test, or when poses
    // computed from joint angles are asked for
    if (M > 0 || (dh && link_T)) {
        PrepArgs a{};
        for (int i = 0; i < L; ++i) a.link[i] = p.link[i];
        if (dh) {
            a.dh = *dh;
            a.q = q;
            a.link_T_out = const_cast<float*>(link_T);   // an output in the fused form
        }
        a.link_T = link_T;
        a.points = points;
        a.spheres = spheres;
        a.qspheres = qspheres;
        a.plan = plan;
        a.maps = maps;
        a.keys = p.keys;
        a.c_off = c_off;
        a.m_off = m_off;
        a.M = M;
        a.C = C;
        a.K = K;
        a.L = L;
        a.chunk_quads = p.chunk_quads;
        // map threads, then (from a wave boundary) one thread per block of
        // every quad, then the plan's workgroup
        a.sphere_base = ((int64_t)C * L + 63) / 64 * 64;
        const int64_t threads = a.sphere_base + kSphereBatch * quad_count(M);
        hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((threads + 255) / 256 + 1)), dim3(256), 0, s, a);
        rc = check_launch(who);
        if (rc != LSDF_OK) return rc;
    }
    if (M > 0) {
        // persistent grid: blocks_per_cu workgroups per CU, a multiple of
        // the XCD count; when the chunk count is known here (one trajectory
        // given by C and M), no more waves than chunks
        int64_t blocks = (int64_t)cus * blocks_per_cu;
        if (!c_off) {
            const int64_t nq = quad_count(M);
            const int64_t chunks = (int64_t)L * ((C + 63) / 64) * ((nq + p.chunk_quads - 1) / p.chunk_quads);
            blocks = std::min<int64_t>(blocks, (chunks + kWavesPerBlock - 1) / kWavesPerBlock);
        }
        blocks = (blocks + kXcds - 1) / kXcds * kXcds;
        p.blocks_per_xcd = (int32_t)(blocks / kXcds);
        const float4* sph = spheres;
        const float4* qsph = qspheres;
        const TrajPlan* pl = plan;
        const dim3 gd((unsigned)blocks), bd(kBlock);
        hipEvent_t ev0, ev1;
        take_kernel_events(&ev0, &ev1);
        if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return fail(LSDF_E_DEVICE, "%s: event record failed", who);
        switch (dtype * 2 + (cubic ? 1 : 0)) {
            case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph, qsph, pl); break;
            case LSDF_F32 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_F32>), gd, bd, 0, s, p, points, static_cast<const float*>(grid_buf), sph, qsph, pl); break;
            case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph, qsph, pl); break;
            case LSDF_BF16 * 2: hipLaunchKernelGGL((query_kernel<false, LSDF_BF16>), gd, bd, 0, s, p, points, static_cast<const uint16_t*>(grid_buf), sph, qsph, pl); break;
            case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((query_kernel<true, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph, qsph, pl); break;
            default: hipLaunchKernelGGL((query_kernel<false, LSDF_F16>), gd, bd, 0, s, p, points, static_cast<const _Float16*>(grid_buf), sph, qsph, pl); break;
        }
        rc = check_launch(who);
        if (rc != LSDF_OK) return rc;
        if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return fail(LSDF_E_DEVICE, "%s: event record failed", who);
    }
    // M = 0: no prep kernel ran and no key is meaningful; every
    // configuration gets +inf and -1
    return launch_query_finalize(M > 0 ? p.keys : nullptr, out_dist, out_link, out_link_dist, C, L, s);
}

}  // namespace

LSDF_API int lsdf_query_workspace_size(int32_t C, int32_t L, int64_t M, uint32_t flags, size_t* bytes) {
    lsdf::clear_error();
    if (flags != 0) return lsdf::fail(LSDF_E_UNSUPPORTED, "query_workspace_size: unsupported flags 0x%x", flags);
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
    *bytes = workspace_bytes(K, C, L, M);
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

namespace {

// Workspace of lsdf_query_min_distance_noalloc: one copy per GPU, loaded with
// the code object.  Host code never names the array itself (on the host it
// is only a stand-in for the symbol); it takes the device address that
// hipGetSymbolAddress gives for the current device, once per device.
constexpr size_t kNoAllocScratch = LSDF_QUERY_NOALLOC_SCRATCH;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(void** out) {
    using namespace lsdf;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LSDF_E_DEVICE, "query_noalloc: no current device");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LSDF_E_DEVICE, "query_noalloc: device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LSDF_E_DEVICE, "query_noalloc: hipGetSymbolAddress of the scratch array failed (%s)",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LSDF_OK;
}

}  // namespace

LSDF_API int lsdf_query_min_distance_noalloc(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                             const void* grid_buf, const float* points, int64_t M, float* out_dist,
                                             int32_t* out_link, float* out_link_dist, uint32_t flags, void* stream) {
    using namespace lsdf;
    clear_error();
    if (flags != 0) return fail(LSDF_E_UNSUPPORTED, "query_noalloc: unsupported flags 0x%x", flags);
    if (C < 0 || M < 0 || M > LSDF_MAX_POINTS)
        return fail(LSDF_E_SHAPE, "query_noalloc: size out of range (C = %d, M = %lld)", (int)C, (long long)M);
    if (L < 1 || L > LSDF_MAX_LINKS)
        return fail(LSDF_E_SHAPE, "query_noalloc: L = %d out of [1, %d]", (int)L, LSDF_MAX_LINKS);
    if (C == 0) return LSDF_OK;
    const size_t need = workspace_bytes(1, C, L, M);
    if (need > kNoAllocScratch)
        return fail(LSDF_E_SHAPE,
                    "query_noalloc: C = %d, L = %d, M = %lld needs %zu bytes of workspace; the library holds %zu "
                    "(use lsdf_query_min_distance with a workspace of your own)",
                    (int)C, (int)L, (long long)M, need, kNoAllocScratch);
    void* ws = nullptr;
    const int rc = noalloc_scratch(&ws);
    if (rc != LSDF_OK) return rc;
    return run_query("query_noalloc", 1, nullptr, nullptr, link_T, C, L, grids, grid_buf, points, M, out_dist,
                     out_link, out_link_dist, nullptr, 0, ws, kNoAllocScratch, stream);
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

LSDF_API int lsdf_query_from_joints(const lsdf_dh* dh, int32_t dof, const float* base_T, const float* q,
                                    int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                                    int32_t C, const lsdf_grid* grids, const void* grid_buf, const float* points,
                                    int64_t M, float* link_T, float* out_dist, int32_t* out_link,
                                    float* out_link_dist, const lsdf_query_tuning* tuning, uint32_t flags,
                                    void* workspace, size_t ws_bytes, void* stream) {
    using namespace lsdf;
    clear_error();
    DhTable t;
    int rc = make_dh_table("query_from_joints", dh, dof, base_T, &t);
    if (rc != LSDF_OK) return rc;
    if ((traj_c_offset == nullptr) != (traj_m_offset == nullptr))
        return fail(LSDF_E_INVALID_ARG, "query_from_joints: give both offset arrays or neither");
    if (!traj_c_offset && K != 1)
        return fail(LSDF_E_SHAPE, "query_from_joints: K = %d without offset arrays (must be 1)", (int)K);
    return run_query("query_from_joints", K, traj_c_offset, traj_m_offset, link_T, C, dof + 1, grids, grid_buf,
                     points, M, out_dist, out_link, out_link_dist, tuning, flags, workspace, ws_bytes, stream, &t, q);
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
    // the default tiling first (so the pick is never a tiling measured
    // slower than it), then chunk sizes over the resident grid, a smaller
    // grid, and the per-XCD slices
    static const lsdf_query_tuning kGrid[] = {
        {0, 0, LSDF_SCHED_DEFAULT, 0},        {64, 0, LSDF_SCHED_INTERLEAVED, 0},
        {128, 0, LSDF_SCHED_INTERLEAVED, 0},  {256, 0, LSDF_SCHED_INTERLEAVED, 0},
        {512, 0, LSDF_SCHED_INTERLEAVED, 0},  {1024, 0, LSDF_SCHED_INTERLEAVED, 0},
        {2048, 0, LSDF_SCHED_INTERLEAVED, 0}, {4096, 0, LSDF_SCHED_INTERLEAVED, 0},
        {256, 4, LSDF_SCHED_INTERLEAVED, 0},  {1024, 4, LSDF_SCHED_INTERLEAVED, 0},
        {256, 0, LSDF_SCHED_XCD_SLICES, 0},   {1024, 0, LSDF_SCHED_XCD_SLICES, 0},
    };
    if (!candidates) {
        candidates = kGrid;
        n_candidates = (int32_t)(sizeof(kGrid) / sizeof(kGrid[0]));
    }
    if (n_candidates < 1) return fail(LSDF_E_INVALID_ARG, "query_autotune: no candidates");
    for (int32_t c = 0; c < n_candidates; ++c) {
        int cb = 0, bpc = 0, sch = 0;
        int rc = check_tuning("query_autotune", &candidates[c], &cb, &bpc, &sch);
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

