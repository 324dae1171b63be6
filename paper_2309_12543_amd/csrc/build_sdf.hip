// Link SDF construction (Sec. III-A: per-link signed distance fields
// precomputed on the link's local grid).  Brute force: every node visits
// every triangle of every closed part of the link mesh.
//   * unsigned distance: closest point on a triangle by the Voronoi-region
//     walk of Ericson, Real-Time Collision Detection (2005), Sec. 5.1.5;
//   * inside/outside: generalised winding number (Jacobson et al. 2013), the
//     sum of signed solid angles (Van Oosterom & Strackee 1983) over 4 pi;
//   * a link made of several closed parts takes the minimum over parts.
// One lane per node; triangles are staged through LDS in chunks.
#include "grid_sample.hpp"

namespace {

using namespace lsdf;

constexpr int kBlock = 256;

struct BuildArgs {
    int32_t comp_first[LSDF_MAX_COMPONENTS + 1];
    float lo[3];
    float h[3];
    int32_t n[3];
    int32_t ncomp;
    int32_t nv;
    int32_t dtype;       // storage type of the output grid
    const float* verts;
    const int32_t* tris;
    void* out;
};

struct V3 {
    float x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline V3 axpy(float s, V3 d, V3 o) { return {o.x + s * d.x, o.y + s * d.y, o.z + s * d.z}; }

// Squared distance from p to triangle (a, b, c), by the Voronoi regions of
// its vertices, edges and face.
__device__ float dist2_point_triangle(V3 p, V3 a, V3 b, V3 c) {
    const V3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    const float d1 = dot(ab, ap), d2 = dot(ac, ap);
    V3 q;
    if (d1 <= 0.0f && d2 <= 0.0f) {
        q = a;
    } else {
        const V3 bp = sub(p, b);
        const float d3 = dot(ab, bp), d4 = dot(ac, bp);
        const V3 cp = sub(p, c);
        const float d5 = dot(ab, cp), d6 = dot(ac, cp);
        const float vc = d1 * d4 - d3 * d2;
        const float vb = d5 * d2 - d1 * d6;
        const float va = d3 * d6 - d5 * d4;
        if (d3 >= 0.0f && d4 <= d3) {
            q = b;
        } else if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {
            q = axpy(d1 / (d1 - d3), ab, a);
        } else if (d6 >= 0.0f && d5 <= d6) {
            q = c;
        } else if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {
            q = axpy(d2 / (d2 - d6), ac, a);
        } else if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {
            q = axpy((d4 - d3) / ((d4 - d3) + (d5 - d6)), sub(c, b), b);
        } else {
            const float s = va + vb + vc;
            if (s > 0.0f) {
                const float inv = 1.0f / s;
                q = axpy(vc * inv, ac, axpy(vb * inv, ab, a));
            } else {
                q = a;   // degenerate triangle: its edges were already tried
            }
        }
    }
    const V3 d = sub(p, q);
    return dot(d, d);
}

// Signed solid angle of triangle (a, b, c) seen from p:
// tan(Omega/2) = det[A B C] / (|A||B||C| + (A.B)|C| + (A.C)|B| + (B.C)|A|).
__device__ float solid_angle(V3 p, V3 a, V3 b, V3 c) {
    const V3 A = sub(a, p), B = sub(b, p), C = sub(c, p);
    const float det = dot(A, cross(B, C));
    const float la = sqrtf(dot(A, A)), lb = sqrtf(dot(B, B)), lc = sqrtf(dot(C, C));
    const float den = la * lb * lc + dot(A, B) * lc + dot(A, C) * lb + dot(B, C) * la;
    return 2.0f * atan2f(det, den);
}

// Signed distance of pt to the mesh (every lane of the block takes part in
// staging triangles through LDS; lanes with want == false skip the math).
__device__ float mesh_sdf(const BuildArgs& p, float (*s_tri)[9], V3 pt, bool want) {
    float sdf = INFINITY;
    for (int comp = 0; comp < p.ncomp; ++comp) {
        const int t0 = p.comp_first[comp], t1 = p.comp_first[comp + 1];
        float best2 = INFINITY;
        float omega = 0.0f;
        for (int base = t0; base < t1; base += kBlock) {
            __syncthreads();
            const int t = base + threadIdx.x;
            if (t < t1) {
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    // vertex indices clamped into range: a bad mesh gives a
                    // wrong grid, never an out-of-bounds read
                    const int vi = min(max(p.tris[3 * t + v], 0), p.nv - 1);
                    s_tri[threadIdx.x][3 * v + 0] = p.verts[3 * vi + 0];
                    s_tri[threadIdx.x][3 * v + 1] = p.verts[3 * vi + 1];
                    s_tri[threadIdx.x][3 * v + 2] = p.verts[3 * vi + 2];
                }
            }
            __syncthreads();
            if (want) {
                const int cnt = min(kBlock, t1 - base);
                for (int k = 0; k < cnt; ++k) {
                    const V3 a = {s_tri[k][0], s_tri[k][1], s_tri[k][2]};
                    const V3 b = {s_tri[k][3], s_tri[k][4], s_tri[k][5]};
                    const V3 c = {s_tri[k][6], s_tri[k][7], s_tri[k][8]};
                    best2 = fminf(best2, dist2_point_triangle(pt, a, b, c));
                    omega += solid_angle(pt, a, b, c);
                }
            }
        }
        const float u = sqrtf(best2);
        const float winding = omega * (float)(0.25 / M_PI);
        sdf = fminf(sdf, winding > 0.5f ? -u : u);
    }
    return sdf;
}

// Grid nodes: node idx of the grid described by p.
__global__ __launch_bounds__(kBlock) void build_sdf_kernel(BuildArgs p) {
    __shared__ float s_tri[kBlock][9];
    const int64_t nodes = (int64_t)p.n[0] * p.n[1] * p.n[2];
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool active = idx < nodes;
    const int64_t kx = idx % p.n[0];
    const int64_t ky = (idx / p.n[0]) % p.n[1];
    const int64_t kz = idx / ((int64_t)p.n[0] * p.n[1]);
    const V3 pt = {fmaf((float)kx, p.h[0], p.lo[0]), fmaf((float)ky, p.h[1], p.lo[1]),
                   fmaf((float)kz, p.h[2], p.lo[2])};
    const float sdf = mesh_sdf(p, s_tri, pt, true);
    if (active) {
        // one rounding, to nearest even, into the storage type
        if (p.dtype == LSDF_BF16)
            static_cast<uint16_t*>(p.out)[idx] = __builtin_bit_cast(uint16_t, (__bf16)sdf);
        else if (p.dtype == LSDF_F16)
            static_cast<_Float16*>(p.out)[idx] = (_Float16)sdf;
        else
            static_cast<float*>(p.out)[idx] = sdf;
    }
}

struct LabelArgs {
    BuildArgs mesh;
    LinkGrid lg;
    const void* grid;
    const float* points;
    float* out;
    int64_t N;
};

// Labels: the grid value inside the grid box, the exact distance outside.
template <bool CUBIC, int DT>
__global__ __launch_bounds__(kBlock) void label_kernel(LabelArgs p) {
    __shared__ float s_tri[kBlock][9];
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool active = j < p.N;
    const int64_t jj = active ? j : p.N - 1;
    const V3 pt = {p.points[3 * jj + 0], p.points[3 * jj + 1], p.points[3 * jj + 2]};
    const float ident[12] = {1.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f};
    const GridMap gm = grid_map(p.lg, ident);
    const float g = sample_or_inf<CUBIC, DT>(static_cast<const typename GridT<DT>::T*>(p.grid) + p.lg.offset, p.lg,
                                             gm, pt.x, pt.y, pt.z);
    const bool exact = active && !(g < INFINITY);
    float v = g;
    if (__syncthreads_or(exact)) {
        const float e = mesh_sdf(p.mesh, s_tri, pt, exact);
        if (exact) v = e;
    }
    if (active) p.out[j] = v;
}

}  // namespace

namespace {

int mesh_args(const float* verts, int32_t nv, const int32_t* tris, int32_t nt, const int32_t* comp_first,
              int32_t ncomp, BuildArgs* p) {
    using namespace lsdf;
    if (nv < 1 || nt < 1) return fail(LSDF_E_SHAPE, "mesh: empty (nv = %d, nt = %d)", (int)nv, (int)nt);
    if (!verts || !tris) return fail(LSDF_E_INVALID_ARG, "mesh: NULL device pointer");
    if (comp_first) {
        if (ncomp < 1 || ncomp > LSDF_MAX_COMPONENTS)
            return fail(LSDF_E_SHAPE, "mesh: ncomp = %d out of [1, %d]", (int)ncomp, LSDF_MAX_COMPONENTS);
        if (comp_first[0] != 0 || comp_first[ncomp] != nt)
            return fail(LSDF_E_SHAPE, "mesh: comp_first must run from 0 to nt");
        for (int k = 0; k <= ncomp; ++k) {
            if (k > 0 && comp_first[k] <= comp_first[k - 1])
                return fail(LSDF_E_SHAPE, "mesh: comp_first must increase strictly");
            p->comp_first[k] = comp_first[k];
        }
        p->ncomp = ncomp;
    } else {
        p->comp_first[0] = 0;
        p->comp_first[1] = nt;
        p->ncomp = 1;
    }
    p->nv = nv;
    p->verts = verts;
    p->tris = tris;
    return LSDF_OK;
}

}  // namespace

LSDF_API int lsdf_sdf_labels(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                             const int32_t* comp_first, int32_t ncomp, const lsdf_grid* desc, const void* grid_buf,
                             const float* points, int64_t N, float* out, void* stream) {
    using namespace lsdf;
    clear_error();
    if (!desc) return fail(LSDF_E_INVALID_ARG, "sdf_labels: desc is NULL");
    if (N < 0) return fail(LSDF_E_SHAPE, "sdf_labels: N < 0");
    LabelArgs a{};
    int rc = mesh_args(verts, nv, tris, nt, comp_first, ncomp, &a.mesh);
    if (rc != LSDF_OK) return rc;
    if ((rc = prepare_link_grid(*desc, 0, &a.lg)) != LSDF_OK) return rc;
    if (N == 0) return LSDF_OK;
    if (!grid_buf || !points || !out) return fail(LSDF_E_INVALID_ARG, "sdf_labels: NULL device pointer");
    a.grid = grid_buf;
    a.points = points;
    a.out = out;
    a.N = N;
    const dim3 grid((unsigned)((N + kBlock - 1) / kBlock));
    hipStream_t st = as_stream(stream);
    switch (a.lg.dtype * 2 + (a.lg.cubic ? 1 : 0)) {
        case LSDF_F32 * 2 + 1: hipLaunchKernelGGL((label_kernel<true, LSDF_F32>), grid, dim3(kBlock), 0, st, a); break;
        case LSDF_F32 * 2: hipLaunchKernelGGL((label_kernel<false, LSDF_F32>), grid, dim3(kBlock), 0, st, a); break;
        case LSDF_BF16 * 2 + 1: hipLaunchKernelGGL((label_kernel<true, LSDF_BF16>), grid, dim3(kBlock), 0, st, a); break;
        case LSDF_BF16 * 2: hipLaunchKernelGGL((label_kernel<false, LSDF_BF16>), grid, dim3(kBlock), 0, st, a); break;
        case LSDF_F16 * 2 + 1: hipLaunchKernelGGL((label_kernel<true, LSDF_F16>), grid, dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL((label_kernel<false, LSDF_F16>), grid, dim3(kBlock), 0, st, a); break;
    }
    return check_launch("sdf_labels");
}

LSDF_API int lsdf_build_link_sdf(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                                 const int32_t* comp_first, int32_t ncomp, const lsdf_grid* desc,
                                 void* grid_buf, void* stream) {
    using namespace lsdf;
    clear_error();
    if (!desc) return fail(LSDF_E_INVALID_ARG, "build_link_sdf: desc is NULL");
    BuildArgs p{};
    int rc0 = mesh_args(verts, nv, tris, nt, comp_first, ncomp, &p);
    if (rc0 != LSDF_OK) return rc0;
    if (!grid_buf) return fail(LSDF_E_INVALID_ARG, "build_link_sdf: grid_buf is NULL");
    LinkGrid g;
    int rc = prepare_link_grid(*desc, 0, &g);
    if (rc != LSDF_OK) return rc;
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = desc->lo[a];
        p.h[a] = (float)(((double)desc->hi[a] - (double)desc->lo[a]) / (double)(desc->n[a] - 1));
        p.n[a] = desc->n[a];
    }
    p.dtype = desc->dtype;
    p.out = static_cast<char*>(grid_buf) + desc->elem_offset * (desc->dtype == LSDF_F32 ? 4 : 2);
    const int64_t nodes = (int64_t)p.n[0] * p.n[1] * p.n[2];
    hipLaunchKernelGGL(build_sdf_kernel, dim3((unsigned)((nodes + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       as_stream(stream), p);
    return check_launch("build_link_sdf");
}
