// Grid sampling in the fixed single-precision order shared by every kernel
// that reads a link grid (plain query, learned-path fallback, labels).
// Coordinates are box-centred grid coordinates v = u - (n - 1) / 2.
#pragma once

#include "lsdf_internal.hpp"

namespace lsdf {

// Storage type of a grid and its exact widening to FP32 (bfloat16: the top
// half of a binary32; binary16: v_cvt_f32_f16).
template <int DT>
struct GridT;
template <>
struct GridT<LSDF_F32> {
    using T = float;
    static __device__ inline float get(const T* p, int i) { return p[i]; }
};
template <>
struct GridT<LSDF_BF16> {
    using T = uint16_t;
    static __device__ inline float get(const T* p, int i) { return __uint_as_float((uint32_t)p[i] << 16); }
};
template <>
struct GridT<LSDF_F16> {
    using T = _Float16;
    static __device__ inline float get(const T* p, int i) { return (float)p[i]; }
};

__device__ inline float lerp_exact_ends(float a, float b, float t) {
    return fmaf(t, b, fmaf(-t, a, a));
}

template <bool CUBIC>
__device__ inline bool inside(const LinkGrid& g, float v0, float v1, float v2) {
    if (CUBIC) return fmaxf(fabsf(v0), fmaxf(fabsf(v1), fabsf(v2))) <= g.half[0];
    return (fabsf(v0) <= g.half[0]) & (fabsf(v1) <= g.half[1]) & (fabsf(v2) <= g.half[2]);
}

// One cell gather: element index of the cell's lower corner and the three
// fractions, from centred coordinates known to be inside the box.
struct Cell {
    int idx;
    float fx, fy, fz;
};

__device__ inline Cell locate(const LinkGrid& g, float v0, float v1, float v2) {
    const float u0 = v0 + g.half[0];
    const float u1 = v1 + g.half[1];
    const float u2 = v2 + g.half[2];
    // u >= 0 here, so truncation is the floor
    const int ix = min((int)u0, g.n[0] - 2);
    const int iy = min((int)u1, g.n[1] - 2);
    const int iz = min((int)u2, g.n[2] - 2);
    Cell c;
    c.fx = u0 - (float)ix;
    c.fy = u1 - (float)iy;
    c.fz = u2 - (float)iz;
    c.idx = (iz * g.n[1] + iy) * g.n[0] + ix;
    return c;
}

// Trilinear value of a cell from its corners (x first, then y, then z).
__device__ inline float interpolate(float c000, float c100, float c010, float c110, float c001, float c101,
                                    float c011, float c111, const Cell& cl) {
    const float e00 = lerp_exact_ends(c000, c100, cl.fx);
    const float e10 = lerp_exact_ends(c010, c110, cl.fx);
    const float e01 = lerp_exact_ends(c001, c101, cl.fx);
    const float e11 = lerp_exact_ends(c011, c111, cl.fx);
    const float e0 = lerp_exact_ends(e00, e10, cl.fy);
    const float e1 = lerp_exact_ends(e01, e11, cl.fy);
    return lerp_exact_ends(e0, e1, cl.fz) + 0.0f;   // -0 -> +0
}

// World-to-grid map of one (pose, link) pair: v = M [x; y; z] + w, in the
// fixed FP32 order (the inverse pose of Eq. 4 with the grid scaling folded
// in).  T is the row-major 3x4 link-to-world pose.
struct GridMap {
    float m00, m01, m02, w0;
    float m10, m11, m12, w1;
    float m20, m21, m22, w2;
};

__device__ inline GridMap grid_map(const LinkGrid& lg, const float* T) {
    const float r00 = T[0], r01 = T[1], r02 = T[2], t0 = T[3];
    const float r10 = T[4], r11 = T[5], r12 = T[6], t1 = T[7];
    const float r20 = T[8], r21 = T[9], r22 = T[10], t2 = T[11];
    GridMap g;
    g.m00 = lg.invh[0] * r00; g.m01 = lg.invh[0] * r10; g.m02 = lg.invh[0] * r20;
    g.m10 = lg.invh[1] * r01; g.m11 = lg.invh[1] * r11; g.m12 = lg.invh[1] * r21;
    g.m20 = lg.invh[2] * r02; g.m21 = lg.invh[2] * r12; g.m22 = lg.invh[2] * r22;
    g.w0 = fmaf(-lg.invh[0], fmaf(r00, t0, fmaf(r10, t1, r20 * t2)), lg.cen[0]);
    g.w1 = fmaf(-lg.invh[1], fmaf(r01, t0, fmaf(r11, t1, r21 * t2)), lg.cen[1]);
    g.w2 = fmaf(-lg.invh[2], fmaf(r02, t0, fmaf(r12, t1, r22 * t2)), lg.cen[2]);
    return g;
}

// Grid value of link-frame or world point x through map gm, +inf outside.
// G points at the link's first element (storage type DT).
template <bool CUBIC, int DT = LSDF_F32>
__device__ inline float sample_or_inf(const typename GridT<DT>::T* __restrict__ G, const LinkGrid& lg,
                                      const GridMap& gm, float x, float y, float z) {
    const float v0 = fmaf(gm.m00, x, fmaf(gm.m01, y, fmaf(gm.m02, z, gm.w0)));
    const float v1 = fmaf(gm.m10, x, fmaf(gm.m11, y, fmaf(gm.m12, z, gm.w1)));
    const float v2 = fmaf(gm.m20, x, fmaf(gm.m21, y, fmaf(gm.m22, z, gm.w2)));
    if (!inside<CUBIC>(lg, v0, v1, v2)) return INFINITY;
    const Cell cl = locate(lg, v0, v1, v2);
    const typename GridT<DT>::T* cp = G + cl.idx;
    const int nx = lg.n[0], nxy = lg.n[0] * lg.n[1];
    using E = GridT<DT>;
    return interpolate(E::get(cp, 0), E::get(cp, 1), E::get(cp, nx), E::get(cp, nx + 1), E::get(cp, nxy),
                       E::get(cp, nxy + 1), E::get(cp, nxy + nx), E::get(cp, nxy + nx + 1), cl);
}

}  // namespace lsdf
