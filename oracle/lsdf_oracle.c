/*
 * lsdf_oracle.c -- plain, slow CPU reference for batched robot-to-obstacle
 * clearance against link-local signed distance grids.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code, header or constant
 * with the HIP library: the two are written independently from the method's
 * definition (paper Sec. III-A) and compared.
 *
 * What it computes (paper Sec. III-A, problem statement and Fig. 3):
 *   for each configuration c, each link i and each obstacle point x_j,
 *   the link-local SDF of link i evaluated at the point expressed in link
 *   i's frame, T_{i,c}^{-1} x_j; the clearance of c is the minimum over
 *   points and links.  The link SDF is a grid of signed distances sampled
 *   at nodes of the link's box (the "Link SDFs" of Sec. III-A) and read
 *   between nodes by trilinear interpolation (the affine-grid sampling the
 *   paper borrows from spatial transformer networks, Sec. III-A).
 *
 * Readings where the paper is silent (listed with their justification in
 * the design notes): nodes sit on the box corners (node-centred grid);
 * points outside a link's box contribute +infinity; the SDF is negative
 * inside; a link made of several closed parts takes the minimum over the
 * parts; argmin ties go to the lowest link index; -0 is returned as +0.
 *
 * Precision: everything is double, except orc_query_f32, the single-
 * precision twin of the query used to take the argmin decision in the
 * precision of the GPU kernel.  Compile with -ffp-contract=off: every fused
 * multiply-add below is written out as fma()/fmaf().
 *
 * Parallelism: OpenMP over independent outer loops only (grid nodes,
 * configurations); the arithmetic of each element is unchanged by it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* small vector helpers (double)                                             */
/* ------------------------------------------------------------------------ */
static void v_sub(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static double v_dot(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void v_cross(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_norm(const double a[3]) { return sqrt(v_dot(a, a)); }

/* ------------------------------------------------------------------------ */
/* Point-to-triangle distance, by definition: the closest point of a         */
/* triangle is either the orthogonal projection onto its plane (when that    */
/* projection lies inside the triangle) or a point of one of its three       */
/* edges.  So the distance is the minimum of those candidates.               */
/* ------------------------------------------------------------------------ */
static double dist_point_segment(const double p[3], const double a[3], const double b[3]) {
    double ab[3], ap[3];
    v_sub(b, a, ab);
    v_sub(p, a, ap);
    double L2 = v_dot(ab, ab);
    double t = L2 > 0.0 ? v_dot(ap, ab) / L2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double q[3] = {a[0] + t * ab[0] - p[0], a[1] + t * ab[1] - p[1], a[2] + t * ab[2] - p[2]};
    return v_norm(q);
}

/* Threads of the OpenMP loops (the timing harness measures one and all). */
ORC_EXPORT void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
ORC_EXPORT int32_t orc_max_threads(void) { return (int32_t)omp_get_max_threads(); }

ORC_EXPORT double orc_point_triangle_distance(const double* p, const double* a,
                                              const double* b, const double* c) {
    double best = dist_point_segment(p, a, b);
    double e = dist_point_segment(p, b, c);
    if (e < best) best = e;
    e = dist_point_segment(p, c, a);
    if (e < best) best = e;
    /* interior candidate: barycentric coordinates of the projection */
    double ab[3], ac[3], ap[3], nrm[3];
    v_sub(b, a, ab);
    v_sub(c, a, ac);
    v_sub(p, a, ap);
    v_cross(ab, ac, nrm);
    double nn = v_dot(nrm, nrm);
    if (nn > 0.0) {
        double h = v_dot(ap, nrm) / nn;                    /* signed height / |n| */
        double proj[3] = {ap[0] - h * nrm[0], ap[1] - h * nrm[1], ap[2] - h * nrm[2]};
        double tmp[3];
        v_cross(proj, ac, tmp);
        double beta = v_dot(tmp, nrm) / nn;                /* weight of b */
        v_cross(ab, proj, tmp);
        double gamma = v_dot(tmp, nrm) / nn;               /* weight of c */
        double alpha = 1.0 - beta - gamma;
        if (alpha >= 0.0 && beta >= 0.0 && gamma >= 0.0) {
            double dplane = fabs(h) * sqrt(nn);
            if (dplane < best) best = dplane;
        }
    }
    return best;
}

/* Solid angle subtended at p by triangle (a, b, c), signed by orientation:
 * tan(Omega / 2) = det[A B C] / (|A||B||C| + (A.B)|C| + (A.C)|B| + (B.C)|A|)
 * with A = a - p etc. (Van Oosterom & Strackee, IEEE TBME 1983). */
static double solid_angle(const double p[3], const double a[3], const double b[3], const double c[3]) {
    double A[3], B[3], C[3], bc[3];
    v_sub(a, p, A);
    v_sub(b, p, B);
    v_sub(c, p, C);
    v_cross(B, C, bc);
    double det = v_dot(A, bc);
    double la = v_norm(A), lb = v_norm(B), lc = v_norm(C);
    double den = la * lb * lc + v_dot(A, B) * lc + v_dot(A, C) * lb + v_dot(B, C) * la;
    return 2.0 * atan2(det, den);
}

/* Generalised winding number of a closed, outward-oriented triangle set
 * (Jacobson et al., SIGGRAPH 2013): total signed solid angle / (4 pi).
 * 1 inside, 0 outside. */
ORC_EXPORT double orc_winding_number(const double* p, const double* V, const int32_t* T,
                                     int32_t t0, int32_t t1) {
    double sum = 0.0;
    for (int32_t t = t0; t < t1; ++t)
        sum += solid_angle(p, V + 3 * T[3 * t], V + 3 * T[3 * t + 1], V + 3 * T[3 * t + 2]);
    return sum / (4.0 * M_PI);
}

/* Signed distance of p to a link made of closed parts [comp_first[k],
 * comp_first[k+1]): each part's distance is the unsigned distance to its
 * triangles, negated when the winding number says p is inside; the link
 * takes the minimum over its parts. */
ORC_EXPORT double orc_mesh_sdf(const double* p, const double* V, const int32_t* T,
                               const int32_t* comp_first, int32_t ncomp) {
    double s = INFINITY;
    for (int32_t k = 0; k < ncomp; ++k) {
        double u = INFINITY;
        for (int32_t t = comp_first[k]; t < comp_first[k + 1]; ++t) {
            double d = orc_point_triangle_distance(p, V + 3 * T[3 * t], V + 3 * T[3 * t + 1],
                                                   V + 3 * T[3 * t + 2]);
            if (d < u) u = d;
        }
        double w = orc_winding_number(p, V, T, comp_first[k], comp_first[k + 1]);
        double sk = (w > 0.5) ? -u : u;
        if (sk < s) s = sk;
    }
    return s;
}

ORC_EXPORT void orc_mesh_sdf_many(const double* P, int64_t np, const double* V, const int32_t* T,
                                  const int32_t* comp_first, int32_t ncomp, double* out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < np; ++j) out[j] = orc_mesh_sdf(P + 3 * j, V, T, comp_first, ncomp);
}

/* Link SDF grid: node k = (kx, ky, kz) sits at lo + k * h with
 * h = (hi - lo) / (n - 1) per axis; storage index (kz * ny + ky) * nx + kx. */
ORC_EXPORT void orc_build_grid(const double* V, const int32_t* T, const int32_t* comp_first,
                               int32_t ncomp, const double* lo, const double* hi, const int32_t* n,
                               double* out) {
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = (hi[a] - lo[a]) / (double)(n[a] - 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t idx = 0; idx < nx * ny * nz; ++idx) {
        int64_t kx = idx % nx, ky = (idx / nx) % ny, kz = idx / (nx * ny);
        double p[3] = {lo[0] + kx * h[0], lo[1] + ky * h[1], lo[2] + kz * h[2]};
        out[idx] = orc_mesh_sdf(p, V, T, comp_first, ncomp);
    }
}

/* ------------------------------------------------------------------------ */
/* Forward kinematics (paper Sec. III-A: link poses T_{i,c} of every link i  */
/* at every configuration c).  Standard DH: frame k = frame k-1 moved by     */
/* Rz(theta) Tz(d) Tx(a) Rx(alpha), theta = q_k + theta_offset_k, written as  */
/* a product of the four elementary 4x4 matrices.                            */
/* ------------------------------------------------------------------------ */
static void m4_mul(const double A[16], const double B[16], double R[16]) {
    double t[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[4 * r + k] * B[4 * k + c];
            t[4 * r + c] = s;
        }
    memcpy(R, t, sizeof(t));
}
static void m4_eye(double M[16]) {
    memset(M, 0, 16 * sizeof(double));
    M[0] = M[5] = M[10] = M[15] = 1.0;
}
static void m4_rotz(double th, double M[16]) {
    m4_eye(M);
    M[0] = cos(th); M[1] = -sin(th);
    M[4] = sin(th); M[5] = cos(th);
}
static void m4_rotx(double al, double M[16]) {
    m4_eye(M);
    M[5] = cos(al); M[6] = -sin(al);
    M[9] = sin(al); M[10] = cos(al);
}
static void m4_trans(double x, double y, double z, double M[16]) {
    m4_eye(M);
    M[3] = x; M[7] = y; M[11] = z;
}

/* dh: [dof][4] rows (a, alpha, d, theta_offset); base: 3x4 link-0 pose or
 * NULL for identity; q: [C][dof]; T out: [C][dof+1][3][4], row-major [R | t],
 * each mapping link-frame coordinates to world coordinates. */
ORC_EXPORT void orc_fk(const double* dh, int32_t dof, const double* base, const double* q,
                       int32_t C, double* T) {
    for (int32_t c = 0; c < C; ++c) {
        double cur[16];
        m4_eye(cur);
        if (base) for (int r = 0; r < 3; ++r) for (int k = 0; k < 4; ++k) cur[4 * r + k] = base[4 * r + k];
        double* out = T + (int64_t)c * (dof + 1) * 12;
        memcpy(out, cur, 12 * sizeof(double));
        for (int32_t k = 0; k < dof; ++k) {
            double a = dh[4 * k], alpha = dh[4 * k + 1], d = dh[4 * k + 2], off = dh[4 * k + 3];
            double th = q[(int64_t)c * dof + k] + off;
            double A[16], E[16];
            m4_rotz(th, A);
            m4_trans(0.0, 0.0, d, E);  m4_mul(A, E, A);
            m4_trans(a, 0.0, 0.0, E);  m4_mul(A, E, A);
            m4_rotx(alpha, E);         m4_mul(A, E, A);
            m4_mul(cur, A, cur);
            memcpy(out + 12 * (k + 1), cur, 12 * sizeof(double));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Query in double: per (c, i) the minimum over points of the trilinear      */
/* interpolant g_i at l = R^T (x - t), +inf when no point lies in the box.   */
/* ------------------------------------------------------------------------ */

/* Trilinear interpolation written as the weighted sum of the 8 cell corners
 * (weights are products of f or 1 - f per axis).  u: grid coordinates,
 * already known to satisfy 0 <= u_a <= n_a - 1. */
ORC_EXPORT double orc_trilinear_f64(const double* grid, const int32_t* n, const double* u) {
    int64_t i[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        int64_t k = (int64_t)floor(u[a]);
        if (k > n[a] - 2) k = n[a] - 2;
        i[a] = k;
        f[a] = u[a] - (double)k;
    }
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
                int64_t idx = ((i[2] + dz) * n[1] + (i[1] + dy)) * (int64_t)n[0] + (i[0] + dx);
                v += w * grid[idx];
            }
    return v;
}

/* T: [C][L][3][4] double poses; lo/hi: [L][3]; n: [L][3]; grids packed with
 * link i starting at offs[i]; P: [M][3]; out: [C][L] per-link minima. */
ORC_EXPORT void orc_query_f64(const double* T, int32_t C, int32_t L, const double* lo,
                              const double* hi, const int32_t* n, const double* grids,
                              const int64_t* offs, const double* P, int64_t M, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < C; ++c) {
        for (int32_t i = 0; i < L; ++i) {
            const double* Ti = T + ((int64_t)c * L + i) * 12;
            const double* lo_i = lo + 3 * i;
            const double* hi_i = hi + 3 * i;
            const int32_t* n_i = n + 3 * i;
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = (hi_i[a] - lo_i[a]) / (double)(n_i[a] - 1);
            double best = INFINITY;
            for (int64_t j = 0; j < M; ++j) {
                double d[3] = {P[3 * j] - Ti[3], P[3 * j + 1] - Ti[7], P[3 * j + 2] - Ti[11]};
                double u[3];
                int inside = 1;
                for (int a = 0; a < 3; ++a) {
                    /* l_a = sum_r R[r][a] d_r  (R^T d) */
                    double l = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];
                    u[a] = (l - lo_i[a]) / h[a];
                    if (!(u[a] >= 0.0 && u[a] <= (double)(n_i[a] - 1))) inside = 0;
                }
                if (!inside) continue;
                double v = orc_trilinear_f64(grids + offs[i], n_i, u);
                if (v < best) best = v;
            }
            out[(int64_t)c * L + i] = best;
        }
    }
}

/* Every pair of the double query, for explaining a disagreement pair by pair
 * (the per-link minimum hides which point set it).  For configuration c,
 * link i and point j, at index e = (c L + i) M + j:
 *   u[3 e + a] = the grid coordinate (R^T (x_j - t) - lo)_a / h_a, in or out
 *                of [0, n_a - 1];
 *   v[e]       = the trilinear interpolant at u clamped into the box (equal
 *                to the query's value when u is inside; a finite value
 *                for every pair).
 * Same arithmetic as orc_query_f64 (definition of Sec. III-A). */
ORC_EXPORT void orc_query_f64_each(const double* T, int32_t C, int32_t L, const double* lo, const double* hi,
                                   const int32_t* n, const double* grids, const int64_t* offs, const double* P,
                                   int64_t M, double* u_out, double* v_out) {
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int32_t c = 0; c < C; ++c) {
        for (int32_t i = 0; i < L; ++i) {
            const double* Ti = T + ((int64_t)c * L + i) * 12;
            const double* lo_i = lo + 3 * i;
            const double* hi_i = hi + 3 * i;
            const int32_t* n_i = n + 3 * i;
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = (hi_i[a] - lo_i[a]) / (double)(n_i[a] - 1);
            const int64_t e0 = ((int64_t)c * L + i) * M;
            for (int64_t j = 0; j < M; ++j) {
                double d[3] = {P[3 * j] - Ti[3], P[3 * j + 1] - Ti[7], P[3 * j + 2] - Ti[11]};
                double u[3], uc[3];
                for (int a = 0; a < 3; ++a) {
                    double l = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];
                    u[a] = (l - lo_i[a]) / h[a];
                    uc[a] = u[a] < 0.0 ? 0.0 : (u[a] > (double)(n_i[a] - 1) ? (double)(n_i[a] - 1) : u[a]);
                    u_out[3 * (e0 + j) + a] = u[a];
                }
                v_out[e0 + j] = orc_trilinear_f64(grids + offs[i], n_i, uc);
            }
        }
    }
}

/* Exact (grid-free) per-link minima: the mesh SDF of link i at every point
 * expressed in link i's frame, over all points (no box).  Brute force, for
 * tiny inputs. */
ORC_EXPORT void orc_exact_min(const double* T, int32_t C, int32_t L, const double* const* Vs,
                              const int32_t* const* Ts, const int32_t* const* comps,
                              const int32_t* ncomps, const double* P, int64_t M, double* out) {
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int32_t c = 0; c < C; ++c) {
        for (int32_t i = 0; i < L; ++i) {
            const double* Ti = T + ((int64_t)c * L + i) * 12;
            double best = INFINITY;
            for (int64_t j = 0; j < M; ++j) {
                double d[3] = {P[3 * j] - Ti[3], P[3 * j + 1] - Ti[7], P[3 * j + 2] - Ti[11]};
                double l[3];
                for (int a = 0; a < 3; ++a) l[a] = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];
                double s = orc_mesh_sdf(l, Vs[i], Ts[i], comps[i], ncomps[i]);
                if (s < best) best = s;
            }
            out[(int64_t)c * L + i] = best;
        }
    }
}

/* Per configuration: minimum over links and the lowest link index that
 * attains it; (+inf, -1) when every link is +inf. */
ORC_EXPORT void orc_reduce_f64(const double* cl, int32_t C, int32_t L, double* d, int32_t* link) {
    for (int32_t c = 0; c < C; ++c) {
        double best = INFINITY;
        int32_t arg = -1;
        for (int32_t i = 0; i < L; ++i) {
            double v = cl[(int64_t)c * L + i];
            if (v < best) { best = v; arg = i; }
        }
        d[c] = best;
        link[c] = arg;
    }
}

/* ------------------------------------------------------------------------ */
/* Single-precision twin of the query.  Every operation is one IEEE binary32 */
/* operation in a fixed order, so that the argmin decision is taken in the   */
/* same precision as the GPU kernel:                                         */
/*   per axis a (double, rounded once):                                       */
/*     invh_a = (float)((n_a - 1) / (hi_a - lo_a)),  half_a = (n_a - 1) / 2    */
/*     cen_a  = (float)(-lo_a * invh_a - half_a)                              */
/*   per (c, i): the world-to-grid map of the inverse pose as one homogeneous */
/*     matrix (the form of paper Eq. 4), centred on the box:                  */
/*       M[a][b] = invh_a * R[b][a]                                           */
/*       w_a = fma(-invh_a, fma(R[0][a], t0, fma(R[1][a], t1, R[2][a]*t2)),   */
/*                 cen_a)                                                     */
/*   per point: v_a = fma(M[a][0], x, fma(M[a][1], y, fma(M[a][2], z, w_a)))  */
/*     inside iff |v_a| <= half_a for every a                                 */
/*     u_a = v_a + half_a (lies in [0, n_a - 1])                              */
/*     i_a = min(floor(u_a), n_a - 2), f_a = u_a - i_a (exact)               */
/*     lerp(p, q, f) = fma(f, q, fma(-f, p, p)) (exact at f = 0 and f = 1):   */
/*     four along x, two along y, one along z                                 */
/*     value + 0.0f (turns -0 into +0); running minimum.                      */
/* ------------------------------------------------------------------------ */
static float lerpf_(float p, float q, float f) { return fmaf(f, q, fmaf(-f, p, p)); }

/* each != NULL also stores every pair's value, [C][L][M] (+inf outside the
 * box). */
static void query_f32_impl(const float* T, int32_t C, int32_t L, const float* lo, const float* hi,
                           const int32_t* n, const float* grids, const int64_t* offs, const float* P, int64_t M,
                           float* out, float* each) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < C; ++c) {
        for (int32_t i = 0; i < L; ++i) {
            const float* Ti = T + ((int64_t)c * L + i) * 12;
            const int32_t* n_i = n + 3 * i;
            const float* G = grids + offs[i];
            float invh[3], half[3], cen[3], Mx[3][3], w[3];
            for (int a = 0; a < 3; ++a) {
                invh[a] = (float)((double)(n_i[a] - 1) / ((double)hi[3 * i + a] - (double)lo[3 * i + a]));
                half[a] = 0.5f * (float)(n_i[a] - 1);
                cen[a] = (float)(-(double)lo[3 * i + a] * (double)invh[a] - (double)half[a]);
            }
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) Mx[a][b] = invh[a] * Ti[4 * b + a];
                float rt = fmaf(Ti[0 + a], Ti[3], fmaf(Ti[4 + a], Ti[7], Ti[8 + a] * Ti[11]));
                w[a] = fmaf(-invh[a], rt, cen[a]);
            }
            float best = INFINITY;
            float* ev = each ? each + ((int64_t)c * L + i) * M : NULL;
            for (int64_t j = 0; j < M; ++j) {
                float x = P[3 * j], y = P[3 * j + 1], z = P[3 * j + 2];
                float v[3];
                int inside = 1;
                if (ev) ev[j] = INFINITY;
                for (int a = 0; a < 3; ++a) {
                    v[a] = fmaf(Mx[a][0], x, fmaf(Mx[a][1], y, fmaf(Mx[a][2], z, w[a])));
                    if (!(fabsf(v[a]) <= half[a])) inside = 0;
                }
                if (!inside) continue;
                int64_t k[3];
                float f[3];
                for (int a = 0; a < 3; ++a) {
                    float u = v[a] + half[a];
                    int64_t q = (int64_t)floorf(u);
                    if (q > n_i[a] - 2) q = n_i[a] - 2;
                    k[a] = q;
                    f[a] = u - (float)q;
                }
                const int64_t nx = n_i[0], ny = n_i[1];
#define GV(dx, dy, dz) G[((k[2] + (dz)) * ny + (k[1] + (dy))) * nx + (k[0] + (dx))]
                float e00 = lerpf_(GV(0, 0, 0), GV(1, 0, 0), f[0]);
                float e10 = lerpf_(GV(0, 1, 0), GV(1, 1, 0), f[0]);
                float e01 = lerpf_(GV(0, 0, 1), GV(1, 0, 1), f[0]);
                float e11 = lerpf_(GV(0, 1, 1), GV(1, 1, 1), f[0]);
#undef GV
                float e0 = lerpf_(e00, e10, f[1]);
                float e1 = lerpf_(e01, e11, f[1]);
                float val = lerpf_(e0, e1, f[2]) + 0.0f;
                if (ev) ev[j] = val;
                if (val < best) best = val;
            }
            out[(int64_t)c * L + i] = best;
        }
    }
}

ORC_EXPORT void orc_query_f32(const float* T, int32_t C, int32_t L, const float* lo, const float* hi,
                              const int32_t* n, const float* grids, const int64_t* offs, const float* P, int64_t M,
                              float* out) {
    query_f32_impl(T, C, L, lo, hi, n, grids, offs, P, M, out, NULL);
}

/* The single-precision twin's value of every (configuration, link, point)
 * triple, [C][L][M]; out receives the per-link minima as orc_query_f32. */
ORC_EXPORT void orc_query_f32_each(const float* T, int32_t C, int32_t L, const float* lo, const float* hi,
                                   const int32_t* n, const float* grids, const int64_t* offs, const float* P,
                                   int64_t M, float* out, float* each) {
    query_f32_impl(T, C, L, lo, hi, n, grids, offs, P, M, out, each);
}

ORC_EXPORT void orc_reduce_f32(const float* cl, int32_t C, int32_t L, float* d, int32_t* link) {
    for (int32_t c = 0; c < C; ++c) {
        float best = INFINITY;
        int32_t arg = -1;
        for (int32_t i = 0; i < L; ++i) {
            float v = cl[(int64_t)c * L + i];
            if (v < best) { best = v; arg = i; }
        }
        d[c] = best;
        link[c] = arg;
    }
}

/* ------------------------------------------------------------------------ */
/* Learned per-link SDF surrogate (not in the paper; the build's learned     */
/* extension, checked against the grid and mesh distances above).            */
/*   m(x) = w4 . h3 + b4,  h_k = SiLU(W_k h_{k-1} + b_k),  h_0 = x (3 values) */
/*   widths 3 -> 128 -> 128 -> 128 -> 1,  SiLU(z) = z / (1 + exp(-z)).       */
/* Parameter vector (33665 values): W1[128][3], b1[128], W2[128][128], b2,    */
/* W3[128][128], b3, w4[128], b4.  Inputs are normalised coordinates.         */
/* Loss: mean absolute error over the batch (the paper trains its own tiny   */
/* network with an L1 loss and Adam, Sec. IV-B); subgradient sign(0) = 0.    */
/*                                                                           */
/* The surrogate's estimate of link i's signed distance at a link-frame     */
/* point l is the network plus a fixed core term (the build's reading):     */
/*   F(l) = m((l - c) / h) + E(l),  E(l) = || max(|l - c| - k, 0) ||,        */
/* c and h the centre and half extent of the network's domain, k the half    */
/* extent of the link's core box (its mesh's bounding box, centred at c).    */
/* E is the distance from l to that box (0 inside it), which the true        */
/* distance approaches far from the link, so the network only learns the     */
/* bounded, slowly varying remainder.  With a remainder bound B > 0 per link */
/* the network's share is B tanh(m / B) (B = +inf: m itself), so that        */
/*   E - B <= F <= E + B,                                                    */
/* which lets a query skip, exactly, the points that cannot hold a minimum.  */
/* ------------------------------------------------------------------------ */
#define ORC_H 128
#define ORC_OFF_W1 0
#define ORC_OFF_B1 (ORC_OFF_W1 + ORC_H * 3)
#define ORC_OFF_W2 (ORC_OFF_B1 + ORC_H)
#define ORC_OFF_B2 (ORC_OFF_W2 + ORC_H * ORC_H)
#define ORC_OFF_W3 (ORC_OFF_B2 + ORC_H)
#define ORC_OFF_B3 (ORC_OFF_W3 + ORC_H * ORC_H)
#define ORC_OFF_W4 (ORC_OFF_B3 + ORC_H)
#define ORC_OFF_B4 (ORC_OFF_W4 + ORC_H)
#define ORC_NPARAM (ORC_OFF_B4 + 1)

ORC_EXPORT int64_t orc_mlp_nparam(void) { return ORC_NPARAM; }

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double silu_grad(double z) {
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* Round a double to the nearest bfloat16 (ties to even), via float. */
static double bf16r(double x) {
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) != 0x7f800000u) {
        uint32_t lsb = (b >> 16) & 1u;
        b = (b + 0x7fffu + lsb) & 0xffff0000u;
    }
    memcpy(&f, &b, 4);
    return (double)f;
}

/* One sample, forward.  bf16 != 0 rounds to bfloat16 where the GPU kernels
 * do (weights W1, W2, W3, w4; activations h1, h2, h3 before they are
 * multiplied); everything else stays double.  Stores pre-activations z1..z3
 * and activations h1..h3 (as used by the next layer). */
static double mlp_forward_one(const double* P, const double* x, int bf16, double* z1, double* h1,
                              double* z2, double* h2, double* z3, double* h3) {
#define R(v) (bf16 ? bf16r(v) : (v))
    for (int u = 0; u < ORC_H; ++u) {
        double s = P[ORC_OFF_B1 + u];
        for (int k = 0; k < 3; ++k) s += R(P[ORC_OFF_W1 + 3 * u + k]) * x[k];
        z1[u] = s;
        h1[u] = R(silu(s));
    }
    for (int u = 0; u < ORC_H; ++u) {
        double s = 0.0;
        for (int k = 0; k < ORC_H; ++k) s += R(P[ORC_OFF_W2 + ORC_H * u + k]) * h1[k];
        z2[u] = s + P[ORC_OFF_B2 + u];
        h2[u] = R(silu(z2[u]));
    }
    for (int u = 0; u < ORC_H; ++u) {
        double s = 0.0;
        for (int k = 0; k < ORC_H; ++k) s += R(P[ORC_OFF_W3 + ORC_H * u + k]) * h2[k];
        z3[u] = s + P[ORC_OFF_B3 + u];
        h3[u] = R(silu(z3[u]));
    }
    double m = P[ORC_OFF_B4];
    for (int k = 0; k < ORC_H; ++k) m += R(P[ORC_OFF_W4 + k]) * h3[k];
    return m;
#undef R
}

ORC_EXPORT void orc_mlp_forward(const double* P, const double* X, int64_t N, int32_t bf16, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double z1[ORC_H], h1[ORC_H], z2[ORC_H], h2[ORC_H], z3[ORC_H], h3[ORC_H];
        out[j] = mlp_forward_one(P, X + 3 * j, bf16, z1, h1, z2, h2, z3, h3);
    }
}

/* Distance from link-frame point l to the core box |l_a - c_a| <= k_a. */
static double core_distance(const double* l, const double* c, const double* k) {
    double q2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = fabs(l[a] - c[a]) - k[a];
        if (e > 0.0) q2 += e * e;
    }
    return sqrt(q2);
}

/* The network's share of the estimate: B tanh(m / B), or m when B = +inf. */
static double bounded(double m, double B) { return isinf(B) ? m : B * tanh(m / B); }

/* The surrogate's estimate F at N link-frame points L [N][3] of one link:   */
/* the network at (l - c) / h, bounded by B, plus the core term E(l)         */
/* (core_k NULL: none).                                                      */
ORC_EXPORT void orc_mlp_value(const double* P, const double* Lp, int64_t N, const double* dom_c,
                              const double* dom_h, const double* core_k, double bound, int32_t bf16, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double z1[ORC_H], h1[ORC_H], z2[ORC_H], h2[ORC_H], z3[ORC_H], h3[ORC_H];
        const double* l = Lp + 3 * j;
        double xh[3];
        for (int a = 0; a < 3; ++a) xh[a] = (l[a] - dom_c[a]) / dom_h[a];
        double m = mlp_forward_one(P, xh, bf16, z1, h1, z2, h2, z3, h3);
        m = bounded(m, bound);
        out[j] = core_k ? m + core_distance(l, dom_c, core_k) : m;
    }
}

/* Mean-absolute-error loss over N samples and its gradient (chain rule,
 * layer by layer).  The estimate of sample j is the network's output m,
 * bounded (B tanh(m / B); bound = +inf: m), plus D[j] (the core term at the
 * sample; D NULL: none), and the loss is mean |estimate - Y|.  With bf16 != 0 the backward pass also rounds where
 * the GPU kernels do: the delta vectors dz3 and dz2 before they are
 * multiplied (weight gradients and the back-propagated deltas). */
ORC_EXPORT double orc_mlp_loss_grad(const double* P, const double* X, const double* D, const double* Y, int64_t N,
                                    double bound, int32_t bf16, double* grad) {
#define R(v) (bf16 ? bf16r(v) : (v))
    memset(grad, 0, ORC_NPARAM * sizeof(double));
    double loss = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        double z1[ORC_H], h1[ORC_H], z2[ORC_H], h2[ORC_H], z3[ORC_H], h3[ORC_H];
        double d3[ORC_H], d2[ORC_H], d1[ORC_H];
        const double* x = X + 3 * j;
        double m = mlp_forward_one(P, x, bf16, z1, h1, z2, h2, z3, h3);
        const double f = bounded(m, bound);
        double r = (D ? f + D[j] : f) - Y[j];
        loss += fabs(r);
        double dm = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / (double)N;
        if (!isinf(bound)) {
            const double t = tanh(m / bound);
            dm *= 1.0 - t * t;   /* d(B tanh(m / B)) / dm */
        }
        grad[ORC_OFF_B4] += dm;
        for (int k = 0; k < ORC_H; ++k) {
            grad[ORC_OFF_W4 + k] += dm * h3[k];
            d3[k] = R(dm * R(P[ORC_OFF_W4 + k]) * silu_grad(z3[k]));
        }
        for (int u = 0; u < ORC_H; ++u) {
            grad[ORC_OFF_B3 + u] += d3[u];
            for (int k = 0; k < ORC_H; ++k) grad[ORC_OFF_W3 + ORC_H * u + k] += d3[u] * h2[k];
        }
        for (int k = 0; k < ORC_H; ++k) {
            double s = 0.0;
            for (int u = 0; u < ORC_H; ++u) s += R(P[ORC_OFF_W3 + ORC_H * u + k]) * d3[u];
            d2[k] = R(s * silu_grad(z2[k]));
        }
        for (int u = 0; u < ORC_H; ++u) {
            grad[ORC_OFF_B2 + u] += d2[u];
            for (int k = 0; k < ORC_H; ++k) grad[ORC_OFF_W2 + ORC_H * u + k] += d2[u] * h1[k];
        }
        for (int k = 0; k < ORC_H; ++k) {
            double s = 0.0;
            for (int u = 0; u < ORC_H; ++u) s += R(P[ORC_OFF_W2 + ORC_H * u + k]) * d2[u];
            d1[k] = s * silu_grad(z1[k]);
        }
        for (int u = 0; u < ORC_H; ++u) {
            grad[ORC_OFF_B1 + u] += d1[u];
            for (int k = 0; k < 3; ++k) grad[ORC_OFF_W1 + 3 * u + k] += d1[u] * x[k];
        }
    }
    return loss / (double)N;
#undef R
}

/* Adam (Kingma & Ba 2015), step t >= 1, bias-corrected moments. */
ORC_EXPORT void orc_adam_step(double* P, double* Mo, double* Vo, const double* G, int64_t n, int64_t t,
                              double lr, double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t k = 0; k < n; ++k) {
        Mo[k] = beta1 * Mo[k] + (1.0 - beta1) * G[k];
        Vo[k] = beta2 * Vo[k] + (1.0 - beta2) * G[k] * G[k];
        double mh = Mo[k] / c1, vh = Vo[k] / c2;
        P[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Judge of the learned surrogate: per (c, i), the minimum over the points   */
/* inside link i's network domain (|(l - dom_c) / dom_h|_a <= 1 on every     */
/* axis) of F_i(l) = the double-precision grid interpolant inside the grid   */
/* box, the exact mesh signed distance outside it.  Exact: points outside    */
/* the box are visited in increasing order of their distance to the mesh's   */
/* bounding box, a lower bound of their mesh distance, and the scan stops    */
/* when that bound reaches the running minimum.  +inf when no point is in    */
/* the domain.                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lb;
    int64_t j;
} orc_lb_t;

static int cmp_lb(const void* a, const void* b) {
    double x = ((const orc_lb_t*)a)->lb, y = ((const orc_lb_t*)b)->lb;
    return (x > y) - (x < y);
}

ORC_EXPORT void orc_judge_min(const double* T, int32_t C, int32_t L, const double* lo, const double* hi,
                              const int32_t* n, const double* grids, const int64_t* offs,
                              const double* const* Vs, const int32_t* const* Ts, const int32_t* const* comps,
                              const int32_t* ncomps, const double* aabb_lo, const double* aabb_hi,
                              const double* dom_c, const double* dom_h, const double* P, int64_t M, double* out) {
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int32_t c = 0; c < C; ++c) {
        for (int32_t i = 0; i < L; ++i) {
            const double* Ti = T + ((int64_t)c * L + i) * 12;
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = (hi[3 * i + a] - lo[3 * i + a]) / (double)(n[3 * i + a] - 1);
            orc_lb_t* outside = (orc_lb_t*)malloc(sizeof(orc_lb_t) * (size_t)(M > 0 ? M : 1));
            int64_t nout = 0;
            double best = INFINITY;
            for (int64_t j = 0; j < M; ++j) {
                double d[3] = {P[3 * j] - Ti[3], P[3 * j + 1] - Ti[7], P[3 * j + 2] - Ti[11]};
                double l[3], u[3];
                int indom = 1, inbox = 1;
                for (int a = 0; a < 3; ++a) {
                    l[a] = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];
                    if (fabs((l[a] - dom_c[3 * i + a]) / dom_h[3 * i + a]) > 1.0) indom = 0;
                    u[a] = (l[a] - lo[3 * i + a]) / h[a];
                    if (!(u[a] >= 0.0 && u[a] <= (double)(n[3 * i + a] - 1))) inbox = 0;
                }
                if (!indom) continue;
                if (inbox) {
                    double v = orc_trilinear_f64(grids + offs[i], n + 3 * i, u);
                    if (v < best) best = v;
                } else {
                    double q2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double e = 0.0;
                        if (l[a] < aabb_lo[3 * i + a]) e = aabb_lo[3 * i + a] - l[a];
                        if (l[a] > aabb_hi[3 * i + a]) e = l[a] - aabb_hi[3 * i + a];
                        q2 += e * e;
                    }
                    outside[nout].lb = sqrt(q2);
                    outside[nout].j = j;
                    ++nout;
                }
            }
            qsort(outside, (size_t)nout, sizeof(orc_lb_t), cmp_lb);
            for (int64_t k = 0; k < nout && outside[k].lb < best; ++k) {
                int64_t j = outside[k].j;
                double d[3] = {P[3 * j] - Ti[3], P[3 * j + 1] - Ti[7], P[3 * j + 2] - Ti[11]};
                double l[3];
                for (int a = 0; a < 3; ++a) l[a] = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];
                double s = orc_mesh_sdf(l, Vs[i], Ts[i], comps[i], ncomps[i]);
                if (s < best) best = s;
            }
            free(outside);
            out[(int64_t)c * L + i] = best;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Clearance with the learned surrogate and its margin fallback (the build's */
/* extension; the safety-margin rule, read as strict).  Per pair (c, i, j):  */
/*   l = R^T (x - t) in double from the FP32 pose; the pair counts only if    */
/*   l lies in link i's network domain, |(l_a - dom_c_a) / dom_h_a| <= 1;    */
/*   m = the network of link i at the normalised point (mlp_forward_one,      */
/*       bfloat16 rounding points when bf16 != 0) plus the core term E(l)    */
/*       (core_k [L][3] the core boxes' half extents; NULL: no core term), */
/*       the network's share bounded by bounds[i] (NULL: unbounded);         */
/*   if m < margin and the single-precision twin places the point in the     */
/*   grid box, the pair's value is the twin's grid value, else it is m (a     */
/*   point outside the box keeps m: the grid has no value there).             */
/* out[c][i] = the minimum over counted pairs (+inf if none).  each_m and     */
/* each_g (optional, [C][L][M]) receive m (evaluated for every pair, in the  */
/* domain or not) and the twin's grid value (+inf outside the box).          */
/* ------------------------------------------------------------------------ */
ORC_EXPORT void orc_query_mlp(const float* T, int32_t C, int32_t L, const float* lo, const float* hi,
                              const int32_t* n, const float* grids, const int64_t* offs, const float* P,
                              int64_t M, const double* params, const double* dom_c, const double* dom_h,
                              const double* core_k, const double* bounds, double margin, int32_t bf16, double* out,
                              double* each_m,
                              double* each_g) {
    float* gl = (float*)malloc(sizeof(float) * (size_t)L);
    float* ge = (float*)malloc(sizeof(float) * (size_t)L * (size_t)(M > 0 ? M : 1));
    for (int32_t c = 0; c < C; ++c) {
        const float* Tc = T + (int64_t)c * L * 12;
        query_f32_impl(Tc, 1, L, lo, hi, n, grids, offs, P, M, gl, ge);
        for (int32_t i = 0; i < L; ++i) {
            const float* Ti = Tc + (int64_t)i * 12;
            const double* Pi = params + (int64_t)i * ORC_NPARAM;
            const int64_t row = (int64_t)c * L + i;
            double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
            for (int64_t j = 0; j < M; ++j) {
                double d[3] = {(double)P[3 * j] - Ti[3], (double)P[3 * j + 1] - Ti[7], (double)P[3 * j + 2] - Ti[11]};
                double xh[3], l[3];
                int indom = 1;
                for (int a = 0; a < 3; ++a) {
                    l[a] = (double)Ti[0 + a] * d[0] + (double)Ti[4 + a] * d[1] + (double)Ti[8 + a] * d[2];
                    xh[a] = (l[a] - dom_c[3 * i + a]) / dom_h[3 * i + a];
                    if (fabs(xh[a]) > 1.0) indom = 0;
                }
                const double g = (double)ge[(int64_t)i * M + j];
                double m = INFINITY;
                if (indom || each_m) {
                    double z1[ORC_H], h1[ORC_H], z2[ORC_H], h2[ORC_H], z3[ORC_H], h3[ORC_H];
                    m = mlp_forward_one(Pi, xh, bf16, z1, h1, z2, h2, z3, h3);
                    if (bounds) m = bounded(m, bounds[i]);
                    if (core_k) m += core_distance(l, dom_c + 3 * i, core_k + 3 * i);
                }
                if (indom) {
                    double v = (m < margin && g < INFINITY) ? g : m;
                    if (v < best) best = v;
                }
                if (each_m) each_m[row * M + j] = m;
                if (each_g) each_g[row * M + j] = g;
            }
            out[row] = best;
        }
    }
    free(ge);
    free(gl);
}

/* ------------------------------------------------------------------------ */
/* The paper's own pipeline (Sec. III-A, Eq. 1-4): Robot SDFs.               */
/*                                                                           */
/* The environment is a voxel grid: voxel v (per axis 0 <= v_a < N_a) spans  */
/* [lo_a + v_a r, lo_a + (v_a + 1) r) and has its centre at                  */
/* lo_a + (v_a + 1/2) r (r = voxel edge; lo = -e_e, the paper's environment  */
/* extent).  Link i's transformed SDF is a block of (2 m_i)^3 voxels         */
/* (m_i r = e_r, the paper's Link SDF extent) aligned to the environment.    */
/* Alignment of link i at configuration c (Eq. 1-3, read as                 */
/*   T_O = t - lo,  k = round(T_O / r) - m,  dt = T_O - (k r + m r)):        */
/* the block covers environment voxels k .. k + 2m - 1 on each axis, its     */
/* centre sits at the grid line nearest to the link origin and dt, the      */
/* origin's offset from that centre, lies in [-r/2, r/2].                    */
/* Euclidean transformation (Eq. 4): block voxel j has centre               */
/* P_j = (j + 1/2 - m) r relative to the block centre, and its link-local    */
/* coordinate is G = R^T (P_j - dt); the transformed SDF value there is the  */
/* link grid's interpolant g_i(G) (+inf outside the grid box).              */
/* Robot SDF of configuration c: per environment voxel, the minimum over    */
/* links of the aligned transformed values (+inf where no block reaches).   */
/* Runtime: obstacle points are voxelised, v_a = floor((x_a - lo_a) / r)    */
/* (in double), points outside the environment are dropped, and the         */
/* distance of c is the minimum of its Robot SDF over the occupied voxels.  */
/* ------------------------------------------------------------------------ */

/* Eq. 1-3 for one link position t: block corner k and residual shift dt. */
ORC_EXPORT void orc_align(const double* t, const double* env_lo, double r, int32_t m, int64_t* k, double* dt) {
    for (int a = 0; a < 3; ++a) {
        const double t_o = t[a] - env_lo[a];                 /* Eq. 1: T_O = T - (-e_e) */
        k[a] = (int64_t)nearbyint(t_o / r) - m;               /* Eq. 2 */
        dt[a] = t_o - ((double)k[a] * r + (double)m * r);     /* Eq. 3 */
    }
}

/* Robot SDFs in double, [C][N_z][N_y][N_x] (x fastest). */
ORC_EXPORT void orc_robot_sdf_f64(const double* T, int32_t C, int32_t L, const double* lo, const double* hi,
                                  const int32_t* n, const double* grids, const int64_t* offs, const int32_t* m,
                                  const double* env_lo, double r, const int32_t* env_n, double* out) {
    const int64_t V = (int64_t)env_n[0] * env_n[1] * env_n[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < C; ++c) {
        double* rs = out + (int64_t)c * V;
        for (int64_t v = 0; v < V; ++v) rs[v] = INFINITY;
        for (int32_t i = 0; i < L; ++i) {
            const double* Ti = T + ((int64_t)c * L + i) * 12;
            const double t[3] = {Ti[3], Ti[7], Ti[11]};
            int64_t k[3];
            double dt[3];
            orc_align(t, env_lo, r, m[i], k, dt);
            double h[3];
            for (int a = 0; a < 3; ++a) h[a] = (hi[3 * i + a] - lo[3 * i + a]) / (double)(n[3 * i + a] - 1);
            const int32_t w = 2 * m[i];
            for (int32_t jz = 0; jz < w; ++jz)
                for (int32_t jy = 0; jy < w; ++jy)
                    for (int32_t jx = 0; jx < w; ++jx) {
                        const int64_t e[3] = {k[0] + jx, k[1] + jy, k[2] + jz};
                        if (e[0] < 0 || e[1] < 0 || e[2] < 0 || e[0] >= env_n[0] || e[1] >= env_n[1] ||
                            e[2] >= env_n[2])
                            continue;                         /* outside the environment */
                        const int32_t j[3] = {jx, jy, jz};
                        double d[3], u[3];
                        for (int a = 0; a < 3; ++a) d[a] = ((double)j[a] + 0.5 - (double)m[i]) * r - dt[a];
                        int inside = 1;
                        for (int a = 0; a < 3; ++a) {
                            const double G = Ti[0 + a] * d[0] + Ti[4 + a] * d[1] + Ti[8 + a] * d[2];   /* Eq. 4 */
                            u[a] = (G - lo[3 * i + a]) / h[a];
                            if (!(u[a] >= 0.0 && u[a] <= (double)(n[3 * i + a] - 1))) inside = 0;
                        }
                        if (!inside) continue;
                        const double val = orc_trilinear_f64(grids + offs[i], n + 3 * i, u);
                        const int64_t idx = (e[2] * env_n[1] + e[1]) * (int64_t)env_n[0] + e[0];
                        if (val < rs[idx]) rs[idx] = val;
                    }
        }
    }
}

/* Environment voxel of a point (double arithmetic), or -1 outside. */
ORC_EXPORT int64_t orc_voxel_index(const double* x, const double* env_lo, double r, const int32_t* env_n) {
    int64_t v[3];
    for (int a = 0; a < 3; ++a) {
        const double q = floor((x[a] - env_lo[a]) / r);
        if (!(q >= 0.0 && q < (double)env_n[a])) return -1;
        v[a] = (int64_t)q;
    }
    return (v[2] * env_n[1] + v[1]) * (int64_t)env_n[0] + v[0];
}

/* Runtime of the Robot-SDF pipeline: per configuration, the minimum of its
 * Robot SDF over the voxels occupied by the points (+inf if none). */
ORC_EXPORT void orc_robot_sdf_query(const double* rs, int32_t C, const double* env_lo, double r,
                                    const int32_t* env_n, const double* P, int64_t M, double* out) {
    const int64_t V = (int64_t)env_n[0] * env_n[1] * env_n[2];
    for (int32_t c = 0; c < C; ++c) out[c] = INFINITY;
    for (int64_t j = 0; j < M; ++j) {
        const int64_t v = orc_voxel_index(P + 3 * j, env_lo, r, env_n);
        if (v < 0) continue;
        for (int32_t c = 0; c < C; ++c) {
            const double x = rs[(int64_t)c * V + v];
            if (x < out[c]) out[c] = x;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The paper's tiny network for the Euclidean grid transformation           */
/* (Sec. III-B-1, Eq. 4-5): f(R) approximates G = R^T P, the rotated         */
/* normalised centres of the (2m)^3 voxels of a transformed Link SDF block.  */
/*   P_j = ((j_x + 1/2) / m - 1, (j_y + 1/2) / m - 1, (j_z + 1/2) / m - 1),  */
/*   voxel j = (j_z * 2m + j_y) * 2m + j_x, output o = 3 j + a:              */
/*   target_o = sum_b R[b][a] P_j[b]   (R^T P_j, axis a)                     */
/* Network: x = R row-major (9 inputs), h = ReLU(W1 x + b1) (32 units),     */
/* out = W2 h + b2 (3 V outputs, V = (2m)^3).  Parameters, in order:         */
/* W1[32][9], b1[32], W2[3V][32], b2[3V].  Loss: mean absolute error over    */
/* the batch and the outputs (the paper trains it with an L1 loss and Adam,  */
/* Sec. IV-B); subgradient sign(0) = 0, ReLU'(0) = 0.                        */
/* ------------------------------------------------------------------------ */
#define ORC_FR_H 32

ORC_EXPORT int64_t orc_frnn_nparam(int32_t m) {
    const int64_t V = (int64_t)(2 * m) * (2 * m) * (2 * m);
    return ORC_FR_H * 9 + ORC_FR_H + 3 * V * ORC_FR_H + 3 * V;
}

/* Exact R^T P for N rotations R [N][9] (row-major): out [N][3V]. */
ORC_EXPORT void orc_frnn_target(int32_t m, const double* R, int64_t N, double* out) {
    const int32_t w = 2 * m;
    const int64_t V = (int64_t)w * w * w;
    for (int64_t s = 0; s < N; ++s) {
        const double* r = R + 9 * s;
        for (int64_t j = 0; j < V; ++j) {
            const int32_t jx = (int32_t)(j % w), jy = (int32_t)((j / w) % w), jz = (int32_t)(j / ((int64_t)w * w));
            const double P[3] = {(jx + 0.5) / m - 1.0, (jy + 0.5) / m - 1.0, (jz + 0.5) / m - 1.0};
            for (int a = 0; a < 3; ++a)
                out[s * 3 * V + 3 * j + a] = r[0 * 3 + a] * P[0] + r[1 * 3 + a] * P[1] + r[2 * 3 + a] * P[2];
        }
    }
}

ORC_EXPORT void orc_frnn_forward(const double* params, int32_t m, const double* R, int64_t N, double* out) {
    const int64_t V = (int64_t)(2 * m) * (2 * m) * (2 * m), O = 3 * V;
    const double* W1 = params;
    const double* b1 = W1 + ORC_FR_H * 9;
    const double* W2 = b1 + ORC_FR_H;
    const double* b2 = W2 + O * ORC_FR_H;
    for (int64_t s = 0; s < N; ++s) {
        double h[ORC_FR_H];
        for (int u = 0; u < ORC_FR_H; ++u) {
            double z = b1[u];
            for (int k = 0; k < 9; ++k) z += W1[u * 9 + k] * R[9 * s + k];
            h[u] = z > 0.0 ? z : 0.0;
        }
        for (int64_t o = 0; o < O; ++o) {
            double y = b2[o];
            for (int u = 0; u < ORC_FR_H; ++u) y += W2[o * ORC_FR_H + u] * h[u];
            out[s * O + o] = y;
        }
    }
}

/* Mean absolute error against R^T P over N rotations, and its gradient. */
ORC_EXPORT double orc_frnn_loss_grad(const double* params, int32_t m, const double* R, int64_t N, double* grad) {
    const int64_t V = (int64_t)(2 * m) * (2 * m) * (2 * m), O = 3 * V;
    const int64_t np = orc_frnn_nparam(m);
    const double* W1 = params;
    const double* b1 = W1 + ORC_FR_H * 9;
    const double* W2 = b1 + ORC_FR_H;
    const double* b2 = W2 + O * ORC_FR_H;
    double* gW1 = grad;
    double* gb1 = gW1 + ORC_FR_H * 9;
    double* gW2 = gb1 + ORC_FR_H;
    double* gb2 = gW2 + O * ORC_FR_H;
    memset(grad, 0, sizeof(double) * (size_t)np);
    double* tgt = (double*)malloc(sizeof(double) * (size_t)O);
    const double scale = 1.0 / ((double)N * (double)O);
    double loss = 0.0;
    for (int64_t s = 0; s < N; ++s) {
        const double* x = R + 9 * s;
        orc_frnn_target(m, x, 1, tgt);
        double z[ORC_FR_H], h[ORC_FR_H], dh[ORC_FR_H];
        for (int u = 0; u < ORC_FR_H; ++u) {
            z[u] = b1[u];
            for (int k = 0; k < 9; ++k) z[u] += W1[u * 9 + k] * x[k];
            h[u] = z[u] > 0.0 ? z[u] : 0.0;
            dh[u] = 0.0;
        }
        for (int64_t o = 0; o < O; ++o) {
            double y = b2[o];
            for (int u = 0; u < ORC_FR_H; ++u) y += W2[o * ORC_FR_H + u] * h[u];
            const double e = y - tgt[o];
            loss += fabs(e) * scale;
            const double g = (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) * scale;
            gb2[o] += g;
            for (int u = 0; u < ORC_FR_H; ++u) {
                gW2[o * ORC_FR_H + u] += g * h[u];
                dh[u] += g * W2[o * ORC_FR_H + u];
            }
        }
        for (int u = 0; u < ORC_FR_H; ++u) {
            const double dz = z[u] > 0.0 ? dh[u] : 0.0;
            gb1[u] += dz;
            for (int k = 0; k < 9; ++k) gW1[u * 9 + k] += dz * x[k];
        }
    }
    free(tgt);
    return loss;
}
