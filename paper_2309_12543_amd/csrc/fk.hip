// Batched forward kinematics (Sec. III-A: link poses T_{i,c} for every
// configuration, computed in parallel).  One lane per configuration; the DH
// table travels in the kernel-argument segment.
#include "lsdf_internal.hpp"

namespace {

struct FkArgs {
    float a[LSDF_MAX_DOF], ca[LSDF_MAX_DOF], sa[LSDF_MAX_DOF], d[LSDF_MAX_DOF], off[LSDF_MAX_DOF];
    float base[12];
    const float* q;
    float* out;
    int32_t C;
    int32_t dof;
};

// Composes cur <- cur * A(theta) with A = Rz(theta) Tz(d) Tx(a) Rx(alpha):
//   A = [[ct, -st*ca,  st*sa, a*ct],
//        [st,  ct*ca, -ct*sa, a*st],
//        [ 0,     sa,     ca,    d]]
__device__ inline void compose_dh(float (&T)[12], float ct, float st, float ca, float sa, float a,
                                  float d) {
    float r[12];
#pragma unroll
    for (int row = 0; row < 3; ++row) {
        const float t0 = T[4 * row + 0], t1 = T[4 * row + 1], t2 = T[4 * row + 2], t3 = T[4 * row + 3];
        r[4 * row + 0] = t0 * ct + t1 * st;
        r[4 * row + 1] = (t1 * ct - t0 * st) * ca + t2 * sa;
        r[4 * row + 2] = (t0 * st - t1 * ct) * sa + t2 * ca;
        r[4 * row + 3] = r[4 * row + 0] * a + t2 * d + t3;
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = r[k];
}

__global__ __launch_bounds__(256) void fk_kernel(FkArgs p) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.C) return;
    float T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = p.base[k];
    float* out = p.out + (int64_t)c * (p.dof + 1) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = T[k];
    const float* q = p.q + (int64_t)c * p.dof;
    for (int j = 0; j < p.dof; ++j) {
        float st, ct;
        sincosf(q[j] + p.off[j], &st, &ct);
        compose_dh(T, ct, st, p.ca[j], p.sa[j], p.a[j], p.d[j]);
        float* o = out + 12 * (j + 1);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = T[k];
    }
}

}  // namespace

LSDF_API int lsdf_fk_batch(const lsdf_dh* dh, int32_t dof, const float* base_T, const float* q,
                           int32_t C, float* link_T, void* stream) {
    using namespace lsdf;
    clear_error();
    if (!dh) return fail(LSDF_E_INVALID_ARG, "fk_batch: dh is NULL");
    if (dof < 1 || dof > LSDF_MAX_DOF) return fail(LSDF_E_SHAPE, "fk_batch: dof = %d out of [1, %d]", (int)dof, LSDF_MAX_DOF);
    if (C < 0) return fail(LSDF_E_SHAPE, "fk_batch: C = %d < 0", (int)C);
    if (C > 0 && (!q || !link_T)) return fail(LSDF_E_INVALID_ARG, "fk_batch: q or link_T is NULL");
    FkArgs p{};
    for (int j = 0; j < dof; ++j) {
        const lsdf_dh& r = dh[j];
        if (!std::isfinite(r.a) || !std::isfinite(r.alpha) || !std::isfinite(r.d) || !std::isfinite(r.theta_offset))
            return fail(LSDF_E_INVALID_ARG, "fk_batch: non-finite DH row %d", j);
        p.a[j] = r.a;
        p.d[j] = r.d;
        p.off[j] = r.theta_offset;
        // cos/sin of the fixed twist: computed once on the host in double
        p.ca[j] = (float)std::cos((double)r.alpha);
        p.sa[j] = (float)std::sin((double)r.alpha);
    }
    for (int k = 0; k < 12; ++k) p.base[k] = (k % 5 == 0) ? 1.0f : 0.0f;  // identity [I | 0]
    if (base_T) {
        for (int k = 0; k < 12; ++k) {
            if (!std::isfinite(base_T[k])) return fail(LSDF_E_INVALID_ARG, "fk_batch: non-finite base_T");
            p.base[k] = base_T[k];
        }
    }
    if (C == 0) return LSDF_OK;
    p.q = q;
    p.out = link_T;
    p.C = C;
    p.dof = dof;
    const int threads = 64;
    hipLaunchKernelGGL(fk_kernel, dim3((C + threads - 1) / threads), dim3(threads), 0, as_stream(stream), p);
    return check_launch("fk_batch");
}
