// Batched forward kinematics (Sec. III-A: link poses T_{i,c} for every
// configuration, computed in parallel).  One lane per configuration; the DH
// table travels in the kernel-argument segment.
#include "fk_chain.hpp"

namespace {

struct FkArgs {
    lsdf::DhTable dh;
    const float* q;
    float* out;
    int32_t C;
};

__global__ __launch_bounds__(256) void fk_kernel(FkArgs p) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.C) return;
    const int dof = p.dh.dof;
    float T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = p.dh.base[k];
    float* out = p.out + (int64_t)c * (dof + 1) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = T[k];
    float st[LSDF_MAX_DOF], ct[LSDF_MAX_DOF];
    lsdf::joint_sincos(p.dh, p.q + (int64_t)c * dof, st, ct);
#pragma unroll
    for (int j = 0; j < LSDF_MAX_DOF; ++j) {
        if (j < dof) {
            lsdf::compose_dh(T, ct[j], st[j], p.dh.ca[j], p.dh.sa[j], p.dh.a[j], p.dh.d[j]);
            float* o = out + 12 * (j + 1);
#pragma unroll
            for (int k = 0; k < 12; ++k) o[k] = T[k];
        }
    }
}

}  // namespace

int lsdf::make_dh_table(const char* who, const lsdf_dh* dh, int32_t dof, const float* base_T, DhTable* t) {
    if (!dh) return fail(LSDF_E_INVALID_ARG, "%s: dh is NULL", who);
    if (dof < 1 || dof > LSDF_MAX_DOF) return fail(LSDF_E_SHAPE, "%s: dof = %d out of [1, %d]", who, (int)dof, LSDF_MAX_DOF);
    *t = DhTable{};
    for (int j = 0; j < dof; ++j) {
        const lsdf_dh& r = dh[j];
        if (!std::isfinite(r.a) || !std::isfinite(r.alpha) || !std::isfinite(r.d) || !std::isfinite(r.theta_offset))
            return fail(LSDF_E_INVALID_ARG, "%s: non-finite DH row %d", who, j);
        t->a[j] = r.a;
        t->d[j] = r.d;
        t->off[j] = r.theta_offset;
        // cos/sin of the fixed twist: computed once on the host in double
        t->ca[j] = (float)std::cos((double)r.alpha);
        t->sa[j] = (float)std::sin((double)r.alpha);
    }
    for (int k = 0; k < 12; ++k) t->base[k] = (k % 5 == 0) ? 1.0f : 0.0f;  // identity [I | 0]
    if (base_T) {
        for (int k = 0; k < 12; ++k) {
            if (!std::isfinite(base_T[k])) return fail(LSDF_E_INVALID_ARG, "%s: non-finite base_T", who);
            t->base[k] = base_T[k];
        }
    }
    t->dof = dof;
    return LSDF_OK;
}

LSDF_API int lsdf_fk_batch(const lsdf_dh* dh, int32_t dof, const float* base_T, const float* q,
                           int32_t C, float* link_T, void* stream) {
    using namespace lsdf;
    clear_error();
    FkArgs p{};
    int rc = make_dh_table("fk_batch", dh, dof, base_T, &p.dh);
    if (rc != LSDF_OK) return rc;
    if (C < 0) return fail(LSDF_E_SHAPE, "fk_batch: C = %d < 0", (int)C);
    if (C > 0 && (!q || !link_T)) return fail(LSDF_E_INVALID_ARG, "fk_batch: q or link_T is NULL");
    if (C == 0) return LSDF_OK;
    p.q = q;
    p.out = link_T;
    p.C = C;
    const int threads = 64;
    hipLaunchKernelGGL(fk_kernel, dim3((C + threads - 1) / threads), dim3(threads), 0, as_stream(stream), p);
    return check_launch("fk_batch");
}
