// Standard-DH chain composition shared by the kinematics kernel and the
// fused kinematics-plus-query set-up kernel, so that both produce the same
// pose bits (Sec. III-A: link transformations T_{i,c} from the joint
// angles by forward kinematics).
#pragma once

#include "lsdf_internal.hpp"

namespace lsdf {

// The DH table as the kernels take it (host-side cos / sin of the twist).
struct DhTable {
    float a[LSDF_MAX_DOF], ca[LSDF_MAX_DOF], sa[LSDF_MAX_DOF], d[LSDF_MAX_DOF], off[LSDF_MAX_DOF];
    float base[12];
    int32_t dof;
};

// Validates dh[0..dof) and base_T (NULL = identity) and fills t.
int make_dh_table(const char* who, const lsdf_dh* dh, int32_t dof, const float* base_T, DhTable* t);

// Composes cur <- cur * A(theta) with A = Rz(theta) Tz(d) Tx(a) Rx(alpha):
//   A = [[ct, -st*ca,  st*sa, a*ct],
//        [st,  ct*ca, -ct*sa, a*st],
//        [ 0,     sa,     ca,    d]]
__device__ inline void compose_dh(float (&T)[12], float ct, float st, float ca, float sa, float a, float d) {
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

// Sine and cosine of every joint angle q[j] + offset_j, j < dof.  They do
// not depend on one another or on the chain, so all the loads and all the
// evaluations are issued together rather than one joint at a time.
__device__ inline void joint_sincos(const DhTable& t, const float* q, float (&st)[LSDF_MAX_DOF],
                                    float (&ct)[LSDF_MAX_DOF]) {
    float qv[LSDF_MAX_DOF];
#pragma unroll
    for (int j = 0; j < LSDF_MAX_DOF; ++j)
        if (j < t.dof) qv[j] = q[j];
#pragma unroll
    for (int j = 0; j < LSDF_MAX_DOF; ++j)
        if (j < t.dof) sincosf(qv[j] + t.off[j], &st[j], &ct[j]);
}

// Pose of frame `link` (0 = base) at joint angles q[0..dof): the base
// composed with joints 0 .. link-1, in the order the kinematics kernel uses.
__device__ inline void chain_pose(const DhTable& t, const float* q, int link, float (&T)[12]) {
    float st[LSDF_MAX_DOF], ct[LSDF_MAX_DOF];
    joint_sincos(t, q, st, ct);
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = t.base[k];
#pragma unroll
    for (int j = 0; j < LSDF_MAX_DOF; ++j)
        if (j < link) compose_dh(T, ct[j], st[j], t.ca[j], t.sa[j], t.a[j], t.d[j]);
}

}  // namespace lsdf
