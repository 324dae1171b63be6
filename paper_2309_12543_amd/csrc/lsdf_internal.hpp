// Internal helpers shared by the HIP translation units of liblsdf.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "lsdf.h"

#define LSDF_API extern "C" __attribute__((visibility("default")))

namespace lsdf {

// Thread-local message of the last failure (lsdf_last_error).
void clear_error();
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

inline int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LSDF_E_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
    return LSDF_OK;
}

inline bool finite3(const float* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---- order-preserving float <-> uint32 map ----------------------------------
// ordered(a) < ordered(b) iff a < b for non-NaN floats (-0 below +0; callers
// canonicalise -0 to +0 first).  Keys in the query workspace are stored
// complemented (~ordered) so that a zero key means "empty" and the
// combining operation is an unsigned atomic max.
__device__ inline uint32_t ordered_bits(float v) {
    uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ inline float from_ordered_bits(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

// Per-link constants of the world-to-grid map, fixed on the host from the
// grid descriptor in double and rounded once to float.  Grid coordinates are
// centred on the box: v_a = u_a - half_a, inside iff |v_a| <= half_a.
struct LinkGrid {
    float invh[3];   // (n_a - 1) / (hi_a - lo_a)
    float cen[3];    // -lo_a * invh_a - half_a
    float half[3];   // (n_a - 1) / 2
    int32_t n[3];
    int32_t dtype;
    int32_t cubic;   // n_x == n_y == n_z
    int64_t offset;  // element offset into the grid buffer
};

int prepare_link_grid(const lsdf_grid& g, int index, LinkGrid* out);

// Events set by lsdf_set_kernel_events for the calling thread's next query
// (both NULL when none); taking them clears the setting.
void take_kernel_events(hipEvent_t* before, hipEvent_t* after);

// Turns the query keys [C][L] into out_dist / out_link / out_link_dist
// (shared by the plain and the learned query); keys == NULL gives +inf and
// -1 everywhere.
int launch_query_finalize(const uint32_t* keys, float* out_dist, int32_t* out_link, float* out_link_dist, int32_t C,
                          int32_t L, hipStream_t s);

// Zeroes n 32-bit words on stream s with a small kernel (no memset node,
// so the call can sit in a captured graph).
int launch_zero_words(uint32_t* w, int64_t n, hipStream_t s);

}  // namespace lsdf
