// Measurement aid: the rate of trilinear-style gathers (8 corners of a
// random cell of an n^3 FP32 grid, x fastest) that one launch sustains, from
// a grid that fits one XCD's L2 (64^3 = 1 MB), one that does not (the seven
// link grids, about 7 MB) or one that only HBM holds.  The query's in-box
// pairs each gather the same 8 corners, so this is the roof their gathers
// are compared against.
#include "lsdf_internal.hpp"

namespace {

// Integer hash with good avalanche ("lowbias32", C. Wellons).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void gather_roof_kernel(const float* __restrict__ g, int32_t n, int32_t iters,
                                                          int64_t threads, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= threads) return;
    const uint32_t m = (uint32_t)(n - 1);
    const uint32_t cells = m * m * m;
    const int64_t nx = n, nxy = (int64_t)n * n;
    float acc = 0.0f;
    for (int32_t it = 0; it < iters; ++it) {
        const uint32_t h = mix32((uint32_t)t * 0x9e3779b9u + (uint32_t)it * 0x85ebca6bu + 0x165667b1u) % cells;
        const uint32_t ix = h % m, iy = (h / m) % m, iz = h / (m * m);
        const float* c = g + (iz * nxy + iy * nx + ix);
        acc += ((c[0] + c[1]) + (c[nx] + c[nx + 1])) + ((c[nxy] + c[nxy + 1]) + (c[nxy + nx] + c[nxy + nx + 1]));
    }
    out[t] = acc;
}

}  // namespace

LSDF_API int lsdf_gather_roof(const float* grid, int32_t n, int32_t iters, int64_t threads, float* out,
                              void* stream) {
    using namespace lsdf;
    clear_error();
    if (n < 2 || n > 1024) return fail(LSDF_E_SHAPE, "gather_roof: n = %d out of [2, 1024]", (int)n);
    if (iters < 1 || threads < 1 || threads > ((int64_t)1 << 31))
        return fail(LSDF_E_SHAPE, "gather_roof: iters = %d, threads = %lld", (int)iters, (long long)threads);
    if (!grid || !out) return fail(LSDF_E_INVALID_ARG, "gather_roof: NULL device pointer");
    hipLaunchKernelGGL(gather_roof_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, as_stream(stream),
                       grid, n, iters, threads, out);
    return check_launch("gather_roof");
}
