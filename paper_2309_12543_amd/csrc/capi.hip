// Host-side plumbing of the C ABI: error state, version, grid descriptors.
#include <cstring>

#include "lsdf_internal.hpp"

namespace lsdf {

namespace {
thread_local char g_err[512] = "";
thread_local hipEvent_t g_ev_before = nullptr;
thread_local hipEvent_t g_ev_after = nullptr;
}

void clear_error() { g_err[0] = '\0'; }

void take_kernel_events(hipEvent_t* before, hipEvent_t* after) {
    *before = g_ev_before;
    *after = g_ev_after;
    g_ev_before = g_ev_after = nullptr;
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int prepare_link_grid(const lsdf_grid& g, int index, LinkGrid* out) {
    if (!finite3(g.lo) || !finite3(g.hi))
        return fail(LSDF_E_INVALID_ARG, "grid %d: non-finite box", index);
    if (g.dtype != LSDF_F32 && g.dtype != LSDF_BF16 && g.dtype != LSDF_F16)
        return fail(LSDF_E_UNSUPPORTED, "grid %d: unsupported dtype %d", index, (int)g.dtype);
    if (g.elem_offset < 0) return fail(LSDF_E_INVALID_ARG, "grid %d: negative elem_offset", index);
    for (int a = 0; a < 3; ++a) {
        if (g.n[a] < 2 || g.n[a] > (1 << 24))
            return fail(LSDF_E_SHAPE, "grid %d: n[%d] = %d out of [2, 2^24]", index, a, (int)g.n[a]);
        if (!(g.hi[a] > g.lo[a])) return fail(LSDF_E_INVALID_ARG, "grid %d: hi[%d] <= lo[%d]", index, a, a);
    }
    if ((int64_t)g.n[0] * g.n[1] * g.n[2] > (int64_t)1 << 31)
        return fail(LSDF_E_SHAPE, "grid %d: more than 2^31 nodes", index);
    for (int a = 0; a < 3; ++a) {
        // fixed once in double from the float box, rounded once to float
        const double invh = (double)(g.n[a] - 1) / ((double)g.hi[a] - (double)g.lo[a]);
        out->invh[a] = (float)invh;
        out->half[a] = 0.5f * (float)(g.n[a] - 1);
        out->cen[a] = (float)(-(double)g.lo[a] * (double)out->invh[a] - (double)out->half[a]);
        out->n[a] = g.n[a];
    }
    out->cubic = (g.n[0] == g.n[1] && g.n[1] == g.n[2]) ? 1 : 0;
    out->dtype = g.dtype;
    out->offset = g.elem_offset;
    return LSDF_OK;
}

}  // namespace lsdf

LSDF_API int lsdf_version(void) { return (0 << 16) | (1 << 8) | 0; }

LSDF_API const char* lsdf_last_error(void) { return lsdf::g_err; }

LSDF_API int lsdf_set_kernel_events(void* before, void* after) {
    lsdf::clear_error();
    if ((before == nullptr) != (after == nullptr))
        return lsdf::fail(LSDF_E_INVALID_ARG, "set_kernel_events: give both events or neither");
    lsdf::g_ev_before = static_cast<hipEvent_t>(before);
    lsdf::g_ev_after = static_cast<hipEvent_t>(after);
    return LSDF_OK;
}
