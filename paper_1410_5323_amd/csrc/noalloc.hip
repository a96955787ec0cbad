// noalloc.hip -- crp_propagate without a caller workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// crp_propagate's workspace holds the work-queue head, the field and
// parameter descriptor tables, the longest-first order and the bucket
// counters.  Here that workspace is a fixed array in the library's device
// image, one per GPU the library runs on, held until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (the
// array's name in host code is a host-side stand-in, never a device address)
// and passed to the same kernels crp_propagate launches.
#include <mutex>

#include "crp_internal.h"

namespace crp {
namespace {

constexpr int64_t NOALLOC_MAX_PARTICLES = CRP_NOALLOC_MAX_PARTICLES;
constexpr int32_t NOALLOC_MAX_FIELDS = CRP_NOALLOC_MAX_FIELDS;
constexpr int32_t NOALLOC_MAX_PARAMS = CRP_NOALLOC_MAX_PARAMS;
constexpr size_t SCRATCH_BYTES = ws_layout(NOALLOC_MAX_PARTICLES, NOALLOC_MAX_FIELDS, NOALLOC_MAX_PARAMS).total;

// The workspace of every call on this device: the queue head and bucket
// counters are cleared by each call (fill kernels), the tables and the order
// are rewritten, so nothing depends on what a previous call left.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void *g_scratch[MAX_DEVICES];  // device address of scratch, per device (null until taken)

// Device address of this device's scratch array, taken on the first call
// with the device current.
crp_status scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(CRP_ERR_DEVICE, "crp_propagate_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= MAX_DEVICES) return report(CRP_ERR_UNSUPPORTED, "crp_propagate_noalloc: device id >= 64");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return report(CRP_ERR_DEVICE, "crp_propagate_noalloc: hipGetSymbolAddress of the scratch array failed");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return CRP_OK;
}

}  // namespace
}  // namespace crp

extern "C" {

size_t crp_noalloc_scratch_bytes(void) { return crp::SCRATCH_BYTES; }

crp_status crp_propagate_noalloc(const crp_field *fields, int32_t n_fields, const crp_params *params,
                                 int32_t n_params, const crp_particles *p, int64_t n, const crp_tape *tape,
                                 int32_t precision, const crp_tuning *tuning, int64_t *counters, void *stream) {
    const char *fn = "crp_propagate_noalloc";
    if (n < 0 || n > crp::NOALLOC_MAX_PARTICLES)
        return crp::report(CRP_ERR_INVALID, "crp_propagate_noalloc: n must be in [0, CRP_NOALLOC_MAX_PARTICLES]");
    if (!fields || n_fields < 1 || n_fields > crp::NOALLOC_MAX_FIELDS)
        return crp::report(CRP_ERR_INVALID, "crp_propagate_noalloc: need 1..CRP_NOALLOC_MAX_FIELDS fields");
    if (!params || n_params < 1 || n_params > crp::NOALLOC_MAX_PARAMS)
        return crp::report(CRP_ERR_INVALID, "crp_propagate_noalloc: need 1..CRP_NOALLOC_MAX_PARAMS params");
    crp::FieldDev fd[crp::NOALLOC_MAX_FIELDS];
    crp::ParamsDev pd[crp::NOALLOC_MAX_PARAMS];
    // every argument is checked before the device is touched
    crp_status st = crp::propagate_impl(fn, fields, n_fields, params, n_params, p, n, tape, precision, tuning,
                                        counters, nullptr, 0, stream, fd, pd, true);
    if (st != CRP_OK || n == 0) return st;
    void *ws = nullptr;
    st = crp::scratch_ptr(&ws);
    if (st != CRP_OK) return st;
    return crp::propagate_impl(fn, fields, n_fields, params, n_params, p, n, tape, precision, tuning, counters, ws,
                               crp::SCRATCH_BYTES, stream, fd, pd, false);
}

}  // extern "C"
