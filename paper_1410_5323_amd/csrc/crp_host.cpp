// crp_host.cpp -- host side of the C ABI declared in include/crp.h.
//
// Validates every argument before anything is enqueued, packs the device
// descriptors, and enqueues the kernels on the caller's stream.  Nothing here
// allocates device memory or blocks on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.h"
#include "crp_internal.h"

namespace {

thread_local std::string g_last_error;

crp_status fail(crp_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
crp_status fail(crp_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

crp_status ok() {
    g_last_error.clear();
    return CRP_OK;
}

crp_status device_error(hipError_t e, const char *what) {
    return fail(CRP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

size_t dtype_size(int32_t d) {
    switch (d) {
        case CRP_F64: return 8;
        case CRP_F32: return 4;
        case CRP_F16: return 2;
        case CRP_BF16: return 2;
        default: return 0;
    }
}

// Checks one field descriptor; data may be NULL only when !need_data.
crp_status check_modulation(const crp_modulation *m, bool need_data, const char *what) {
    if (!m) return fail(CRP_ERR_INVALID, "%s: null modulation descriptor", what);
    for (int a = 0; a < 3; ++a) {
        if (m->n[a] < 2 || m->n[a] > (1 << 20))
            return fail(CRP_ERR_INVALID, "%s: modulation n[%d] = %d out of range [2, 2^20]", what, a, m->n[a]);
        if (!std::isfinite(m->origin[a])) return fail(CRP_ERR_INVALID, "%s: modulation origin not finite", what);
    }
    if (!(m->spacing > 0.0) || !std::isfinite(m->spacing))
        return fail(CRP_ERR_INVALID, "%s: modulation spacing must be finite and > 0", what);
    if (m->dtype != CRP_F64 && m->dtype != CRP_F32)
        return fail(CRP_ERR_INVALID, "%s: modulation dtype must be F64 or F32", what);
    if (((uint64_t)m->n[0] + 1) * ((uint64_t)m->n[1] + 1) * ((uint64_t)m->n[2] + 1) >= (1ull << 32))
        return fail(CRP_ERR_UNSUPPORTED, "%s: modulation grid limited to 2^32 stored values", what);
    if (need_data && !m->data) return fail(CRP_ERR_INVALID, "%s: null modulation data pointer", what);
    return CRP_OK;
}

void fill_modulation_dev(crp::FieldDev &d, const crp_modulation &m) {
    d.mod_data = m.data;
    for (int a = 0; a < 3; ++a) {
        d.mod_n[a] = m.n[a];
        d.mod_origin[a] = m.origin[a];
    }
    d.mod_pow2 = is_pow2(m.n[0]) && is_pow2(m.n[1]) && is_pow2(m.n[2]);
    d.mod_inv_spacing = 1.0 / m.spacing;
    d.mod_sy = (uint32_t)(m.n[2] + 1);
    d.mod_sx = (uint32_t)((m.n[1] + 1) * (m.n[2] + 1));
    d.mod_dtype = m.dtype;
}

crp_status check_field(const crp_field *f, bool need_data, const char *what) {
    if (!f) return fail(CRP_ERR_INVALID, "%s: null field descriptor", what);
    for (int a = 0; a < 3; ++a) {
        if (f->n[a] < 2 || f->n[a] > (1 << 20))
            return fail(CRP_ERR_INVALID, "%s: n[%d] = %d out of range [2, 2^20]", what, a, f->n[a]);
        if (!std::isfinite(f->origin[a])) return fail(CRP_ERR_INVALID, "%s: origin not finite", what);
    }
    if (!(f->spacing > 0.0) || !std::isfinite(f->spacing))
        return fail(CRP_ERR_INVALID, "%s: spacing must be finite and > 0", what);
    if (!(f->value_scale > 0.0) || !std::isfinite(f->value_scale))
        return fail(CRP_ERR_INVALID, "%s: value_scale must be finite and > 0", what);
    if (dtype_size(f->dtype) == 0) return fail(CRP_ERR_INVALID, "%s: unknown dtype %d", what, f->dtype);
    if (f->layout != CRP_LAYOUT_LINEAR && f->layout != CRP_LAYOUT_CELL8)
        return fail(CRP_ERR_INVALID, "%s: unknown layout %d", what, f->layout);
    uint64_t n0 = f->n[0], n1 = f->n[1], n2 = f->n[2];
    if (f->layout == CRP_LAYOUT_LINEAR && 3ull * (n0 + 1) * (n1 + 1) * (n2 + 1) >= (1ull << 32))
        return fail(CRP_ERR_UNSUPPORTED, "%s: LINEAR layout limited to 2^32 stored values", what);
    if (f->layout == CRP_LAYOUT_CELL8 && n0 * n1 * n2 >= (1ull << 32))
        return fail(CRP_ERR_UNSUPPORTED, "%s: CELL8 layout limited to 2^32 cells", what);
    if (need_data && !f->data) return fail(CRP_ERR_INVALID, "%s: null data pointer", what);
    if (need_data && f->modulation) return check_modulation(f->modulation, true, what);
    return CRP_OK;
}

crp::FieldDev make_field_dev(const crp_field &f) {
    crp::FieldDev d;
    std::memset(&d, 0, sizeof d);
    d.data = f.data;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = f.n[a];
        d.origin[a] = f.origin[a];
    }
    d.pow2 = is_pow2(f.n[0]) && is_pow2(f.n[1]) && is_pow2(f.n[2]);
    d.inv_spacing = 1.0 / f.spacing;
    d.value_scale = f.value_scale;
    d.sy = (uint32_t)(f.n[2] + 1);
    d.sx = (uint32_t)((f.n[1] + 1) * (f.n[2] + 1));
    d.cy = (uint32_t)f.n[2];
    d.cx = (uint32_t)((uint64_t)f.n[1] * f.n[2]);
    d.dtype = f.dtype;
    d.layout = f.layout;
    if (f.modulation) fill_modulation_dev(d, *f.modulation);
    return d;
}

crp_status check_params(const crp_params *p, int32_t n_fields, int i) {
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(CRP_ERR_INVALID, "params[%d]: tol must be > 0", i);
    if (!(p->h_min > 0.0) || !std::isfinite(p->h_max) || !(p->h_max >= p->h_min))
        return fail(CRP_ERR_INVALID, "params[%d]: need 0 < h_min <= h_max < inf", i);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->obs_center[a])) return fail(CRP_ERR_INVALID, "params[%d]: centre not finite", i);
    if (!std::isfinite(p->obs_radius)) return fail(CRP_ERR_INVALID, "params[%d]: radius not finite", i);
    if (std::isnan(p->l_max) || !(p->l_max > 0.0))
        return fail(CRP_ERR_INVALID, "params[%d]: l_max must be > 0 (or +inf)", i);
    if (p->max_steps < 0) return fail(CRP_ERR_INVALID, "params[%d]: max_steps < 0", i);
    if (!std::isfinite(p->l_max) && p->max_steps == 0)
        return fail(CRP_ERR_INVALID, "params[%d]: without l_max a max_steps budget is required", i);
    if (std::isfinite(p->l_max) && p->h_min < p->l_max * 1e-14)
        return fail(CRP_ERR_INVALID, "params[%d]: h_min below the FP64 resolution of l_max", i);
    if (p->field_index < 0 || p->field_index >= n_fields)
        return fail(CRP_ERR_INVALID, "params[%d]: field_index %d out of range", i, p->field_index);
    if (p->reflect != 0 && p->reflect != 1) return fail(CRP_ERR_INVALID, "params[%d]: reflect must be 0 or 1", i);
    if (p->backtrack != 0 && p->backtrack != 1)
        return fail(CRP_ERR_INVALID, "params[%d]: backtrack must be 0 or 1", i);
    if (p->reflect)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(p->box_lo[a]) || !std::isfinite(p->box_hi[a]) || !(p->box_lo[a] < p->box_hi[a]))
                return fail(CRP_ERR_INVALID, "params[%d]: reflective box needs finite lo < hi on every axis", i);
    return CRP_OK;
}

crp::ParamsDev make_params_dev(const crp_params &p) {
    crp::ParamsDev d;
    std::memset(&d, 0, sizeof d);
    d.tol = p.tol;
    d.h_min = p.h_min;
    d.h_max = p.h_max;
    for (int a = 0; a < 3; ++a) d.center[a] = p.obs_center[a];
    d.radius = p.obs_radius;
    d.r2 = p.obs_radius * p.obs_radius;
    d.l_max = p.l_max;
    d.max_steps = p.max_steps;
    d.field_index = p.field_index;
    d.sphere_on = p.obs_radius > 0.0;
    d.lmax_on = std::isfinite(p.l_max);
    d.reflect_on = p.reflect != 0;
    d.backtrack_on = p.backtrack != 0;
    for (int a = 0; a < 3; ++a) {
        d.box_lo[a] = p.box_lo[a];
        d.box_hi[a] = p.box_hi[a];
    }
    return d;
}

int cu_count() {
    static thread_local int dev_cached = -1, cus_cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != dev_cached) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        dev_cached = dev;
        cus_cached = cus;
    }
    return cus_cached;
}

}  // namespace

namespace crp {

crp_status report(crp_status st, const char *msg) {
    if (st == CRP_OK) return ok();
    return fail(st, "%s", msg);
}

}  // namespace crp

extern "C" {

const char *crp_last_error(void) { return g_last_error.c_str(); }

const char *crp_version(void) { return "crp-mi355x 0.1 (gfx950)"; }

size_t crp_field_bytes(const crp_field *f) {
    if (check_field(f, false, "crp_field_bytes") != CRP_OK) return 0;
    uint64_t n0 = f->n[0], n1 = f->n[1], n2 = f->n[2];
    uint64_t vals = f->layout == CRP_LAYOUT_CELL8 ? n0 * n1 * n2 * 32ull : 3ull * (n0 + 1) * (n1 + 1) * (n2 + 1);
    return (size_t)(vals * dtype_size(f->dtype));
}

crp_status crp_field_upload(const crp_field *f, const void *src, int32_t src_dtype, void *stream) {
    crp_status st = check_field(f, true, "crp_field_upload");
    if (st != CRP_OK) return st;
    if (!src) return fail(CRP_ERR_INVALID, "crp_field_upload: null source");
    if (src_dtype != CRP_F64 && src_dtype != CRP_F32)
        return fail(CRP_ERR_INVALID, "crp_field_upload: source dtype must be F64 or F32");
    uint64_t src_bytes = 3ull * f->n[0] * f->n[1] * f->n[2] * dtype_size(src_dtype);
    const char *s0 = static_cast<const char *>(src);
    const char *d0 = static_cast<const char *>(f->data);
    if (s0 < d0 + crp_field_bytes(f) && d0 < s0 + src_bytes)
        return fail(CRP_ERR_INVALID, "crp_field_upload: source and destination overlap");
    crp::FieldDev d = make_field_dev(*f);
    hipError_t e = crp::launch_upload(d, src, src_dtype, f->data, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_field_upload");
    return ok();
}

size_t crp_modulation_bytes(const crp_modulation *m) {
    if (check_modulation(m, false, "crp_modulation_bytes") != CRP_OK) return 0;
    uint64_t vals = ((uint64_t)m->n[0] + 1) * ((uint64_t)m->n[1] + 1) * ((uint64_t)m->n[2] + 1);
    return (size_t)(vals * dtype_size(m->dtype));
}

crp_status crp_modulation_upload(const crp_modulation *m, const void *src, int32_t src_dtype, void *stream) {
    crp_status st = check_modulation(m, true, "crp_modulation_upload");
    if (st != CRP_OK) return st;
    if (!src) return fail(CRP_ERR_INVALID, "crp_modulation_upload: null source");
    if (src_dtype != CRP_F64 && src_dtype != CRP_F32)
        return fail(CRP_ERR_INVALID, "crp_modulation_upload: source dtype must be F64 or F32");
    size_t sb = (size_t)m->n[0] * m->n[1] * m->n[2] * dtype_size(src_dtype);
    size_t db = crp_modulation_bytes(m);
    const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(m->data);
    if (a < b + db && b < a + sb) return fail(CRP_ERR_INVALID, "crp_modulation_upload: source and destination overlap");
    if (cu_count() <= 0) return fail(CRP_ERR_DEVICE, "crp_modulation_upload: no HIP device available");
    crp::FieldDev d;
    std::memset(&d, 0, sizeof d);
    fill_modulation_dev(d, *m);
    hipError_t e = crp::launch_upload_modulation(d, src, src_dtype, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_modulation_upload");
    return ok();
}

size_t crp_workspace_bytes(int64_t n, int32_t n_fields, int32_t n_params) {
    if (n < 0 || n_fields < 1 || n_params < 1) return 0;
    return crp::ws_layout(n, n_fields, n_params).total;
}

crp_status crp_propagate(const crp_field *fields, int32_t n_fields, const crp_params *params, int32_t n_params,
                         const crp_particles *p, int64_t n, const crp_tape *tape, int32_t precision,
                         const crp_tuning *tuning, int64_t *counters, void *workspace, size_t workspace_bytes,
                         void *stream) {
    if (!fields || n_fields < 1 || n_fields > 4096) return fail(CRP_ERR_INVALID, "crp_propagate: need 1..4096 fields");
    if (!params || n_params < 1 || n_params > 65536)
        return fail(CRP_ERR_INVALID, "crp_propagate: need 1..65536 params");
    std::vector<crp::FieldDev> fd(n_fields);
    std::vector<crp::ParamsDev> pd(n_params);
    return crp::propagate_impl("crp_propagate", fields, n_fields, params, n_params, p, n, tape, precision, tuning,
                               counters, workspace, workspace_bytes, stream, fd.data(), pd.data(), false);
}

}  // extern "C"

namespace crp {

crp_status propagate_impl(const char *fn, const crp_field *fields, int32_t n_fields, const crp_params *params,
                          int32_t n_params, const crp_particles *p, int64_t n, const crp_tape *tape,
                          int32_t precision, const crp_tuning *tuning, int64_t *counters, void *workspace,
                          size_t workspace_bytes, void *stream, FieldDev *fd, ParamsDev *pd, bool check_only) {
    if (!fields || n_fields < 1 || n_fields > 4096) return fail(CRP_ERR_INVALID, "%s: need 1..4096 fields", fn);
    if (!params || n_params < 1 || n_params > 65536) return fail(CRP_ERR_INVALID, "%s: need 1..65536 params", fn);
    if (!p) return fail(CRP_ERR_INVALID, "%s: null particles", fn);
    if (n < 0 || n > (int64_t)0x7fffffff) return fail(CRP_ERR_INVALID, "%s: n = %lld out of range", fn, (long long)n);
    for (int i = 0; i < n_fields; ++i) {
        crp_status st = check_field(&fields[i], true, fn);
        if (st != CRP_OK) return st;
        if (fields[i].dtype != fields[0].dtype || fields[i].layout != fields[0].layout)
            return fail(CRP_ERR_INVALID, "%s: all fields of one call must share dtype and layout", fn);
    }
    for (int i = 0; i < n_params; ++i) {
        crp_status st = check_params(&params[i], n_fields, i);
        if (st != CRP_OK) return st;
    }
    if (n > 0 && (!p->x || !p->y || !p->z || !p->ux || !p->uy || !p->uz || !p->energy || !p->charge ||
                  !p->length || !p->h_next || !p->status || !p->n_accepted || !p->n_rejected))
        return fail(CRP_ERR_INVALID, "%s: a required particle array is null", fn);
    if (n > 0 && n_params > 1 && !p->param_index)
        return fail(CRP_ERR_INVALID, "%s: param_index is required with several parameter groups", fn);
    if (precision != CRP_PREC_FP64 && precision != CRP_PREC_MIXED_F64ACC && precision != CRP_PREC_MIXED_DFACC)
        return fail(CRP_ERR_INVALID, "%s: unknown precision %d", fn, precision);
    bool modulated = false;
    for (int i = 0; i < n_fields; ++i) modulated = modulated || fields[i].modulation != nullptr;
    if (modulated && precision == CRP_PREC_FP64 && fields[0].dtype != CRP_F64 && fields[0].dtype != CRP_F32)
        return fail(CRP_ERR_UNSUPPORTED, "%s: modulated fields in FP64 precision need F64 or F32 storage", fn);
    bool reflective = false;
    for (int i = 0; i < n_params; ++i) reflective = reflective || params[i].reflect != 0;
    if (tape) {
        if (precision != CRP_PREC_FP64) return fail(CRP_ERR_UNSUPPORTED, "%s: a tape needs FP64 precision", fn);
        if (n_params > 1 || (n > 0 && p->param_index) || n_fields > 1)
            return fail(CRP_ERR_UNSUPPORTED, "%s: a tape is recorded for one field and one parameter group", fn);
        if (fields[0].dtype != CRP_F64 && fields[0].dtype != CRP_F32)
            return fail(CRP_ERR_UNSUPPORTED, "%s: a tape needs an F64 or F32 field", fn);
        if (tape->every_k < 1 || tape->every_k > 4096)
            return fail(CRP_ERR_INVALID, "%s: tape interval must be in [1, 4096]", fn);
        if (tape->capacity < 1) return fail(CRP_ERR_INVALID, "%s: the tape needs at least one record", fn);
        if (n > 0 && (!tape->head || !tape->finals || !tape->checkpoints || !tape->links))
            return fail(CRP_ERR_INVALID, "%s: tape arrays must not be null", fn);
    }
    crp_tuning t = {256, 4, 32, 1, 0, 0, nullptr};
    if (tuning) t = *tuning;
    if (t.block_size != 64 && t.block_size != 128 && t.block_size != 256)
        return fail(CRP_ERR_INVALID, "%s: block_size must be 64, 128 or 256", fn);
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64)
        return fail(CRP_ERR_INVALID, "%s: blocks_per_cu must be in [0, 64]", fn);
    if (t.refill_threshold < 1 || t.refill_threshold > 64)
        return fail(CRP_ERR_INVALID, "%s: refill_threshold must be in [1, 64]", fn);
    if (t.cache_cells < -1 || t.cache_cells > 1)
        return fail(CRP_ERR_INVALID, "%s: cache_cells must be -1, 0 or 1", fn);
    crp::WsLayout wl = crp::ws_layout(n, n_fields, n_params);
    if (n == 0 || check_only) return ok();
    if (!workspace || workspace_bytes < wl.total)
        return fail(CRP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed, %zu given", fn, wl.total,
                    workspace ? workspace_bytes : (size_t)0);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(CRP_ERR_WORKSPACE, "%s: workspace must be 256-byte aligned", fn);

    int cus = cu_count();
    if (cus <= 0) return fail(CRP_ERR_DEVICE, "%s: no HIP device available", fn);

    hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    for (int i = 0; i < n_fields; ++i) fd[i] = make_field_dev(fields[i]);
    for (int i = 0; i < n_params; ++i) pd[i] = make_params_dev(params[i]);
    hipError_t e = crp::launch_write_table(ws + wl.fields, fd, size_t(n_fields) * sizeof(crp::FieldDev), s);
    if (e == hipSuccess) e = crp::launch_write_table(ws + wl.params, pd, size_t(n_params) * sizeof(crp::ParamsDev), s);
    if (e == hipSuccess) e = crp::launch_fill_u64(reinterpret_cast<unsigned long long *>(ws), 0ull, 1, s);
    int32_t *order = nullptr;
    if (e == hipSuccess && t.order_by_rigidity) {
        order = reinterpret_cast<int32_t *>(ws + wl.order);
        e = crp::launch_order_by_rigidity(p->energy, p->charge, p->status, n, order,
                                          reinterpret_cast<unsigned int *>(ws + wl.buckets), s);
    }
    if (e != hipSuccess) return device_error(e, fn);

    crp::PropArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = p->x;
    a.y = p->y;
    a.z = p->z;
    a.ux = p->ux;
    a.uy = p->uy;
    a.uz = p->uz;
    a.energy = p->energy;
    a.charge = p->charge;
    a.length = p->length;
    a.h_next = p->h_next;
    a.time = p->time;
    a.status = p->status;
    a.param_index = p->param_index;
    a.n_acc = p->n_accepted;
    a.n_rej = p->n_rejected;
    a.n = n;
    a.fields = reinterpret_cast<const crp::FieldDev *>(ws + wl.fields);
    a.params = reinterpret_cast<const crp::ParamsDev *>(ws + wl.params);
    a.F0 = fd[params[0].field_index];  // the field of the single parameter group
    a.P0 = pd[0];
    a.order = order;
    a.queue = reinterpret_cast<unsigned long long *>(ws);
    a.counters = reinterpret_cast<unsigned long long *>(counters);
    a.refill_threshold = t.refill_threshold;
    a.n_params = n_params;
    a.modulated = modulated ? 1 : 0;
    a.reflective = reflective ? 1 : 0;
    a.cancel = t.cancel;
    a.tape_ckpt = tape ? tape->checkpoints : nullptr;
    a.tape_link = tape ? tape->links : nullptr;
    a.tape_head = tape ? tape->head : nullptr;
    a.tape_fin = tape ? tape->finals : nullptr;
    a.tape_cap = tape ? tape->capacity : 0;
    a.tape_k = tape ? tape->every_k : 1;

    int64_t need_blocks = (n + t.block_size - 1) / t.block_size;
    int64_t blocks = t.blocks_per_cu == 0 ? need_blocks : (int64_t)cus * t.blocks_per_cu;
    if (blocks > need_blocks) blocks = need_blocks;
    bool multi = n_params > 1 || p->param_index != nullptr;
    // Cell cache (the last cell's values in each lane's registers, or in LDS
    // for the FP64 kernel with per-particle groups), automatic.  The LINEAR
    // layout spreads a cell over several lines and gains.  A CELL8 record is
    // one line; there the cache pays only with more than 2048 particles per
    // compute unit: then the texture path is congested, and skipping it
    // shortens the longest trajectories' dependent lookups, which set the
    // launch time.  With fewer particles its extra instructions cost more than
    // the queues it avoids (measured break-even between 2000 and 2900
    // particles per compute unit).
    const bool cache_auto = fields[0].layout == CRP_LAYOUT_LINEAR || n > 2048 * (int64_t)cus;
    const bool cache = t.cache_cells == 0 ? cache_auto : t.cache_cells > 0;
    if (precision == CRP_PREC_FP64)
        e = crp::launch_propagate_fp64(a, fields[0].dtype, fields[0].layout, multi, cache, (int)blocks,
                                       t.block_size, s);
    else
        e = crp::launch_propagate_mixed(a, fields[0].dtype, fields[0].layout, multi, precision, cache, (int)blocks,
                                        t.block_size, s);
    if (e != hipSuccess) return device_error(e, fn);
    return ok();
}

}  // namespace crp

extern "C" {

// Threads of the adjoint's sweep launch (each keeps a column of replay
// records): at most 16384, one wavefront per compute unit of an MI355X.  The
// sweep runs one wavefront per SIMD at most (it takes all 512 registers), and
// wavefronts sharing a compute unit slow each other down more than they add:
// on a 1e5-particle workload with parallel replay the sweep took 1333 ms with
// 65536 threads, 992 with 32768, 907 with 24576, 852 with 16384, 899 with
// 12288 and 1051 with 8192.
static int64_t adjoint_lanes(int64_t n) { return n < 16384 ? ((n + 63) / 64) * 64 : 16384; }

size_t crp_adjoint_replay_workspace_bytes(int64_t n, int32_t every_k, int64_t replay_steps) {
    if (n < 0 || every_k < 1 || every_k > 4096 || replay_steps < 0) return 0;
    return crp::adjoint_ws_layout(n, every_k, adjoint_lanes(n), replay_steps).total;
}

size_t crp_adjoint_workspace_bytes(int64_t n, int32_t every_k) {
    return crp_adjoint_replay_workspace_bytes(n, every_k, 0);
}

crp_status crp_propagate_adjoint(const crp_field *field, const crp_params *params, const crp_particles *initial,
                                 int64_t n, const crp_tape *tape, const double *gbar_dir, const double *gbar_time,
                                 const double *gbar_energy, double *grad_u0, double *grad_x0, double *grad_energy,
                                 void *grad_field, int32_t grad_dtype,
                                 void *workspace, size_t workspace_bytes, void *stream) {
    const char *fn = "crp_propagate_adjoint";
    crp_status st = check_field(field, true, fn);
    if (st != CRP_OK) return st;
    if (field->dtype != CRP_F64 && field->dtype != CRP_F32)
        return fail(CRP_ERR_UNSUPPORTED, "%s: the adjoint reads F64 or F32 grids", fn);
    if (!params) return fail(CRP_ERR_INVALID, "%s: null params", fn);
    st = check_params(params, 1, 0);
    if (st != CRP_OK) return st;
    if (!initial || !tape) return fail(CRP_ERR_INVALID, "%s: null particles or tape", fn);
    if (n < 0 || n > (int64_t)0x7fffffff) return fail(CRP_ERR_INVALID, "%s: n out of range", fn);
    if (grad_dtype != CRP_F64 && grad_dtype != CRP_F32)
        return fail(CRP_ERR_INVALID, "%s: grad_dtype must be CRP_F64 or CRP_F32", fn);
    if (tape->every_k < 1 || tape->every_k > 4096) return fail(CRP_ERR_INVALID, "%s: bad tape interval", fn);
    if (n == 0) return ok();
    if (tape->capacity < 1) return fail(CRP_ERR_INVALID, "%s: the tape needs at least one record", fn);
    if (!initial->ux || !initial->uy || !initial->uz || !initial->energy || !initial->charge || !tape->finals ||
        !tape->checkpoints || !tape->links || !gbar_dir || !grad_u0 || !grad_field)
        return fail(CRP_ERR_INVALID, "%s: a required array is null", fn);
    int64_t lanes = adjoint_lanes(n);
    size_t need = crp::adjoint_ws_layout(n, tape->every_k, lanes, 0).total;
    if (!workspace || workspace_bytes < need)
        return fail(CRP_ERR_WORKSPACE, "%s: workspace of %zu bytes needed", fn, need);
    // the parallel-replay space: the most records the rest of the workspace
    // holds (at most 2^36, 40 TB of records, which keeps every size and grid
    // dimension derived from it in range)
    int64_t lo = 0, hi = (int64_t)(workspace_bytes / (8 * crp::ADJ_RECORD_DOUBLES));
    if (hi > ((int64_t)1 << 36)) hi = (int64_t)1 << 36;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (crp::adjoint_ws_layout(n, tape->every_k, lanes, mid).total <= workspace_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    const crp::AdjWs L = crp::adjoint_ws_layout(n, tape->every_k, lanes, lo);
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(CRP_ERR_WORKSPACE, "%s: workspace alignment", fn);
    if (cu_count() <= 0) return fail(CRP_ERR_DEVICE, "%s: no HIP device available", fn);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    crp::AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.F = make_field_dev(*field);
    a.P = make_params_dev(*params);
    a.x0 = initial->x;
    a.y0 = initial->y;
    a.z0 = initial->z;
    a.ux0 = initial->ux;
    a.uy0 = initial->uy;
    a.uz0 = initial->uz;
    a.energy = initial->energy;
    a.charge = initial->charge;
    a.ckpt = tape->checkpoints;
    a.link = tape->links;
    a.fin = tape->finals;
    a.fin_out = tape->finals;
    a.cap = tape->capacity;
    a.K = tape->every_k;
    a.gbar_dir = gbar_dir;
    a.gbar_time = gbar_time;
    a.gbar_energy = gbar_energy;
    a.grad_u0 = grad_u0;
    a.grad_x0 = grad_x0;
    a.grad_energy = grad_energy;
    a.grad_field = grad_field;
    a.grad_f32 = grad_dtype == CRP_F32;
    a.segbuf = reinterpret_cast<double *>(ws + L.seg);
    a.lanes = lanes;
    a.queue = reinterpret_cast<unsigned long long *>(ws);
    a.order = reinterpret_cast<const int32_t *>(ws + L.order);
    a.n = n;
    a.R = L.R;
    a.rows = L.rows;
    if (L.R > 0) {
        a.grp_rec = reinterpret_cast<int64_t *>(ws + L.grp_rec);
        a.grp_row = reinterpret_cast<int64_t *>(ws + L.grp_row);
        a.pre_ok = reinterpret_cast<int32_t *>(ws + L.pre_ok);
        a.seg_slot = reinterpret_cast<int64_t *>(ws + L.seg_slot);
        a.prerec = reinterpret_cast<double *>(ws + L.prerec);
        a.prebar = reinterpret_cast<double *>(ws + L.prebar);
    }
    // queue head and parallel-replay cuts (0: none) cleared by a fill kernel
    hipError_t e = crp::launch_fill_u64(a.queue, 0ull, 3, s);
    if (e == hipSuccess)
        e = crp::launch_order_by_steps(tape->finals, n, reinterpret_cast<int32_t *>(ws + L.order),
                                       reinterpret_cast<unsigned int *>(ws + L.buckets), s);
    if (e == hipSuccess) e = crp::launch_adjoint_fp64(a, (int)(lanes / 64), s);
    if (e != hipSuccess) return device_error(e, fn);
    return ok();
}

struct crp_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

crp_status crp_graph_create(const crp_field *fields, int32_t n_fields, const crp_params *params, int32_t n_params,
                            const crp_particles *p, int64_t n, int32_t precision, const crp_tuning *tuning,
                            int64_t *counters, void *workspace, size_t workspace_bytes, void *stream,
                            crp_graph **out) {
    const char *fn = "crp_graph_create";
    if (!out) return fail(CRP_ERR_INVALID, "%s: null output handle", fn);
    *out = nullptr;
    if (!stream) return fail(CRP_ERR_INVALID, "%s: capture needs a non-default stream", fn);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_error(e, fn);
    crp_status st = crp_propagate(fields, n_fields, params, n_params, p, n, nullptr, precision, tuning, counters,
                                  workspace, workspace_bytes, stream);
    std::string msg = g_last_error;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st != CRP_OK) {
        if (graph) hipGraphDestroy(graph);
        g_last_error = msg;
        return st;
    }
    if (e != hipSuccess) return device_error(e, fn);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return device_error(e, fn);
    }
    *out = new crp_graph{graph, exec};
    return ok();
}

crp_status crp_graph_launch(crp_graph *g, void *stream) {
    if (!g) return fail(CRP_ERR_INVALID, "crp_graph_launch: null graph");
    hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_graph_launch");
    return ok();
}

crp_status crp_graph_destroy(crp_graph *g) {
    if (!g) return ok();
    hipError_t e1 = hipGraphExecDestroy(g->exec);
    hipError_t e2 = hipGraphDestroy(g->graph);
    delete g;
    if (e1 != hipSuccess) return device_error(e1, "crp_graph_destroy");
    if (e2 != hipSuccess) return device_error(e2, "crp_graph_destroy");
    return ok();
}

crp_status crp_selftest_arith(const double *in, double *out, int64_t n, int32_t op, void *stream) {
    if (n < 0) return fail(CRP_ERR_INVALID, "crp_selftest_arith: n < 0");
    if (n > 0 && (!in || !out)) return fail(CRP_ERR_INVALID, "crp_selftest_arith: null pointer");
    if (op < 0 || op > 6) return fail(CRP_ERR_INVALID, "crp_selftest_arith: unknown op %d", op);
    hipError_t e = crp::launch_selftest(in, out, n, op, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_selftest_arith");
    return ok();
}

crp_status crp_bench_gather(const crp_field *f, int64_t lanes, int64_t lookups_per_lane, double spread,
                            uint64_t seed, double *sink, void *stream) {
    crp_status st = check_field(f, true, "crp_bench_gather");
    if (st != CRP_OK) return st;
    if (lanes < 1 || lanes > (int64_t)1 << 30 || lookups_per_lane < 0 || !sink || !std::isfinite(spread))
        return fail(CRP_ERR_INVALID, "crp_bench_gather: bad lanes, lookups, spread or sink");
    hipError_t e = crp::launch_gather_bench(make_field_dev(*f), lanes, lookups_per_lane, spread, (uint32_t)seed,
                                            sink, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_bench_gather");
    return ok();
}

crp_status crp_bench_gather_replay(const crp_field *f, const double *rec, int64_t lanes, int64_t steps,
                                   int32_t cache_cells, double *sink, int64_t *misses, void *stream) {
    crp_status st = check_field(f, true, "crp_bench_gather_replay");
    if (st != CRP_OK) return st;
    if (f->dtype != CRP_F64 && f->dtype != CRP_F32)
        return fail(CRP_ERR_UNSUPPORTED, "crp_bench_gather_replay: F64 or F32 grids only");
    if (lanes < 1 || lanes > (int64_t)1 << 30 || steps < 0 || !rec || !sink || (cache_cells != 0 && cache_cells != 1))
        return fail(CRP_ERR_INVALID, "crp_bench_gather_replay: bad lanes, steps, records, cache flag or sink");
    hipError_t e = crp::launch_gather_replay(make_field_dev(*f), rec, lanes, steps, cache_cells != 0, sink, misses,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_bench_gather_replay");
    return ok();
}

crp_status crp_bench_stream(const void *src, void *dst, size_t bytes, double *sink, int32_t blocks, void *stream) {
    if (!src || bytes < 16 || (bytes & 15) || blocks < 1 || blocks > (1 << 20) || (!dst && !sink))
        return fail(CRP_ERR_INVALID, "crp_bench_stream: bad arguments");
    if (reinterpret_cast<uintptr_t>(src) & 15 || reinterpret_cast<uintptr_t>(dst) & 15)
        return fail(CRP_ERR_INVALID, "crp_bench_stream: buffers must be 16-byte aligned");
    hipError_t e = crp::launch_stream(src, dst, bytes, sink, blocks, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, "crp_bench_stream");
    return ok();
}

crp_status crp_healpix_pixels(int32_t nside, const double *ux, const double *uy, const double *uz, int64_t n,
                              int32_t *pix, void *stream) {
    const char *fn = "crp_healpix_pixels";
    if (nside < 1 || nside > 8192) return fail(CRP_ERR_INVALID, "%s: nside must be in [1, 8192]", fn);
    if (n < 0 || n > (int64_t)1 << 40) return fail(CRP_ERR_INVALID, "%s: n out of range", fn);
    if (n > 0 && (!ux || !uy || !uz || !pix)) return fail(CRP_ERR_INVALID, "%s: null pointer", fn);
    hipError_t e = crp::launch_healpix(nside, ux, uy, uz, n, 1.0, pix, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, fn);
    return ok();
}

size_t crp_lens_workspace_bytes(int32_t nside, int64_t n) {
    if (nside < 1 || nside > 1024 || n < 0 || n > (int64_t)0x7fffffff) return 0;
    return crp::lens_ws_layout(nside, n).total;
}

crp_status crp_lens_build(int32_t nside, const int32_t *row, const double *ux, const double *uy, const double *uz,
                          const int32_t *status, int64_t n, int64_t *row_ptr, int32_t *col, float *val,
                          int64_t capacity, int64_t *nnz, void *workspace, size_t workspace_bytes, void *stream) {
    const char *fn = "crp_lens_build";
    if (nside < 1 || nside > 1024) return fail(CRP_ERR_INVALID, "%s: nside must be in [1, 1024]", fn);
    if (n < 0 || n > (int64_t)0x7fffffff) return fail(CRP_ERR_INVALID, "%s: n out of range", fn);
    if (!row_ptr || !nnz) return fail(CRP_ERR_INVALID, "%s: null row_ptr or nnz", fn);
    if (n > 0 && (!row || !ux || !uy || !uz || !status || !col || !val))
        return fail(CRP_ERR_INVALID, "%s: null pointer", fn);
    if (capacity < n) return fail(CRP_ERR_INVALID, "%s: capacity must be at least n", fn);
    const crp::LensWs wl = crp::lens_ws_layout(nside, n);
    if (!workspace || workspace_bytes < wl.total)
        return fail(CRP_ERR_WORKSPACE, "%s: need %zu workspace bytes", fn, wl.total);
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(CRP_ERR_WORKSPACE, "%s: workspace alignment", fn);
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    hipError_t e = crp::launch_lens_build(nside, row, ux, uy, uz, status, n, row_ptr, col, val, ws, s);
    uint32_t flag = 0;
    int64_t total = 0;
    const int64_t npix = 12 * (int64_t)nside * nside;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, ws + wl.flag, sizeof flag, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&total, row_ptr + npix, sizeof total, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(e, fn);
    *nnz = total;
    if (flag & 1u) return fail(CRP_ERR_INVALID, "%s: a row index is outside [0, npix)", fn);
    if (flag & 2u) return fail(CRP_ERR_UNSUPPORTED, "%s: a row reaches more than 4096 distinct border pixels", fn);
    return ok();
}

crp_status crp_lens_apply(int32_t nside, const int64_t *row_ptr, const int32_t *col, const float *val, int64_t nnz,
                          const float *x, float *y, int32_t nvec, void *stream) {
    const char *fn = "crp_lens_apply";
    if (nside < 1 || nside > 8192) return fail(CRP_ERR_INVALID, "%s: nside must be in [1, 8192]", fn);
    if (nvec < 1 || nvec > 4096) return fail(CRP_ERR_INVALID, "%s: nvec must be in [1, 4096]", fn);
    if (nnz < 0) return fail(CRP_ERR_INVALID, "%s: nnz < 0", fn);
    if (!row_ptr || !x || !y || (nnz > 0 && (!col || !val))) return fail(CRP_ERR_INVALID, "%s: null pointer", fn);
    const int64_t npix = 12 * (int64_t)nside * nside;
    hipError_t e = crp::launch_lens_apply(row_ptr, col, val, x, y, npix, nvec, nnz, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_error(e, fn);
    return ok();
}

}  // extern "C"
