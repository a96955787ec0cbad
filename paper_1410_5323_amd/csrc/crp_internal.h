// crp_internal.h -- descriptors shared by the host ABI and the gfx950 kernels of libcrp.
//
// Device-side copies of the field and parameter descriptors live in the
// caller's workspace; the host packs them (crp_host.cpp) and a small kernel
// writes them there, so every call is a pure sequence of stream operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/crp.h"

namespace crp {

// Device descriptor of one field grid (192 bytes).
struct FieldDev {
    const void *data;
    int32_t n[3];          // nodes per axis
    int32_t pow2;          // 1 if every n is a power of two (wrap by mask)
    double origin[3];
    double inv_spacing;    // 1.0 / spacing (one FP64 division on the host)
    double value_scale;    // nG per stored unit
    uint32_t sx, sy;       // LINEAR: node strides of the padded grid, (n1+1)(n2+1) and (n2+1)
    uint32_t cy, cx;       // CELL8: cell strides n2 and n1*n2
    int32_t dtype, layout;
    // modulation (mod_data NULL: none): padded [m0+1][m1+1][m2+1] scalars
    const void *mod_data;
    int32_t mod_n[3];
    int32_t mod_pow2;
    double mod_origin[3];
    double mod_inv_spacing;
    uint32_t mod_sx, mod_sy;
    int32_t mod_dtype;
    int32_t pad_[9];
};
static_assert(sizeof(FieldDev) == 192, "FieldDev layout");

// Device descriptor of one parameter group (128 bytes).
struct ParamsDev {
    double tol, h_min, h_max;
    double center[3];
    double radius, r2;     // r2 = radius * radius
    double l_max;
    int64_t max_steps;
    double box_lo[3], box_hi[3];  // reflective box faces
    int32_t field_index;
    int32_t sphere_on;     // radius > 0
    int32_t lmax_on;       // l_max finite
    int32_t reflect_on;    // reflective box on
    int32_t backtrack_on;  // propagate the antiparticle backwards
    int32_t pad_[3];
};
static_assert(sizeof(ParamsDev) == 160, "ParamsDev layout");

// Workspace layout (offsets in bytes from the 256-byte aligned base).
//   [0, 256)                 control: queue head (uint64 at 0)
//   [256, 256 + 192*nf)      FieldDev table
//   then 160*np              ParamsDev table
//   then 4*n                 order (int32 particle indices, rigidity buckets ascending)
//   then 4*(NBUCKET+1)*2     bucket counts and cursors
constexpr int NBUCKET = 256;

struct WsLayout {
    size_t fields, params, order, buckets, total;
};

constexpr size_t ws_round_up(size_t v) { return (v + 255) & ~size_t(255); }

constexpr WsLayout ws_layout(int64_t n, int32_t nf, int32_t np) {
    auto up = ws_round_up;
    WsLayout w{};
    w.fields = 256;
    w.params = up(w.fields + sizeof(FieldDev) * size_t(nf));
    w.order = up(w.params + sizeof(ParamsDev) * size_t(np));
    w.buckets = up(w.order + 4 * size_t(n > 0 ? n : 0));
    w.total = up(w.buckets + 8 * size_t(NBUCKET + 1));
    return w;
}

// Kernel arguments of the propagation kernels (passed by value).
struct PropArgs {
    double *x, *y, *z, *ux, *uy, *uz;
    const double *energy;
    const int32_t *charge;
    double *length, *h_next, *time;
    int32_t *status;
    const int32_t *param_index;
    int64_t *n_acc, *n_rej;
    int64_t n;
    const FieldDev *fields;
    const ParamsDev *params;
    const int32_t *order;            // NULL: particles in index order
    unsigned long long *queue;       // work-queue head
    unsigned long long *counters;    // NULL or CRP_NCOUNTERS accumulators
    double *tape_ckpt;               // NULL: no tape; else the pool of 8-double records
    int64_t *tape_link;              // previous record of the same particle
    unsigned long long *tape_head;   // pool head
    double *tape_fin;                // 4 doubles per particle
    int64_t tape_cap;                // records in the pool
    int32_t tape_k;                  // checkpoint interval
    int32_t refill_threshold;
    int32_t n_params;
    int32_t modulated;               // some field carries a modulation grid
    int32_t reflective;              // some parameter group has a reflective box
    const int32_t *cancel;           // NULL, or the caller's cancel word (nonzero: stop)
    // The first field and parameter group by value: a launch with one of each
    // reads them from the kernel arguments with scalar loads, which never wait
    // behind the lanes' field gathers as vector loads of the tables would.
    FieldDev F0;
    ParamsDev P0;
};

// crp_propagate's checks and launches (crp_host.cpp), given host staging
// arrays fd and pd of at least n_fields and n_params descriptors.  fn names
// the entry point in error messages.  check_only: validate the arguments
// (everything but the workspace) and return without touching the device.
crp_status propagate_impl(const char *fn, const crp_field *fields, int32_t n_fields, const crp_params *params,
                          int32_t n_params, const crp_particles *p, int64_t n, const crp_tape *tape,
                          int32_t precision, const crp_tuning *tuning, int64_t *counters, void *workspace,
                          size_t workspace_bytes, void *stream, FieldDev *fd, ParamsDev *pd, bool check_only);

// Sets the thread's last-error message (msg) for a failing status, clears it
// for CRP_OK; returns st.
crp_status report(crp_status st, const char *msg);

// Launchers (defined in the .hip files, called by crp_host.cpp).
hipError_t launch_write_table(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *dst, unsigned long long v, int count, hipStream_t s);
hipError_t launch_order_by_rigidity(const double *energy, const int32_t *charge, const int32_t *status,
                                    int64_t n, int32_t *order, unsigned int *buckets, hipStream_t s);
hipError_t launch_propagate_fp64(const PropArgs &a, int dtype, int layout, bool multi, bool cache, int blocks,
                                 int block_size, hipStream_t s);
hipError_t launch_propagate_mixed(const PropArgs &a, int dtype, int layout, bool multi, int precision, bool cache,
                                  int blocks, int block_size, hipStream_t s);
hipError_t launch_order_by_steps(const double *fin, int64_t n, int32_t *order, unsigned int *buckets, hipStream_t s);
hipError_t launch_upload_modulation(const FieldDev &f, const void *src, int src_dtype, hipStream_t s);
hipError_t launch_upload(const FieldDev &f, const void *src, int src_dtype, void *dst, hipStream_t s);
hipError_t launch_selftest(const double *in, double *out, int64_t n, int op, hipStream_t s);
hipError_t launch_gather_bench(const FieldDev &F, int64_t lanes, int64_t lookups, double spread, uint32_t seed,
                               double *sink, hipStream_t s);
hipError_t launch_gather_replay(const FieldDev &F, const double *rec, int64_t lanes, int64_t steps, bool cache,
                                double *sink, int64_t *misses, hipStream_t s);
// Lens construction workspace (byte offsets): device flag, launches per row,
// cursors, row segment starts, the grouped border pixels and the run-length
// encoded entries per row segment.
struct LensWs {
    size_t flag, counts, cursor, starts, colbuf, scol, sval, total;
};
LensWs lens_ws_layout(int32_t nside, int64_t n);
hipError_t launch_healpix(int32_t nside, const double *ux, const double *uy, const double *uz, int64_t n,
                          double sign, int32_t *pix, hipStream_t s);
hipError_t launch_lens_build(int32_t nside, const int32_t *row, const double *ux, const double *uy,
                             const double *uz, const int32_t *status, int64_t n, int64_t *row_ptr, int32_t *col,
                             float *val, uint8_t *ws, hipStream_t s);
hipError_t launch_lens_apply(const int64_t *row_ptr, const int32_t *col, const float *val, const float *x, float *y,
                             int64_t npix, int32_t nvec, int64_t nnz, hipStream_t s);
hipError_t launch_stream(const void *src, void *dst, size_t bytes, double *sink, int blocks, hipStream_t s);

}  // namespace crp
