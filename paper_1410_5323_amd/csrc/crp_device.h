// crp_device.h -- device arithmetic of the FP64 propagation path (gfx950).
//
// Everything here is written for the GPU library alone.  The arithmetic
// follows one fixed contract so that the result of every particle is
// reproducible bit for bit:
//   * IEEE FP64, round to nearest even, compiled with -ffp-contract=off; a
//     fused multiply-add only where fma() is written;
//   * sqrt and division are the correctly rounded device sequences;
//   * the controller's fifth root is a fixed Newton iteration, not pow().
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crp_internal.h"

namespace crp {
namespace dev {

// Lorentz-force constant: kappa = Z*K/E gives kappa*B = 1/r_gyro with B in nG,
// E in eV and lengths in Mpc; K = c * 1e-13 T/nG * 1 Mpc, c = 299792458 m/s,
// 1 Mpc = 1e6 * 648000/pi au, au = 149597870700 m.
constexpr double K_LORENTZ = 9.250628667507923e17;
// Seconds of light travel per Mpc.
constexpr double SEC_PER_MPC = 102927125054339.0;

// Cash-Karp 5(4) tableau (Cash & Karp 1990), each entry the FP64 rounding of
// its rational value.  Fifth-order weights B5*, error weights E* = b5 - b4.
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 3.0 / 10.0, A42 = -9.0 / 10.0, A43 = 6.0 / 5.0;
constexpr double A51 = -11.0 / 54.0, A52 = 5.0 / 2.0, A53 = -70.0 / 27.0, A54 = 35.0 / 27.0;
constexpr double A61 = 1631.0 / 55296.0, A62 = 175.0 / 512.0, A63 = 575.0 / 13824.0,
                 A64 = 44275.0 / 110592.0, A65 = 253.0 / 4096.0;
constexpr double B51 = 37.0 / 378.0, B53 = 250.0 / 621.0, B54 = 125.0 / 594.0, B56 = 512.0 / 1771.0;
constexpr double E1 = -277.0 / 64512.0, E3 = 6925.0 / 370944.0, E4 = -6925.0 / 202752.0,
                 E5 = -277.0 / 14336.0, E6 = 277.0 / 7084.0;

// 2^(-j/5), j = 0..4, nearest FP64.
__device__ __forceinline__ double two_pow_neg_fifth(int j) {
    switch (j) {
        case 0: return 0x1.0000000000000p+0;
        case 1: return 0x1.bdb8cdadbe120p-1;
        case 2: return 0x1.8406003b2ae5cp-1;
        case 3: return 0x1.51cb453b9536cp-1;
        default: return 0x1.2611186bae675p-1;
    }
}

// x^(-1/5) for finite x > 0: x = m 2^e, m in [0.5, 1); e = 5q + j with j in
// 0..4; six Newton steps r <- r (6 - m r^5) / 5 from r = 1 give m^(-1/5)
// (monotone from below); the result is r * 2^(-j/5) * 2^(-q).
__device__ __forceinline__ double inv_fifth_root(double x) {
    int e;
    double m = frexp(x, &e);
    int q = e >= 0 ? e / 5 : -((-e + 4) / 5);
    int j = e - 5 * q;
    double r = 1.0;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        double r2 = r * r;
        double r5 = (r2 * r2) * r;
        r = r * (6.0 - m * r5) * 0.2;
    }
    return ldexp(r * two_pow_neg_fifth(j), -q);
}

__device__ __forceinline__ double lerp(double a, double b, double t) { return fma(t, b - a, a); }

template <class T> __device__ __forceinline__ double to_f64(T v);
template <> __device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<__half>(__half v) { return (double)__half2float(v); }
template <> __device__ __forceinline__ double to_f64<__hip_bfloat16>(__hip_bfloat16 v) {
    return (double)__bfloat162float(v);
}

// Cell index and fraction along one axis: f = (X - o) * inv_spacing,
// i = floor(f) wrapped into [0, n), t = f - floor(f).
__device__ __forceinline__ int cell_axis(double X, double o, double inv, int n, int pow2, double &t) {
    double f = (X - o) * inv;
    double fl = floor(f);
    t = f - fl;
    int i = (int)fl;
    if (pow2) return i & (n - 1);
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Grid data is read through global-address-space pointers: the data pointer
// comes from a descriptor table in memory, so without the cast the compiler
// would emit flat loads, which also hold up the LDS counter.
template <class T>
using global_ptr = const __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ global_ptr<T> as_global(const void *p) {
    return (global_ptr<T>)(p);
}

// Raw storage type of a grid value (16-bit types are loaded as bits).
template <class T> struct raw_of { using type = T; };
template <> struct raw_of<__half> { using type = unsigned short; };
template <> struct raw_of<__hip_bfloat16> { using type = unsigned short; };
template <class T> using raw_t = typename raw_of<T>::type;

template <class T> __device__ __forceinline__ T from_raw(raw_t<T> r) { return r; }
template <> __device__ __forceinline__ __half from_raw<__half>(unsigned short r) { return __ushort_as_half(r); }
template <> __device__ __forceinline__ __hip_bfloat16 from_raw<__hip_bfloat16>(unsigned short r) {
    return __ushort_as_bfloat16(r);
}

// Corner values of cell (i, j, k) in the order v[((dz*2 + dy)*2 + dx)*3 + c].
// LINEAR (wrap-padded) layout: corner (dx,dy,dz) is node (i+dx, j+dy, k+dz) of
// the padded grid, so no corner needs a wrap.  CELL8 layout: one record of 32
// values per cell holding the 8 corners in that order (24 used).
template <class T, int LAYOUT>
__device__ __forceinline__ void load_corners(const FieldDev &F, int i, int j, int k, T (&v)[24]) {
    if (LAYOUT == CRP_LAYOUT_CELL8) {
        const global_ptr<raw_t<T>> p = as_global<raw_t<T>>(F.data) +
                                       32ull * (uint64_t)((uint32_t)i * F.cx + (uint32_t)j * F.cy + (uint32_t)k);
#pragma unroll
        for (int w = 0; w < 24; ++w) v[w] = from_raw<T>(p[w]);
    } else {
        const global_ptr<raw_t<T>> p =
            as_global<raw_t<T>>(F.data) + 3u * ((uint32_t)i * F.sx + (uint32_t)j * F.sy + (uint32_t)k);
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const global_ptr<raw_t<T>> q = p + 3u * ((uint32_t)dx * F.sx + (uint32_t)dy * F.sy);
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                    for (int c = 0; c < 3; ++c) v[((dz * 2 + dy) * 2 + dx) * 3 + c] = from_raw<T>(q[3 * dz + c]);
            }
    }
}

// Trilinear interpolation of stored corner values, converted exactly to FP64,
// one component at a time, then scaled by value_scale (a multiplication by 1
// for FP64/FP32 grids).
template <class T>
__device__ __forceinline__ void interp_corners(const FieldDev &F, const T (&v)[24], double tx, double ty, double tz,
                                               double B[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double c00 = lerp(to_f64<T>(v[0 + c]), to_f64<T>(v[3 + c]), tx);    // (dy, dz) = (0, 0)
        double c10 = lerp(to_f64<T>(v[6 + c]), to_f64<T>(v[9 + c]), tx);    // (1, 0)
        double c01 = lerp(to_f64<T>(v[12 + c]), to_f64<T>(v[15 + c]), tx);  // (0, 1)
        double c11 = lerp(to_f64<T>(v[18 + c]), to_f64<T>(v[21 + c]), tx);  // (1, 1)
        double c0 = lerp(c00, c10, ty);
        double c1 = lerp(c01, c11, ty);
        B[c] = lerp(c0, c1, tz);
    }
    if (F.value_scale != 1.0) {
        B[0] = B[0] * F.value_scale;
        B[1] = B[1] * F.value_scale;
        B[2] = B[2] * F.value_scale;
    }
}

// fma(t, d, a) into a register of its own.  The compiler's two-address form
// of fma overwrites its addend, which for the cached edges would cost a copy
// of every cached value at every lookup; this form leaves them in place.  The
// same rounding as fma().
__device__ __forceinline__ double fma_keep(double t, double d, double a) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(t), "v"(d), "v"(a));
    return r;
}

// The cached form of a cell: edge e = (dz*2 + dy)*3 + c runs along x from
// corner (0, dy, dz) to (1, dy, dz) of component c; a holds its lower value,
// d the upper minus the lower, both as interp_corners forms them.
template <class T>
__device__ __forceinline__ void edges_of_corners(const T (&v)[24], double (&a)[12], double (&d)[12]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[3 * e + c] = to_f64<T>(v[6 * e + c]);
            d[3 * e + c] = to_f64<T>(v[6 * e + 3 + c]) - a[3 * e + c];
        }
}

// interp_corners on the cached edges: the same operations in the same order.
__device__ __forceinline__ void interp_edges(const FieldDev &F, const double (&a)[12], const double (&d)[12],
                                             double tx, double ty, double tz, double B[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double c00 = fma_keep(tx, d[0 + c], a[0 + c]);
        double c10 = fma_keep(tx, d[3 + c], a[3 + c]);
        double c01 = fma_keep(tx, d[6 + c], a[6 + c]);
        double c11 = fma_keep(tx, d[9 + c], a[9 + c]);
        double c0 = lerp(c00, c10, ty);
        double c1 = lerp(c01, c11, ty);
        B[c] = lerp(c0, c1, tz);
    }
    if (F.value_scale != 1.0) {
        B[0] = B[0] * F.value_scale;
        B[1] = B[1] * F.value_scale;
        B[2] = B[2] * F.value_scale;
    }
}

// Field lookup at X (Mpc) -> B (nG), reading the corners from memory.
template <class T, int LAYOUT>
__device__ __forceinline__ void lookup(const FieldDev &F, const double X[3], double B[3]) {
    double tx, ty, tz;
    int i = cell_axis(X[0], F.origin[0], F.inv_spacing, F.n[0], F.pow2, tx);
    int j = cell_axis(X[1], F.origin[1], F.inv_spacing, F.n[1], F.pow2, ty);
    int k = cell_axis(X[2], F.origin[2], F.inv_spacing, F.n[2], F.pow2, tz);
    T v[24];
    load_corners<T, LAYOUT>(F, i, j, k, v);
    interp_corners<T>(F, v, tx, ty, tz, B);
}

// Per-lane cache of the corner values of the last cell looked up.  A particle
// whose steps are small compared with the grid spacing looks up the same cell
// many times in a row; those lookups then issue no global memory instruction,
// so the longest trajectories' dependent lookups skip the texture path's
// queues.  The values are held in the lane's registers, or (IN_LDS) in one
// LDS column per lane ([value][thread], so the reads of a wavefront hit
// distinct banks) where the kernel has no registers to spare.  The values are
// the stored ones: results are bit-identical with or without it.
constexpr int CACHE_BLOCK = 256;

template <class T, bool IN_LDS = false>
struct CellCache {
    uint32_t key;   // cell index (i*n1 + j)*n2 + k, 0xffffffff = empty
    int32_t field;  // field the cell belongs to
    T v[24];        // the cell's stored corner values
    double a[12];   // or, for paired lookups (lookup_pair), the cell's x-edges: lower corner
    double d[12];   // values converted exactly, and upper minus lower
    float fa[12];   // the same in FP32 for the mixed kernel's paired lookups
    float fd[12];
    uint32_t mkey;  // FP32 modulation grid: its last cell, 0xffffffff = empty
    float mv[8];    // that cell's 8 stored values
    int misses;     // lookups that read global memory (diagnostic)
};

template <class T>
struct CellCache<T, true> {
    uint32_t key;
    int32_t field;
    T (*v)[CACHE_BLOCK];  // LDS [24][CACHE_BLOCK]
    int t;                // the thread's column
    int misses;
};

template <class T>
__device__ __forceinline__ void cache_reset(CellCache<T, false> &c) {
    c.key = 0xffffffffu;
    c.field = -1;
    c.mkey = 0xffffffffu;
    c.misses = 0;
}

template <class T>
__device__ __forceinline__ void cache_reset(CellCache<T, true> &c, T (*lds)[CACHE_BLOCK], int t) {
    c.key = 0xffffffffu;
    c.field = -1;
    c.v = lds;
    c.t = t;
    c.misses = 0;
}

// Modulation corners of the cell holding X (section 3.2, modulated grids):
// the padded scalar grid's 8 stored values and the cell fractions.
template <class M>
struct ModCorners {
    M v000, v001, v100, v101, v010, v011, v110, v111;
    double t[3];
};

template <class M>
__device__ __forceinline__ void mod_load(const FieldDev &F, const double X[3], ModCorners<M> &m) {
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = cell_axis(X[a], F.mod_origin[a], F.mod_inv_spacing, F.mod_n[a], F.mod_pow2, m.t[a]);
    const global_ptr<M> p = as_global<M>(F.mod_data) + ((uint32_t)c[0] * F.mod_sx + (uint32_t)c[1] * F.mod_sy + (uint32_t)c[2]);
    const uint32_t sx = F.mod_sx, sy = F.mod_sy;
    m.v000 = p[0];
    m.v001 = p[1];
    m.v100 = p[sx];
    m.v101 = p[sx + 1];
    m.v010 = p[sy];
    m.v011 = p[sy + 1];
    m.v110 = p[sx + sy];
    m.v111 = p[sx + sy + 1];
}

// Modulation value from its corners: trilinear, x then y then z, as the
// vector components.
template <class M>
__device__ __forceinline__ double mod_value(const ModCorners<M> &m) {
    const double c00 = lerp((double)m.v000, (double)m.v100, m.t[0]);
    const double c10 = lerp((double)m.v010, (double)m.v110, m.t[0]);
    const double c01 = lerp((double)m.v001, (double)m.v101, m.t[0]);
    const double c11 = lerp((double)m.v011, (double)m.v111, m.t[0]);
    return lerp(lerp(c00, c10, m.t[1]), lerp(c01, c11, m.t[1]), m.t[2]);
}

template <class M>
__device__ __forceinline__ double mod_interp(const FieldDev &F, const double X[3]) {
    ModCorners<M> m;
    mod_load<M>(F, X, m);
    return mod_value<M>(m);
}

// B <- B * m(X) when the field carries a modulation grid.
__device__ __forceinline__ void modulate(const FieldDev &F, const double X[3], double B[3]) {
    if (!F.mod_data) return;
    const double m = F.mod_dtype == CRP_F64 ? mod_interp<double>(F, X) : mod_interp<float>(F, X);
    B[0] = B[0] * m;
    B[1] = B[1] * m;
    B[2] = B[2] * m;
}

// Field value times modulation at X, the same arithmetic as lookup() then
// modulate(), with both grids' corner loads issued before either
// interpolation: the lookup waits for memory once, the two gathers' latencies
// overlap instead of adding up.
template <class T, int LAYOUT, class M>
__device__ __forceinline__ void lookup_mod(const FieldDev &F, const double X[3], double B[3]) {
    ModCorners<M> m;
    mod_load<M>(F, X, m);
    double tx, ty, tz;
    int i = cell_axis(X[0], F.origin[0], F.inv_spacing, F.n[0], F.pow2, tx);
    int j = cell_axis(X[1], F.origin[1], F.inv_spacing, F.n[1], F.pow2, ty);
    int k = cell_axis(X[2], F.origin[2], F.inv_spacing, F.n[2], F.pow2, tz);
    T v[24];
    load_corners<T, LAYOUT>(F, i, j, k, v);
    interp_corners<T>(F, v, tx, ty, tz, B);
    const double mv = mod_value<M>(m);
    B[0] = B[0] * mv;
    B[1] = B[1] * mv;
    B[2] = B[2] * mv;
}

// MOD: the launch has modulated fields (then each field's modulation, if any,
// multiplies its value); without it no modulation code is compiled in.
template <class T, int LAYOUT, bool CACHE, bool MOD = false, bool L = false>
__device__ __forceinline__ void lookup_cached(const FieldDev &F, int fid, const double X[3], double B[3],
                                              CellCache<T, L> &cache) {
    if (!CACHE) {
        if (!MOD || !F.mod_data)
            lookup<T, LAYOUT>(F, X, B);
        else if (F.mod_dtype == CRP_F64)
            lookup_mod<T, LAYOUT, double>(F, X, B);
        else
            lookup_mod<T, LAYOUT, float>(F, X, B);
        cache.misses++;
        return;
    }
    double tx, ty, tz;
    int i = cell_axis(X[0], F.origin[0], F.inv_spacing, F.n[0], F.pow2, tx);
    int j = cell_axis(X[1], F.origin[1], F.inv_spacing, F.n[1], F.pow2, ty);
    int k = cell_axis(X[2], F.origin[2], F.inv_spacing, F.n[2], F.pow2, tz);
    uint32_t key = ((uint32_t)i * (uint32_t)F.n[1] + (uint32_t)j) * (uint32_t)F.n[2] + (uint32_t)k;
    if constexpr (L) {
        T v[24];
        if (key != cache.key || fid != cache.field) {
            load_corners<T, LAYOUT>(F, i, j, k, v);
#pragma unroll
            for (int w = 0; w < 24; ++w) cache.v[w][cache.t] = v[w];
            cache.key = key;
            cache.field = fid;
            cache.misses++;
        } else {
#pragma unroll
            for (int w = 0; w < 24; ++w) v[w] = cache.v[w][cache.t];
        }
        interp_corners<T>(F, v, tx, ty, tz, B);
    } else {
        if (key != cache.key || fid != cache.field) {
            load_corners<T, LAYOUT>(F, i, j, k, cache.v);
            cache.key = key;
            cache.field = fid;
            cache.misses++;
        }
        interp_corners<T>(F, cache.v, tx, ty, tz, B);
    }
    if (MOD) {
        if constexpr (!L) {
            // an FP32 modulation grid's last cell is kept too (its cells are
            // larger than the vector grid's, so it is revisited longer)
            if (F.mod_data && F.mod_dtype == CRP_F32) {
                ModCorners<float> mc;
                int c[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    c[a] = cell_axis(X[a], F.mod_origin[a], F.mod_inv_spacing, F.mod_n[a], F.mod_pow2, mc.t[a]);
                const uint32_t mkey = ((uint32_t)c[0] * (uint32_t)F.mod_n[1] + (uint32_t)c[1]) * (uint32_t)F.mod_n[2] +
                                      (uint32_t)c[2];
                if (mkey != cache.mkey) {
                    const global_ptr<float> p = as_global<float>(F.mod_data) +
                                                ((uint32_t)c[0] * F.mod_sx + (uint32_t)c[1] * F.mod_sy + (uint32_t)c[2]);
                    const uint32_t sx = F.mod_sx, sy = F.mod_sy;
                    cache.mv[0] = p[0];
                    cache.mv[1] = p[1];
                    cache.mv[2] = p[sx];
                    cache.mv[3] = p[sx + 1];
                    cache.mv[4] = p[sy];
                    cache.mv[5] = p[sy + 1];
                    cache.mv[6] = p[sx + sy];
                    cache.mv[7] = p[sx + sy + 1];
                    cache.mkey = mkey;
                }
                mc.v000 = cache.mv[0];
                mc.v001 = cache.mv[1];
                mc.v100 = cache.mv[2];
                mc.v101 = cache.mv[3];
                mc.v010 = cache.mv[4];
                mc.v011 = cache.mv[5];
                mc.v110 = cache.mv[6];
                mc.v111 = cache.mv[7];
                const double m = mod_value<float>(mc);
                B[0] = B[0] * m;
                B[1] = B[1] * m;
                B[2] = B[2] * m;
                return;
            }
        }
        modulate(F, X, B);
    }
}

// Direction part of the right-hand side: k[3..5] = kappa * U x B for Y = (X, U).
__device__ __forceinline__ void lorentz(double kap, const double Y[6], const double B[3], double k[6]) {
    double cx = Y[4] * B[2] - Y[5] * B[1];
    double cy = Y[5] * B[0] - Y[3] * B[2];
    double cz = Y[3] * B[1] - Y[4] * B[0];
    k[3] = kap * cx;
    k[4] = kap * cy;
    k[5] = kap * cz;
}

// Right-hand side in path length: k = (U, kappa * U x B(X)) for Y = (X, U).
template <class T, int LAYOUT, bool CACHE, bool MOD = false, bool L = false>
__device__ __forceinline__ void rhs(const FieldDev &F, int fid, CellCache<T, L> &cache, double kap, const double Y[6],
                                    double k[6], double B[3]) {
    lookup_cached<T, LAYOUT, CACHE, MOD>(F, fid, Y, B, cache);
    k[0] = Y[3];
    k[1] = Y[4];
    k[2] = Y[5];
    lorentz(kap, Y, B, k);
}

__device__ __forceinline__ double norm3(double a, double b, double c) { return sqrt(a * a + b * b + c * c); }

// Stage recorder of ck_eval: receives each stage state Y_i (i = 1..5; Y_0 is
// y itself) and each stage's field value B_i (i = 0..5).  The default records
// nothing (records = false) and compiles away.  A recorder with deferred = true is instead
// handed the step's inputs and stage derivatives once, after the last stage
// (flush), so that its stores come after every field gather of the step.
struct NoStageRecord {
    static constexpr bool records = false;
    static constexpr bool deferred = false;
    __device__ __forceinline__ void stage(int, const double *) const {}
    __device__ __forceinline__ void field(int, const double *) const {}
    __device__ __forceinline__ void flush(const double *, double, const double *, const double *, const double *,
                                          const double *, const double *) const {}
};

// Component c of the Cash-Karp stage states Y_1..Y_5 from the stage
// derivatives k_1..k_i: sums over j in increasing order with fma from zero.
__device__ __forceinline__ double ck_y1(const double *y, double h, const double *k1, int c) {
    return fma(h, fma(A21, k1[c], 0.0), y[c]);
}
__device__ __forceinline__ double ck_y2(const double *y, double h, const double *k1, const double *k2, int c) {
    return fma(h, fma(A32, k2[c], fma(A31, k1[c], 0.0)), y[c]);
}
__device__ __forceinline__ double ck_y3(const double *y, double h, const double *k1, const double *k2,
                                        const double *k3, int c) {
    return fma(h, fma(A43, k3[c], fma(A42, k2[c], fma(A41, k1[c], 0.0))), y[c]);
}
__device__ __forceinline__ double ck_y4(const double *y, double h, const double *k1, const double *k2,
                                        const double *k3, const double *k4, int c) {
    return fma(h, fma(A54, k4[c], fma(A53, k3[c], fma(A52, k2[c], fma(A51, k1[c], 0.0)))), y[c]);
}
__device__ __forceinline__ double ck_y5(const double *y, double h, const double *k1, const double *k2,
                                        const double *k3, const double *k4, const double *k5, int c) {
    return fma(h, fma(A65, k5[c], fma(A64, k4[c], fma(A63, k3[c], fma(A62, k2[c], fma(A61, k1[c], 0.0))))), y[c]);
}

// The cell of the grid holding X and the fractions within it, as
// lookup_cached finds them.
struct CellAt {
    uint32_t key;
    int i, j, k;
    double tx, ty, tz;
};

__device__ __forceinline__ void cell_at(const FieldDev &F, const double X[3], CellAt &c) {
    c.i = cell_axis(X[0], F.origin[0], F.inv_spacing, F.n[0], F.pow2, c.tx);
    c.j = cell_axis(X[1], F.origin[1], F.inv_spacing, F.n[1], F.pow2, c.ty);
    c.k = cell_axis(X[2], F.origin[2], F.inv_spacing, F.n[2], F.pow2, c.tz);
    c.key = ((uint32_t)c.i * (uint32_t)F.n[1] + (uint32_t)c.j) * (uint32_t)F.n[2] + (uint32_t)c.k;
}

// The corner values of cell (i, j, k) with key (i*n1 + j)*n2 + k (use), or
// of the grid's first cell.  In CELL8 storage the key is the record index.
template <class T, int LAYOUT>
__device__ __forceinline__ void load_cell(const FieldDev &F, uint32_t key, int i, int j, int k, bool use,
                                          T (&v)[24]) {
    if (LAYOUT == CRP_LAYOUT_CELL8) {
        const global_ptr<raw_t<T>> p = as_global<raw_t<T>>(F.data) + 32ull * (uint64_t)(use ? key : 0u);
#pragma unroll
        for (int w = 0; w < 24; ++w) v[w] = from_raw<T>(p[w]);
    } else {
        load_corners<T, LAYOUT>(F, use ? i : 0, use ? j : 0, use ? k : 0, v);
    }
}

// Two lookups whose positions are both known, through the register cell
// cache: the corner loads of both cells are issued before the first is
// waited for, so the two gathers' latencies overlap.  Every lane issues both
// loads; a lane whose cell is already held reads the grid's first record
// instead (the same line for the whole wavefront, so one cache access), which
// keeps the loads out of branches: the wait for the first cell then does not
// also wait for the second.  The cache holds A's cell after A and B's after
// B, as two calls of lookup_cached would leave it; the values, and so B, are
// the same.
template <class T, int LAYOUT>
__device__ __forceinline__ void lookup_pair(const FieldDev &F, int fid, const double XA[3], const double XB[3],
                                            double BA[3], double BB[3], CellCache<T, false> &cache) {
    CellAt a, b;
    cell_at(F, XA, a);
    cell_at(F, XB, b);
    const bool missA = a.key != cache.key || fid != cache.field;
    const bool missB = b.key != a.key;
    T va[24], vb[24];
    load_cell<T, LAYOUT>(F, a.key, a.i, a.j, a.k, missA, va);
    load_cell<T, LAYOUT>(F, b.key, b.i, b.j, b.k, missB, vb);
    // keeps both loads here: without it the compiler moves each into the
    // branch that uses it, where it is waited for at once
    asm volatile("" ::: "memory");
    if (missA) {
        edges_of_corners<T>(va, cache.a, cache.d);
        cache.key = a.key;
        cache.field = fid;
        cache.misses++;
    }
    interp_edges(F, cache.a, cache.d, a.tx, a.ty, a.tz, BA);
    if (missB) {
        edges_of_corners<T>(vb, cache.a, cache.d);
        cache.key = b.key;
        cache.misses++;
    }
    interp_edges(F, cache.a, cache.d, b.tx, b.ty, b.tz, BB);
}

// ck_eval's six stages in three levels of two lookups (register cell cache,
// no modulation, nothing recorded).  The position of stage i+1 needs only the
// stage directions up to stage i, that is the fields up to stage i-1, so
// stages (1, 2), (3, 4) and (5, 6) can look up their fields together.  Every
// component is computed by the same expression as in ck_eval; only the order
// in which components are formed differs, so the results are the same bits.
template <class T, int LAYOUT>
__device__ __forceinline__ void ck_stages_paired(const FieldDev &F, int fid, CellCache<T, false> &cache, double kap,
                                                 const double y[6], double h, double k1[6], double k2[6],
                                                 double k3[6], double k4[6], double k5[6], double k6[6]) {
    double Ya[6], Yb[6], BA[3], BB[3];
    // stages 1 and 2: X_1 = x; X_2 needs k1[0..2] = u only
    k1[0] = y[3];
    k1[1] = y[4];
    k1[2] = y[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) Yb[c] = ck_y1(y, h, k1, c);
    lookup_pair<T, LAYOUT>(F, fid, y, Yb, BA, BB, cache);
    lorentz(kap, y, BA, k1);
#pragma unroll
    for (int c = 3; c < 6; ++c) Yb[c] = ck_y1(y, h, k1, c);
    k2[0] = Yb[3];
    k2[1] = Yb[4];
    k2[2] = Yb[5];
    lorentz(kap, Yb, BB, k2);
    // stages 3 and 4: X_3 needs k1, k2; X_4 needs k3[0..2] = U_3, which needs k1, k2
#pragma unroll
    for (int c = 0; c < 6; ++c) Ya[c] = ck_y2(y, h, k1, k2, c);
    k3[0] = Ya[3];
    k3[1] = Ya[4];
    k3[2] = Ya[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) Yb[c] = ck_y3(y, h, k1, k2, k3, c);
    lookup_pair<T, LAYOUT>(F, fid, Ya, Yb, BA, BB, cache);
    lorentz(kap, Ya, BA, k3);
#pragma unroll
    for (int c = 3; c < 6; ++c) Yb[c] = ck_y3(y, h, k1, k2, k3, c);
    k4[0] = Yb[3];
    k4[1] = Yb[4];
    k4[2] = Yb[5];
    lorentz(kap, Yb, BB, k4);
    // stages 5 and 6
#pragma unroll
    for (int c = 0; c < 6; ++c) Ya[c] = ck_y4(y, h, k1, k2, k3, k4, c);
    k5[0] = Ya[3];
    k5[1] = Ya[4];
    k5[2] = Ya[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) Yb[c] = ck_y5(y, h, k1, k2, k3, k4, k5, c);
    lookup_pair<T, LAYOUT>(F, fid, Ya, Yb, BA, BB, cache);
    lorentz(kap, Ya, BA, k5);
#pragma unroll
    for (int c = 3; c < 6; ++c) Yb[c] = ck_y5(y, h, k1, k2, k3, k4, k5, c);
    k6[0] = Yb[3];
    k6[1] = Yb[4];
    k6[2] = Yb[5];
    lorentz(kap, Yb, BB, k6);
}

// One Cash-Karp evaluation of step h from y: fifth-order solution y5 and the
// norms of the embedded error vector delta = h * sum_i e_i k_i split into
// position (ex) and direction (eu) parts.  Stage sums accumulate over j in
// increasing order with fma starting from zero; terms with a zero weight are
// omitted (they only add a signed zero).
template <class T, int LAYOUT, bool CACHE, class Rec = NoStageRecord, bool MOD = false, bool L = false>
__device__ __forceinline__ void ck_eval(const FieldDev &F, int fid, CellCache<T, L> &cache, double kap,
                                        const double y[6], double h, double y5[6], double &ex, double &eu,
                                        const Rec &rec = Rec()) {
    double k1[6], k2[6], k3[6], k4[6], k5[6], k6[6];
    if constexpr (CACHE && !MOD && !L && !Rec::records) {
        ck_stages_paired<T, LAYOUT>(F, fid, cache, kap, y, h, k1, k2, k3, k4, k5, k6);
    } else {
    double Y[6], B[3];
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, y, k1, B);
    rec.field(0, B);
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = ck_y1(y, h, k1, c);
    rec.stage(1, Y);
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, Y, k2, B);
    rec.field(1, B);
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = ck_y2(y, h, k1, k2, c);
    rec.stage(2, Y);
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, Y, k3, B);
    rec.field(2, B);
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = ck_y3(y, h, k1, k2, k3, c);
    rec.stage(3, Y);
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, Y, k4, B);
    rec.field(3, B);
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = ck_y4(y, h, k1, k2, k3, k4, c);
    rec.stage(4, Y);
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, Y, k5, B);
    rec.field(4, B);
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = ck_y5(y, h, k1, k2, k3, k4, k5, c);
    rec.stage(5, Y);
    rhs<T, LAYOUT, CACHE, MOD>(F, fid, cache, kap, Y, k6, B);
    rec.field(5, B);
    if constexpr (Rec::deferred) rec.flush(y, h, k1, k2, k3, k4, k5);
    }
    double d[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double a5 = fma(B56, k6[c], fma(B54, k4[c], fma(B53, k3[c], fma(B51, k1[c], 0.0))));
        double ae = fma(E6, k6[c], fma(E5, k5[c], fma(E4, k4[c], fma(E3, k3[c], fma(E1, k1[c], 0.0)))));
        y5[c] = fma(h, a5, y[c]);
        d[c] = h * ae;
    }
    ex = norm3(d[0], d[1], d[2]);
    eu = norm3(d[3], d[4], d[5]);
}

// A kernel's arguments (one struct A by value, its only argument, so at the
// start of the kernel-argument segment) read again where this is called,
// with scalar loads from that segment, instead of held in scalar registers
// across the main loop: for values used only on rare paths (a particle
// starting or ending), which would otherwise be spilled to vector-register
// lanes.  The empty asm hides the pointer's origin, so the compiler cannot
// hoist those loads out of the loop.
template <class A>
using KernArg = const __attribute__((address_space(4))) A;
template <class A>
__device__ __forceinline__ KernArg<A> &kernel_args() {
    KernArg<A> *q = (KernArg<A> *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(q));
    return *q;
}

}  // namespace dev
}  // namespace crp
