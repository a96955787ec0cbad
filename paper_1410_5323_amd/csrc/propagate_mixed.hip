// propagate_mixed.hip -- mixed-precision propagation kernel for gfx950.
//
// Same method and control flow as the FP64-state kernel (one Cash-Karp
// evaluation per loop iteration, modes NORMAL / EVENT / FINAL, ballot refill
// from the work queue), with the arithmetic split by what each quantity needs:
//   * the Runge-Kutta stages, the trilinear lookups, the direction and the
//     error control run in FP32 (the grid may be stored in FP16/BF16/FP32);
//   * position and trajectory length are accumulated in FP64 (ACC_F64) or as
//     compensated double-float pairs (ACC_DF), because Gpc paths at kpc
//     resolution exceed FP32's 24-bit mantissa;
//   * lookups use cell-relative coordinates: the base cell and the FP32
//     fraction inside it are taken from the accumulated position once per
//     evaluation, and each stage adds its small FP32 offset to that fraction,
//     so a lookup is resolved to ~1e-7 of a cell at any distance.
// The results are not bitwise comparable with the FP64 oracle; their angular,
// length and time errors are measured against it.
#include "crp_device.h"

namespace crp {
namespace {

using namespace dev;

enum { ACC_F64 = 0, ACC_DF = 1 };
enum { MODE_NORMAL = 0, MODE_EVENT = 1, MODE_FINAL = 2 };
enum { F_EVAL = 1, F_ACC = 2, F_REJ = 4, F_EVENT = 8, F_FLOOR = 16 };
constexpr int MAX_BLOCK = 256;

// FP32 Cash-Karp tableau, each entry rounded once from its rational value.
constexpr float a21 = 1.0f / 5.0f;
constexpr float a31 = 3.0f / 40.0f, a32 = 9.0f / 40.0f;
constexpr float a41 = 3.0f / 10.0f, a42 = -9.0f / 10.0f, a43 = 6.0f / 5.0f;
constexpr float a51 = -11.0f / 54.0f, a52 = 5.0f / 2.0f, a53 = -70.0f / 27.0f, a54 = 35.0f / 27.0f;
constexpr float a61 = 1631.0f / 55296.0f, a62 = 175.0f / 512.0f, a63 = 575.0f / 13824.0f,
                a64 = 44275.0f / 110592.0f, a65 = 253.0f / 4096.0f;
constexpr float b51 = 37.0f / 378.0f, b53 = 250.0f / 621.0f, b54 = 125.0f / 594.0f, b56 = 512.0f / 1771.0f;
constexpr float e1 = -277.0f / 64512.0f, e3 = 6925.0f / 370944.0f, e4 = -6925.0f / 202752.0f,
                e5 = -277.0f / 14336.0f, e6 = 277.0f / 7084.0f;

template <class T> __device__ __forceinline__ float to_f32(T v);
template <> __device__ __forceinline__ float to_f32<double>(double v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<__half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float to_f32<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ int wrap(int i, int n, int pow2) {
    if (pow2) return i & (n - 1);
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Base cell of a step's start in the modulation grid (section 3.2, modulated
// grids), with the FP32 fraction: the stages add their offsets to it in FP32
// as they do for the vector grid.
struct ModRel {
    int ib[3];
    float tb[3];
};

// Double-float helpers (Knuth two-sum; Dekker split replaced by fma).
struct df {
    float hi, lo;
};
__device__ __forceinline__ df df_add(df a, float b) {
    float s = a.hi + b;
    float bb = s - a.hi;
    float err = (a.hi - (s - bb)) + (b - bb);
    float lo = a.lo + err;
    float hi = s + lo;
    return {hi, lo - (hi - s)};
}
__device__ __forceinline__ double df_val(df a) { return (double)a.hi + (double)a.lo; }

// Position and length accumulator, FP64 or double-float.
template <int ACC> struct Acc;
template <> struct Acc<ACC_F64> {
    double x[3], L;
    __device__ __forceinline__ void set(const double p[3], double len) {
        x[0] = p[0];
        x[1] = p[1];
        x[2] = p[2];
        L = len;
    }
    __device__ __forceinline__ void add_x(const float d[3]) {
        x[0] += (double)d[0];
        x[1] += (double)d[1];
        x[2] += (double)d[2];
    }
    __device__ __forceinline__ void add_L(float h) { L += (double)h; }
    __device__ __forceinline__ double X(int a) const { return x[a]; }
    __device__ __forceinline__ double len() const { return L; }
    __device__ __forceinline__ void set_len(double v) { L = v; }
    // base cell index and FP32 fraction of (x - o) / spacing
    __device__ __forceinline__ void cell(const FieldDev &F, int a, int &i, float &t) const {
        double f = (x[a] - F.origin[a]) * F.inv_spacing;
        double fl = floor(f);
        t = (float)(f - fl);
        i = wrap((int)fl, F.n[a], F.pow2);
    }
    // base cell and FP32 fraction in the modulation grid
    __device__ __forceinline__ void mod_cell(const FieldDev &F, int a, int &i, float &t) const {
        double f = (x[a] - F.mod_origin[a]) * F.mod_inv_spacing;
        double fl = floor(f);
        t = (float)(f - fl);
        i = wrap((int)fl, F.mod_n[a], F.mod_pow2);
    }
    // reflective box: mirror the position on a face it crossed, negate that
    // direction component
    __device__ __forceinline__ void reflect(const ParamsDev &P, float u[3]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (x[a] > P.box_hi[a]) {
                x[a] = 2.0 * P.box_hi[a] - x[a];
                u[a] = -u[a];
            } else if (x[a] < P.box_lo[a]) {
                x[a] = 2.0 * P.box_lo[a] - x[a];
                u[a] = -u[a];
            }
        }
    }
    // |x + d - c|^2 - R^2
    __device__ __forceinline__ double sphere(const ParamsDev &P, const float d[3]) const {
        double q0 = (x[0] + (double)d[0]) - P.center[0];
        double q1 = (x[1] + (double)d[1]) - P.center[1];
        double q2 = (x[2] + (double)d[2]) - P.center[2];
        return (q0 * q0 + q1 * q1 + q2 * q2) - P.r2;
    }
};
template <> struct Acc<ACC_DF> {
    df x[3], L;
    __device__ __forceinline__ void set(const double p[3], double len) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a].hi = (float)p[a];
            x[a].lo = (float)(p[a] - (double)x[a].hi);
        }
        L.hi = (float)len;
        L.lo = (float)(len - (double)L.hi);
    }
    __device__ __forceinline__ void add_x(const float d[3]) {
        x[0] = df_add(x[0], d[0]);
        x[1] = df_add(x[1], d[1]);
        x[2] = df_add(x[2], d[2]);
    }
    __device__ __forceinline__ void add_L(float h) { L = df_add(L, h); }
    __device__ __forceinline__ double X(int a) const { return df_val(x[a]); }
    __device__ __forceinline__ double len() const { return df_val(L); }
    __device__ __forceinline__ void set_len(double v) {
        L.hi = (float)v;
        L.lo = (float)(v - (double)L.hi);
    }
    // (hi + lo - o) * inv with an exact FP32 product error term (origin taken in FP32)
    __device__ __forceinline__ void cell(const FieldDev &F, int a, int &i, float &t) const {
        float inv = (float)F.inv_spacing;
        float d = x[a].hi - (float)F.origin[a];
        float p = d * inv;
        float e = fmaf(d, inv, -p) + x[a].lo * inv;
        float fl = floorf(p);
        float fr = (p - fl) + e;
        if (fr < 0.0f) {
            fr += 1.0f;
            fl -= 1.0f;
        } else if (fr >= 1.0f) {
            fr -= 1.0f;
            fl += 1.0f;
        }
        t = fr;
        i = wrap((int)fl, F.n[a], F.pow2);
    }
    // base cell and FP32 fraction in the modulation grid (from the FP64 value)
    __device__ __forceinline__ void mod_cell(const FieldDev &F, int a, int &i, float &t) const {
        double f = (df_val(x[a]) - F.mod_origin[a]) * F.mod_inv_spacing;
        double fl = floor(f);
        t = (float)(f - fl);
        i = wrap((int)fl, F.mod_n[a], F.mod_pow2);
    }
    // reflective box: the mirrored position in FP64, split again into hi + lo
    __device__ __forceinline__ void reflect(const ParamsDev &P, float u[3]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = df_val(x[a]);
            double m = v;
            if (v > P.box_hi[a])
                m = 2.0 * P.box_hi[a] - v;
            else if (v < P.box_lo[a])
                m = 2.0 * P.box_lo[a] - v;
            if (m != v) {
                x[a].hi = (float)m;
                x[a].lo = (float)(m - (double)x[a].hi);
                u[a] = -u[a];
            }
        }
    }
    __device__ __forceinline__ double sphere(const ParamsDev &P, const float d[3]) const {
        float q0 = ((x[0].hi - (float)P.center[0]) + x[0].lo) + d[0];
        float q1 = ((x[1].hi - (float)P.center[1]) + x[1].lo) + d[1];
        float q2 = ((x[2].hi - (float)P.center[2]) + x[2].lo) + d[2];
        return (double)((q0 * q0 + q1 * q1 + q2 * q2) - (float)P.r2);
    }
};

// FP32 trilinear interpolation of a cell's stored corner values at
// fractions t (along x, then y, then z), times the grid's value scale.
template <class T>
__device__ __forceinline__ void interp_rel(const T (&v)[24], const float t[3], float sc, float B[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float c00 = lerpf(to_f32<T>(v[0 + c]), to_f32<T>(v[3 + c]), t[0]);
        float c10 = lerpf(to_f32<T>(v[6 + c]), to_f32<T>(v[9 + c]), t[0]);
        float c01 = lerpf(to_f32<T>(v[12 + c]), to_f32<T>(v[15 + c]), t[0]);
        float c11 = lerpf(to_f32<T>(v[18 + c]), to_f32<T>(v[21 + c]), t[0]);
        B[c] = lerpf(lerpf(c00, c10, t[1]), lerpf(c01, c11, t[1]), t[2]);
    }
    B[0] *= sc;
    B[1] *= sc;
    B[2] *= sc;
}

// Cell-relative FP32 lookup: base cell ib, fraction tb, stage offset d (Mpc).
// With CACHE, the last cell's corner values are kept in the lane's registers
// and a repeated lookup of that cell reads no global memory; those instances
// run at 2 waves per SIMD, whose register budget holds the cell unspilled.
template <class T, int LAYOUT, bool CACHE, bool MOD>
__device__ __forceinline__ void lookup_rel(const FieldDev &F, int fid, const int ib[3], const float tb[3],
                                           const ModRel &mr, const float d[3], float B[3], CellCache<T> &cache) {
    // modulation corners first, so that their loads and the vector grid's are in flight together
    float mv[8], mt[3];
    const bool mod = MOD && F.mod_data != nullptr;
    if (mod) {
        int mc[3];
        const float minv = (float)F.mod_inv_spacing;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float f = fmaf(d[a], minv, mr.tb[a]);
            float fl = floorf(f);
            mt[a] = f - fl;
            mc[a] = wrap(mr.ib[a] + (int)fl, F.mod_n[a], F.mod_pow2);
        }
        const uint32_t o = (uint32_t)mc[0] * F.mod_sx + (uint32_t)mc[1] * F.mod_sy + (uint32_t)mc[2];
        const uint32_t sx = F.mod_sx, sy = F.mod_sy;
        const uint32_t off[8] = {0, 1, sx, sx + 1, sy, sy + 1, sx + sy, sx + sy + 1};
        // with CACHE the modulation's last cell is kept too (as the FP32 values
        // used here); its cells are larger than the vector grid's
        const uint32_t mkey = ((uint32_t)mc[0] * (uint32_t)F.mod_n[1] + (uint32_t)mc[1]) * (uint32_t)F.mod_n[2] +
                              (uint32_t)mc[2];
        if (!CACHE || mkey != cache.mkey) {
            if (F.mod_dtype == CRP_F64) {
                const global_ptr<double> q = as_global<double>(F.mod_data) + o;
#pragma unroll
                for (int k = 0; k < 8; ++k) mv[k] = (float)q[off[k]];
            } else {
                const global_ptr<float> q = as_global<float>(F.mod_data) + o;
#pragma unroll
                for (int k = 0; k < 8; ++k) mv[k] = q[off[k]];
            }
            if constexpr (CACHE) {
#pragma unroll
                for (int k = 0; k < 8; ++k) cache.mv[k] = mv[k];
                cache.mkey = mkey;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) mv[k] = cache.mv[k];
        }
    }
    const float inv = (float)F.inv_spacing;
    int ci[3];
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = fmaf(d[a], inv, tb[a]);
        float fl = floorf(f);
        t[a] = f - fl;
        ci[a] = wrap(ib[a] + (int)fl, F.n[a], F.pow2);
    }
    T v[24];
    if constexpr (CACHE) {
        uint32_t key = ((uint32_t)ci[0] * (uint32_t)F.n[1] + (uint32_t)ci[1]) * (uint32_t)F.n[2] + (uint32_t)ci[2];
        if (key != cache.key || fid != cache.field) {
            load_corners<T, LAYOUT>(F, ci[0], ci[1], ci[2], cache.v);
            cache.key = key;
            cache.field = fid;
            cache.misses++;
        }
#pragma unroll
        for (int w = 0; w < 24; ++w) v[w] = cache.v[w];
    } else {
        load_corners<T, LAYOUT>(F, ci[0], ci[1], ci[2], v);
        cache.misses++;
    }
    interp_rel<T>(v, t, (float)F.value_scale, B);
    if (mod) {
        // trilinear as the FP64 path: along x, then y, then z
        const float c00 = lerpf(mv[0], mv[2], mt[0]);  // (y, z) = (0, 0)
        const float c10 = lerpf(mv[4], mv[6], mt[0]);  // (1, 0)
        const float c01 = lerpf(mv[1], mv[3], mt[0]);  // (0, 1)
        const float c11 = lerpf(mv[5], mv[7], mt[0]);  // (1, 1)
        const float m = lerpf(lerpf(c00, c10, mt[1]), lerpf(c01, c11, mt[1]), mt[2]);
        B[0] *= m;
        B[1] *= m;
        B[2] *= m;
    }
}

// fmaf(t, d, a) into a register of its own (the two-address fma would
// overwrite the cached addend a; same rounding as fmaf).
__device__ __forceinline__ float fmaf_keep(float t, float d, float a) {
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(t), "v"(d), "v"(a));
    return r;
}

// interp_rel on a cell held as FP32 x-edges: edge e = (dz*2 + dy)*3 + c has
// lower value fa[e] and upper minus lower fd[e], as interp_rel forms them.
__device__ __forceinline__ void interp_rel_edges(const float (&fa)[12], const float (&fd)[12], const float t[3],
                                                 float sc, float B[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float c00 = fmaf_keep(t[0], fd[0 + c], fa[0 + c]);
        float c10 = fmaf_keep(t[0], fd[3 + c], fa[3 + c]);
        float c01 = fmaf_keep(t[0], fd[6 + c], fa[6 + c]);
        float c11 = fmaf_keep(t[0], fd[9 + c], fa[9 + c]);
        B[c] = lerpf(lerpf(c00, c10, t[1]), lerpf(c01, c11, t[1]), t[2]);
    }
    B[0] *= sc;
    B[1] *= sc;
    B[2] *= sc;
}

template <class T>
__device__ __forceinline__ void edges_rel(const T (&v)[24], float (&fa)[12], float (&fd)[12]) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            fa[3 * e + c] = to_f32<T>(v[6 * e + c]);
            fd[3 * e + c] = to_f32<T>(v[6 * e + 3 + c]) - fa[3 * e + c];
        }
}

// Two cell-relative lookups whose offsets are both known (register cell
// cache, no modulation): the corner loads of both cells are issued before
// the first is waited for.  Every lane issues both loads, a lane whose cell
// is already cached reading the grid's first record instead (one line for
// the whole wavefront), so that the wait for the first cell is not also a
// wait for the second; the empty asm keeps the compiler from moving each load
// into the branch that uses it.  Cells, fractions and interpolation are those
// of lookup_rel (the cell cached as its FP32 x-edges), and the cache holds
// the cell two calls of it would leave it holding.
template <class T, int LAYOUT>
__device__ __forceinline__ void lookup_pair_rel(const FieldDev &F, int fid, const int ib[3], const float tb[3],
                                                const float dA[3], const float dB[3], float BA[3], float BB[3],
                                                CellCache<T> &cache) {
    const float inv = (float)F.inv_spacing;
    int ca[3], cb[3];
    float ta[3], tbb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float f = fmaf(dA[a], inv, tb[a]);
        float fl = floorf(f);
        ta[a] = f - fl;
        ca[a] = wrap(ib[a] + (int)fl, F.n[a], F.pow2);
        float g = fmaf(dB[a], inv, tb[a]);
        float gl = floorf(g);
        tbb[a] = g - gl;
        cb[a] = wrap(ib[a] + (int)gl, F.n[a], F.pow2);
    }
    const uint32_t ka = ((uint32_t)ca[0] * (uint32_t)F.n[1] + (uint32_t)ca[1]) * (uint32_t)F.n[2] + (uint32_t)ca[2];
    const uint32_t kb = ((uint32_t)cb[0] * (uint32_t)F.n[1] + (uint32_t)cb[1]) * (uint32_t)F.n[2] + (uint32_t)cb[2];
    const bool missA = ka != cache.key || fid != cache.field;
    const bool missB = kb != ka;
    T va[24], vb[24];
    load_cell<T, LAYOUT>(F, ka, ca[0], ca[1], ca[2], missA, va);
    load_cell<T, LAYOUT>(F, kb, cb[0], cb[1], cb[2], missB, vb);
    asm volatile("" ::: "memory");
    const float sc = (float)F.value_scale;
    if (missA) {
        edges_rel<T>(va, cache.fa, cache.fd);
        cache.key = ka;
        cache.field = fid;
        cache.misses++;
    }
    interp_rel_edges(cache.fa, cache.fd, ta, sc, BA);
    if (missB) {
        edges_rel<T>(vb, cache.fa, cache.fd);
        cache.key = kb;
        cache.misses++;
    }
    interp_rel_edges(cache.fa, cache.fd, tbb, sc, BB);
}

__device__ __forceinline__ void lorentz(float kap, const float U[3], const float B[3], float F[3]) {
    F[0] = kap * (U[1] * B[2] - U[2] * B[1]);
    F[1] = kap * (U[2] * B[0] - U[0] * B[2]);
    F[2] = kap * (U[0] * B[1] - U[1] * B[0]);
}

// One FP32 Cash-Karp evaluation from (x, u) with step h: the position offset
// dx5, the new direction u5 (unnormalised), and the error norms.
template <class T, int LAYOUT, bool CACHE, bool MOD>
__device__ __forceinline__ void ck_eval_f32(const FieldDev &F, int fid, CellCache<T> &cache, const int ib[3],
                                            const float tb[3], const ModRel &mr, float kap, const float u[3], float h, float dx5[3],
                                            float u5[3], float &ex, float &eu) {
    float U2[3], U3[3], U4[3], U5[3], U6[3];
    float F1[3], F2[3], F3[3], F4[3], F5[3], F6[3];
    float d[3], B[3];
    const float z[3] = {0.f, 0.f, 0.f};
    if constexpr (CACHE && !MOD) {
        // stages (1, 2), (3, 4), (5, 6) in pairs: the offset of stage i+1
        // needs the directions up to stage i, so the fields only up to i-1;
        // each quantity is the same expression as below
        float e[3], B2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) e[c] = h * (a21 * u[c]);
        lookup_pair_rel<T, LAYOUT>(F, fid, ib, tb, z, e, B, B2, cache);
        lorentz(kap, u, B, F1);
#pragma unroll
        for (int c = 0; c < 3; ++c) U2[c] = fmaf(h, a21 * F1[c], u[c]);
        lorentz(kap, U2, B2, F2);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d[c] = h * fmaf(a32, U2[c], a31 * u[c]);
            U3[c] = fmaf(h, fmaf(a32, F2[c], a31 * F1[c]), u[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) e[c] = h * fmaf(a43, U3[c], fmaf(a42, U2[c], a41 * u[c]));
        lookup_pair_rel<T, LAYOUT>(F, fid, ib, tb, d, e, B, B2, cache);
        lorentz(kap, U3, B, F3);
#pragma unroll
        for (int c = 0; c < 3; ++c) U4[c] = fmaf(h, fmaf(a43, F3[c], fmaf(a42, F2[c], a41 * F1[c])), u[c]);
        lorentz(kap, U4, B2, F4);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d[c] = h * fmaf(a54, U4[c], fmaf(a53, U3[c], fmaf(a52, U2[c], a51 * u[c])));
            U5[c] = fmaf(h, fmaf(a54, F4[c], fmaf(a53, F3[c], fmaf(a52, F2[c], a51 * F1[c]))), u[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            e[c] = h * fmaf(a65, U5[c], fmaf(a64, U4[c], fmaf(a63, U3[c], fmaf(a62, U2[c], a61 * u[c]))));
        lookup_pair_rel<T, LAYOUT>(F, fid, ib, tb, d, e, B, B2, cache);
        lorentz(kap, U5, B, F5);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            U6[c] = fmaf(h, fmaf(a65, F5[c], fmaf(a64, F4[c], fmaf(a63, F3[c], fmaf(a62, F2[c], a61 * F1[c])))), u[c]);
        lorentz(kap, U6, B2, F6);
    } else {
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, z, B, cache);
    lorentz(kap, u, B, F1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = h * (a21 * u[c]);
        U2[c] = fmaf(h, a21 * F1[c], u[c]);
    }
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, d, B, cache);
    lorentz(kap, U2, B, F2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = h * fmaf(a32, U2[c], a31 * u[c]);
        U3[c] = fmaf(h, fmaf(a32, F2[c], a31 * F1[c]), u[c]);
    }
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, d, B, cache);
    lorentz(kap, U3, B, F3);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = h * fmaf(a43, U3[c], fmaf(a42, U2[c], a41 * u[c]));
        U4[c] = fmaf(h, fmaf(a43, F3[c], fmaf(a42, F2[c], a41 * F1[c])), u[c]);
    }
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, d, B, cache);
    lorentz(kap, U4, B, F4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = h * fmaf(a54, U4[c], fmaf(a53, U3[c], fmaf(a52, U2[c], a51 * u[c])));
        U5[c] = fmaf(h, fmaf(a54, F4[c], fmaf(a53, F3[c], fmaf(a52, F2[c], a51 * F1[c]))), u[c]);
    }
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, d, B, cache);
    lorentz(kap, U5, B, F5);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        d[c] = h * fmaf(a65, U5[c], fmaf(a64, U4[c], fmaf(a63, U3[c], fmaf(a62, U2[c], a61 * u[c]))));
        U6[c] = fmaf(h, fmaf(a65, F5[c], fmaf(a64, F4[c], fmaf(a63, F3[c], fmaf(a62, F2[c], a61 * F1[c])))), u[c]);
    }
    lookup_rel<T, LAYOUT, CACHE, MOD>(F, fid, ib, tb, mr, d, B, cache);
    lorentz(kap, U6, B, F6);
    }
    float exx[3], euu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dx5[c] = h * fmaf(b56, U6[c], fmaf(b54, U4[c], fmaf(b53, U3[c], b51 * u[c])));
        u5[c] = fmaf(h, fmaf(b56, F6[c], fmaf(b54, F4[c], fmaf(b53, F3[c], b51 * F1[c]))), u[c]);
        exx[c] = h * fmaf(e6, U6[c], fmaf(e5, U5[c], fmaf(e4, U4[c], fmaf(e3, U3[c], e1 * u[c]))));
        euu[c] = h * fmaf(e6, F6[c], fmaf(e5, F5[c], fmaf(e4, F4[c], fmaf(e3, F3[c], e1 * F1[c]))));
    }
    ex = sqrtf(exx[0] * exx[0] + exx[1] * exx[1] + exx[2] * exx[2]);
    eu = sqrtf(euu[0] * euu[0] + euu[1] * euu[1] + euu[2] * euu[2]);
}

template <int ACC>
struct Lane {
    Acc<ACC> acc;
    float u[3];
    float kap, hctrl, h;
    int32_t dacc, drej, mode, binding, pidx;
};

struct EventLDS {
    float lo[MAX_BLOCK], hi[MAX_BLOCK], hacc[MAX_BLOCK];
    double glo[MAX_BLOCK], ghi[MAX_BLOCK], lacc[MAX_BLOCK];
    int32_t side[MAX_BLOCK], eit[MAX_BLOCK];
};

template <int ACC, bool RFL>
__device__ __forceinline__ void bid(const ParamsDev &P, Lane<ACC> &s) {
    float h = s.hctrl;
    const float hmax = (float)P.h_max, hmin = (float)P.h_min;
    if (h > hmax) h = hmax;
    if (P.sphere_on) {
        const float z[3] = {0.f, 0.f, 0.f};
        double g = s.acc.sphere(P, z);  // |x - c|^2 - R^2
        // g + R^2 is |x - c|^2 up to the rounding of R^2 inside g: at the
        // centre it can come out a few ulp below zero, which is clamped
        double r = sqrt(fmax(g + P.r2, 0.0));
        float dist = (float)(P.radius - r);
        if (dist < h) h = dist;
    }
    if (RFL && P.reflect_on) {
        // the distance to the nearest face of the reflective box bids too
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double xa = s.acc.X(a);
            const float dlo = (float)(xa - P.box_lo[a]), dhi = (float)(P.box_hi[a] - xa);
            if (dlo < h) h = dlo;
            if (dhi < h) h = dhi;
        }
    }
    if (h < hmin) h = hmin;
    s.binding = 0;
    if (P.lmax_on) {
        double rem = P.l_max - s.acc.len();
        if (rem <= (double)h) {
            h = (float)rem;
            s.binding = 1;
        }
    }
    s.h = h;
}

template <int ACC>
__device__ __forceinline__ void store(const ParamsDev &P, int64_t p, const Lane<ACC> &s, double hnext, int st) {
    KernArg<PropArgs> &a = kernel_args<PropArgs>();
    a.x[p] = s.acc.X(0);
    a.y[p] = s.acc.X(1);
    a.z[p] = s.acc.X(2);
    // backtracking carries the antiparticle's direction: reverse it back
    const double sg = P.backtrack_on ? -1.0 : 1.0;
    a.ux[p] = sg * (double)s.u[0];
    a.uy[p] = sg * (double)s.u[1];
    a.uz[p] = sg * (double)s.u[2];
    // a length stop lands on l_max exactly, as in the FP64 path (a double-float
    // length cannot hold every FP64 l_max)
    double L = st == CRP_ST_MAX_LENGTH && P.lmax_on ? P.l_max : s.acc.len();
    a.length[p] = L;
    a.h_next[p] = hnext;
    if (s.dacc) a.n_acc[p] += s.dacc;
    if (s.drej) a.n_rej[p] += s.drej;
    if (a.time) a.time[p] = L * SEC_PER_MPC;
    a.status[p] = st;
}

template <int ACC>
__device__ __forceinline__ void event_next(const ParamsDev &P, Lane<ACC> &s, EventLDS &e, int t) {
    float lo = e.lo[t], hi = e.hi[t];
    double glo = e.glo[t], ghi = e.ghi[t];
    // FP32 stages resolve the crossing to ~1e-6 R; stop there or on a small bracket
    if (ghi <= 1e-7 * P.r2 || (hi - lo) <= 1e-6f * e.hacc[t] || e.eit[t] >= 30) {
        s.mode = MODE_FINAL;
        s.h = hi;
    } else {
        s.h = (float)(((double)lo * ghi - (double)hi * glo) / (ghi - glo));
    }
}

template <bool MULTI, int ACC, bool RFL>
__device__ __forceinline__ bool start(const PropArgs &args, int64_t p, Lane<ACC> &s) {
    KernArg<PropArgs> &a = kernel_args<PropArgs>();  // the particle arrays
    if (a.status[p] != CRP_ST_ACTIVE) return false;
    s.pidx = MULTI && a.param_index ? a.param_index[p] : 0;
    if (MULTI && (s.pidx < 0 || s.pidx >= a.n_params)) {
        a.status[p] = CRP_ST_BAD_INPUT;
        return false;
    }
    const ParamsDev &P = MULTI ? args.params[s.pidx] : args.P0;
    double E = a.energy[p];
    int Z = a.charge[p];
    double x[3] = {a.x[p], a.y[p], a.z[p]};
    double u[3] = {a.ux[p], a.uy[p], a.uz[p]};
    if (P.backtrack_on) {  // the antiparticle, moving the other way
        u[0] = -u[0];
        u[1] = -u[1];
        u[2] = -u[2];
    }
    double L = a.length[p];
    double hn = a.h_next[p];
    s.dacc = 0;
    s.drej = 0;
    bool ok = E > 0.0 && isfinite(E) && isfinite(L) && hn >= 0.0 && isfinite(hn);
#pragma unroll
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(x[c]) && isfinite(u[c]);
    if (ok && hn == 0.0) {
        double n2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        if (n2 > 0.0) {
            double nrm = sqrt(n2);
            u[0] /= nrm;
            u[1] /= nrm;
            u[2] /= nrm;
        } else {
            ok = false;
        }
    }
    if (!ok) {
        a.status[p] = CRP_ST_BAD_INPUT;
        return false;
    }
    s.acc.set(x, L);
    s.u[0] = (float)u[0];
    s.u[1] = (float)u[1];
    s.u[2] = (float)u[2];
    const float z[3] = {0.f, 0.f, 0.f};
    if (P.sphere_on && s.acc.sphere(P, z) >= 0.0) {
        store(P, p, s, hn, CRP_ST_ARRIVED);
        return false;
    }
    if (P.lmax_on && L >= P.l_max) {
        store(P, p, s, hn, CRP_ST_MAX_LENGTH);
        return false;
    }
    s.hctrl = hn == 0.0 ? (float)P.h_max : (float)hn;
    s.kap = (float)(((double)(P.backtrack_on ? -Z : Z) * K_LORENTZ) / E);
    s.mode = MODE_NORMAL;
    bid<ACC, RFL>(P, s);
    return true;
}

template <class T, int LAYOUT, bool MULTI, int ACC, bool CACHE, bool RFL, bool MOD>
__device__ __forceinline__ int advance(const PropArgs &a, int64_t p, Lane<ACC> &s, CellCache<T> &cache, EventLDS &e,
                                       int &flags, bool cancel) {
    const int t = threadIdx.x;
    // per-particle groups: the lane's descriptors, read from the tables once
    // per iteration into registers (the lanes of a wavefront may differ)
    ParamsDev Pm;
    FieldDev Fm;
    if (MULTI) {
        Pm = a.params[s.pidx];
        Fm = a.fields[Pm.field_index];
    }
    const ParamsDev &P = MULTI ? Pm : a.P0;
    const int fid = MULTI ? P.field_index : 0;
    const FieldDev &F = MULTI ? Fm : a.F0;
    int ib[3];
    float tb[3];
    s.acc.cell(F, 0, ib[0], tb[0]);
    s.acc.cell(F, 1, ib[1], tb[1]);
    s.acc.cell(F, 2, ib[2], tb[2]);
    ModRel mr;
    if (MOD && F.mod_data) {
        s.acc.mod_cell(F, 0, mr.ib[0], mr.tb[0]);
        s.acc.mod_cell(F, 1, mr.ib[1], mr.tb[1]);
        s.acc.mod_cell(F, 2, mr.ib[2], mr.tb[2]);
    }
    float dx5[3], u5[3], ex, eu;
    ck_eval_f32<T, LAYOUT, CACHE, MOD>(F, fid, cache, ib, tb, mr, s.kap, s.u, s.h, dx5, u5, ex, eu);
    flags = F_EVAL;

    if (s.mode == MODE_NORMAL) {
        float exh = ex / s.h;
        if (!isfinite(eu) || !isfinite(exh)) {
            store(P, p, s, (double)s.hctrl, CRP_ST_NONFINITE);
            return CRP_ST_NONFINITE;
        }
        float err = (eu > exh ? eu : exh) / (float)P.tol;
        const float hmin = (float)P.h_min, hmax = (float)P.h_max;
        if (err > 1.0f && s.h > hmin) {
            float fac = 0.9f / sqrtf(sqrtf(err));
            if (fac < 0.1f) fac = 0.1f;
            float h = s.h * fac;
            if (h < hmin) h = hmin;
            s.h = h;
            s.binding = 0;
            s.drej++;
            flags |= F_REJ;
            return CRP_ST_ACTIVE;
        }
        float g;
        if (err > 1.0f) {
            g = 1.0f;
            flags |= F_FLOOR;
        } else if (err == 0.0f) {
            g = 5.0f;
        } else {
            g = 0.9f * exp2f(-0.2f * log2f(err));
            if (g > 5.0f) g = 5.0f;
        }
        float hc = s.h * g;
        if (hc < hmin) hc = hmin;
        if (hc > hmax) hc = hmax;
        s.hctrl = hc;
        double Lnew = s.binding ? P.l_max : s.acc.len() + (double)s.h;
        s.dacc++;
        flags |= F_ACC;
        if (P.sphere_on && s.acc.sphere(P, dx5) >= 0.0) {
            const float z[3] = {0.f, 0.f, 0.f};
            s.mode = MODE_EVENT;
            e.lo[t] = 0.0f;
            e.glo[t] = s.acc.sphere(P, z);
            e.hi[t] = s.h;
            e.ghi[t] = s.acc.sphere(P, dx5);
            e.hacc[t] = s.h;
            e.lacc[t] = Lnew;
            e.side[t] = 0;
            e.eit[t] = 0;
            event_next(P, s, e, t);
            return CRP_ST_ACTIVE;
        }
        float un = sqrtf(u5[0] * u5[0] + u5[1] * u5[1] + u5[2] * u5[2]);
        s.acc.add_x(dx5);
        if (s.binding)
            s.acc.set_len(P.l_max);
        else
            s.acc.add_L(s.h);
        s.u[0] = u5[0] / un;
        s.u[1] = u5[1] / un;
        s.u[2] = u5[2] / un;
        if (RFL && P.reflect_on) s.acc.reflect(P, s.u);
        // the step that took the remaining length ends the particle: a double-float
        // length may stay a rounding below an l_max it cannot represent
        if (P.lmax_on && (s.binding || s.acc.len() >= P.l_max)) {
            store(P, p, s, (double)s.hctrl, CRP_ST_MAX_LENGTH);
            return CRP_ST_MAX_LENGTH;
        }
        if (P.max_steps > 0 && s.dacc >= P.max_steps) {
            store(P, p, s, (double)s.hctrl, CRP_ST_MAX_STEPS);
            return CRP_ST_MAX_STEPS;
        }
        if (cancel) {  // the caller's cancel flag: stop here, resumable like a used-up budget
            store(P, p, s, (double)s.hctrl, CRP_ST_CANCELLED);
            return CRP_ST_CANCELLED;
        }
        bid<ACC, RFL>(P, s);
        return CRP_ST_ACTIVE;
    }

    flags |= F_EVENT;
    if (s.mode == MODE_EVENT) {
        double gs = s.acc.sphere(P, dx5);
        if (!isfinite(gs)) {
            store(P, p, s, (double)s.hctrl, CRP_ST_NONFINITE);
            return CRP_ST_NONFINITE;
        }
        if (gs >= 0.0) {
            e.hi[t] = s.h;
            e.ghi[t] = gs;
            if (e.side[t] == 1) e.glo[t] = e.glo[t] * 0.5;
            e.side[t] = 1;
        } else {
            e.lo[t] = s.h;
            e.glo[t] = gs;
            if (e.side[t] == -1) e.ghi[t] = e.ghi[t] * 0.5;
            e.side[t] = -1;
        }
        e.eit[t] += 1;
        event_next(P, s, e, t);
        return CRP_ST_ACTIVE;
    }

    // MODE_FINAL
    float sn = sqrtf(u5[0] * u5[0] + u5[1] * u5[1] + u5[2] * u5[2]);
    double Lf = e.hi[t] == e.hacc[t] ? e.lacc[t] : s.acc.len() + (double)e.hi[t];
    s.acc.add_x(dx5);
    s.acc.set_len(Lf);
    s.u[0] = u5[0] / sn;
    s.u[1] = u5[1] / sn;
    s.u[2] = u5[2] / sn;
    store(P, p, s, (double)s.hctrl, CRP_ST_ARRIVED);
    return CRP_ST_ARRIVED;
}

template <class T, int LAYOUT, bool MULTI, int ACC, bool CACHE, bool RFL, bool MOD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CACHE ? 2 : 4, 8))) k_propagate_mixed(PropArgs a) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int64_t pid = -1;
    __shared__ EventLDS ev;
    CellCache<T> cache;
    cache_reset(cache);
    Lane<ACC> s;
    unsigned long long n_eval = 0, n_acc = 0, n_rej = 0, n_ev = 0, n_fl = 0, n_taken = 0, n_iter = 0;
    bool cancel = false;  // the caller's cancel flag was seen set (read every 64 iterations)

    for (;;) {
        if ((n_iter & 63u) == 0 && !cancel) {
            // the pointer is read from the kernel-argument segment here, not held in
            // registers across the loop
            const int32_t *cw = kernel_args<PropArgs>().cancel;
            if (cw) cancel = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
        }
        for (;;) {
            unsigned long long want = __ballot(pid == -1);
            if (want == 0ull) break;
            unsigned long long busy = __ballot(pid >= 0);
            int nwant = __popcll(want);
            if (busy != 0ull && nwant < a.refill_threshold) break;
            int leader = __ffsll((long long)want) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)nwant);
            base = __shfl(base, leader, 64);
            unsigned long long got = 0;
            if (pid == -1) {
                unsigned long long q = base + (unsigned long long)__popcll(want & below);
                if (q < (unsigned long long)a.n && !cancel) {
                    int64_t p = a.order ? (int64_t)a.order[q] : (int64_t)q;
                    got = 1;
                    pid = start<MULTI, ACC, RFL>(a, p, s) ? p : -1;
                } else {
                    pid = -2;
                }
            }
            n_taken += __popcll(__ballot(got != 0));
        }
        if (__ballot(pid >= 0) == 0ull) {
            if (__ballot(pid == -1) == 0ull) break;
            continue;
        }
        n_iter++;
        int flags = 0;
        if (pid >= 0) {
            int st = advance<T, LAYOUT, MULTI, ACC, CACHE, RFL, MOD>(a, pid, s, cache, ev, flags, cancel);
            if (st != CRP_ST_ACTIVE) pid = -1;
        }
        n_eval += __popcll(__ballot(flags & F_EVAL));
        n_acc += __popcll(__ballot(flags & F_ACC));
        n_rej += __popcll(__ballot(flags & F_REJ));
        n_ev += __popcll(__ballot(flags & F_EVENT));
        n_fl += __popcll(__ballot(flags & F_FLOOR));
    }
    if (a.counters) {
        unsigned long long m = (unsigned long long)cache.misses;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
        if (lane == 0) {
            unsigned long long v[8] = {n_eval, n_acc, n_rej, n_ev, n_fl, n_taken, m, n_iter};
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (v[i]) atomicAdd(a.counters + i, v[i]);
        }
    }
}

template <class T, int LAYOUT, bool MULTI, int ACC>
hipError_t launch_feat(const PropArgs &a, bool cache, const dim3 &g, const dim3 &b, hipStream_t s) {
    // the reflective box and the modulation each have their own instances;
    // with them the cell cache is instantiated for one parameter group only
    constexpr bool C = !MULTI;
    if (a.reflective && a.modulated) {
        if (C && cache)
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, C, true, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, false, true, true>), g, b, 0, s, a);
    } else if (a.reflective) {
        if (C && cache)
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, C, true, false>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, false, true, false>), g, b, 0, s, a);
    } else if (a.modulated) {
        if (C && cache)
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, C, false, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, false, false, true>), g, b, 0, s, a);
    } else if (cache)
        hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, true, false, false>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((k_propagate_mixed<T, LAYOUT, MULTI, ACC, false, false, false>), g, b, 0, s, a);
    return hipGetLastError();
}

template <class T, int LAYOUT, bool MULTI>
hipError_t launch_acc(const PropArgs &a, int acc, bool cache, int blocks, int bs, hipStream_t s) {
    const dim3 g(blocks), b(bs);
    return acc == ACC_DF ? launch_feat<T, LAYOUT, MULTI, ACC_DF>(a, cache, g, b, s)
                         : launch_feat<T, LAYOUT, MULTI, ACC_F64>(a, cache, g, b, s);
}

template <class T>
hipError_t launch_layout(const PropArgs &a, int layout, bool multi, int acc, bool cache, int blocks, int bs,
                         hipStream_t s) {
    if (layout == CRP_LAYOUT_CELL8)
        return multi ? launch_acc<T, CRP_LAYOUT_CELL8, true>(a, acc, cache, blocks, bs, s)
                     : launch_acc<T, CRP_LAYOUT_CELL8, false>(a, acc, cache, blocks, bs, s);
    return multi ? launch_acc<T, CRP_LAYOUT_LINEAR, true>(a, acc, cache, blocks, bs, s)
                 : launch_acc<T, CRP_LAYOUT_LINEAR, false>(a, acc, cache, blocks, bs, s);
}

}  // namespace

hipError_t launch_propagate_mixed(const PropArgs &a, int dtype, int layout, bool multi, int precision, bool cache,
                                  int blocks, int block_size, hipStream_t s) {
    int acc = precision == CRP_PREC_MIXED_DFACC ? ACC_DF : ACC_F64;
    switch (dtype) {
        case CRP_F64: return launch_layout<double>(a, layout, multi, acc, cache, blocks, block_size, s);
        case CRP_F32: return launch_layout<float>(a, layout, multi, acc, cache, blocks, block_size, s);
        case CRP_F16: return launch_layout<__half>(a, layout, multi, acc, cache, blocks, block_size, s);
        case CRP_BF16: return launch_layout<__hip_bfloat16>(a, layout, multi, acc, cache, blocks, block_size, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace crp
