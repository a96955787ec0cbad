// adjoint_fp64.hip -- reverse-mode derivatives of a taped FP64 propagation
// (gfx950).
//
// The derivative is that of the replayed map: the accepted step sizes of the
// taped forward run are held fixed and the sphere crossing in the last step is
// differentiated through its defining equation (implicit function theorem).
// A particle's accepted steps are replayed from its checkpoints with the
// propagation kernel's own step logic (so the states are bit-identical),
// recording every accepted step's stage states and stage field values; the
// records are then swept in reverse.  The reverse sweep reads the recorded
// stages instead of recomputing them, so it gathers each stage's cell once
// (for the field gradient) and adds the grid-gradient contributions to a
// natural-layout FP64 or FP32 array with atomics.
//
// Where the replay happens:
//  * in the sweep kernel, one checkpoint segment at a time, into its
//    wavefront's block of records (every particle, when no parallel-replay
//    space is given);
//  * before the sweep, for the particles with the most accepted steps that
//    fit in the workspace's parallel-replay space: every checkpoint segment
//    of theirs is replayed by a thread of its own (segments are independent
//    given their checkpoints), so the sweep of those particles is only the
//    reverse pass, and their grid contributions are added after it.  Their
//    records are the same bits either way.
#include "adjoint.h"
#include "lane.h"

namespace crp {
namespace {

// Record of one accepted step, its fields `stride` doubles apart (64: the
// records of a wavefront's lanes interleave, so that a field's loads and
// stores are contiguous across the wavefront): the
// pre-step state y (6), the step size (1), the stage states Y_1..Y_5 (30),
// the stage field values B_0..B_5 (18), the unnormalised output direction
// (3) and, in a reflective box, the axes mirrored after the step (1).
constexpr int REC_Y = 0, REC_H = 6, REC_STAGE = 7, REC_FIELD = 37, REC_ZU = 55, REC_MIR = 58,
              REC_SIZE = ADJ_RECORD_DOUBLES;
static_assert(REC_MIR + 1 == REC_SIZE, "record layout");

// Stage recorder of a replayed step.  Vector-memory loads and stores retire
// through one in-order counter, so a store issued before a field gather would
// hold up the wait for that gather: the stage fields are kept in registers
// and every record store is issued after the step's last gather, the stage
// states recomputed from the stage derivatives with the step's own formulas
// (the same bits).
struct RecordWriter {
    static constexpr bool records = true;
    static constexpr bool deferred = true;
    double *r;       // field 0 of the record
    int64_t stride;  // doubles between its fields
    mutable double B[6][3];
    __device__ __forceinline__ void stage(int, const double *) const {}
    __device__ __forceinline__ void field(int i, const double *b) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) B[i][c] = b[c];
    }
    __device__ __forceinline__ void flush(const double *y, double h, const double *k1, const double *k2,
                                          const double *k3, const double *k4, const double *k5) const {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            r[(REC_STAGE + c) * stride] = ck_y1(y, h, k1, c);
            r[(REC_STAGE + 6 + c) * stride] = ck_y2(y, h, k1, k2, c);
            r[(REC_STAGE + 12 + c) * stride] = ck_y3(y, h, k1, k2, k3, c);
            r[(REC_STAGE + 18 + c) * stride] = ck_y4(y, h, k1, k2, k3, k4, c);
            r[(REC_STAGE + 24 + c) * stride] = ck_y5(y, h, k1, k2, k3, k4, k5, c);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) r[(REC_FIELD + 3 * i + c) * stride] = B[i][c];
    }
};

// Stage i's state (i = 0 is the pre-step state) and field value from a record.
__device__ __forceinline__ void rec_stage(const double *r, int64_t stride, int i, double Y[6]) {
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = r[(i == 0 ? REC_Y + c : REC_STAGE + 6 * (i - 1) + c) * stride];
}
__device__ __forceinline__ void rec_field(const double *r, int64_t stride, int i, double B[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) B[c] = r[(REC_FIELD + 3 * i + c) * stride];
}

// Component c of the stage derivative k_i = (U_i, kappa U_i x B_i), evaluated
// exactly as the forward right-hand side does.
__device__ __forceinline__ double stage_k(double kap, const double Y[6], const double B[3], int c) {
    switch (c) {
        case 0: return Y[3];
        case 1: return Y[4];
        case 2: return Y[5];
        case 3: return kap * (Y[4] * B[2] - Y[5] * B[1]);
        case 4: return kap * (Y[5] * B[0] - Y[3] * B[2]);
        default: return kap * (Y[3] * B[1] - Y[4] * B[0]);
    }
}

// One attempt of the replay of a step from lane state s, exactly as advance()
// takes it (the caller bids before a step's first attempt): one Cash-Karp
// evaluation recorded at r (this lane's record), then either a rejection
// (smaller step, returns false) or the acceptance (controller, normalisation,
// the mirror in a reflective box, the pre-step state, step size and mirrored
// axes recorded; returns true).
template <class T, int LAYOUT, bool RFL, bool MOD>
__device__ __forceinline__ bool replay_attempt(const FieldDev &F, const ParamsDev &P, Lane &s, double *r, int64_t stride) {
    CellCache<T> cache;
    cache_reset(cache);
    const RecordWriter rec{r, stride};
    double y5[6], ex, eu;
    ck_eval<T, LAYOUT, false, RecordWriter, MOD>(F, 0, cache, s.kap, s.y, s.h, y5, ex, eu, rec);
    double exh = ex / s.h;
    double em = eu > exh ? eu : exh;
    double err = em / P.tol;
    if (err > 1.0 && s.h > P.h_min) {
        double fac = 0.9 * (1.0 / sqrt(sqrt(err)));
        if (fac < 0.1) fac = 0.1;
        double h = s.h * fac;
        if (h < P.h_min) h = P.h_min;
        s.h = h;
        s.binding = 0;
        return false;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) r[(REC_Y + c) * stride] = s.y[c];
    r[REC_H * stride] = s.h;
#pragma unroll
    for (int c = 0; c < 3; ++c) r[(REC_ZU + c) * stride] = y5[3 + c];
    double g;
    if (err > 1.0) {
        g = 1.0;
    } else if (err == 0.0) {
        g = 5.0;
    } else {
        g = 0.9 * inv_fifth_root(err);
        if (g > 5.0) g = 5.0;
    }
    double hc = s.h * g;
    if (hc < P.h_min) hc = P.h_min;
    if (hc > P.h_max) hc = P.h_max;
    s.hctrl = hc;
    double Lnew = s.binding ? P.l_max : s.L + s.h;
    double un = sqrt(y5[3] * y5[3] + y5[4] * y5[4] + y5[5] * y5[5]);
    s.y[0] = y5[0];
    s.y[1] = y5[1];
    s.y[2] = y5[2];
    s.y[3] = y5[3] / un;
    s.y[4] = y5[4] / un;
    s.y[5] = y5[5] / un;
    if (RFL) r[REC_MIR * stride] = (double)reflect(P, s.y);
    s.L = Lnew;
    return true;
}

// Cotangent through the mirror of a recorded step: on each mirrored axis the
// map is x -> 2 face - x, u -> -u, so both cotangent components change sign.
__device__ __forceinline__ void mirror_cotangent(const double *r, int64_t stride, double lam[6]) {
    const int m = (int)r[REC_MIR * stride];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (m >> c & 1) {
            lam[c] = -lam[c];
            lam[3 + c] = -lam[3 + c];
        }
}

// Cell of X with its trilinear fractions and the cell's stored corner values.
template <class T, int LAYOUT>
__device__ __forceinline__ void cell_of(const FieldDev &F, const double X[3], int ci[3], double t[3], T (&raw)[24]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) ci[a] = cell_axis(X[a], F.origin[a], F.inv_spacing, F.n[a], F.pow2, t[a]);
    load_corners<T, LAYOUT>(F, ci[0], ci[1], ci[2], raw);
}

// Corner q (bit 0: +x, bit 1: +y, bit 2: +z) of the cell: its trilinear
// weight, the weight's gradient (per Mpc) and the node's index in the natural
// [n0][n1][n2] layout.
__device__ __forceinline__ double corner_weight(const FieldDev &F, const int ci[3], const double t[3], int q,
                                                double dw[3], int64_t &node) {
    const int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
    const double wx = dx ? t[0] : 1.0 - t[0], wy = dy ? t[1] : 1.0 - t[1], wz = dz ? t[2] : 1.0 - t[2];
    const double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
    dw[0] = sx * wy * wz * F.inv_spacing;
    dw[1] = wx * sy * wz * F.inv_spacing;
    dw[2] = wx * wy * sz * F.inv_spacing;
    const int ix = dx ? (ci[0] + 1 == F.n[0] ? 0 : ci[0] + 1) : ci[0];
    const int iy = dy ? (ci[1] + 1 == F.n[1] ? 0 : ci[1] + 1) : ci[1];
    const int iz = dz ? (ci[2] + 1 == F.n[2] ? 0 : ci[2] + 1) : ci[2];
    node = ((int64_t)ix * F.n[1] + iy) * F.n[2] + iz;
    return wx * wy * wz;
}

// Modulation at X (section 3.2, modulated grids) as the forward lookup
// computes it, and its gradient dm/dX (per Mpc) summed over the corners
// (dx fastest, then dy, then dz).
template <class M>
__device__ __forceinline__ double mod_value_grad_t(const FieldDev &F, const double X[3], double dm[3]) {
    ModCorners<M> mc;
    mod_load<M>(F, X, mc);
    const double v[8] = {(double)mc.v000, (double)mc.v100, (double)mc.v010, (double)mc.v110,
                         (double)mc.v001, (double)mc.v101, (double)mc.v011, (double)mc.v111};
    dm[0] = dm[1] = dm[2] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
        const double wx = dx ? mc.t[0] : 1.0 - mc.t[0], wy = dy ? mc.t[1] : 1.0 - mc.t[1],
                     wz = dz ? mc.t[2] : 1.0 - mc.t[2];
        const double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        dm[0] += sx * wy * wz * F.mod_inv_spacing * v[q];
        dm[1] += wx * sy * wz * F.mod_inv_spacing * v[q];
        dm[2] += wx * wy * sz * F.mod_inv_spacing * v[q];
    }
    return mod_value<M>(mc);
}

__device__ __forceinline__ double mod_value_grad(const FieldDev &F, const double X[3], double dm[3]) {
    return F.mod_dtype == CRP_F64 ? mod_value_grad_t<double>(F, X, dm) : mod_value_grad_t<float>(F, X, dm);
}

constexpr double ADJ_A[6][5] = {{0, 0, 0, 0, 0},
                                {A21, 0, 0, 0, 0},
                                {A31, A32, 0, 0, 0},
                                {A41, A42, A43, 0, 0},
                                {A51, A52, A53, A54, 0},
                                {A61, A62, A63, A64, A65}};
constexpr double ADJ_B5[6] = {B51, 0.0, B53, B54, 0.0, B56};

// Unnormalised output z = Phi(y, h) of a recorded step: the fifth-order sum
// over the recorded stages, evaluated as the forward step does.
__device__ __forceinline__ void rec_output(double kap, const double *r, int64_t stride, double z[6]) {
    double a5[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double Y[6], B[3];
        rec_stage(r, stride, i, Y);
        rec_field(r, stride, i, B);
#pragma unroll
        for (int c = 0; c < 6; ++c) a5[c] = fma(ADJ_B5[i], stage_k(kap, Y, B, c), a5[c]);
    }
    const double h = r[REC_H * stride];
#pragma unroll
    for (int c = 0; c < 6; ++c) z[c] = fma(h, a5[c], r[(REC_Y + c) * stride]);
}

// Derivative in the step size of the recorded step's output, dz/ds at s = h
// (forward mode through the stages; dB/ds from the trilinear gradient of the
// stage's cell, and for a modulated field B = b m, b-dot m + b m-dot).  kd:
// scratch column of 36 values for the stage derivatives, kstride apart.
template <class T, int LAYOUT, bool MOD>
__device__ __forceinline__ void rec_output_ds(const FieldDev &F, double kap, const double *r, int64_t stride, double *kd,
                              int64_t kstride, double zs[6]) {
    const double s = r[REC_H * stride];
    double a5[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, a5d[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 6; ++i) {
        double Yd[6];
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Yd[c] = 0.0;
                continue;
            }
            double acc = 0.0, accd = 0.0;
            for (int j = 0; j < i; ++j) {
                double Yj[6], Bj[3];
                rec_stage(r, stride, j, Yj);
                rec_field(r, stride, j, Bj);
                acc = fma(ADJ_A[i][j], stage_k(kap, Yj, Bj, c), acc);
                accd = ADJ_A[i][j] * kd[(6 * j + c) * kstride] + accd;
            }
            Yd[c] = acc + s * accd;
        }
        double Y[6];
        rec_stage(r, stride, i, Y);
        int ci[3];
        double t[3];
        T raw[24];
        cell_of<T, LAYOUT>(F, Y, ci, t, raw);
        // the vector grid's value, interpolated as the forward lookup does
        double Bs[3], Bd[3] = {0.0, 0.0, 0.0};
        interp_corners<T>(F, raw, t[0], t[1], t[2], Bs);
        for (int q = 0; q < 8; ++q) {
            double dw[3];
            int64_t node;
            corner_weight(F, ci, t, q, dw, node);
            const double gd = dw[0] * Yd[0] + dw[1] * Yd[1] + dw[2] * Yd[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) Bd[c] += gd * (to_f64<T>(raw[q * 3 + c]) * F.value_scale);
        }
        if constexpr (MOD) {
            double dm[3];
            const double mv = mod_value_grad(F, Y, dm);
            const double mdot = dm[0] * Yd[0] + dm[1] * Yd[1] + dm[2] * Yd[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Bd[c] = Bd[c] * mv + Bs[c] * mdot;
                Bs[c] = Bs[c] * mv;
            }
        }
        const double *U = Y + 3, *Ud = Yd + 3;
        double kdi[6] = {Ud[0], Ud[1], Ud[2],
                         kap * ((Ud[1] * Bs[2] + U[1] * Bd[2]) - (Ud[2] * Bs[1] + U[2] * Bd[1])),
                         kap * ((Ud[2] * Bs[0] + U[2] * Bd[0]) - (Ud[0] * Bs[2] + U[0] * Bd[2])),
                         kap * ((Ud[0] * Bs[1] + U[0] * Bd[1]) - (Ud[1] * Bs[0] + U[1] * Bd[0]))};
        double B[3];
        rec_field(r, stride, i, B);
        for (int c = 0; c < 6; ++c) {
            kd[(6 * i + c) * kstride] = kdi[c];
            a5[c] = fma(ADJ_B5[i], stage_k(kap, Y, B, c), a5[c]);
            a5d[c] = ADJ_B5[i] * kdi[c] + a5d[c];
        }
    }
    for (int c = 0; c < 6; ++c) zs[c] = a5[c] + s * a5d[c];
}

// Grid-gradient accumulator of one lane: the contributions to the 8 corners of
// the last cell touched, held in LDS (one column per lane, so no two lanes
// share a slot) and added to the global gradient with atomics only when the
// lane moves to another cell or finishes its particle.  Small steps visit the
// same cell for many stages in a row, so most contributions never leave LDS.
struct GradAccum {
    double (*v)[64];  // LDS [24][64]: corner q, component c at row 3 q + c
    int t;            // lane within the wavefront
    uint32_t key;     // cell (i n1 + j) n2 + k, 0xffffffff when empty
    int ci[3];
    int dropped;      // a contribution of the lane's particle was not finite and was left out
};

// The grid gradient: FP64 or FP32 values in the natural [n0][n1][n2][3] layout.
struct GradOut {
    void *p;
    int f32;
};

__device__ __forceinline__ void grad_flush(const FieldDev &F, GradAccum &g, GradOut gbar) {
    if (g.key == 0xffffffffu) return;
    const double t0[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double dw[3];
        int64_t node;
        corner_weight(F, g.ci, t0, q, dw, node);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // a cotangent beyond the FP64 range (a chaotic trajectory) would
            // poison every particle's sum: its contribution is left out
            const double v = g.v[3 * q + c][g.t];
            if (gbar.f32) {
                const float v32 = (float)v;
                if (isfinite(v32))
                    unsafeAtomicAdd(static_cast<float *>(gbar.p) + 3 * node + c, v32);
                else
                    g.dropped = 1;
            } else if (isfinite(v)) {
                unsafeAtomicAdd(static_cast<double *>(gbar.p) + 3 * node + c, v);
            } else {
                g.dropped = 1;
            }
        }
    }
    g.key = 0xffffffffu;
}

// Make ci the accumulator's cell, flushing and clearing the slots when it
// changes.
__device__ __forceinline__ void grad_select(const FieldDev &F, GradAccum &g, const int ci[3], GradOut gbar) {
    const uint32_t key = ((uint32_t)ci[0] * (uint32_t)F.n[1] + (uint32_t)ci[1]) * (uint32_t)F.n[2] + (uint32_t)ci[2];
    if (key == g.key) return;
    grad_flush(F, g, gbar);
    g.key = key;
    g.ci[0] = ci[0];
    g.ci[1] = ci[1];
    g.ci[2] = ci[2];
#pragma unroll
    for (int r = 0; r < 24; ++r) g.v[r][g.t] = 0.0;
}

// Reverse sweep of one recorded step y -> normalise(Phi(y, h)).  lam: in, the
// cotangent of the normalised output; out, the cotangent of y.  comb (three
// values or NULL): extra cotangent of the unnormalised output position (the
// crossing term).  Grid-gradient contributions go to gbar through the lane's
// accumulator, or, with bbar given, each stage's cotangent of the vector
// grid's value is stored there instead (stage i's component c at
// bbar[(3 i + c) stride]) for a later scatter.  A modulated field B = b m
// (MOD): the vector grid's value takes b-bar = m B-bar, the position also
// (b . B-bar) dm/dX.
template <class T, int LAYOUT, bool MOD>
__device__ __forceinline__ void reverse_step(const FieldDev &F, double kap, const double *r, int64_t stride, double lam[6],
                             const double *comb, GradAccum &acc, GradOut gbar, double &kbar, double *bbar) {
    const double s = r[REC_H * stride];
    double z[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) z[3 + c] = r[(REC_ZU + c) * stride];
    const double zn = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
    const double u[3] = {z[3] / zn, z[4] / zn, z[5] / zn};
    const double lu = lam[3] * u[0] + lam[4] * u[1] + lam[5] * u[2];
    double zb[6] = {lam[0], lam[1], lam[2], (lam[3] - lu * u[0]) / zn, (lam[4] - lu * u[1]) / zn,
                    (lam[5] - lu * u[2]) / zn};
    if (comb)
        for (int c = 0; c < 3; ++c) zb[c] += comb[c];
    double Yb[6][6];
    double bbs[6][3];  // the stages' b-bar, stored after the step's last gather
    double yb[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) yb[c] = zb[c];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double kb[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double v = s * ADJ_B5[i] * zb[c];
#pragma unroll
            for (int j = i + 1; j < 6; ++j) v += s * ADJ_A[j][i] * Yb[j][c];
            kb[c] = v;
        }
        double Y[6], B[3];
        rec_stage(r, stride, i, Y);
        rec_field(r, stride, i, B);
        const double *U = Y + 3;
        const double Bb[3] = {kap * (kb[4] * U[2] - kb[5] * U[1]), kap * (kb[5] * U[0] - kb[3] * U[2]),
                              kap * (kb[3] * U[1] - kb[4] * U[0])};
        // kappa enters the stage as kappa U x B: kappa-bar += ku . (U x B)
        kbar += kb[3] * (U[1] * B[2] - U[2] * B[1]) + kb[4] * (U[2] * B[0] - U[0] * B[2]) +
                kb[5] * (U[0] * B[1] - U[1] * B[0]);
        Yb[i][3] = kb[0] + kap * (B[1] * kb[5] - B[2] * kb[4]);
        Yb[i][4] = kb[1] + kap * (B[2] * kb[3] - B[0] * kb[5]);
        Yb[i][5] = kb[2] + kap * (B[0] * kb[4] - B[1] * kb[3]);
        Yb[i][0] = Yb[i][1] = Yb[i][2] = 0.0;
        int ci[3];
        double t[3];
        T raw[24];
        cell_of<T, LAYOUT>(F, Y, ci, t, raw);
        if (!bbar) grad_select(F, acc, ci, gbar);
        // cotangent of the vector grid's interpolated value: b-bar = m B-bar
        double bb[3] = {Bb[0], Bb[1], Bb[2]}, dm[3], bB = 0.0;
        if constexpr (MOD) {
            const double mv = mod_value_grad(F, Y, dm);
            double b[3];
            interp_corners<T>(F, raw, t[0], t[1], t[2], b);
            bB = b[0] * Bb[0] + b[1] * Bb[1] + b[2] * Bb[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) bb[c] = Bb[c] * mv;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double dw[3];
            int64_t node;
            const double w = corner_weight(F, ci, t, q, dw, node);
            // X-bar += (db/dX)^T b-bar: this corner's value dotted with b-bar, times dw
            const double vb = (to_f64<T>(raw[q * 3 + 0]) * F.value_scale) * bb[0] +
                              (to_f64<T>(raw[q * 3 + 1]) * F.value_scale) * bb[1] +
                              (to_f64<T>(raw[q * 3 + 2]) * F.value_scale) * bb[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) Yb[i][a] += dw[a] * vb;
            if (!bbar)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    // the lane owns its slot: an LDS add without return, no wait on a read
                    __hip_atomic_fetch_add(&acc.v[3 * q + c][acc.t], w * bb[c], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) bbs[i][c] = bb[c];
        if constexpr (MOD) {
            // X-bar += (b . B-bar) dm/dX
#pragma unroll
            for (int a = 0; a < 3; ++a) Yb[i][a] += dm[a] * bB;
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) yb[c] += Yb[i][c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) lam[c] = yb[c];
    // stores retire through the same in-order counter as the gathers: issued
    // here, none of this step's gathers waits for them
    if (bbar)
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int c = 0; c < 3; ++c) bbar[(3 * i + c) * stride] = bbs[i][c];
}

// Wavefront-wide maximum of a lane value (inactive lanes contribute 0).
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Adjoint state of the particle a lane works on.
struct AdjLane {
    int64_t p;        // particle, -1 none
    int64_t N;        // accepted steps of the forward run
    int64_t seg;      // segment being processed (from the last down to 0)
    int64_t slot;     // tape record of that segment's first state
    int flags;
    double kap, Lbar;
    double kbar;      // cotangent of kappa, summed from the last step back
    double lam[6];    // cotangent of the state after the segment being processed
    const double *pre;  // the particle's parallel-replayed records, NULL: replayed here
    double *bar;        // and their grid-value cotangents (scattered after the sweep)
};

// Gradients of the lane's finished particle: the direction entering the map
// is normalised on a fresh start.
__device__ __forceinline__ void adj_finish(const AdjLane &L, int dropped) {
    KernArg<AdjArgs> &a = kernel_args<AdjArgs>();  // read here: once per particle
    const int64_t p = L.p;
    // a cotangent that left the FP64 range is reported in the particle's tape flags
    bool finite = isfinite(L.kbar);
    for (int c = 0; c < 6; ++c) finite = finite && isfinite(L.lam[c]);
    if (dropped || !finite) a.fin_out[4 * p + 3] = (double)(L.flags | CRP_TAPE_GRAD_OVERFLOW);
    // a backtracked run is the forward run of the antiparticle with the
    // direction reversed: its direction gradient is reversed back
    const double sg = a.P.backtrack_on ? -1.0 : 1.0;
    if (L.flags & CRP_TAPE_FRESH) {
        const double u0[3] = {sg * a.ux0[p], sg * a.uy0[p], sg * a.uz0[p]};
        double un = sqrt(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
        double uh[3] = {u0[0] / un, u0[1] / un, u0[2] / un};
        double lu = L.lam[3] * uh[0] + L.lam[4] * uh[1] + L.lam[5] * uh[2];
        for (int c = 0; c < 3; ++c) a.grad_u0[3 * p + c] = sg * ((L.lam[3 + c] - lu * uh[c]) / un);
    } else {
        for (int c = 0; c < 3; ++c) a.grad_u0[3 * p + c] = sg * L.lam[3 + c];
    }
    if (a.grad_x0)
        for (int c = 0; c < 3; ++c) a.grad_x0[3 * p + c] = L.lam[c];
    if (a.grad_energy) {
        // d kappa / d E = -kappa / E
        const double ge = L.kbar * (-(L.kap / a.energy[p]));
        a.grad_energy[p] = a.gbar_energy ? a.gbar_energy[p] + ge : ge;
    }
}

// A particle with no adjoint (incomplete tape or broken record chain): zero gradients.
__device__ __forceinline__ void adj_zero(int64_t p) {
    KernArg<AdjArgs> &a = kernel_args<AdjArgs>();
    for (int c = 0; c < 3; ++c) {
        a.grad_u0[3 * p + c] = 0.0;
        if (a.grad_x0) a.grad_x0[3 * p + c] = 0.0;
    }
    if (a.grad_energy) a.grad_energy[p] = 0.0;
}

// The last step of a particle that arrived, recorded again: taken from the
// recorded pre-step state to the located crossing s* (its record then holds
// the crossing step's stages, step s* and output direction).
template <class T, int LAYOUT, bool MOD>
__device__ __forceinline__ void rerecord_crossing(const FieldDev &F, double kap, double *r, int64_t stride,
                                                  double sstar) {
    double y[6], y5[6], ex, eu;
    for (int c = 0; c < 6; ++c) y[c] = r[(REC_Y + c) * stride];
    CellCache<T> cache;
    cache_reset(cache);
    ck_eval<T, LAYOUT, false, RecordWriter, MOD>(F, 0, cache, kap, y, sstar, y5, ex, eu, RecordWriter{r, stride});
    r[REC_H * stride] = sstar;
    for (int c = 0; c < 3; ++c) r[(REC_ZU + c) * stride] = y5[3 + c];
}

// ---------------------------------------------------------------- parallel replay
//
// Order position q (the sweep's queue order, most steps first) is eligible
// for parallel replay if its tape is complete with a record at its head and
// it took steps.  Positions go in groups of 64 (G = q / 64, lane l = q % 64):
// a group's records are blocks of 64 (one record per lane, padded to the
// group's most steps), and its replay threads rows of 64 (one row per
// segment index, padded to its most segments), so replay stores and sweep
// loads of a field are contiguous across a wavefront.  The parallel-replayed
// groups are those before the first one whose blocks no longer fit in the
// workspace (the cut).

struct Eligible {
    int64_t p, N, nseg, slot;
    int flags;
    bool ok;
};

__device__ __forceinline__ Eligible eligible(const AdjArgs &a, int64_t q) {
    Eligible e;
    e.p = a.order ? (int64_t)a.order[q] : q;
    const double *f = a.fin + 4 * e.p;
    e.N = (int64_t)f[0];
    e.slot = (int64_t)f[2];
    e.flags = (int)f[3];
    e.ok = (e.flags & CRP_TAPE_COMPLETE) && !(e.flags & CRP_TAPE_OVERFLOW) && e.N > 0 && e.slot >= 0 &&
           e.slot < a.cap;
    e.nseg = e.ok ? (e.N + a.K - 1) / a.K : 0;
    if (!e.ok) e.N = 0;
    return e;
}

// Most steps of group G's eligible positions.
__device__ __forceinline__ int64_t group_steps(const AdjArgs &a, int64_t G) {
    int64_t m = 0;
    const int64_t q1 = (G + 1) * ADJ_GROUP < a.n ? (G + 1) * ADJ_GROUP : a.n;
    for (int64_t q = G * ADJ_GROUP; q < q1; ++q) {
        const int64_t N = eligible(a, q).N;
        m = N > m ? N : m;
    }
    return m;
}

// Record blocks and replay rows of every group (exclusive sums), and the cut
// (one block: each thread takes a contiguous run of groups, the block scans
// the runs' sums, each thread writes its run's offsets).
constexpr int PREFIX_THREADS = 1024;

__global__ void __launch_bounds__(PREFIX_THREADS) k_adj_prefix(AdjArgs a) {
    __shared__ int64_t sr[PREFIX_THREADS], ss[PREFIX_THREADS];
    __shared__ unsigned long long cut;
    const int t = threadIdx.x;
    // the scan covers the first R / 64 + 1 groups: a group with steps takes at
    // least one block, so a later group can fit only after empty ones (then
    // it is left to the sweep)
    const int64_t ng_all = (a.n + ADJ_GROUP - 1) / ADJ_GROUP, blocks = a.R / ADJ_GROUP;
    const int64_t ng = ng_all < blocks + 1 ? ng_all : blocks + 1;
    const int64_t chunk = (ng + PREFIX_THREADS - 1) / PREFIX_THREADS;
    const int64_t g0 = (int64_t)t * chunk < ng ? (int64_t)t * chunk : ng;
    const int64_t g1 = g0 + chunk < ng ? g0 + chunk : ng;
    int64_t r = 0, w = 0;
    for (int64_t G = g0; G < g1; ++G) {
        const int64_t m = group_steps(a, G);
        r += m;
        w += (m + a.K - 1) / a.K;
    }
    sr[t] = r;
    ss[t] = w;
    if (t == 0) cut = (unsigned long long)ng;
    __syncthreads();
    for (int off = 1; off < PREFIX_THREADS; off <<= 1) {
        const int64_t vr = t >= off ? sr[t - off] : 0, vs = t >= off ? ss[t - off] : 0;
        __syncthreads();
        sr[t] += vr;
        ss[t] += vs;
        __syncthreads();
    }
    r = sr[t] - r;  // exclusive
    w = ss[t] - w;
    for (int64_t G = g0; G < g1; ++G) {
        const int64_t m = group_steps(a, G);
        a.grp_rec[G] = r;
        a.grp_row[G] = w;
        if (r + m > blocks) atomicMin(&cut, (unsigned long long)G);
        r += m;
        w += (m + a.K - 1) / a.K;
    }
    if (t == PREFIX_THREADS - 1) {
        a.grp_rec[ng] = sr[t];
        a.grp_row[ng] = ss[t];
    }
    __syncthreads();
    if (t == 0) {
        const int64_t G = (int64_t)cut;
        a.queue[1] = (unsigned long long)(G * ADJ_GROUP < a.n ? G * ADJ_GROUP : a.n);
        a.queue[2] = (unsigned long long)G;
    }
}

// One thread per order position before the cut: the checkpoint record of each
// of its segments in its lane of the group's rows, walking the tape's links
// from the last segment back, -1 in the rows past its segments.  A broken
// chain leaves the particle to the sweep.
__global__ void __launch_bounds__(256) k_adj_walk(AdjArgs a) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= (int64_t)a.queue[1]) return;
    const Eligible e = eligible(a, q);
    const int64_t G = q / ADJ_GROUP, l = q % ADJ_GROUP;
    const int64_t row0 = a.grp_row[G], nrow = a.grp_row[G + 1] - row0;
    int64_t *slots = a.seg_slot + row0 * ADJ_GROUP + l;
    for (int64_t s = e.nseg; s < nrow; ++s) slots[s * ADJ_GROUP] = -1;
    int64_t slot = e.slot;
    int ok = e.ok;
    for (int64_t s = e.nseg - 1; s >= 0; --s) {
        if (slot < 0 || slot >= a.cap) {
            ok = 0;
            break;
        }
        slots[s * ADJ_GROUP] = slot;
        if (s > 0) slot = a.link[slot];
    }
    a.pre_ok[q] = ok;
}

// The group and lane of replay thread g (its row's group: the last G with
// grp_row[G] <= row); false if the thread has no segment.
__device__ __forceinline__ bool replay_slot(const AdjArgs &a, int64_t g, int64_t &G, int64_t &q, int64_t &sg) {
    const int64_t gcut = (int64_t)a.queue[2];
    const int64_t row = g / ADJ_GROUP, l = g % ADJ_GROUP;
    G = 0;
    q = l;
    sg = 0;
    if (row >= a.grp_row[gcut]) return false;
    int64_t lo = 0, hi = gcut - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (a.grp_row[mid] <= row)
            lo = mid;
        else
            hi = mid - 1;
    }
    G = lo;
    q = G * ADJ_GROUP + l;
    sg = row - a.grp_row[G];
    return q < (int64_t)a.queue[1] && a.pre_ok[q] && a.seg_slot[g] >= 0;
}

// One thread per (row, lane) of the parallel-replayed groups: replay segment
// s = row - first row of the group of position q = 64 G + lane from its
// checkpoint, one attempt per loop iteration, into the position's records
// (and record a crossing step again at s*).
template <class T, int LAYOUT, bool RFL, bool MOD>
__global__ void __launch_bounds__(256) k_adj_replay(AdjArgs a) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t G, q, sg;
    const bool busy = replay_slot(a, g, G, q, sg);
    const int64_t l = q % ADJ_GROUP;
    int m = 0;
    double *r0 = nullptr;
    Lane s;
    int64_t p = 0, nseg = 0;
    int flags = 0;
    if (busy) {
        const Eligible e = eligible(a, q);
        p = e.p;
        flags = e.flags;
        nseg = e.nseg;
        m = (int)(sg == nseg - 1 ? e.N - sg * a.K : a.K);
        r0 = a.prerec + (a.grp_rec[G] + sg * a.K) * ADJ_BLOCK_DOUBLES + l;
        const double *ck = a.ckpt + 8 * a.seg_slot[g];
        for (int c = 0; c < 6; ++c) s.y[c] = ck[c];
        s.L = ck[6];
        s.hctrl = ck[7];
        s.kap = ((double)(a.P.backtrack_on ? -a.charge[p] : a.charge[p]) * K_LORENTZ) / a.energy[p];
    }
    int j = 0;
    if (m > 0) bid<RFL>(a.P, s);
    while (__ballot(j < m) != 0ull) {
        if (j < m && replay_attempt<T, LAYOUT, RFL, MOD>(a.F, a.P, s, r0 + (int64_t)j * ADJ_BLOCK_DOUBLES, ADJ_GROUP))
            if (++j < m) bid<RFL>(a.P, s);
    }
    if (busy && sg == nseg - 1 && (flags & CRP_TAPE_EVENT))
        rerecord_crossing<T, LAYOUT, MOD>(a.F, s.kap, r0 + (int64_t)(m - 1) * ADJ_BLOCK_DOUBLES, ADJ_GROUP,
                                          a.fin[4 * p + 1]);
}

// After the sweep, one thread per parallel-replayed segment: the grid-gradient
// contributions w_q b-bar of its steps' stages, summed per cell in the
// thread's LDS column and added to the grid gradient with atomics when the
// cell changes (the sweep of these particles only stored b-bar).
__global__ void __launch_bounds__(64) k_adj_scatter(AdjArgs a) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double acc_lds[24][64];
    GradAccum acc{acc_lds, (int)threadIdx.x, 0xffffffffu, {0, 0, 0}, 0};
    const GradOut gout{a.grad_field, a.grad_f32};
    int64_t G, q, sg;
    if (!replay_slot(a, g, G, q, sg)) return;
    const Eligible e = eligible(a, q);
    const int64_t l = q % ADJ_GROUP;
    const int m = (int)(sg == e.nseg - 1 ? e.N - sg * a.K : a.K);
    const int64_t blk = a.grp_rec[G] + sg * a.K;
    for (int j = 0; j < m; ++j) {
        const double *r = a.prerec + (blk + j) * ADJ_BLOCK_DOUBLES + l;
        const double *bb = a.prebar + (blk + j) * ADJ_BAR_BLOCK + l;
        for (int i = 0; i < 6; ++i) {
            double Y[6];
            rec_stage(r, ADJ_GROUP, i, Y);
            int ci[3];
            double t[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) ci[c] = cell_axis(Y[c], a.F.origin[c], a.F.inv_spacing, a.F.n[c], a.F.pow2, t[c]);
            grad_select(a.F, acc, ci, gout);
            const double b[3] = {bb[(3 * i) * ADJ_GROUP], bb[(3 * i + 1) * ADJ_GROUP], bb[(3 * i + 2) * ADJ_GROUP]};
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
                double dw[3];
                int64_t node;
                const double w = corner_weight(a.F, ci, t, qq, dw, node);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    __hip_atomic_fetch_add(&acc.v[3 * qq + c][acc.t], w * b[c], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    grad_flush(a.F, acc, gout);
    if (acc.dropped) a.fin_out[4 * e.p + 3] = (double)(e.flags | CRP_TAPE_GRAD_OVERFLOW);
}

// ------------------------------------------------------------------ reverse sweep

// One lane per particle; the lanes of a wavefront move through their
// particles' segments in lockstep: every lane replays its current segment
// (one attempt per loop iteration, lanes that are done idle), then every lane
// sweeps its records in reverse, so no lane replays while another one is in
// the reverse sweep.  A parallel-replayed particle skips the replay and reads
// its records where the replay kernel left them.  Finished lanes take the
// next particle from a queue ordered by step count, most steps first.
template <class T, int LAYOUT, bool RFL, bool MOD>
__global__ void __launch_bounds__(64) k_adjoint_fp64(AdjArgs a) {
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double acc_lds[24][64];
    GradAccum acc{acc_lds, (int)threadIdx.x, 0xffffffffu, {0, 0, 0}, 0};
    const GradOut gout{a.grad_field, a.grad_f32};
    // this wavefront's block of segment records, the lane's records in it
    double *col = a.segbuf + (lane / ADJ_GROUP) * (int64_t)a.K * ADJ_BLOCK_DOUBLES + lane % ADJ_GROUP;
    double *kdcol = a.segbuf + (int64_t)a.K * REC_SIZE * a.lanes + lane;
    AdjLane L;
    L.p = -1;
    bool exhausted = false;
    for (;;) {
        // take particles until one needs a sweep (or the queue is empty)
        while (L.p < 0 && !exhausted) {
            // the particle's inputs: kernel arguments read here, not held across the loop
            KernArg<AdjArgs> &k = kernel_args<AdjArgs>();
            unsigned long long q = atomicAdd(k.queue, 1ull);
            if (q >= (unsigned long long)k.n) {
                exhausted = true;
                break;
            }
            const int64_t p = k.order ? (int64_t)k.order[q] : (int64_t)q;
            const double *fin = k.fin + 4 * p;
            L.p = p;
            L.flags = (int)fin[3];
            L.N = (int64_t)fin[0];
            for (int c = 0; c < 3; ++c) L.lam[c] = 0.0;
            // backtracking: the cotangent of the antiparticle's (reversed) direction
            for (int c = 0; c < 3; ++c) L.lam[3 + c] = k.P.backtrack_on ? -k.gbar_dir[3 * p + c] : k.gbar_dir[3 * p + c];
            if (!(L.flags & CRP_TAPE_COMPLETE) || (L.flags & CRP_TAPE_OVERFLOW)) {
                adj_zero(p);
                L.p = -1;
                continue;
            }
            L.kap = ((double)(k.P.backtrack_on ? -k.charge[p] : k.charge[p]) * K_LORENTZ) / k.energy[p];
            L.kbar = 0.0;
            acc.dropped = 0;
            if (L.N == 0) {
                adj_finish(L, 0);
                L.p = -1;
                continue;
            }
            L.slot = (int64_t)fin[2];
            if (L.slot < 0 || L.slot >= k.cap) {  // no record although steps were taken: no adjoint
                adj_zero(p);
                L.p = -1;
                continue;
            }
            L.Lbar = k.gbar_time ? k.gbar_time[p] * SEC_PER_MPC : 0.0;
            L.seg = (L.N + k.K - 1) / k.K - 1;
            // positions before the cut were replayed in parallel if their chain was whole
            const bool pre = (int64_t)q < (int64_t)k.queue[1] && k.pre_ok[q];
            L.pre = pre ? k.prerec + k.grp_rec[q / ADJ_GROUP] * ADJ_BLOCK_DOUBLES + q % ADJ_GROUP : nullptr;
            L.bar = pre ? k.prebar + k.grp_rec[q / ADJ_GROUP] * ADJ_BAR_BLOCK + q % ADJ_GROUP : nullptr;
        }
        const bool busy = L.p >= 0;
        if (__ballot(busy) == 0ull) break;

        // this segment's records: the wavefront's block, replayed here, or the
        // parallel-replayed ones (the same layout: fields 64 apart)
        const bool pre = busy && L.pre != nullptr;
        const int64_t nseg = busy ? (L.N + a.K - 1) / a.K : 0;
        const int m = busy ? (int)(L.seg == nseg - 1 ? L.N - L.seg * a.K : a.K) : 0;
        const bool event = busy && L.seg == nseg - 1 && (L.flags & CRP_TAPE_EVENT);
        double *rb = pre ? const_cast<double *>(L.pre) + L.seg * a.K * ADJ_BLOCK_DOUBLES : col;
        double *bb0 = pre ? L.bar + L.seg * a.K * ADJ_BAR_BLOCK : nullptr;
        constexpr int64_t fs = ADJ_GROUP, ss = ADJ_BLOCK_DOUBLES;
        Lane s;
        if (busy && !pre) {
            const double *ck = a.ckpt + 8 * L.slot;
            for (int c = 0; c < 6; ++c) s.y[c] = ck[c];
            s.L = ck[6];
            s.hctrl = ck[7];
            s.kap = L.kap;
        }
        // one attempt per loop iteration, so a lane's rejections cost the others nothing
        int j = pre ? m : 0;
        if (j < m) bid<RFL>(a.P, s);
        while (__ballot(j < m) != 0ull) {
            if (j < m && replay_attempt<T, LAYOUT, RFL, MOD>(a.F, a.P, s, col + (int64_t)j * ss, fs))
                if (++j < m) bid<RFL>(a.P, s);
        }
        const int mmax = wave_max(m);
        if (event) {
            double *r = rb + (int64_t)(m - 1) * ss;
            // the crossing step, taken to s* (already so in parallel-replayed records)
            if (!pre) rerecord_crossing<T, LAYOUT, MOD>(a.F, L.kap, r, fs, a.fin[4 * L.p + 1]);
            // crossing: psi = zbar . Phi_s + Lbar, cotangent zbar - (psi / g_s) dg/dz
            double z[6], zs[6];
            rec_output(L.kap, r, fs, z);
            rec_output_ds<T, LAYOUT, MOD>(a.F, L.kap, r, fs, kdcol, a.lanes, zs);
            double zn = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
            double u[3] = {z[3] / zn, z[4] / zn, z[5] / zn};
            double lu = L.lam[3] * u[0] + L.lam[4] * u[1] + L.lam[5] * u[2];
            double zb[6] = {L.lam[0], L.lam[1], L.lam[2], (L.lam[3] - lu * u[0]) / zn, (L.lam[4] - lu * u[1]) / zn,
                            (L.lam[5] - lu * u[2]) / zn};
            double psi = L.Lbar, gs = 0.0, dg[3];
            for (int c = 0; c < 6; ++c) psi += zb[c] * zs[c];
            for (int c = 0; c < 3; ++c) {
                dg[c] = 2.0 * (z[c] - a.P.center[c]);
                gs += dg[c] * zs[c];
            }
            double comb[3] = {-(psi / gs) * dg[0], -(psi / gs) * dg[1], -(psi / gs) * dg[2]};
            reverse_step<T, LAYOUT, MOD>(a.F, L.kap, r, fs, L.lam, comb, acc, gout, L.kbar,
                                         bb0 ? bb0 + (int64_t)(m - 1) * ADJ_BAR_BLOCK : nullptr);
        }
        // reverse sweep (the crossing step, if any, is done above; it ends on
        // the sphere, unmirrored)
        const int mrev = event ? m - 1 : m;
        for (int j = mmax - 1; j >= 0; --j)
            if (j < mrev) {
                const double *r = rb + (int64_t)j * ss;
                if (RFL) mirror_cotangent(r, fs, L.lam);
                reverse_step<T, LAYOUT, MOD>(a.F, L.kap, r, fs, L.lam, nullptr, acc, gout, L.kbar,
                                             bb0 ? bb0 + (int64_t)j * ADJ_BAR_BLOCK : nullptr);
            }
        if (busy) {
            if (--L.seg < 0) {
                grad_flush(a.F, acc, gout);
                adj_finish(L, acc.dropped);
                L.p = -1;
            } else if (!pre) {
                L.slot = a.link[L.slot];
                if (L.slot < 0 || L.slot >= a.cap) {  // a broken chain: no adjoint for this particle
                    grad_flush(a.F, acc, gout);
                    adj_zero(L.p);
                    L.p = -1;
                }
            }
        }
    }
}

}  // namespace

template <class T, int LAYOUT, bool RFL, bool MOD>
hipError_t launch_adjoint_one(const AdjArgs &a, int blocks, hipStream_t s) {
    if (a.R > 0) {
        hipLaunchKernelGGL(k_adj_prefix, dim3(1), dim3(PREFIX_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_adj_walk, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_adj_replay<T, LAYOUT, RFL, MOD>), dim3((unsigned)((a.rows * ADJ_GROUP + 255) / 256)),
                           dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL((k_adjoint_fp64<T, LAYOUT, RFL, MOD>), dim3(blocks), dim3(64), 0, s, a);
    if (a.R > 0) hipLaunchKernelGGL(k_adj_scatter, dim3((unsigned)a.rows), dim3(ADJ_GROUP), 0, s, a);
    return hipGetLastError();
}

template <bool RFL, bool MOD>
hipError_t launch_adjoint_feat(const AdjArgs &a, int blocks, hipStream_t s) {
    switch (a.F.dtype * 2 + (a.F.layout == CRP_LAYOUT_CELL8)) {
        case CRP_F64 * 2: return launch_adjoint_one<double, CRP_LAYOUT_LINEAR, RFL, MOD>(a, blocks, s);
        case CRP_F64 * 2 + 1: return launch_adjoint_one<double, CRP_LAYOUT_CELL8, RFL, MOD>(a, blocks, s);
        case CRP_F32 * 2: return launch_adjoint_one<float, CRP_LAYOUT_LINEAR, RFL, MOD>(a, blocks, s);
        case CRP_F32 * 2 + 1: return launch_adjoint_one<float, CRP_LAYOUT_CELL8, RFL, MOD>(a, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

// Instances per feature: a reflective box (RFL) and a modulated field (MOD).
hipError_t launch_adjoint_fp64(const AdjArgs &a, int blocks, hipStream_t s) {
    const bool mod = a.F.mod_data != nullptr;
    if (a.P.reflect_on)
        return mod ? launch_adjoint_feat<true, true>(a, blocks, s) : launch_adjoint_feat<true, false>(a, blocks, s);
    return mod ? launch_adjoint_feat<false, true>(a, blocks, s) : launch_adjoint_feat<false, false>(a, blocks, s);
}

}  // namespace crp
