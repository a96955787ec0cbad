// propagate_fp64.hip -- FP64-state propagation kernel for gfx950.
//
// One particle per lane, structure-of-arrays state.  A lane performs exactly
// one Cash-Karp evaluation per loop iteration, whatever it is doing:
//   NORMAL  an attempt of the bid step from the current state (accept or
//           reject under the error controller, then the stop checks);
//   EVENT   one Illinois iteration locating the observer-sphere crossing
//           inside the accepted step (section 3.1: observers end the
//           propagation; the crossing point, not the first point outside);
//   FINAL   the evaluation at the located crossing, which ends the particle.
// Keeping every lane on the same instruction stream avoids divergent inner
// loops.  When lanes finish, the wavefront ballots them and refills them from
// a device work queue (one atomic per wavefront), so waves stay full while
// trajectories of very different lengths (tens to tens of thousands of
// steps) run side by side; the grid is persistent (a few blocks per CU).
#include "crp_device.h"

namespace crp {
namespace {

using namespace dev;

enum { MODE_NORMAL = 0, MODE_EVENT = 1, MODE_FINAL = 2 };

constexpr int MAX_BLOCK = 256;

// Per-lane state kept in registers for the whole loop.
struct Lane {
    double y[6];          // current state (x, u); the pre-step state while locating an event
    double kap, L, hctrl, h;
    int32_t dacc, drej;   // accepted / rejected attempts of this call
    int32_t mode, binding, pidx;
    int32_t tflags;       // tape flags of this particle (fresh start, overflow)
};

// Tape: checkpoint c of particle p (state before accepted step c*K).
__device__ __forceinline__ void tape_checkpoint(const PropArgs &a, int64_t p, Lane &s, int64_t c) {
    int64_t base = a.tape_off[p], cap = a.tape_off[p + 1] - base;
    if (c >= cap) {
        s.tflags |= CRP_TAPE_OVERFLOW;
        return;
    }
    double *r = a.tape_ckpt + 8 * (base + c);
    r[0] = s.y[0];
    r[1] = s.y[1];
    r[2] = s.y[2];
    r[3] = s.y[3];
    r[4] = s.y[4];
    r[5] = s.y[5];
    r[6] = s.L;
    r[7] = s.hctrl;
}

__device__ __forceinline__ void tape_final(const PropArgs &a, int64_t p, const Lane &s, double sstar, double hlast,
                                           int flags) {
    double *f = a.tape_fin + 4 * p;
    f[0] = (double)s.dacc;
    f[1] = sstar;
    f[2] = hlast;
    f[3] = (double)(s.tflags | flags);
}

// Event-location state, used once per particle: kept in LDS, one slot per
// thread, so it costs no registers in the main loop.
struct EventLDS {
    double lo[MAX_BLOCK], hi[MAX_BLOCK], glo[MAX_BLOCK], ghi[MAX_BLOCK], hacc[MAX_BLOCK], lacc[MAX_BLOCK];
    int32_t side[MAX_BLOCK], eit[MAX_BLOCK];
};

__device__ __forceinline__ double sphere_g(const ParamsDev &P, const double x[3]) {
    double d0 = x[0] - P.center[0], d1 = x[1] - P.center[1], d2 = x[2] - P.center[2];
    return (d0 * d0 + d1 * d1 + d2 * d2) - P.r2;
}

// Bid of the next step: controller, h_max and sphere distance, floored by
// h_min; then the remaining length (not floored), which lands exactly on l_max.
__device__ __forceinline__ void bid(const ParamsDev &P, Lane &s) {
    double h = s.hctrl;
    if (h > P.h_max) h = P.h_max;
    if (P.sphere_on) {
        double d0 = s.y[0] - P.center[0], d1 = s.y[1] - P.center[1], d2 = s.y[2] - P.center[2];
        double dist = P.radius - sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (dist < h) h = dist;
    }
    if (h < P.h_min) h = P.h_min;
    s.binding = 0;
    if (P.lmax_on) {
        double rem = P.l_max - s.L;
        if (rem <= h) {
            h = rem;
            s.binding = 1;
        }
    }
    s.h = h;
}

// Write the particle's state back (its own slots only).
__device__ __forceinline__ void store(const PropArgs &a, int64_t p, const Lane &s, double hnext, int st) {
    a.x[p] = s.y[0];
    a.y[p] = s.y[1];
    a.z[p] = s.y[2];
    a.ux[p] = s.y[3];
    a.uy[p] = s.y[4];
    a.uz[p] = s.y[5];
    a.length[p] = s.L;
    a.h_next[p] = hnext;
    if (s.dacc) a.n_acc[p] += s.dacc;
    if (s.drej) a.n_rej[p] += s.drej;
    if (a.time) a.time[p] = s.L * SEC_PER_MPC;
    a.status[p] = st;
}

// Event step decision after entering EVENT mode or after an Illinois
// iteration: stop when the outside end is on the sphere to 1e-14 R^2, the
// bracket is below 1e-15 h, or after 30 iterations; otherwise the next
// regula-falsi point.
__device__ __forceinline__ void event_next(const ParamsDev &P, Lane &s, EventLDS &e, int t) {
    double lo = e.lo[t], hi = e.hi[t], glo = e.glo[t], ghi = e.ghi[t];
    if (ghi <= 1e-14 * P.r2 || (hi - lo) <= 1e-15 * e.hacc[t] || e.eit[t] >= 30) {
        s.mode = MODE_FINAL;
        s.h = hi;
    } else {
        s.h = (lo * ghi - hi * glo) / (ghi - glo);
    }
}

// Per-iteration outcome bits of a lane; the wavefront sums them with ballots
// into wave-uniform (scalar) counters.
enum { F_EVAL = 1, F_ACC = 2, F_REJ = 4, F_EVENT = 8, F_FLOOR = 16 };

// Start particle p in lane state s.  Returns true if it needs steps; false if
// it was skipped (not ACTIVE) or finished at once (its result is stored).
template <bool MULTI>
__device__ __forceinline__ bool start(const PropArgs &a, int64_t p, Lane &s) {
    int st = a.status[p];
    if (a.tape_ckpt) {
        double *f = a.tape_fin + 4 * p;  // overwritten when the particle completes
        f[0] = f[1] = f[2] = f[3] = 0.0;
    }
    if (st != CRP_ST_ACTIVE) return false;
    s.pidx = MULTI && a.param_index ? a.param_index[p] : 0;
    if (MULTI && (s.pidx < 0 || s.pidx >= a.n_params)) {
        a.status[p] = CRP_ST_BAD_INPUT;
        return false;
    }
    const ParamsDev &P = a.params[MULTI ? s.pidx : 0];
    double E = a.energy[p];
    int Z = a.charge[p];
    s.y[0] = a.x[p];
    s.y[1] = a.y[p];
    s.y[2] = a.z[p];
    s.y[3] = a.ux[p];
    s.y[4] = a.uy[p];
    s.y[5] = a.uz[p];
    s.L = a.length[p];
    s.dacc = 0;
    s.drej = 0;
    double hn = a.h_next[p];
    bool ok = E > 0.0 && isfinite(E) && isfinite(s.L) && hn >= 0.0 && isfinite(hn);
#pragma unroll
    for (int c = 0; c < 6; ++c) ok = ok && isfinite(s.y[c]);
    if (ok && hn == 0.0) {
        double n2 = s.y[3] * s.y[3] + s.y[4] * s.y[4] + s.y[5] * s.y[5];
        if (n2 > 0.0) {
            double nrm = sqrt(n2);
            s.y[3] = s.y[3] / nrm;
            s.y[4] = s.y[4] / nrm;
            s.y[5] = s.y[5] / nrm;
        } else {
            ok = false;
        }
    }
    if (!ok) {
        a.status[p] = CRP_ST_BAD_INPUT;
        return false;
    }
    s.tflags = hn == 0.0 ? CRP_TAPE_FRESH : 0;
    if (P.sphere_on && sphere_g(P, s.y) >= 0.0) {
        store(a, p, s, hn, CRP_ST_ARRIVED);
        if (a.tape_ckpt) tape_final(a, p, s, 0.0, 0.0, CRP_TAPE_COMPLETE);
        return false;
    }
    if (P.lmax_on && s.L >= P.l_max) {
        store(a, p, s, hn, CRP_ST_MAX_LENGTH);
        if (a.tape_ckpt) tape_final(a, p, s, 0.0, 0.0, CRP_TAPE_COMPLETE);
        return false;
    }
    s.hctrl = hn == 0.0 ? P.h_max : hn;
    s.kap = ((double)Z * K_LORENTZ) / E;
    s.mode = MODE_NORMAL;
    if (a.tape_ckpt) tape_checkpoint(a, p, s, 0);
    bid(P, s);
    return true;
}

// One loop iteration of a working lane.  Returns a status != ACTIVE when the
// particle ended (its result already stored).
template <class T, int LAYOUT, bool MULTI, bool CACHE>
__device__ __forceinline__ int advance(const PropArgs &a, int64_t p, Lane &s, CellCache<T> &cache, EventLDS &e,
                                       int &flags) {
    const int t = threadIdx.x;
    const ParamsDev &P = a.params[MULTI ? s.pidx : 0];
    const int fid = MULTI ? P.field_index : 0;
    const FieldDev &F = a.fields[fid];
    double y5[6], ex, eu;
    ck_eval<T, LAYOUT, CACHE>(F, fid, cache, s.kap, s.y, s.h, y5, ex, eu);
    flags = F_EVAL;

    if (s.mode == MODE_NORMAL) {
        double exh = ex / s.h;
        if (!isfinite(eu) || !isfinite(exh)) {
            store(a, p, s, s.hctrl, CRP_ST_NONFINITE);
            if (a.tape_ckpt) tape_final(a, p, s, 0.0, 0.0, 0);
            return CRP_ST_NONFINITE;
        }
        double em = eu > exh ? eu : exh;
        double err = em / P.tol;
        if (err > 1.0 && s.h > P.h_min) {
            double fac = 0.9 * (1.0 / sqrt(sqrt(err)));
            if (fac < 0.1) fac = 0.1;
            double h = s.h * fac;
            if (h < P.h_min) h = P.h_min;
            s.h = h;
            s.binding = 0;
            s.drej++;
            flags |= F_REJ;
            return CRP_ST_ACTIVE;
        }
        // accepted: next controller bid
        double g;
        if (err > 1.0) {
            g = 1.0;
            flags |= F_FLOOR;
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
        s.dacc++;
        flags |= F_ACC;
        if (P.sphere_on && sphere_g(P, y5) >= 0.0) {
            s.mode = MODE_EVENT;
            e.lo[t] = 0.0;
            e.glo[t] = sphere_g(P, s.y);
            e.hi[t] = s.h;
            e.ghi[t] = sphere_g(P, y5);
            e.hacc[t] = s.h;
            e.lacc[t] = Lnew;
            e.side[t] = 0;
            e.eit[t] = 0;
            event_next(P, s, e, t);
            return CRP_ST_ACTIVE;
        }
        double un = sqrt(y5[3] * y5[3] + y5[4] * y5[4] + y5[5] * y5[5]);
        s.y[0] = y5[0];
        s.y[1] = y5[1];
        s.y[2] = y5[2];
        s.y[3] = y5[3] / un;
        s.y[4] = y5[4] / un;
        s.y[5] = y5[5] / un;
        s.L = Lnew;
        if (P.lmax_on && s.L >= P.l_max) {
            store(a, p, s, s.hctrl, CRP_ST_MAX_LENGTH);
            if (a.tape_ckpt) tape_final(a, p, s, 0.0, s.h, CRP_TAPE_COMPLETE);
            return CRP_ST_MAX_LENGTH;
        }
        if (P.max_steps > 0 && s.dacc >= P.max_steps) {
            store(a, p, s, s.hctrl, CRP_ST_MAX_STEPS);
            if (a.tape_ckpt) tape_final(a, p, s, 0.0, s.h, 0);
            return CRP_ST_MAX_STEPS;
        }
        if (a.tape_ckpt && s.dacc % a.tape_k == 0) tape_checkpoint(a, p, s, s.dacc / a.tape_k);
        bid(P, s);
        return CRP_ST_ACTIVE;
    }

    flags |= F_EVENT;
    if (s.mode == MODE_EVENT) {
        double gs = sphere_g(P, y5);
        if (!isfinite(gs)) {
            store(a, p, s, s.hctrl, CRP_ST_NONFINITE);
            if (a.tape_ckpt) tape_final(a, p, s, 0.0, 0.0, 0);
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

    // MODE_FINAL: the state at the located crossing
    double sn = sqrt(y5[3] * y5[3] + y5[4] * y5[4] + y5[5] * y5[5]);
    s.y[0] = y5[0];
    s.y[1] = y5[1];
    s.y[2] = y5[2];
    s.y[3] = y5[3] / sn;
    s.y[4] = y5[4] / sn;
    s.y[5] = y5[5] / sn;
    s.L = e.hi[t] == e.hacc[t] ? e.lacc[t] : s.L + e.hi[t];
    store(a, p, s, s.hctrl, CRP_ST_ARRIVED);
    if (a.tape_ckpt) tape_final(a, p, s, e.hi[t], e.hacc[t], CRP_TAPE_COMPLETE | CRP_TAPE_EVENT);
    return CRP_ST_ARRIVED;
}

// Minimum resident waves per SIMD the register allocation must allow (the
// kernel is bound by gather latency, so occupancy is what hides it).
#ifndef CRP_FP64_MIN_WAVES
#define CRP_FP64_MIN_WAVES 2
#endif

template <class T, int LAYOUT, bool MULTI, bool CACHE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CRP_FP64_MIN_WAVES, 8)))
k_propagate_fp64(PropArgs a) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int64_t pid = -1;  // >= 0 working, -1 wants work, -2 queue exhausted
    __shared__ EventLDS ev;
    __shared__ T cache_lds[CACHE ? 24 : 1][CACHE_BLOCK];
    Lane s;
    CellCache<T> cache;
    cache_reset(cache, cache_lds, threadIdx.x);
    // wave-uniform counters, summed from ballots (scalar registers)
    unsigned long long n_eval = 0, n_acc = 0, n_rej = 0, n_ev = 0, n_fl = 0, n_taken = 0, n_iter = 0;

    for (;;) {
        // refill idle lanes from the work queue
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
                if (q < (unsigned long long)a.n) {
                    int64_t p = a.order ? (int64_t)a.order[q] : (int64_t)q;
                    got = 1;
                    pid = start<MULTI>(a, p, s) ? p : -1;
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
            int st = advance<T, LAYOUT, MULTI, CACHE>(a, pid, s, cache, ev, flags);
            if (st != CRP_ST_ACTIVE) pid = -1;
        }
        n_eval += __popcll(__ballot(flags & F_EVAL));
        n_acc += __popcll(__ballot(flags & F_ACC));
        n_rej += __popcll(__ballot(flags & F_REJ));
        n_ev += __popcll(__ballot(flags & F_EVENT));
        n_fl += __popcll(__ballot(flags & F_FLOOR));
    }

    if (a.counters) {
        // cell loads: per-lane totals summed across the wavefront
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

template <class T, int LAYOUT, bool MULTI>
hipError_t launch_c(const PropArgs &a, bool cache, int blocks, int bs, hipStream_t s) {
    if (cache)
        hipLaunchKernelGGL((k_propagate_fp64<T, LAYOUT, MULTI, true>), dim3(blocks), dim3(bs), 0, s, a);
    else
        hipLaunchKernelGGL((k_propagate_fp64<T, LAYOUT, MULTI, false>), dim3(blocks), dim3(bs), 0, s, a);
    return hipGetLastError();
}

template <class T>
hipError_t launch_layout(const PropArgs &a, int layout, bool multi, bool cache, int blocks, int bs, hipStream_t s) {
    if (layout == CRP_LAYOUT_CELL8)
        return multi ? launch_c<T, CRP_LAYOUT_CELL8, true>(a, cache, blocks, bs, s)
                     : launch_c<T, CRP_LAYOUT_CELL8, false>(a, cache, blocks, bs, s);
    return multi ? launch_c<T, CRP_LAYOUT_LINEAR, true>(a, cache, blocks, bs, s)
                 : launch_c<T, CRP_LAYOUT_LINEAR, false>(a, cache, blocks, bs, s);
}

// ============================ adjoint ======================================
//
// The derivative is that of the replayed map: the accepted step sizes of the
// taped forward run are held fixed and the sphere crossing in the last step
// is differentiated through its defining equation (implicit function theorem).
// Each lane takes one particle; from its last checkpoint segment to its first
// it replays the segment's accepted steps with the forward kernel's own step
// logic (so the states are bit-identical), then sweeps them in reverse.
// Grid-gradient contributions go to a natural-layout FP64 array by atomics.

// Replay m accepted steps from lane state s exactly as advance() takes them,
// writing (state before the step, step size) into the lane's record column.
template <class T, int LAYOUT>
__device__ void replay_segment(const FieldDev &F, const ParamsDev &P, Lane &s, int m, double *buf, int64_t stride,
                               int64_t lane) {
    CellCache<T> cache;
    cache_reset(cache, (T(*)[CACHE_BLOCK]) nullptr, 0);
    for (int j = 0; j < m; ++j) {
        bid(P, s);
        double y5[6], ex, eu, err;
        for (;;) {
            ck_eval<T, LAYOUT, false>(F, 0, cache, s.kap, s.y, s.h, y5, ex, eu);
            double exh = ex / s.h;
            double em = eu > exh ? eu : exh;
            err = em / P.tol;
            if (err > 1.0 && s.h > P.h_min) {
                double fac = 0.9 * (1.0 / sqrt(sqrt(err)));
                if (fac < 0.1) fac = 0.1;
                double h = s.h * fac;
                if (h < P.h_min) h = P.h_min;
                s.h = h;
                s.binding = 0;
                continue;
            }
            break;
        }
        double *r = buf + (int64_t)j * 7 * stride + lane;
#pragma unroll
        for (int c = 0; c < 6; ++c) r[c * stride] = s.y[c];
        r[6 * stride] = s.h;
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
        s.L = Lnew;
    }
}

// Trilinear stencil of the cell containing X: weights w, their gradients dw
// (per Mpc), corner values v[corner][c] and flat node indices (natural layout).
template <class T, int LAYOUT>
__device__ __forceinline__ void stencil(const FieldDev &F, const double X[3], double w[8], double dw[3][8],
                                        double v[8][3], int64_t node[8]) {
    double t[3];
    int ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ci[a] = cell_axis(X[a], F.origin[a], F.inv_spacing, F.n[a], F.pow2, t[a]);
    T raw[24];
    load_corners<T, LAYOUT>(F, ci[0], ci[1], ci[2], raw);
    int i1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) i1[a] = ci[a] + 1 == F.n[a] ? 0 : ci[a] + 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        double wx = dx ? t[0] : 1.0 - t[0], wy = dy ? t[1] : 1.0 - t[1], wz = dz ? t[2] : 1.0 - t[2];
        double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        w[k] = wx * wy * wz;
        dw[0][k] = sx * wy * wz * F.inv_spacing;
        dw[1][k] = wx * sy * wz * F.inv_spacing;
        dw[2][k] = wx * wy * sz * F.inv_spacing;
#pragma unroll
        for (int c = 0; c < 3; ++c) v[k][c] = to_f64<T>(raw[k * 3 + c]) * F.value_scale;
        node[k] = ((int64_t)(dx ? i1[0] : ci[0]) * F.n[1] + (dy ? i1[1] : ci[1])) * F.n[2] + (dz ? i1[2] : ci[2]);
    }
}

// Step map and its derivative in the step size at s: z = Phi(y, s), zs = dPhi/ds.
template <class T, int LAYOUT>
__device__ void ck_eval_ds(const FieldDev &F, double kap, const double y[6], double s, double z[6], double zs[6]) {
    CellCache<T> cache;
    cache_reset(cache, (T(*)[CACHE_BLOCK]) nullptr, 0);
    constexpr double A[6][5] = {{0, 0, 0, 0, 0},
                                {A21, 0, 0, 0, 0},
                                {A31, A32, 0, 0, 0},
                                {A41, A42, A43, 0, 0},
                                {A51, A52, A53, A54, 0},
                                {A61, A62, A63, A64, A65}};
    constexpr double Bw[6] = {B51, 0.0, B53, B54, 0.0, B56};
    double k[6][6], kd[6][6];
    for (int i = 0; i < 6; ++i) {
        double Y[6], Yd[6];
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Y[c] = y[c];
                Yd[c] = 0.0;
                continue;
            }
            double acc = 0.0, accd = 0.0;
            for (int j = 0; j < i; ++j) {
                acc = fma(A[i][j], k[j][c], acc);
                accd = A[i][j] * kd[j][c] + accd;
            }
            Y[c] = fma(s, acc, y[c]);
            Yd[c] = acc + s * accd;
        }
        rhs<T, LAYOUT, false>(F, 0, cache, kap, Y, k[i]);
        double w[8], dw[3][8], v[8][3];
        int64_t node[8];
        stencil<T, LAYOUT>(F, Y, w, dw, v, node);
        double B[3], Bd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double b = 0.0, bd = 0.0;
            for (int q = 0; q < 8; ++q) {
                b += w[q] * v[q][c];
                bd += (dw[0][q] * Yd[0] + dw[1][q] * Yd[1] + dw[2][q] * Yd[2]) * v[q][c];
            }
            B[c] = b;
            Bd[c] = bd;
        }
        const double *U = Y + 3;
        const double *Ud = Yd + 3;
        kd[i][0] = Ud[0];
        kd[i][1] = Ud[1];
        kd[i][2] = Ud[2];
        kd[i][3] = kap * ((Ud[1] * B[2] + U[1] * Bd[2]) - (Ud[2] * B[1] + U[2] * Bd[1]));
        kd[i][4] = kap * ((Ud[2] * B[0] + U[2] * Bd[0]) - (Ud[0] * B[2] + U[0] * Bd[2]));
        kd[i][5] = kap * ((Ud[0] * B[1] + U[0] * Bd[1]) - (Ud[1] * B[0] + U[1] * Bd[0]));
    }
    for (int c = 0; c < 6; ++c) {
        double a5 = 0.0, a5d = 0.0;
        for (int i = 0; i < 6; ++i) {
            a5 = fma(Bw[i], k[i][c], a5);
            a5d = Bw[i] * kd[i][c] + a5d;
        }
        z[c] = fma(s, a5, y[c]);
        zs[c] = a5 + s * a5d;
    }
}

// Reverse sweep of one step y -> normalise(Phi(y, s)).  lam: in, cotangent of
// the normalised output; out, cotangent of y.  comb: optional extra cotangent
// of the unnormalised output (the crossing term).
template <class T, int LAYOUT>
__device__ void step_vjp(const FieldDev &F, double kap, const double y[6], double s, double lam[6],
                         const double *comb, double *gbar) {
    CellCache<T> cache;
    cache_reset(cache, (T(*)[CACHE_BLOCK]) nullptr, 0);
    constexpr double A[6][5] = {{0, 0, 0, 0, 0},
                                {A21, 0, 0, 0, 0},
                                {A31, A32, 0, 0, 0},
                                {A41, A42, A43, 0, 0},
                                {A51, A52, A53, A54, 0},
                                {A61, A62, A63, A64, A65}};
    constexpr double Bw[6] = {B51, 0.0, B53, B54, 0.0, B56};
    double k[6][6], Y[6][6];
    for (int i = 0; i < 6; ++i) {
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Y[i][c] = y[c];
                continue;
            }
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc = fma(A[i][j], k[j][c], acc);
            Y[i][c] = fma(s, acc, y[c]);
        }
        rhs<T, LAYOUT, false>(F, 0, cache, kap, Y[i], k[i]);
    }
    double z[6];
    for (int c = 0; c < 6; ++c) {
        double a5 = 0.0;
        for (int i = 0; i < 6; ++i) a5 = fma(Bw[i], k[i][c], a5);
        z[c] = fma(s, a5, y[c]);
    }
    double zn = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
    double u[3] = {z[3] / zn, z[4] / zn, z[5] / zn};
    double lu = lam[3] * u[0] + lam[4] * u[1] + lam[5] * u[2];
    double zb[6] = {lam[0], lam[1], lam[2], (lam[3] - lu * u[0]) / zn, (lam[4] - lu * u[1]) / zn,
                    (lam[5] - lu * u[2]) / zn};
    if (comb)
        for (int c = 0; c < 6; ++c) zb[c] += comb[c];
    double Yb[6][6];
    double yb[6];
    for (int c = 0; c < 6; ++c) yb[c] = zb[c];
    for (int i = 5; i >= 0; --i) {
        double kb[6];
        for (int c = 0; c < 6; ++c) {
            double v = s * Bw[i] * zb[c];
            for (int j = i + 1; j < 6; ++j) v += s * A[j][i] * Yb[j][c];
            kb[c] = v;
        }
        double w[8], dw[3][8], v[8][3];
        int64_t node[8];
        stencil<T, LAYOUT>(F, Y[i], w, dw, v, node);
        double B[3];
        lookup<T, LAYOUT>(F, Y[i], B);
        const double *U = Y[i] + 3;
        double Bb[3] = {kap * (kb[4] * U[2] - kb[5] * U[1]), kap * (kb[5] * U[0] - kb[3] * U[2]),
                        kap * (kb[3] * U[1] - kb[4] * U[0])};
        Yb[i][3] = kb[0] + kap * (B[1] * kb[5] - B[2] * kb[4]);
        Yb[i][4] = kb[1] + kap * (B[2] * kb[3] - B[0] * kb[5]);
        Yb[i][5] = kb[2] + kap * (B[0] * kb[4] - B[1] * kb[3]);
        Yb[i][0] = Yb[i][1] = Yb[i][2] = 0.0;
        for (int q = 0; q < 8; ++q) {
            for (int c = 0; c < 3; ++c) {
                for (int a = 0; a < 3; ++a) Yb[i][a] += dw[a][q] * v[q][c] * Bb[c];
                unsafeAtomicAdd(gbar + 3 * node[q] + c, w[q] * Bb[c]);
            }
        }
        for (int c = 0; c < 6; ++c) yb[c] += Yb[i][c];
    }
    for (int c = 0; c < 6; ++c) lam[c] = yb[c];
}

template <class T, int LAYOUT>
__global__ void __launch_bounds__(64) k_adjoint_fp64(AdjArgs a) {
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (;;) {
        unsigned long long q = atomicAdd(a.queue, 1ull);
        if (q >= (unsigned long long)a.n) break;
        const int64_t p = a.order ? (int64_t)a.order[q] : (int64_t)q;
        const double *fin = a.fin + 4 * p;
        const int flags = (int)fin[3];
        const int64_t N = (int64_t)fin[0];
        double u0[3] = {a.ux0[p], a.uy0[p], a.uz0[p]};
        double lam[6] = {0.0, 0.0, 0.0, a.gbar_dir[3 * p], a.gbar_dir[3 * p + 1], a.gbar_dir[3 * p + 2]};
        if (!(flags & CRP_TAPE_COMPLETE) || (flags & CRP_TAPE_OVERFLOW)) {
            for (int c = 0; c < 3; ++c) {
                a.grad_u0[3 * p + c] = 0.0;
                if (a.grad_x0) a.grad_x0[3 * p + c] = 0.0;
            }
            continue;
        }
        const double kap = ((double)a.charge[p] * K_LORENTZ) / a.energy[p];
        const double Lbar = a.gbar_time ? a.gbar_time[p] * SEC_PER_MPC : 0.0;
        const int64_t nseg = N > 0 ? (N + a.K - 1) / a.K : 0;
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const double *r = a.ckpt + 8 * (a.off[p] + seg);
            Lane s;
            for (int c = 0; c < 6; ++c) s.y[c] = r[c];
            s.L = r[6];
            s.hctrl = r[7];
            s.kap = kap;
            const int m = (int)(seg == nseg - 1 ? N - seg * a.K : a.K);
            replay_segment<T, LAYOUT>(a.F, a.P, s, m, a.segbuf, a.lanes, lane);
            for (int j = m - 1; j >= 0; --j) {
                const double *rj = a.segbuf + (int64_t)j * 7 * a.lanes + lane;
                double y[6];
                for (int c = 0; c < 6; ++c) y[c] = rj[c * a.lanes];
                double h = rj[6 * a.lanes];
                if (seg == nseg - 1 && j == m - 1 && (flags & CRP_TAPE_EVENT)) {
                    // crossing: psi = zbar . Phi_s + Lbar, cotangent zbar - (psi / g_s) dg/dz
                    const double sstar = fin[1];
                    double z[6], zs[6];
                    ck_eval_ds<T, LAYOUT>(a.F, kap, y, sstar, z, zs);
                    double zn = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
                    double u[3] = {z[3] / zn, z[4] / zn, z[5] / zn};
                    double lu = lam[3] * u[0] + lam[4] * u[1] + lam[5] * u[2];
                    double zb[6] = {lam[0], lam[1], lam[2], (lam[3] - lu * u[0]) / zn, (lam[4] - lu * u[1]) / zn,
                                    (lam[5] - lu * u[2]) / zn};
                    double psi = Lbar, gs = 0.0, dg[3];
                    for (int c = 0; c < 6; ++c) psi += zb[c] * zs[c];
                    for (int c = 0; c < 3; ++c) {
                        dg[c] = 2.0 * (z[c] - a.P.center[c]);
                        gs += dg[c] * zs[c];
                    }
                    double comb[6] = {-(psi / gs) * dg[0], -(psi / gs) * dg[1], -(psi / gs) * dg[2], 0.0, 0.0, 0.0};
                    step_vjp<T, LAYOUT>(a.F, kap, y, sstar, lam, comb, a.grad_field);
                } else {
                    step_vjp<T, LAYOUT>(a.F, kap, y, h, lam, nullptr, a.grad_field);
                }
            }
        }
        // the direction entering the map: normalised on a fresh start
        if (flags & CRP_TAPE_FRESH) {
            double un = sqrt(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
            double uh[3] = {u0[0] / un, u0[1] / un, u0[2] / un};
            double lu = lam[3] * uh[0] + lam[4] * uh[1] + lam[5] * uh[2];
            for (int c = 0; c < 3; ++c) a.grad_u0[3 * p + c] = (lam[3 + c] - lu * uh[c]) / un;
        } else {
            for (int c = 0; c < 3; ++c) a.grad_u0[3 * p + c] = lam[3 + c];
        }
        if (a.grad_x0)
            for (int c = 0; c < 3; ++c) a.grad_x0[3 * p + c] = lam[c];
    }
}

}  // namespace

hipError_t launch_adjoint_fp64(const AdjArgs &a, int blocks, hipStream_t s) {
    switch (a.F.dtype * 2 + (a.F.layout == CRP_LAYOUT_CELL8)) {
        case CRP_F64 * 2: hipLaunchKernelGGL((k_adjoint_fp64<double, CRP_LAYOUT_LINEAR>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F64 * 2 + 1: hipLaunchKernelGGL((k_adjoint_fp64<double, CRP_LAYOUT_CELL8>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F32 * 2: hipLaunchKernelGGL((k_adjoint_fp64<float, CRP_LAYOUT_LINEAR>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F32 * 2 + 1: hipLaunchKernelGGL((k_adjoint_fp64<float, CRP_LAYOUT_CELL8>), dim3(blocks), dim3(64), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_propagate_fp64(const PropArgs &a, int dtype, int layout, bool multi, bool cache, int blocks,
                                 int block_size, hipStream_t s) {
    switch (dtype) {
        case CRP_F64: return launch_layout<double>(a, layout, multi, cache, blocks, block_size, s);
        case CRP_F32: return launch_layout<float>(a, layout, multi, cache, blocks, block_size, s);
        case CRP_F16: return launch_layout<__half>(a, layout, multi, cache, blocks, block_size, s);
        case CRP_BF16: return launch_layout<__hip_bfloat16>(a, layout, multi, cache, blocks, block_size, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace crp
