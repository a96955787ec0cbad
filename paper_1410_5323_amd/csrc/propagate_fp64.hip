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

struct Lane {
    double y[6];          // current state (x, u); the pre-step state while locating an event
    double kap, L, hctrl, h;
    double lo, hi, glo, ghi, hacc, lacc;
    int64_t nacc, nrej, ncall;
    int mode, binding, side, eit, pidx;
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

__device__ __forceinline__ void store(const PropArgs &a, int64_t p, const Lane &s, int st, bool state) {
    if (state) {
        a.x[p] = s.y[0];
        a.y[p] = s.y[1];
        a.z[p] = s.y[2];
        a.ux[p] = s.y[3];
        a.uy[p] = s.y[4];
        a.uz[p] = s.y[5];
        a.length[p] = s.L;
        a.h_next[p] = s.hctrl;
        a.n_acc[p] = s.nacc;
        a.n_rej[p] = s.nrej;
        if (a.time) a.time[p] = s.L * SEC_PER_MPC;
    }
    a.status[p] = st;
}

// Event step decision after entering EVENT mode or after an Illinois
// iteration: stop when the outside end is on the sphere to 1e-14 R^2, the
// bracket is below 1e-15 h, or after 30 iterations; otherwise the next
// regula-falsi point.
__device__ __forceinline__ void event_next(const ParamsDev &P, Lane &s) {
    if (s.ghi <= 1e-14 * P.r2 || (s.hi - s.lo) <= 1e-15 * s.hacc || s.eit >= 30) {
        s.mode = MODE_FINAL;
        s.h = s.hi;
    } else {
        s.h = (s.lo * s.ghi - s.hi * s.glo) / (s.ghi - s.glo);
    }
}

struct LocalCounters {
    unsigned int evals, acc, rej, ev, fl, taken;
};

// Start particle p in lane state s.  Returns true if it needs steps; false if
// it was skipped (not ACTIVE) or finished at once (its result is stored).
template <bool MULTI>
__device__ __forceinline__ bool start(const PropArgs &a, int64_t p, Lane &s) {
    int st = a.status[p];
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
    double hn = a.h_next[p];
    s.nacc = a.n_acc[p];
    s.nrej = a.n_rej[p];
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
    s.hctrl = hn == 0.0 ? P.h_max : hn;
    if (P.sphere_on && sphere_g(P, s.y) >= 0.0) {
        double keep = s.hctrl;
        s.hctrl = hn;
        store(a, p, s, CRP_ST_ARRIVED, true);
        s.hctrl = keep;
        return false;
    }
    if (P.lmax_on && s.L >= P.l_max) {
        s.hctrl = hn;
        store(a, p, s, CRP_ST_MAX_LENGTH, true);
        return false;
    }
    s.kap = ((double)Z * K_LORENTZ) / E;
    s.ncall = 0;
    s.mode = MODE_NORMAL;
    bid(P, s);
    return true;
}

// One loop iteration of a working lane.  Returns a status != ACTIVE when the
// particle ended (its result already stored).
template <class T, int LAYOUT, bool MULTI>
__device__ __forceinline__ int advance(const PropArgs &a, int64_t p, Lane &s, LocalCounters &cnt) {
    const ParamsDev &P = a.params[MULTI ? s.pidx : 0];
    const FieldDev &F = a.fields[MULTI ? P.field_index : 0];
    double y5[6], ex, eu;
    ck_eval<T, LAYOUT>(F, s.kap, s.y, s.h, y5, ex, eu);
    cnt.evals++;

    if (s.mode == MODE_NORMAL) {
        double exh = ex / s.h;
        if (!isfinite(eu) || !isfinite(exh)) {
            store(a, p, s, CRP_ST_NONFINITE, true);
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
            s.nrej++;
            cnt.rej++;
            return CRP_ST_ACTIVE;
        }
        // accepted: next controller bid
        double g;
        if (err > 1.0) {
            g = 1.0;
            cnt.fl++;
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
        s.nacc++;
        s.ncall++;
        cnt.acc++;
        if (P.sphere_on && sphere_g(P, y5) >= 0.0) {
            s.mode = MODE_EVENT;
            s.lo = 0.0;
            s.glo = sphere_g(P, s.y);
            s.hi = s.h;
            s.ghi = sphere_g(P, y5);
            s.hacc = s.h;
            s.lacc = Lnew;
            s.side = 0;
            s.eit = 0;
            event_next(P, s);
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
            store(a, p, s, CRP_ST_MAX_LENGTH, true);
            return CRP_ST_MAX_LENGTH;
        }
        if (P.max_steps > 0 && s.ncall >= P.max_steps) {
            store(a, p, s, CRP_ST_MAX_STEPS, true);
            return CRP_ST_MAX_STEPS;
        }
        bid(P, s);
        return CRP_ST_ACTIVE;
    }

    cnt.ev++;
    if (s.mode == MODE_EVENT) {
        double gs = sphere_g(P, y5);
        if (!isfinite(gs)) {
            store(a, p, s, CRP_ST_NONFINITE, true);
            return CRP_ST_NONFINITE;
        }
        if (gs >= 0.0) {
            s.hi = s.h;
            s.ghi = gs;
            if (s.side == 1) s.glo = s.glo * 0.5;
            s.side = 1;
        } else {
            s.lo = s.h;
            s.glo = gs;
            if (s.side == -1) s.ghi = s.ghi * 0.5;
            s.side = -1;
        }
        s.eit++;
        event_next(P, s);
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
    s.L = s.hi == s.hacc ? s.lacc : s.L + s.hi;
    store(a, p, s, CRP_ST_ARRIVED, true);
    return CRP_ST_ARRIVED;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class T, int LAYOUT, bool MULTI>
__global__ void __launch_bounds__(256) k_propagate_fp64(PropArgs a) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int64_t pid = -1;  // >= 0 working, -1 wants work, -2 queue exhausted
    Lane s;
    LocalCounters cnt = {0, 0, 0, 0, 0, 0};

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
            if (pid == -1) {
                unsigned long long q = base + (unsigned long long)__popcll(want & below);
                if (q < (unsigned long long)a.n) {
                    int64_t p = a.order ? (int64_t)a.order[q] : (int64_t)q;
                    cnt.taken++;
                    pid = start<MULTI>(a, p, s) ? p : -1;
                } else {
                    pid = -2;
                }
            }
        }
        if (__ballot(pid >= 0) == 0ull) {
            if (__ballot(pid == -1) == 0ull) break;
            continue;
        }
        if (pid >= 0) {
            int st = advance<T, LAYOUT, MULTI>(a, pid, s, cnt);
            if (st != CRP_ST_ACTIVE) pid = -1;
        }
    }

    if (a.counters) {
        unsigned long long v[6] = {cnt.evals, cnt.acc, cnt.rej, cnt.ev, cnt.fl, cnt.taken};
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            unsigned long long t = wave_sum(v[i]);
            if (lane == 0 && t) atomicAdd(a.counters + i, t);
        }
    }
}

template <class T, int LAYOUT>
hipError_t launch_t(const PropArgs &a, bool multi, int blocks, int bs, hipStream_t s) {
    if (multi)
        hipLaunchKernelGGL((k_propagate_fp64<T, LAYOUT, true>), dim3(blocks), dim3(bs), 0, s, a);
    else
        hipLaunchKernelGGL((k_propagate_fp64<T, LAYOUT, false>), dim3(blocks), dim3(bs), 0, s, a);
    return hipGetLastError();
}

template <class T>
hipError_t launch_layout(const PropArgs &a, int layout, bool multi, int blocks, int bs, hipStream_t s) {
    if (layout == CRP_LAYOUT_CELL8) return launch_t<T, CRP_LAYOUT_CELL8>(a, multi, blocks, bs, s);
    return launch_t<T, CRP_LAYOUT_LINEAR>(a, multi, blocks, bs, s);
}

}  // namespace

hipError_t launch_propagate_fp64(const PropArgs &a, int dtype, int layout, bool multi, int blocks,
                                 int block_size, hipStream_t s) {
    switch (dtype) {
        case CRP_F64: return launch_layout<double>(a, layout, multi, blocks, block_size, s);
        case CRP_F32: return launch_layout<float>(a, layout, multi, blocks, block_size, s);
        case CRP_F16: return launch_layout<__half>(a, layout, multi, blocks, block_size, s);
        case CRP_BF16: return launch_layout<__hip_bfloat16>(a, layout, multi, blocks, block_size, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace crp
