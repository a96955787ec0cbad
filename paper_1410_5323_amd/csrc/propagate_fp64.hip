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
};

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
    if (P.sphere_on && sphere_g(P, s.y) >= 0.0) {
        store(a, p, s, hn, CRP_ST_ARRIVED);
        return false;
    }
    if (P.lmax_on && s.L >= P.l_max) {
        store(a, p, s, hn, CRP_ST_MAX_LENGTH);
        return false;
    }
    s.hctrl = hn == 0.0 ? P.h_max : hn;
    s.kap = ((double)Z * K_LORENTZ) / E;
    s.mode = MODE_NORMAL;
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
            return CRP_ST_MAX_LENGTH;
        }
        if (P.max_steps > 0 && s.dacc >= P.max_steps) {
            store(a, p, s, s.hctrl, CRP_ST_MAX_STEPS);
            return CRP_ST_MAX_STEPS;
        }
        bid(P, s);
        return CRP_ST_ACTIVE;
    }

    flags |= F_EVENT;
    if (s.mode == MODE_EVENT) {
        double gs = sphere_g(P, y5);
        if (!isfinite(gs)) {
            store(a, p, s, s.hctrl, CRP_ST_NONFINITE);
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
    return CRP_ST_ARRIVED;
}

template <class T, int LAYOUT, bool MULTI, bool CACHE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_propagate_fp64(PropArgs a) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int64_t pid = -1;  // >= 0 working, -1 wants work, -2 queue exhausted
    __shared__ EventLDS ev;
    __shared__ T cache_lds[CACHE ? 24 : 1][CACHE_BLOCK];
    Lane s;
    CellCache<T> cache;
    cache_reset(cache, cache_lds, threadIdx.x);
    // wave-uniform counters, summed from ballots (scalar registers)
    unsigned long long n_eval = 0, n_acc = 0, n_rej = 0, n_ev = 0, n_fl = 0, n_taken = 0;

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
            unsigned long long v[7] = {n_eval, n_acc, n_rej, n_ev, n_fl, n_taken, m};
#pragma unroll
            for (int i = 0; i < 7; ++i)
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

}  // namespace

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
