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
#include <type_traits>

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
    int64_t tlast;        // the particle's last tape record, -1 none
};

// Tape: take the next record of the pool for the lane's current state (the
// state before its next accepted step) and link it to the particle's previous
// record.
__device__ __forceinline__ void tape_checkpoint(const PropArgs &a, Lane &s) {
    const unsigned long long slot = atomicAdd(a.tape_head, 1ull);
    if (slot >= (unsigned long long)a.tape_cap) {
        s.tflags |= CRP_TAPE_OVERFLOW;
        return;
    }
    double *r = a.tape_ckpt + 8 * (int64_t)slot;
    r[0] = s.y[0];
    r[1] = s.y[1];
    r[2] = s.y[2];
    r[3] = s.y[3];
    r[4] = s.y[4];
    r[5] = s.y[5];
    r[6] = s.L;
    r[7] = s.hctrl;
    a.tape_link[slot] = s.tlast;
    s.tlast = (int64_t)slot;
}

__device__ __forceinline__ void tape_final(const PropArgs &a, int64_t p, const Lane &s, double sstar, int flags) {
    double *f = a.tape_fin + 4 * p;
    f[0] = (double)s.dacc;
    f[1] = sstar;
    f[2] = (double)s.tlast;
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
template <bool RFL>
__device__ __forceinline__ void bid(const ParamsDev &P, Lane &s) {
    double h = s.hctrl;
    if (h > P.h_max) h = P.h_max;
    if (P.sphere_on) {
        double d0 = s.y[0] - P.center[0], d1 = s.y[1] - P.center[1], d2 = s.y[2] - P.center[2];
        double dist = P.radius - sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (dist < h) h = dist;
    }
    if (RFL && P.reflect_on) {
        // the distance to the nearest face of the reflective box bids too
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double dlo = s.y[c] - P.box_lo[c], dhi = P.box_hi[c] - s.y[c];
            if (dlo < h) h = dlo;
            if (dhi < h) h = dhi;
        }
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

// Reflective box: an accepted step that ends outside the box on an axis is
// mirrored on that face (position 2 face - x, that direction component
// negated).  Returns the mirrored axes (bit c for axis c).
__device__ __forceinline__ int reflect(const ParamsDev &P, double y[6]) {
    int m = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (y[c] > P.box_hi[c]) {
            y[c] = 2.0 * P.box_hi[c] - y[c];
            y[3 + c] = -y[3 + c];
            m |= 1 << c;
        } else if (y[c] < P.box_lo[c]) {
            y[c] = 2.0 * P.box_lo[c] - y[c];
            y[3 + c] = -y[3 + c];
            m |= 1 << c;
        }
    }
    return m;
}

// Write the particle's state back (its own slots only).
__device__ __forceinline__ void store(const ParamsDev &P, int64_t p, const Lane &s, double hnext, int st) {
    KernArg<PropArgs> &a = kernel_args<PropArgs>();
    a.x[p] = s.y[0];
    a.y[p] = s.y[1];
    a.z[p] = s.y[2];
    // backtracking carries the antiparticle's direction: reverse it back
    a.ux[p] = P.backtrack_on ? -s.y[3] : s.y[3];
    a.uy[p] = P.backtrack_on ? -s.y[4] : s.y[4];
    a.uz[p] = P.backtrack_on ? -s.y[5] : s.y[5];
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

// The cancel flag is read once every CANCEL_POLL loop iterations of a wavefront.
constexpr unsigned int CANCEL_POLL = 64;

// Per-iteration outcome bits of a lane; the wavefront sums them with ballots
// into wave-uniform (scalar) counters.
enum { F_EVAL = 1, F_ACC = 2, F_REJ = 4, F_EVENT = 8, F_FLOOR = 16 };

// Start particle p in lane state s.  Returns true if it needs steps; false if
// it was skipped (not ACTIVE) or finished at once (its result is stored).
template <bool MULTI, bool TAPE, bool RFL>
__device__ __forceinline__ bool start(const PropArgs &args, int64_t p, Lane &s) {
    KernArg<PropArgs> &a = kernel_args<PropArgs>();  // the particle arrays
    int st = a.status[p];
    if (TAPE) {
        double *f = a.tape_fin + 4 * p;  // overwritten when the particle completes
        f[0] = f[1] = f[3] = 0.0;
        f[2] = -1.0;
        s.tlast = -1;
    }
    if (st != CRP_ST_ACTIVE) return false;
    s.pidx = MULTI && a.param_index ? a.param_index[p] : 0;
    if (MULTI && (s.pidx < 0 || s.pidx >= a.n_params)) {
        a.status[p] = CRP_ST_BAD_INPUT;
        return false;
    }
    const ParamsDev &P = MULTI ? args.params[s.pidx] : args.P0;
    double E = a.energy[p];
    int Z = a.charge[p];
    s.y[0] = a.x[p];
    s.y[1] = a.y[p];
    s.y[2] = a.z[p];
    s.y[3] = a.ux[p];
    s.y[4] = a.uy[p];
    s.y[5] = a.uz[p];
    if (P.backtrack_on) {  // the antiparticle, moving the other way
        s.y[3] = -s.y[3];
        s.y[4] = -s.y[4];
        s.y[5] = -s.y[5];
    }
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
        store(P, p, s, hn, CRP_ST_ARRIVED);
        if (TAPE) tape_final(args, p, s, 0.0, CRP_TAPE_COMPLETE);
        return false;
    }
    if (P.lmax_on && s.L >= P.l_max) {
        store(P, p, s, hn, CRP_ST_MAX_LENGTH);
        if (TAPE) tape_final(args, p, s, 0.0, CRP_TAPE_COMPLETE);
        return false;
    }
    s.hctrl = hn == 0.0 ? P.h_max : hn;
    s.kap = ((double)(P.backtrack_on ? -Z : Z) * K_LORENTZ) / E;
    s.mode = MODE_NORMAL;
    if (TAPE) tape_checkpoint(args, s);
    bid<RFL>(P, s);
    return true;
}

// One loop iteration of a working lane.  Returns a status != ACTIVE when the
// particle ended (its result already stored).
template <class T, int LAYOUT, bool MULTI, bool CACHE, bool TAPE, bool MOD, bool RFL>
__device__ __forceinline__ int advance(const PropArgs &a, int64_t p, Lane &s, CellCache<T, MULTI> &cache, EventLDS &e,
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
    double y5[6], ex, eu;
    ck_eval<T, LAYOUT, CACHE, NoStageRecord, MOD>(F, fid, cache, s.kap, s.y, s.h, y5, ex, eu);
    flags = F_EVAL;

    if (s.mode == MODE_NORMAL) {
        double exh = ex / s.h;
        if (!isfinite(eu) || !isfinite(exh)) {
            store(P, p, s, s.hctrl, CRP_ST_NONFINITE);
            if (TAPE) tape_final(a, p, s, 0.0, 0);
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
        if (RFL && P.reflect_on && reflect(P, s.y) && TAPE) s.tflags |= CRP_TAPE_MIRRORED;
        s.L = Lnew;
        if (P.lmax_on && s.L >= P.l_max) {
            store(P, p, s, s.hctrl, CRP_ST_MAX_LENGTH);
            if (TAPE) tape_final(a, p, s, 0.0, CRP_TAPE_COMPLETE);
            return CRP_ST_MAX_LENGTH;
        }
        if (P.max_steps > 0 && s.dacc >= P.max_steps) {
            store(P, p, s, s.hctrl, CRP_ST_MAX_STEPS);
            if (TAPE) tape_final(a, p, s, 0.0, 0);
            return CRP_ST_MAX_STEPS;
        }
        if (cancel) {  // the caller's cancel flag: stop here, resumable like a used-up budget
            store(P, p, s, s.hctrl, CRP_ST_CANCELLED);
            if (TAPE) tape_final(a, p, s, 0.0, 0);
            return CRP_ST_CANCELLED;
        }
        if (TAPE && s.dacc % a.tape_k == 0) tape_checkpoint(a, s);
        bid<RFL>(P, s);
        return CRP_ST_ACTIVE;
    }

    flags |= F_EVENT;
    if (s.mode == MODE_EVENT) {
        double gs = sphere_g(P, y5);
        if (!isfinite(gs)) {
            store(P, p, s, s.hctrl, CRP_ST_NONFINITE);
            if (TAPE) tape_final(a, p, s, 0.0, 0);
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
    store(P, p, s, s.hctrl, CRP_ST_ARRIVED);
    if (TAPE) tape_final(a, p, s, e.hi[t], CRP_TAPE_COMPLETE | CRP_TAPE_EVENT);
    return CRP_ST_ARRIVED;
}

// Minimum resident waves per SIMD the register allocation must allow (the
// kernel is bound by gather latency, so occupancy is what hides it).
#ifndef CRP_FP64_MIN_WAVES
#define CRP_FP64_MIN_WAVES 2
#endif

template <class T, int LAYOUT, bool MULTI, bool CACHE, bool TAPE, bool MOD, bool RFL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CRP_FP64_MIN_WAVES, 8)))
k_propagate_fp64(PropArgs a) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int64_t pid = -1;  // >= 0 working, -1 wants work, -2 queue exhausted
    __shared__ EventLDS ev;
    Lane s;
    // the cell cache in registers; with per-particle group tables (MULTI)
    // the registers are taken, and it lives in LDS
    __shared__ T cache_lds[CACHE && MULTI ? 24 : 1][CACHE_BLOCK];
    CellCache<T, MULTI> cache;
    if constexpr (MULTI)
        cache_reset(cache, cache_lds, threadIdx.x);
    else
        cache_reset(cache);
    // wave-uniform counters, summed from ballots (scalar registers)
    unsigned long long n_eval = 0, n_acc = 0, n_rej = 0, n_ev = 0, n_fl = 0, n_taken = 0, n_iter = 0;
    bool cancel = false;  // the caller's cancel flag was seen set

    for (;;) {
        if ((n_iter & (CANCEL_POLL - 1)) == 0 && !cancel) {
            // the pointer is read from the kernel-argument segment here, not held in
            // registers across the loop
            const int32_t *cw = kernel_args<PropArgs>().cancel;
            if (cw) cancel = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
        }
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
                if (q < (unsigned long long)a.n && !cancel) {
                    int64_t p = a.order ? (int64_t)a.order[q] : (int64_t)q;
                    got = 1;
                    pid = start<MULTI, TAPE, RFL>(a, p, s) ? p : -1;
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
            int st = advance<T, LAYOUT, MULTI, CACHE, TAPE, MOD, RFL>(a, pid, s, cache, ev, flags, cancel);
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

template <class T, int LAYOUT, bool MULTI, bool CACHE, bool TAPE, bool MOD, bool RFL = false>
hipError_t launch_one(const PropArgs &a, int blocks, int bs, hipStream_t s) {
    hipLaunchKernelGGL((k_propagate_fp64<T, LAYOUT, MULTI, CACHE, TAPE, MOD, RFL>), dim3(blocks), dim3(bs), 0, s, a);
    return hipGetLastError();
}

template <class T, int LAYOUT, bool MULTI>
hipError_t launch_c(const PropArgs &a, bool cache, int blocks, int bs, hipStream_t s) {
    constexpr bool wide = std::is_same<T, double>::value || std::is_same<T, float>::value;
    if (a.tape_ckpt) {
        // taped runs (for the adjoint): one field, FP64 or FP32 storage, with
        // or without a modulation and a reflective box
        if constexpr (!MULTI && wide) {
            if (a.modulated)
                return a.reflective ? launch_one<T, LAYOUT, false, false, true, true, true>(a, blocks, bs, s)
                                    : launch_one<T, LAYOUT, false, false, true, true, false>(a, blocks, bs, s);
            if (a.reflective) return launch_one<T, LAYOUT, false, false, true, false, true>(a, blocks, bs, s);
            return cache ? launch_one<T, LAYOUT, false, true, true, false>(a, blocks, bs, s)
                         : launch_one<T, LAYOUT, false, false, true, false>(a, blocks, bs, s);
        }
        return hipErrorInvalidValue;
    }
    if (a.reflective) {
        // a reflective box, with or without modulation; the cell cache is
        // instantiated for one parameter group only (with per-particle groups
        // its registers spill, and the automatic setting leaves it off)
        if (a.modulated) {
            if constexpr (wide) {
                if constexpr (!MULTI)
                    if (cache) return launch_one<T, LAYOUT, false, true, false, true, true>(a, blocks, bs, s);
                return launch_one<T, LAYOUT, MULTI, false, false, true, true>(a, blocks, bs, s);
            }
            return hipErrorInvalidValue;
        }
        if constexpr (!MULTI)
            if (cache) return launch_one<T, LAYOUT, false, true, false, false, true>(a, blocks, bs, s);
        return launch_one<T, LAYOUT, MULTI, false, false, false, true>(a, blocks, bs, s);
    }
    if (a.modulated) {
        // modulated fields: FP64 or FP32 storage
        if constexpr (wide)
            return cache ? launch_one<T, LAYOUT, MULTI, true, false, true>(a, blocks, bs, s)
                         : launch_one<T, LAYOUT, MULTI, false, false, true>(a, blocks, bs, s);
        return hipErrorInvalidValue;
    }
    return cache ? launch_one<T, LAYOUT, MULTI, true, false, false>(a, blocks, bs, s)
                 : launch_one<T, LAYOUT, MULTI, false, false, false>(a, blocks, bs, s);
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
// taped forward run are held fixed and the sphere crossing in the last step is
// differentiated through its defining equation (implicit function theorem).
// Each lane takes one particle; from its last checkpoint segment to its first
// it replays the segment's accepted steps with the forward kernel's own step
// logic (so the states are bit-identical), recording every accepted step's
// stage states and stage field values in its own column of the workspace,
// then sweeps the records in reverse.  The reverse sweep reads the recorded
// stages instead of recomputing them, so it gathers each stage's cell once
// (for the field gradient) and scatters the grid-gradient contributions to a
// natural-layout FP64 array with atomics.

// Record of one accepted step, one column per thread (stride = lanes): the
// pre-step state y (6), the step size (1), the stage states Y_1..Y_5 (30),
// the stage field values B_0..B_5 (18), the unnormalised output direction
// (3) and, in a reflective box, the axes mirrored after the step (1).
constexpr int REC_Y = 0, REC_H = 6, REC_STAGE = 7, REC_FIELD = 37, REC_ZU = 55, REC_MIR = 58,
              REC_SIZE = ADJ_RECORD_DOUBLES;
static_assert(REC_MIR + 1 == REC_SIZE, "record layout");

struct RecordWriter {
    double *r;       // field 0 of the record in this thread's column
    int64_t stride;  // threads in the launch
    __device__ __forceinline__ void stage(int i, const double *Y) const {
#pragma unroll
        for (int c = 0; c < 6; ++c) r[(REC_STAGE + 6 * (i - 1) + c) * stride] = Y[c];
    }
    __device__ __forceinline__ void field(int i, const double *B) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[(REC_FIELD + 3 * i + c) * stride] = B[c];
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
// evaluation recorded at r (this thread's column), then either a rejection
// (smaller step, returns false) or the acceptance (controller, normalisation,
// the mirror in a reflective box, the pre-step state, step size and mirrored
// axes recorded; returns true).
template <class T, int LAYOUT, bool RFL, bool MOD>
__device__ bool replay_attempt(const FieldDev &F, const ParamsDev &P, Lane &s, double *r, int64_t stride) {
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
// scratch column of 36 values for the stage derivatives.
template <class T, int LAYOUT, bool MOD>
__device__ void rec_output_ds(const FieldDev &F, double kap, const double *r, int64_t stride, double *kd,
                              double zs[6]) {
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
                accd = ADJ_A[i][j] * kd[(6 * j + c) * stride] + accd;
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
            kd[(6 * i + c) * stride] = kdi[c];
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

__device__ __forceinline__ void grad_flush(const FieldDev &F, GradAccum &g, double *gbar) {
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
            if (isfinite(v))
                unsafeAtomicAdd(gbar + 3 * node + c, v);
            else
                g.dropped = 1;
        }
    }
    g.key = 0xffffffffu;
}

// Make ci the accumulator's cell, flushing and clearing the slots when it
// changes.
__device__ __forceinline__ void grad_select(const FieldDev &F, GradAccum &g, const int ci[3], double *gbar) {
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
// crossing term).  Grid-gradient contributions go to gbar.  A modulated field
// B = b m (MOD): the vector grid's value takes b-bar = m B-bar, the position
// also (b . B-bar) dm/dX.
template <class T, int LAYOUT, bool MOD>
__device__ void reverse_step(const FieldDev &F, double kap, const double *r, int64_t stride, double lam[6],
                             const double *comb, GradAccum &acc, double *gbar, double &kbar) {
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
        grad_select(F, acc, ci, gbar);
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
#pragma unroll
            for (int c = 0; c < 3; ++c)
                // the lane owns its slot: an LDS add without return, no wait on a read
                __hip_atomic_fetch_add(&acc.v[3 * q + c][acc.t], w * bb[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
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

// One lane per particle; the lanes of a wavefront move through their
// particles' segments in lockstep: every lane replays its current segment
// (one attempt per loop iteration, lanes that are done idle), then every lane
// sweeps its records in reverse, so no lane replays while another one is in
// the reverse sweep.  Finished lanes take the next particle from a queue
// ordered by step count, longest first.
template <class T, int LAYOUT, bool RFL, bool MOD>
__global__ void __launch_bounds__(64) k_adjoint_fp64(AdjArgs a) {
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double acc_lds[24][64];
    GradAccum acc{acc_lds, (int)threadIdx.x, 0xffffffffu, {0, 0, 0}, 0};
    double *col = a.segbuf + lane;
    double *kdcol = a.segbuf + (int64_t)a.K * REC_SIZE * a.lanes + lane;
    const int64_t rstride = (int64_t)REC_SIZE * a.lanes;  // doubles between consecutive records
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
        }
        const bool busy = L.p >= 0;
        if (__ballot(busy) == 0ull) break;

        // replay the current segment from its checkpoint
        const int64_t nseg = busy ? (L.N + a.K - 1) / a.K : 0;
        const int m = busy ? (int)(L.seg == nseg - 1 ? L.N - L.seg * a.K : a.K) : 0;
        const bool event = busy && L.seg == nseg - 1 && (L.flags & CRP_TAPE_EVENT);
        Lane s;
        if (busy) {
            const double *ck = a.ckpt + 8 * L.slot;
            for (int c = 0; c < 6; ++c) s.y[c] = ck[c];
            s.L = ck[6];
            s.hctrl = ck[7];
            s.kap = L.kap;
        }
        // one attempt per loop iteration, so a lane's rejections cost the others nothing
        int j = 0;
        if (m > 0) bid<RFL>(a.P, s);
        while (__ballot(j < m) != 0ull) {
            if (j < m && replay_attempt<T, LAYOUT, RFL, MOD>(a.F, a.P, s, col + (int64_t)j * rstride, a.lanes))
                if (++j < m) bid<RFL>(a.P, s);
        }
        const int mmax = wave_max(m);
        if (event) {
            // record the last step again, taken to the located crossing s*
            double *r = col + (int64_t)(m - 1) * rstride;
            const double sstar = a.fin[4 * L.p + 1];
            double y[6], y5[6], ex, eu;
            for (int c = 0; c < 6; ++c) y[c] = r[(REC_Y + c) * a.lanes];
            CellCache<T> cache;
            cache_reset(cache);
            ck_eval<T, LAYOUT, false, RecordWriter, MOD>(a.F, 0, cache, L.kap, y, sstar, y5, ex, eu,
                                                    RecordWriter{r, a.lanes});
            r[REC_H * a.lanes] = sstar;
            for (int c = 0; c < 3; ++c) r[(REC_ZU + c) * a.lanes] = y5[3 + c];
            // crossing: psi = zbar . Phi_s + Lbar, cotangent zbar - (psi / g_s) dg/dz
            double z[6], zs[6];
            rec_output(L.kap, r, a.lanes, z);
            rec_output_ds<T, LAYOUT, MOD>(a.F, L.kap, r, a.lanes, kdcol, zs);
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
            reverse_step<T, LAYOUT, MOD>(a.F, L.kap, r, a.lanes, L.lam, comb, acc, a.grad_field, L.kbar);
        }
        // reverse sweep (the crossing step, if any, is done above; it ends on
        // the sphere, unmirrored)
        const int mrev = event ? m - 1 : m;
        for (int j = mmax - 1; j >= 0; --j)
            if (j < mrev) {
                if (RFL) mirror_cotangent(col + (int64_t)j * rstride, a.lanes, L.lam);
                reverse_step<T, LAYOUT, MOD>(a.F, L.kap, col + (int64_t)j * rstride, a.lanes, L.lam, nullptr, acc,
                                        a.grad_field, L.kbar);
            }
        if (busy) {
            if (--L.seg < 0) {
                grad_flush(a.F, acc, a.grad_field);
                adj_finish(L, acc.dropped);
                L.p = -1;
            } else {
                L.slot = a.link[L.slot];
                if (L.slot < 0 || L.slot >= a.cap) {  // a broken chain: no adjoint for this particle
                    grad_flush(a.F, acc, a.grad_field);
                    adj_zero(L.p);
                    L.p = -1;
                }
            }
        }
    }
}

}  // namespace

template <bool RFL, bool MOD>
hipError_t launch_adjoint_feat(const AdjArgs &a, int blocks, hipStream_t s) {
    switch (a.F.dtype * 2 + (a.F.layout == CRP_LAYOUT_CELL8)) {
        case CRP_F64 * 2: hipLaunchKernelGGL((k_adjoint_fp64<double, CRP_LAYOUT_LINEAR, RFL, MOD>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F64 * 2 + 1: hipLaunchKernelGGL((k_adjoint_fp64<double, CRP_LAYOUT_CELL8, RFL, MOD>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F32 * 2: hipLaunchKernelGGL((k_adjoint_fp64<float, CRP_LAYOUT_LINEAR, RFL, MOD>), dim3(blocks), dim3(64), 0, s, a); break;
        case CRP_F32 * 2 + 1: hipLaunchKernelGGL((k_adjoint_fp64<float, CRP_LAYOUT_CELL8, RFL, MOD>), dim3(blocks), dim3(64), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Instances per feature: a reflective box (RFL) and a modulated field (MOD).
hipError_t launch_adjoint_fp64(const AdjArgs &a, int blocks, hipStream_t s) {
    const bool mod = a.F.mod_data != nullptr;
    if (a.P.reflect_on)
        return mod ? launch_adjoint_feat<true, true>(a, blocks, s) : launch_adjoint_feat<true, false>(a, blocks, s);
    return mod ? launch_adjoint_feat<false, true>(a, blocks, s) : launch_adjoint_feat<false, false>(a, blocks, s);
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
