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

#include "lane.h"

namespace crp {
namespace {

using namespace dev;

enum { MODE_NORMAL = 0, MODE_EVENT = 1, MODE_FINAL = 2 };

constexpr int MAX_BLOCK = 256;

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
