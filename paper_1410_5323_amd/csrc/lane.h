// lane.h -- the per-lane FP64 particle state and the step bid, shared by the
// propagation kernel and the adjoint's replay (which must take every step
// exactly as the propagation did).
#pragma once

#include "crp_device.h"

namespace crp {
namespace {

using namespace dev;

// Per-lane state kept in registers for the whole loop.
struct Lane {
    double y[6];          // current state (x, u); the pre-step state while locating an event
    double kap, L, hctrl, h;
    int32_t dacc, drej;   // accepted / rejected attempts of this call
    int32_t mode, binding, pidx;
    int32_t tflags;       // tape flags of this particle (fresh start, overflow)
    int64_t tlast;        // the particle's last tape record, -1 none
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
}  // namespace
}  // namespace crp
