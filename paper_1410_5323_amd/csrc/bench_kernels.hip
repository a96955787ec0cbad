// bench_kernels.hip -- measurement kernels for the roofline of the field lookups (gfx950).
//
// k_gather_bench: the lookup of the propagation kernel (same layout, dtype and
//   FP64 trilinear arithmetic) at pseudo-random positions, independent from one
//   lookup to the next, with few registers so that many waves are resident:
//   the achievable rate of field lookups for a given grid, layout and spread
//   of positions.
// k_stream_read / k_stream_copy: plain streaming reads (and copies) of a
//   buffer, the bandwidth ceiling of each memory level, and a transfer of
//   known size that calibrates hardware byte counters.
#include "crp_device.h"

namespace crp {
namespace {

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Uniform double in [0, 1) from a 32-bit state (xorshift32 step).
__device__ __forceinline__ double next_u01(uint32_t &s) {
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return (double)s * 0x1.0p-32;
}

// Positions: spread <= 0 -> uniform over the periodic box; spread > 0 -> a
// Gaussian-like cloud (sum of 3 uniforms, std ~ spread Mpc) around the origin.
template <class T, int LAYOUT>
__global__ void __launch_bounds__(256) k_gather_bench(FieldDev F, int64_t lookups, double spread, uint32_t seed,
                                                      double *sink) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t s = hash32((uint32_t)tid * 2654435761u ^ seed) | 1u;
    const double box0 = F.n[0] / F.inv_spacing, box1 = F.n[1] / F.inv_spacing, box2 = F.n[2] / F.inv_spacing;
    double acc = 0.0;
    for (int64_t i = 0; i < lookups; ++i) {
        double X[3];
        if (spread <= 0.0) {
            X[0] = F.origin[0] + next_u01(s) * box0;
            X[1] = F.origin[1] + next_u01(s) * box1;
            X[2] = F.origin[2] + next_u01(s) * box2;
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double g = next_u01(s) + next_u01(s) + next_u01(s) - 1.5;  // variance 1/4
                X[a] = 2.0 * spread * g;
            }
        }
        double B[3];
        dev::lookup<T, LAYOUT>(F, X, B);
        acc += B[0] + B[1] + B[2];
    }
    sink[tid] = acc;
}

// Replayed lookups: each lane walks a recorded stream of accepted steps
// (state x, u and step size h, layout [step][7][lane]) and looks the field up
// at the six Cash-Karp stage points of each step along the straight line,
// x + c_i h u, with the propagation kernel's lookup and (CACHE) its per-lane
// cell cache.  The lookups do not depend on one another, so many are in
// flight: the achievable lookup rate for the cell sequences a real run
// visits, including the locality the cell cache exploits.
template <class T, int LAYOUT, bool CACHE>
__global__ void __launch_bounds__(256) k_gather_replay(FieldDev F, const double *rec, int64_t lanes, int64_t steps,
                                                       double *sink, int64_t *misses) {
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (lane >= lanes) return;
    constexpr double C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
    dev::CellCache<T> cache;
    dev::cache_reset(cache);
    double acc = 0.0;
    for (int64_t s = 0; s < steps; ++s) {
        const double *r = rec + s * 7 * lanes + lane;
        const double x[3] = {r[0], r[lanes], r[2 * lanes]};
        const double u[3] = {r[3 * lanes], r[4 * lanes], r[5 * lanes]};
        const double h = r[6 * lanes];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const double X[3] = {fma(C[i] * h, u[0], x[0]), fma(C[i] * h, u[1], x[1]), fma(C[i] * h, u[2], x[2])};
            double B[3];
            dev::lookup_cached<T, LAYOUT, CACHE>(F, 0, X, B, cache);
            acc += B[0] + B[1] + B[2];
        }
    }
    sink[lane] = acc;
    if (misses) misses[lane] = cache.misses;
}

__global__ void __launch_bounds__(256) k_stream_read(const float4 *src, uint64_t n4, double *sink) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    float a = 0.f;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
        float4 v = src[i];
        a += (v.x + v.y) + (v.z + v.w);
    }
    sink[blockIdx.x * (uint64_t)blockDim.x + threadIdx.x] = a;
}

__global__ void __launch_bounds__(256) k_stream_copy(const float4 *src, float4 *dst, uint64_t n4) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

template <class T>
hipError_t gather_t(const FieldDev &F, int64_t lanes, int64_t lookups, double spread, uint32_t seed, double *sink,
                    hipStream_t s) {
    unsigned blocks = (unsigned)((lanes + 255) / 256);
    if (F.layout == CRP_LAYOUT_CELL8)
        hipLaunchKernelGGL((k_gather_bench<T, CRP_LAYOUT_CELL8>), dim3(blocks), dim3(256), 0, s, F, lookups, spread,
                           seed, sink);
    else
        hipLaunchKernelGGL((k_gather_bench<T, CRP_LAYOUT_LINEAR>), dim3(blocks), dim3(256), 0, s, F, lookups, spread,
                           seed, sink);
    return hipGetLastError();
}

template <class T>
hipError_t replay_t(const FieldDev &F, const double *rec, int64_t lanes, int64_t steps, bool cache, double *sink,
                    int64_t *misses, hipStream_t s) {
    const unsigned blocks = (unsigned)((lanes + 255) / 256);
    if (F.layout == CRP_LAYOUT_CELL8) {
        if (cache)
            hipLaunchKernelGGL((k_gather_replay<T, CRP_LAYOUT_CELL8, true>), dim3(blocks), dim3(256), 0, s, F, rec,
                               lanes, steps, sink, misses);
        else
            hipLaunchKernelGGL((k_gather_replay<T, CRP_LAYOUT_CELL8, false>), dim3(blocks), dim3(256), 0, s, F, rec,
                               lanes, steps, sink, misses);
    } else {
        if (cache)
            hipLaunchKernelGGL((k_gather_replay<T, CRP_LAYOUT_LINEAR, true>), dim3(blocks), dim3(256), 0, s, F, rec,
                               lanes, steps, sink, misses);
        else
            hipLaunchKernelGGL((k_gather_replay<T, CRP_LAYOUT_LINEAR, false>), dim3(blocks), dim3(256), 0, s, F, rec,
                               lanes, steps, sink, misses);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gather_replay(const FieldDev &F, const double *rec, int64_t lanes, int64_t steps, bool cache,
                                double *sink, int64_t *misses, hipStream_t s) {
    switch (F.dtype) {
        case CRP_F64: return replay_t<double>(F, rec, lanes, steps, cache, sink, misses, s);
        case CRP_F32: return replay_t<float>(F, rec, lanes, steps, cache, sink, misses, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_bench(const FieldDev &F, int64_t lanes, int64_t lookups, double spread, uint32_t seed,
                               double *sink, hipStream_t s) {
    switch (F.dtype) {
        case CRP_F64: return gather_t<double>(F, lanes, lookups, spread, seed, sink, s);
        case CRP_F32: return gather_t<float>(F, lanes, lookups, spread, seed, sink, s);
        case CRP_F16: return gather_t<__half>(F, lanes, lookups, spread, seed, sink, s);
        case CRP_BF16: return gather_t<__hip_bfloat16>(F, lanes, lookups, spread, seed, sink, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stream(const void *src, void *dst, size_t bytes, double *sink, int blocks, hipStream_t s) {
    uint64_t n4 = bytes / 16;
    if (dst)
        hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, s, static_cast<const float4 *>(src),
                           static_cast<float4 *>(dst), n4);
    else
        hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, s, static_cast<const float4 *>(src), n4, sink);
    return hipGetLastError();
}

}  // namespace crp
