// upload.hip -- field grid conversion into the device layouts (gfx950).
//
// Source: C-order [n0][n1][n2][3] values in nG (FP64 or FP32), on the device.
// LINEAR: (n0+1)(n1+1)(n2+1) nodes, node (i,j,k) holds source node
//         (i mod n0, j mod n1, k mod n2): the wrap is stored once, so a cell
//         lookup never needs to wrap its +1 corners.
// CELL8:  per cell a record of the 8 corner vectors, order (dz, dy, dx, c),
//         padded with zeros to 32 values (one 128-byte line for FP32).
// Values are divided by value_scale in FP64, then rounded to nearest even:
// FP64 -> FP32 directly; FP16/BF16 from the FP32 value.
// Modulation grids (scalars) are stored like LINEAR with one component.
#include "crp_device.h"

namespace crp {
namespace {

template <class T> __device__ __forceinline__ T from_scaled(double v);
template <> __device__ __forceinline__ double from_scaled<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_scaled<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ __half from_scaled<__half>(double v) { return __float2half((float)v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_scaled<__hip_bfloat16>(double v) {
    return __float2bfloat16((float)v);
}

template <class S>
__device__ __forceinline__ double src_val(const S *src, uint64_t node, int c) {
    return (double)src[3 * node + c];
}

template <class T, class S>
__global__ void k_upload_linear(FieldDev f, const S *src, T *dst, uint64_t total) {
    const uint64_t n1p = (uint64_t)f.n[1] + 1, n2p = (uint64_t)f.n[2] + 1;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t node = e / 3;
        int c = (int)(e - node * 3);
        uint64_t k = node % n2p;
        uint64_t t = node / n2p;
        uint64_t j = t % n1p;
        uint64_t i = t / n1p;
        uint64_t si = i % (uint64_t)f.n[0], sj = j % (uint64_t)f.n[1], sk = k % (uint64_t)f.n[2];
        uint64_t snode = (si * f.n[1] + sj) * f.n[2] + sk;
        double v = src_val(src, snode, c);
        dst[e] = from_scaled<T>(v / f.value_scale);
    }
}

template <class T, class S>
__global__ void k_upload_cell8(FieldDev f, const S *src, T *dst, uint64_t total) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t cell = e >> 5;
        int w = (int)(e & 31);
        if (w >= 24) {
            dst[e] = from_scaled<T>(0.0);
            continue;
        }
        int c = w % 3;
        int corner = w / 3;  // (dz*2 + dy)*2 + dx
        int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
        uint64_t k = cell % (uint64_t)f.n[2];
        uint64_t t = cell / (uint64_t)f.n[2];
        uint64_t j = t % (uint64_t)f.n[1];
        uint64_t i = t / (uint64_t)f.n[1];
        uint64_t si = (i + dx) % (uint64_t)f.n[0], sj = (j + dy) % (uint64_t)f.n[1],
                 sk = (k + dz) % (uint64_t)f.n[2];
        uint64_t snode = (si * f.n[1] + sj) * f.n[2] + sk;
        double v = src_val(src, snode, c);
        dst[e] = from_scaled<T>(v / f.value_scale);
    }
}

template <class T, class S>
hipError_t launch_ts(const FieldDev &f, const S *src, void *dst, hipStream_t s) {
    uint64_t total;
    if (f.layout == CRP_LAYOUT_CELL8)
        total = (uint64_t)f.n[0] * f.n[1] * f.n[2] * 32ull;
    else
        total = ((uint64_t)f.n[0] + 1) * ((uint64_t)f.n[1] + 1) * ((uint64_t)f.n[2] + 1) * 3ull;
    uint64_t nb = (total + 255) / 256;
    unsigned blocks = (unsigned)(nb < 65536 ? nb : 65536);
    if (f.layout == CRP_LAYOUT_CELL8)
        hipLaunchKernelGGL((k_upload_cell8<T, S>), dim3(blocks), dim3(256), 0, s, f, src, static_cast<T *>(dst),
                           total);
    else
        hipLaunchKernelGGL((k_upload_linear<T, S>), dim3(blocks), dim3(256), 0, s, f, src, static_cast<T *>(dst),
                           total);
    return hipGetLastError();
}

// Modulation grid: source C-order [m0][m1][m2] scalars, stored padded
// (m0+1)(m1+1)(m2+1) with the wrap, rounded to nearest even into T.
template <class T, class S>
__global__ void k_upload_mod(FieldDev f, const S *src, T *dst, uint64_t total) {
    const uint64_t n1p = (uint64_t)f.mod_n[1] + 1, n2p = (uint64_t)f.mod_n[2] + 1;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t k = e % n2p;
        uint64_t t = e / n2p;
        uint64_t j = t % n1p;
        uint64_t i = t / n1p;
        uint64_t si = i % (uint64_t)f.mod_n[0], sj = j % (uint64_t)f.mod_n[1], sk = k % (uint64_t)f.mod_n[2];
        dst[e] = from_scaled<T>((double)src[(si * f.mod_n[1] + sj) * f.mod_n[2] + sk]);
    }
}

template <class T, class S>
hipError_t launch_mod(const FieldDev &f, const S *src, hipStream_t s) {
    uint64_t total = ((uint64_t)f.mod_n[0] + 1) * ((uint64_t)f.mod_n[1] + 1) * ((uint64_t)f.mod_n[2] + 1);
    uint64_t nb = (total + 255) / 256;
    unsigned blocks = (unsigned)(nb < 65536 ? nb : 65536);
    hipLaunchKernelGGL((k_upload_mod<T, S>), dim3(blocks), dim3(256), 0, s, f, src,
                       static_cast<T *>(const_cast<void *>(f.mod_data)), total);
    return hipGetLastError();
}

template <class S>
hipError_t launch_s(const FieldDev &f, const S *src, void *dst, hipStream_t s) {
    switch (f.dtype) {
        case CRP_F64: return launch_ts<double, S>(f, src, dst, s);
        case CRP_F32: return launch_ts<float, S>(f, src, dst, s);
        case CRP_F16: return launch_ts<__half, S>(f, src, dst, s);
        case CRP_BF16: return launch_ts<__hip_bfloat16, S>(f, src, dst, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_upload_modulation(const FieldDev &f, const void *src, int src_dtype, hipStream_t s) {
    const bool d64 = f.mod_dtype == CRP_F64;
    if (src_dtype == CRP_F64)
        return d64 ? launch_mod<double, double>(f, static_cast<const double *>(src), s)
                   : launch_mod<float, double>(f, static_cast<const double *>(src), s);
    if (src_dtype == CRP_F32)
        return d64 ? launch_mod<double, float>(f, static_cast<const float *>(src), s)
                   : launch_mod<float, float>(f, static_cast<const float *>(src), s);
    return hipErrorInvalidValue;
}

hipError_t launch_upload(const FieldDev &f, const void *src, int src_dtype, void *dst, hipStream_t s) {
    if (src_dtype == CRP_F64) return launch_s<double>(f, static_cast<const double *>(src), dst, s);
    if (src_dtype == CRP_F32) return launch_s<float>(f, static_cast<const float *>(src), dst, s);
    return hipErrorInvalidValue;
}

}  // namespace crp
