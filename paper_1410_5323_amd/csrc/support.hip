// support.hip -- small kernels around the propagation kernel (gfx950):
// descriptor-table writes, queue reset, longest-first ordering and the
// device arithmetic self-test.
#include <cstring>

#include "crp_device.h"

namespace crp {
namespace {

// A chunk of a descriptor table passed by value (1 KiB), written by one block.
struct TableChunk {
    uint32_t words[256];
};

__global__ void k_write_table(uint32_t *dst, TableChunk c, int nwords) {
    int t = threadIdx.x;
    if (t < nwords) dst[t] = c.words[t];
}

__global__ void k_fill_u64(unsigned long long *dst, unsigned long long v, int count) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = v;
}

// Work-ordering key: lower magnetic rigidity E/|Z| means stronger deflection,
// smaller steps and longer trajectories, so those particles are handed out
// first (longest-processing-time-first keeps the tail of the launch short).
// Buckets of 1/8 in log2(rigidity / eV) starting at 2^40 eV; Z = 0 and
// inactive particles go last.
__device__ __forceinline__ int rigidity_bucket(double E, int Z, int st) {
    if (st != CRP_ST_ACTIVE || Z == 0 || !(E > 0.0)) return NBUCKET - 1;
    float lr = __log2f((float)(E / (double)(Z < 0 ? -Z : Z)));
    int b = (int)((lr - 40.0f) * 8.0f);
    return b < 0 ? 0 : (b > NBUCKET - 1 ? NBUCKET - 1 : b);
}

// Adjoint work order: most accepted steps first (buckets of 1/8 in log2 N).
__device__ __forceinline__ int steps_bucket(const double *fin, int64_t i) {
    double N = fin[4 * i];
    float l = __log2f((float)N + 1.0f);
    int b = NBUCKET - 1 - (int)(l * 8.0f);
    return b < 0 ? 0 : (b > NBUCKET - 1 ? NBUCKET - 1 : b);
}

struct RigidityKey {
    const double *E;
    const int32_t *Z;
    const int32_t *st;
    __device__ int operator()(int64_t i) const { return rigidity_bucket(E[i], Z[i], st[i]); }
};

struct StepsKey {
    const double *fin;
    __device__ int operator()(int64_t i) const { return steps_bucket(fin, i); }
};

template <class Key>
__global__ void __launch_bounds__(256) k_bucket_count(Key key, int64_t n, unsigned int *counts) {
    __shared__ unsigned int h[NBUCKET];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[key(i)], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

// Exclusive scan of the bucket counts into cursors (one block of NBUCKET threads).
__global__ void __launch_bounds__(256) k_bucket_scan(const unsigned int *counts, unsigned int *cursors) {
    __shared__ unsigned int s[NBUCKET];
    int t = threadIdx.x;
    s[t] = counts[t];
    __syncthreads();
    for (int off = 1; off < NBUCKET; off <<= 1) {
        unsigned int v = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    cursors[t] = t == 0 ? 0u : s[t - 1];
}

template <class Key>
__global__ void __launch_bounds__(256) k_bucket_scatter(Key key, int64_t n, unsigned int *cursors, int32_t *order) {
    __shared__ unsigned int h[NBUCKET];
    __shared__ unsigned int base[NBUCKET];
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
        h[threadIdx.x] = 0;
        __syncthreads();
        int64_t i = i0 + threadIdx.x;
        int b = 0;
        unsigned int r = 0;
        if (i < n) {
            b = key(i);
            r = atomicAdd(&h[b], 1u);
        }
        __syncthreads();
        if (h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursors[threadIdx.x], h[threadIdx.x]);
        __syncthreads();
        if (i < n) order[base[b] + r] = (int32_t)i;
        __syncthreads();
    }
}

// Device arithmetic probes (op codes as in crp_selftest_arith).
__global__ void k_selftest(const double *in, double *out, int64_t n, int op) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r;
    switch (op) {
        case 0: r = sqrt(in[i]); break;
        case 1: r = 1.0 / in[i]; break;
        case 2: r = fma(in[3 * i], in[3 * i + 1], in[3 * i + 2]); break;
        case 3: r = floor(in[i]); break;
        case 4: r = dev::inv_fifth_root(in[i]); break;
        case 5: r = 1.0 / sqrt(sqrt(in[i])); break;
        default: r = in[2 * i] / in[2 * i + 1]; break;
    }
    out[i] = r;
}

}  // namespace

hipError_t launch_write_table(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const uint8_t *p = static_cast<const uint8_t *>(src);
    uint8_t *d = static_cast<uint8_t *>(dst);
    for (size_t off = 0; off < bytes; off += sizeof(TableChunk)) {
        TableChunk c;
        size_t nb = bytes - off < sizeof(TableChunk) ? bytes - off : sizeof(TableChunk);
        std::memset(&c, 0, sizeof c);
        std::memcpy(&c, p + off, nb);
        int nwords = (int)((nb + 3) / 4);
        hipLaunchKernelGGL(k_write_table, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t *>(d + off), c,
                           nwords);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long *dst, unsigned long long v, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3((count + 255) / 256), dim3(256), 0, s, dst, v, count);
    return hipGetLastError();
}

template <class Key>
hipError_t bucket_order(Key key, int64_t n, int32_t *order, unsigned int *buckets, hipStream_t s) {
    unsigned int *counts = buckets;
    unsigned int *cursors = buckets + NBUCKET;
    hipError_t e = launch_fill_u64(reinterpret_cast<unsigned long long *>(counts), 0ull, NBUCKET / 2, s);
    if (e != hipSuccess) return e;
    int64_t nb = (n + 255) / 256;
    int blocks = (int)(nb < 2048 ? nb : 2048);
    hipLaunchKernelGGL((k_bucket_count<Key>), dim3(blocks), dim3(256), 0, s, key, n, counts);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(NBUCKET), 0, s, counts, cursors);
    hipLaunchKernelGGL((k_bucket_scatter<Key>), dim3(blocks), dim3(256), 0, s, key, n, cursors, order);
    return hipGetLastError();
}

hipError_t launch_order_by_rigidity(const double *energy, const int32_t *charge, const int32_t *status,
                                    int64_t n, int32_t *order, unsigned int *buckets, hipStream_t s) {
    return bucket_order(RigidityKey{energy, charge, status}, n, order, buckets, s);
}

hipError_t launch_order_by_steps(const double *fin, int64_t n, int32_t *order, unsigned int *buckets, hipStream_t s) {
    return bucket_order(StepsKey{fin}, n, order, buckets, s);
}

hipError_t launch_selftest(const double *in, double *out, int64_t n, int op, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_selftest, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n, op);
    return hipGetLastError();
}

}  // namespace crp
