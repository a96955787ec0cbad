// lens.hip -- HEALPix binning, lens construction and lens application (gfx950).
//
// The lensing technique of section 3.3 (the PARSEC method): particles traced
// back from Earth (backtracking) to the galactic border give, per rigidity, a
// sparse matrix over sky pixels that maps directions at the border to the
// directions observed at Earth; whole arrival distributions are transformed
// by matrix-vector products.  The sky is pixelised with HEALPix (Gorski et
// al. 2005, ApJ 622:759) in its RING numbering.
//
// Construction: a counting sort of the launches by observed pixel (row),
// then one block per row sorts its border pixels in LDS (bitonic), run-length
// encodes them into (column, count) pairs and writes count / launches (a row
// of more than 4096 launches counts its columns in an LDS hash table
// instead); a scan of the per-row entry counts gives the CSR row pointers.  Application: one
// team of lanes per row, lanes split between the row's entries and the
// vectors, FP64 sums, HBM-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crp_internal.h"

namespace crp {
namespace {

constexpr double HALF_PI = 1.5707963267948966;
constexpr double TWO_PI = 6.283185307179586;
constexpr int32_t SENTINEL = 0x7fffffff;  // launches that did not reach the border sort last

// RING-scheme pixel of the direction (x, y, z) (any non-zero finite length),
// FP64, operations in this order: z/r decides the belt or the caps, phi =
// atan2 in [0, 2 pi), tt = phi / (pi/2); in the belt the two edge-line indices
// give the ring and the position in it; in the caps the distance from the
// pole does.  -1 for a zero or non-finite direction.
__device__ __forceinline__ int64_t ring_pixel(int64_t nside, double x, double y, double z) {
    const double ns = (double)nside;
    const double r = sqrt(x * x + y * y + z * z);
    if (!(r > 0.0) || !isfinite(r)) return -1;
    const double zz = z / r;
    const double za = fabs(zz);
    double phi = atan2(y, x);
    if (phi < 0.0) phi = phi + TWO_PI;
    double tt = phi / HALF_PI;
    if (tt >= 4.0) tt = 0.0;
    if (za <= 2.0 / 3.0) {
        const double t1 = ns * (0.5 + tt);
        const double t2 = ns * (zz * 0.75);
        const int64_t jp = (int64_t)floor(t1 - t2);
        const int64_t jm = (int64_t)floor(t1 + t2);
        int64_t ir = nside + 1 + jp - jm;  // belt ring; kept in range where rounding puts z on the edge
        ir = ir < 1 ? 1 : (ir > 2 * nside + 1 ? 2 * nside + 1 : ir);
        const int64_t kshift = 1 - (ir & 1);
        int64_t q = jp + jm - nside + kshift + 1;
        q = q < 0 ? 0 : q;
        const int64_t ip = (q / 2) % (4 * nside);
        return 2 * nside * (nside - 1) + 4 * nside * (ir - 1) + ip;
    }
    const double tp = tt - floor(tt);
    const double s = ns * sqrt(3.0 * (1.0 - za));
    const int64_t jp = (int64_t)floor(tp * s);
    const int64_t jm = (int64_t)floor((1.0 - tp) * s);
    int64_t ir = jp + jm + 1;
    ir = ir < 1 ? 1 : (ir > nside ? nside : ir);
    const int64_t ip = ((int64_t)floor(tt * (double)ir)) % (4 * ir);
    return zz > 0.0 ? 2 * ir * (ir - 1) + ip : 12 * nside * nside - 2 * ir * (ir + 1) + ip;
}

__global__ void __launch_bounds__(256) k_healpix(int32_t nside, const double *ux, const double *uy,
                                                 const double *uz, int64_t n, double sign, int32_t *pix) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = ux[i], y = uy[i], z = uz[i];
    if (sign < 0.0) {
        x = -x;
        y = -y;
        z = -z;
    }
    pix[i] = (int32_t)ring_pixel(nside, x, y, z);
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Launches per row; a row index outside [0, npix) raises flag bit 1 and is skipped.
__global__ void __launch_bounds__(256) k_lens_count(const int32_t *row, int64_t n, int64_t npix, uint32_t *counts,
                                                    uint32_t *flag) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = row[i];
    if (r < 0 || r >= npix) {
        atomicOr(flag, 1u);
        return;
    }
    atomicAdd(&counts[r], 1u);
}

// Exclusive scan of m counts into out[0..m] (out[m] = total), one block of
// 1024 threads walking tiles of 8192 values with a running carry.
__global__ void __launch_bounds__(1024) k_scan(const uint32_t *in, int64_t m, int64_t *out) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < m; base += 8192) {
        int64_t v[8];
        int64_t sum = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = base + 8 * t + k;
            v[k] = i < m ? (int64_t)in[i] : 0;
            sum += v[k];
        }
        part[t] = sum;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t a = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += a;
            __syncthreads();
        }
        int64_t run = carry + part[t] - sum;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = base + 8 * t + k;
            if (i < m) out[i] = run;
            run += v[k];
        }
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) out[m] = carry;
}

// Group the launches by row: each writes its border pixel (the pixel of the
// reversed velocity) or the sentinel into its row's segment.
__global__ void __launch_bounds__(256) k_lens_scatter(int32_t nside, const int32_t *row, const double *ux,
                                                      const double *uy, const double *uz, const int32_t *status,
                                                      int64_t n, int64_t npix, const int64_t *starts,
                                                      uint32_t *cursor, int32_t *colbuf) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = row[i];
    if (r < 0 || r >= npix) return;
    int32_t c = SENTINEL;
    if (status[i] == CRP_ST_ARRIVED) {
        const int64_t j = ring_pixel(nside, -ux[i], -uy[i], -uz[i]);
        if (j >= 0) c = (int32_t)j;
    }
    const uint32_t k = atomicAdd(&cursor[r], 1u);
    colbuf[starts[r] + k] = c;
}

constexpr int ROW_CAP = 4096;  // launches per row sorted in LDS; distinct columns of a larger row

// In-place bitonic sort of P (a power of two, <= ROW_CAP) keys in LDS by the
// block, carrying a value along when val is not null.
__device__ __forceinline__ void lds_bitonic(int32_t *key, int32_t *val, int P) {
    const int t = threadIdx.x;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = t; i < P; i += 256) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t a = key[i], b = key[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[l] = a;
                        if (val) {
                            const int32_t va = val[i];
                            val[i] = val[l];
                            val[l] = va;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// A row with more than ROW_CAP launches: its border pixels are counted in an
// LDS hash table of ROW_CAP slots (open addressing, linear probing), whose
// (column, count) pairs are then sorted by column and written as
// (column, count / launches).  More than ROW_CAP distinct columns raise flag
// bit 2 and give the row no entries.
__device__ void lens_row_counted(const int32_t *colbuf, int64_t s0, int64_t m, int64_t r, int32_t *scol, float *sval,
                                 uint32_t *nnz_row, uint32_t *flag, int32_t *key, int32_t *cnt) {
    __shared__ int full;
    __shared__ int nvalid;
    const int t = threadIdx.x;
    for (int i = t; i < ROW_CAP; i += 256) {
        key[i] = SENTINEL;
        cnt[i] = 0;
    }
    if (t == 0) {
        full = 0;
        nvalid = ROW_CAP;
    }
    __syncthreads();
    for (int64_t i = t; i < m; i += 256) {
        const int32_t c = colbuf[s0 + i];
        if (c == SENTINEL) continue;  // did not reach the border: denominator only
        uint32_t slot = ((uint32_t)c * 2654435761u) >> 20;  // 12 bits: ROW_CAP slots
        int probe = 0;
        for (; probe < ROW_CAP; ++probe, slot = (slot + 1) & (ROW_CAP - 1)) {
            const int32_t old = atomicCAS(&key[slot], SENTINEL, c);
            if (old == SENTINEL || old == c) {
                atomicAdd(&cnt[slot], 1);
                break;
            }
        }
        if (probe == ROW_CAP) full = 1;
    }
    __syncthreads();
    if (full) {
        if (t == 0) {
            atomicOr(flag, 2u);
            nnz_row[r] = 0;
        }
        return;
    }
    lds_bitonic(key, cnt, ROW_CAP);
    // the occupied slots now lead, in ascending column order
    for (int i = t; i < ROW_CAP; i += 256)
        if (key[i] != SENTINEL && (i + 1 == ROW_CAP || key[i + 1] == SENTINEL)) nvalid = i + 1;
    __syncthreads();
    const int total = key[0] == SENTINEL ? 0 : nvalid;
    for (int q = t; q < total; q += 256) {
        scol[s0 + q] = key[q];
        sval[s0 + q] = (float)((double)cnt[q] / (double)m);
    }
    if (t == 0) nnz_row[r] = (uint32_t)total;
}

// One block per row: bitonic sort of the row's border pixels in LDS, then
// run-length encoding into (column, count / launches), written at the row's
// segment start; the number of entries goes to nnz_row.  A row with more
// than ROW_CAP launches is counted in an LDS hash table instead.
__global__ void __launch_bounds__(256) k_lens_rows(const int32_t *colbuf, const int64_t *starts, int64_t npix,
                                                   int32_t *scol, float *sval, uint32_t *nnz_row, uint32_t *flag) {
    __shared__ int32_t key[ROW_CAP];
    __shared__ int32_t pos[ROW_CAP + 1];
    __shared__ int32_t wsum[4];
    const int64_t r = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t s0 = starts[r];
    const int64_t m64 = starts[r + 1] - s0;
    if (m64 > ROW_CAP) {
        lens_row_counted(colbuf, s0, m64, r, scol, sval, nnz_row, flag, key, pos);
        return;
    }
    const int m = (int)m64;
    if (m == 0) {
        if (t == 0) nnz_row[r] = 0;
        return;
    }
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = t; i < P; i += 256) key[i] = i < m ? colbuf[s0 + i] : SENTINEL;
    __syncthreads();
    lds_bitonic(key, nullptr, P);
    // heads of runs among the valid keys; each thread owns a contiguous chunk
    const int chunk = (P + 255) / 256;
    const int b0 = t * chunk;
    int local = 0;
    for (int i = b0; i < b0 + chunk && i < P; ++i)
        local += key[i] != SENTINEL && (i == 0 || key[i] != key[i - 1]);
    // block exclusive scan of the per-thread head counts (wave scans, then waves)
    const int lane = t & 63, w = t >> 6;
    int incl = local;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < w; ++q) before += wsum[q];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    int rank = before + incl - local;
    int valid_end = 0;  // number of valid keys = position of the first sentinel
    for (int i = b0; i < b0 + chunk && i < P; ++i) {
        if (key[i] != SENTINEL && (i == 0 || key[i] != key[i - 1])) pos[rank++] = i;
        if (key[i] != SENTINEL && (i + 1 == P || key[i + 1] == SENTINEL)) valid_end = i + 1;
    }
    if (valid_end) pos[total] = valid_end;
    __syncthreads();
    for (int q = t; q < total; q += 256) {
        const int count = pos[q + 1] - pos[q];
        scol[s0 + q] = key[pos[q]];
        sval[s0 + q] = (float)((double)count / (double)m);
    }
    if (t == 0) nnz_row[r] = (uint32_t)total;
}

// Copy each row's entries from its segment to its CSR position.
__global__ void __launch_bounds__(64) k_lens_compact(const int32_t *scol, const float *sval, const int64_t *starts,
                                                     const int64_t *row_ptr, int32_t *col, float *val) {
    const int64_t r = blockIdx.x;
    const int64_t s0 = starts[r], d0 = row_ptr[r], m = row_ptr[r + 1] - d0;
    for (int64_t q = threadIdx.x; q < m; q += 64) {
        col[d0 + q] = scol[s0 + q];
        val[d0 + q] = sval[s0 + q];
    }
}

// y[i][v] = sum over the row's entries e of val[e] * x[col[e]][v], x and y
// pixel-major with nvec values per pixel.  A team of S lanes takes one row:
// V lanes across the vectors and G = S / V across the entries; the G partial
// FP64 sums are combined with shuffles.
__global__ void __launch_bounds__(256) k_lens_apply(const int64_t *row_ptr, const int32_t *col, const float *val,
                                                    const float *x, float *y, int64_t npix, int32_t nvec, int S,
                                                    int V) {
    const int lane = threadIdx.x & 63;
    const int64_t team = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / S;
    const int sl = lane % S;  // lane within the team
    const int g = sl / V, vl = sl % V, G = S / V;
    const bool live = team < npix;
    const int64_t e0 = live ? row_ptr[team] : 0, e1 = live ? row_ptr[team + 1] : 0;
    for (int v0 = 0; v0 < nvec; v0 += V) {  // same trip count in every lane of the wave
        const int v = v0 + vl;
        double acc = 0.0;
        if (v < nvec) {
            // four entries' gathers in flight at once, summed in entry order
            int64_t e = e0 + g;
            for (; e + 3 * G < e1; e += 4 * G) {
                const int64_t c0 = col[e], c1 = col[e + G], c2 = col[e + 2 * G], c3 = col[e + 3 * G];
                const float w0 = val[e], w1 = val[e + G], w2 = val[e + 2 * G], w3 = val[e + 3 * G];
                const float x0 = x[c0 * nvec + v], x1 = x[c1 * nvec + v], x2 = x[c2 * nvec + v],
                            x3 = x[c3 * nvec + v];
                acc += (double)w0 * (double)x0;
                acc += (double)w1 * (double)x1;
                acc += (double)w2 * (double)x2;
                acc += (double)w3 * (double)x3;
            }
            for (; e < e1; e += G) acc += (double)val[e] * (double)x[(int64_t)col[e] * nvec + v];
        }
        for (int off = V; off < S; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if (live && g == 0 && v < nvec) y[team * nvec + v] = (float)acc;
    }
}

}  // namespace

hipError_t launch_healpix(int32_t nside, const double *ux, const double *uy, const double *uz, int64_t n,
                          double sign, int32_t *pix, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_healpix, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nside, ux, uy, uz, n, sign,
                       pix);
    return hipGetLastError();
}

LensWs lens_ws_layout(int32_t nside, int64_t n) {
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t npix = 12 * (size_t)nside * (size_t)nside;
    LensWs w;
    w.flag = 0;
    w.counts = 256;
    w.cursor = up(w.counts + 4 * npix);
    w.starts = up(w.cursor + 4 * npix);
    w.colbuf = up(w.starts + 8 * (npix + 1));
    w.scol = up(w.colbuf + 4 * (size_t)n);
    w.sval = up(w.scol + 4 * (size_t)n);
    w.total = up(w.sval + 4 * (size_t)n);
    return w;
}

hipError_t launch_lens_build(int32_t nside, const int32_t *row, const double *ux, const double *uy,
                             const double *uz, const int32_t *status, int64_t n, int64_t *row_ptr, int32_t *col,
                             float *val, uint8_t *ws, hipStream_t s) {
    const LensWs w = lens_ws_layout(nside, n);
    const int64_t npix = 12 * (int64_t)nside * nside;
    uint32_t *flag = reinterpret_cast<uint32_t *>(ws + w.flag);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + w.counts);
    uint32_t *cursor = reinterpret_cast<uint32_t *>(ws + w.cursor);
    int64_t *starts = reinterpret_cast<int64_t *>(ws + w.starts);
    int32_t *colbuf = reinterpret_cast<int32_t *>(ws + w.colbuf);
    int32_t *scol = reinterpret_cast<int32_t *>(ws + w.scol);
    float *sval = reinterpret_cast<float *>(ws + w.sval);
    const unsigned pb = (unsigned)((npix + 255) / 256), nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, flag, 0u, (int64_t)1);
    hipLaunchKernelGGL(k_fill_u32, dim3(pb), dim3(256), 0, s, counts, 0u, npix);
    hipLaunchKernelGGL(k_fill_u32, dim3(pb), dim3(256), 0, s, cursor, 0u, npix);
    if (n > 0) hipLaunchKernelGGL(k_lens_count, dim3(nb), dim3(256), 0, s, row, n, npix, counts, flag);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, npix, starts);
    if (n > 0)
        hipLaunchKernelGGL(k_lens_scatter, dim3(nb), dim3(256), 0, s, nside, row, ux, uy, uz, status, n, npix, starts,
                           cursor, colbuf);
    // cursor now holds the launches per row again; reuse it for the entries per row
    hipLaunchKernelGGL(k_lens_rows, dim3((unsigned)npix), dim3(256), 0, s, colbuf, starts, npix, scol, sval, cursor,
                       flag);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cursor, npix, row_ptr);
    hipLaunchKernelGGL(k_lens_compact, dim3((unsigned)npix), dim3(64), 0, s, scol, sval, starts, row_ptr, col, val);
    return hipGetLastError();
}

hipError_t launch_lens_apply(const int64_t *row_ptr, const int32_t *col, const float *val, const float *x, float *y,
                             int64_t npix, int32_t nvec, int64_t nnz, hipStream_t s) {
    // V lanes across the vectors (the power of two >= nvec, at most 64), the
    // team wide enough for about one entry per lane
    int V = 1;
    while (V < nvec && V < 64) V <<= 1;
    const double per_row = npix > 0 ? (double)nnz / (double)npix : 0.0;
    int S = V;
    while (S < 64 && (double)(S / V) < per_row) S <<= 1;
    const int64_t threads = npix * S;
    hipLaunchKernelGGL(k_lens_apply, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, row_ptr, col, val, x,
                       y, npix, nvec, S, V);
    return hipGetLastError();
}

}  // namespace crp
