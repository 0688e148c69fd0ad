// Binning of the charges into the cell list used by the near part and by the
// spreading step: fixed-point encoding of the positions, cell histogram,
// scan, scatter and a per-cell ranking that makes the order deterministic.
//
// Positions are stored as uint32 fractions of the cell edge (u = x/L * 2^32),
// so a periodic wrap is an integer overflow and the int32 difference of two
// encodings is the exact minimum-image separation.
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

__global__ void __launch_bounds__(256) k_encode(BinArgs a, const float* __restrict__ xyz,
                                                const float* __restrict__ q,
                                                uint4* __restrict__ coord,
                                                int* __restrict__ cell_of,
                                                int* __restrict__ cell_count,
                                                double* __restrict__ qpart) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double qs = 0.0, q2 = 0.0;
    if (i < a.n) {
        uint32_t u[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = to_fixed((double)xyz[3 * i + k], a.inv_box[k]);
        const float qi = q[i];
        const int c = (cell_coord(u[2], a.nc[2]) * a.nc[1] + cell_coord(u[1], a.nc[1])) * a.nc[0] +
                      cell_coord(u[0], a.nc[0]);
        coord[i] = make_uint4(u[0], u[1], u[2], __float_as_uint(qi));
        cell_of[i] = c;
        atomicAdd(&cell_count[c], 1);
        qs = qi;
        q2 = (double)qi * (double)qi;
    }
    __shared__ double s1[256], s2[256];
    s1[threadIdx.x] = qs;
    s2[threadIdx.x] = q2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        qpart[2 * blockIdx.x] = s1[0];
        qpart[2 * blockIdx.x + 1] = s2[0];
    }
}

// One block of 1024 threads: exclusive scan of the cell counts (each thread
// owns a contiguous chunk; wavefront scans by shuffles, then a scan of the 16
// wavefront totals), zero the fill counters, and reduce the charge partials
// in a fixed order (sum q, sum q^2).
__global__ void __launch_bounds__(1024) k_scan(int ncell, const int* __restrict__ count,
                                               int* __restrict__ start, int* __restrict__ fill,
                                               const double* __restrict__ qpart, int nqpart,
                                               double* __restrict__ qstats) {
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int chunk = (ncell + 1023) / 1024;
    const int lo = min(t * chunk, ncell), hi = min(lo + chunk, ncell);
    int s = 0;
    for (int c = lo; c < hi; ++c) s += count[c];
    int v = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    if (wv == 0) {
        int x = lane < 16 ? wsum[lane] : 0;
        const int own = x;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int u = __shfl_up(x, off, 64);
            if (lane >= off) x += u;
        }
        if (lane < 16) wsum[lane] = x - own;
    }
    __syncthreads();
    int run = wsum[wv] + v - s;   // exclusive prefix of this chunk
    for (int c = lo; c < hi; ++c) {
        start[c] = run;
        run += count[c];
        fill[c] = 0;
    }
    if (t == 1023) start[ncell] = run;
    if (wv == 1) {
        double a = 0.0, b = 0.0;
        for (int k = lane; k < nqpart; k += 64) {
            a += qpart[2 * k];
            b += qpart[2 * k + 1];
        }
        a = wave_sum_d(a);
        b = wave_sum_d(b);
        if (lane == 0) {
            qstats[0] = a;
            qstats[1] = b;
        }
    }
}

__global__ void __launch_bounds__(256) k_scatter(int n, const int* __restrict__ cell_of,
                                                 const int* __restrict__ start,
                                                 int* __restrict__ fill, int* __restrict__ perm) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int slot = atomicAdd(&fill[c], 1);
    perm[start[c] + slot] = i;
}

// One thread per charge: its rank inside its cell is the number of charges of
// the same cell with a smaller input index, so the order inside a cell does
// not depend on the timing of the scatter atomics.  Writes the permutation
// (sorted slot -> input index) and the sorted encoded positions.
__global__ void __launch_bounds__(256) k_rank(int n, const int* __restrict__ cell_of,
                                              const int* __restrict__ start,
                                              const int* __restrict__ slots,
                                              const uint4* __restrict__ coord,
                                              int* __restrict__ perm,
                                              uint4* __restrict__ sorted) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int lo = start[c], hi = start[c + 1];
    int rank = 0;
    for (int k = lo; k < hi; ++k) rank += slots[k] < i;
    perm[lo + rank] = i;
    sorted[lo + rank] = coord[i];
}

hipError_t launch_encode(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                         int* cell_of, int* cell_count, double* qpart, int nqpart,
                         hipStream_t st) {
    if (a.n > 0)
        hipLaunchKernelGGL(k_encode, dim3(nqpart), dim3(256), 0, st, a, xyz, q, coord, cell_of,
                           cell_count, qpart);
    return hipGetLastError();
}

hipError_t launch_scan(int ncell, const int* cell_count, int* cell_start, int* cell_fill,
                       const double* qpart, int nqpart, double* qstats, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, ncell, cell_count, cell_start,
                       cell_fill, qpart, nqpart, qstats);
    return hipGetLastError();
}

hipError_t launch_scatter(int n, const int* cell_of, const int* cell_start, int* cell_fill,
                          int* perm, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, st, n, cell_of,
                           cell_start, cell_fill, perm);
    return hipGetLastError();
}

hipError_t launch_rank(int n, const int* cell_of, const int* cell_start, const int* slots,
                       const uint4* coord, int* perm, uint4* sorted, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_rank, dim3((n + 255) / 256), dim3(256), 0, st, n, cell_of,
                           cell_start, slots, coord, perm, sorted);
    return hipGetLastError();
}

}  // namespace useries
