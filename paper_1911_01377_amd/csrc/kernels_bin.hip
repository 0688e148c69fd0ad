// Binning of the charges into x-y columns, sorted by z inside each column,
// and cut into clusters of up to 8 consecutive charges (spatially compact:
// one column cross-section by about the same extent in z).  Used by the near
// part (cluster-pair tiles) and by the spreading step (z-ranges per column).
//
// Positions are stored as uint32 fractions of the cell edge (u = x/L * 2^32),
// so a periodic wrap is an integer overflow and the int32 difference of two
// encodings is the exact minimum-image separation.
//
// Two sequences produce the same sorted charges, permutation and z-plane
// index; the clusters differ only in their numbering.
//
// Two launches (bin_local -> colbuild), when the column counts fit in LDS and
// the blocks' column prefixes are few enough for every column to read:
//   bin_local: block b of 256 charges ranks its charges within their columns
//     in LDS and writes them grouped by column into its own segment
//     [256 b, 256 b + 256) of the records, with its exclusive column prefix
//     P[b][0 .. ncol] (no global atomics, no counters);
//   colbuild: block c reads P[b][c] and P[b][c + 1] of every block b: its
//     first sorted position sum_b P[b][c], its count, and where its charges
//     lie in each segment; it gathers them, sorts them and writes the column.
//   Column c's clusters are numbered from floor(lo_c / 8) + c (lo_c its first
//   sorted position), so no prefix over the cluster counts of all columns is
//   needed; numbers left between two columns are clusters of no charge.
//
// Otherwise four: encode -> scan (column and cluster offsets) -> scatter
// (atomic slots) -> colsort, with consecutive cluster numbers.  When the
// column counts fit in LDS and are few enough to be read by every scatter
// block, each scatter block takes the offsets itself (block 0 also publishes
// them) and the scan launch is skipped; colsort clears the counters either
// way, ready for the next evaluation.
//
// Either way each column is sorted by (z, input index): a deterministic
// order.  Cluster numbers up to the pair kernel's block count that hold no
// charge have a count of 0.
#include <algorithm>

#include "useries_internal.h"
#include "device_common.h"

namespace useries {

// Column histograms are first taken in LDS per block (many charges share a
// column), then added to the global counters once per (block, column).
constexpr int kHistCols = 4096;

__device__ __forceinline__ void encode_body(const BinArgs& a, int bid, const float* __restrict__ xyz,
                                            const float* __restrict__ q,
                                            uint4* __restrict__ coord,
                                            int* __restrict__ col_count,
                                            double* __restrict__ qpart) {
    __shared__ double red[2][4];
    __shared__ int hist[kHistCols];
    const int ncol = a.nc[0] * a.nc[1];
    const bool local = ncol <= kHistCols;
    if (local)
        for (int k = threadIdx.x; k < ncol; k += 256) hist[k] = 0;
    __syncthreads();
    const int i = bid * 256 + threadIdx.x;
    double qs = 0.0, q2 = 0.0;
    if (i < a.n) {
        uint32_t u[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = to_fixed((double)xyz[3 * i + k], a.inv_box[k]);
        const float qi = q[i];
        const int c = cell_coord(u[1], a.nc[1]) * a.nc[0] + cell_coord(u[0], a.nc[0]);
        coord[i] = make_uint4(u[0], u[1], u[2], __float_as_uint(qi));
        if (local) atomicAdd(&hist[c], 1);
        else atomicAdd(&col_count[c], 1);
        qs = qi;
        q2 = (double)qi * (double)qi;
    }
    __syncthreads();
    if (local)
        for (int k = threadIdx.x; k < ncol; k += 256)
            if (hist[k] > 0) atomicAdd(&col_count[k], hist[k]);
    // charge sums: wavefront sums, then the 4 wavefront sums in order
    qs = wave_sum_d(qs);
    q2 = wave_sum_d(q2);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = qs;
        red[1][wv] = q2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        qpart[2 * bid] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        qpart[2 * bid + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

__global__ void __launch_bounds__(256) k_encode(const float* __restrict__ xyz,
                                                const float* __restrict__ q,
                                                uint4* __restrict__ coord,
                                                int* __restrict__ col_count,
                                                double* __restrict__ qpart, BinArgs a) {
    encode_body(a, blockIdx.x, xyz, q, coord, col_count, qpart);
}

__global__ void __launch_bounds__(256) k_encode_batch(const BatchTable* __restrict__ tab,
                                                      const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_ENCODE, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        encode_body(d.bin, item, d.xyz, d.q, d.coord, d.col_count, d.qpart);
    });
}

// One block of 1024 threads: exclusive scans of the column counts and of the
// cluster counts ceil(count / 8) (each thread owns a contiguous chunk;
// wavefront scans by DPP lane moves, then a scan of the 16 wavefront totals), zero
// the fill counters, and reduce the charge partials in a fixed order.  The
// column counts are cleared once read, ready for the next evaluation (they
// start at zero when the workspace is allocated).
__device__ __forceinline__ void scan_body(int ncol, int* __restrict__ count,
                                          int* __restrict__ start, int* __restrict__ cstart,
                                          int* __restrict__ fill,
                                          const double* __restrict__ qpart, int nqpart,
                                          double* __restrict__ qstats) {
    __shared__ int wsum[2][16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int chunk = (ncol + 1023) / 1024;
    const int lo = min(t * chunk, ncol), hi = min(lo + chunk, ncol);
    int s = 0, sc = 0;
    for (int c = lo; c < hi; ++c) {
        const int k = count[c];
        s += k;
        sc += (k + 7) >> 3;
    }
    const int v = wave_incl_scan(s), vc = wave_incl_scan(sc);
    if (lane == 63) {
        wsum[0][wv] = v;
        wsum[1][wv] = vc;
    }
    __syncthreads();
    if (wv == 0) {
        const int own = lane < 16 ? wsum[0][lane] : 0, ownc = lane < 16 ? wsum[1][lane] : 0;
        const int x = wave_incl_scan(own), xc = wave_incl_scan(ownc);
        if (lane < 16) {
            wsum[0][lane] = x - own;
            wsum[1][lane] = xc - ownc;
        }
    }
    __syncthreads();
    int run = wsum[0][wv] + v - s, runc = wsum[1][wv] + vc - sc;   // exclusive prefixes
    for (int c = lo; c < hi; ++c) {
        const int k = count[c];
        start[c] = run;
        cstart[c] = runc;
        run += k;
        runc += (k + 7) >> 3;
        fill[c] = 0;
        count[c] = 0;
    }
    if (t == 1023) {
        start[ncol] = run;
        cstart[ncol] = runc;
    }
    if (wv == 1) {
        double qa = 0.0, qb = 0.0;
        for (int k = lane; k < nqpart; k += 64) {
            qa += qpart[2 * k];
            qb += qpart[2 * k + 1];
        }
        qa = wave_sum_d(qa);
        qb = wave_sum_d(qb);
        if (lane == 0) {
            qstats[0] = qa;
            qstats[1] = qb;
        }
    }
}

__global__ void __launch_bounds__(1024) k_scan(int ncol, int* __restrict__ count,
                                               int* __restrict__ start, int* __restrict__ cstart,
                                               int* __restrict__ fill,
                                               const double* __restrict__ qpart, int nqpart,
                                               double* __restrict__ qstats) {
    scan_body(ncol, count, start, cstart, fill, qpart, nqpart, qstats);
}

__global__ void __launch_bounds__(1024) k_scan_batch(const BatchTable* __restrict__ tab,
                                                     const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_SCAN, [&](int i, int) {
        const BoxDesc& d = desc[tab->slot[i]];
        scan_body(d.ncol, d.col_count, d.col_start, d.clus_start, d.col_fill, d.qpart, d.nq,
                  d.qstats);
    });
}

// Slots inside a column: the rank among the block's charges of that column
// (LDS atomic) plus a base reserved once per (block, column).  The order they
// produce is arbitrary; colsort makes it deterministic.  Each slot gets the
// charge's input index and its encoded record (the record into `sorted`,
// which colsort then reorders within the column).  With `fused`, the
// block first takes the exclusive prefix sums of the column counts (256
// threads, a contiguous run of at most kHistCols / 256 columns each) as its
// column starts; block 0 also writes them, the cluster starts and the charge
// sums, in place of the scan kernel.
constexpr int kPrefixRun = kHistCols / 256;

__device__ __forceinline__ void scatter_body(const BinArgs& a, int bid, bool fused,
                                             const uint4* __restrict__ coord,
                                             uint4* __restrict__ sorted,
                                             const int* __restrict__ count,
                                             int* __restrict__ start, int* __restrict__ cstart,
                                             int* __restrict__ fill, int* __restrict__ slots,
                                             const double* __restrict__ qpart, int nqpart,
                                             double* __restrict__ qstats) {
    __shared__ int hist[kHistCols];
    __shared__ int base[kHistCols];
    __shared__ int wsum[2][4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int n = a.n, ncol = a.nc[0] * a.nc[1];
    const bool local = ncol <= kHistCols;
    if (local)
        for (int k = t; k < ncol; k += 256) hist[k] = 0;
    const int i = bid * 256 + t;
    const uint4 rec = i < n ? coord[i] : make_uint4(0, 0, 0, 0);
    const int c = cell_coord(rec.y, a.nc[1]) * a.nc[0] + cell_coord(rec.x, a.nc[0]);
    if (fused) {
        const int run_len = (ncol + 255) / 256;
        const int lo = min(t * run_len, ncol), hi = min(lo + run_len, ncol);
        int kc[kPrefixRun];
        int s = 0, sc = 0;
#pragma unroll
        for (int u = 0; u < kPrefixRun; ++u) kc[u] = lo + u < hi ? count[lo + u] : 0;
#pragma unroll
        for (int u = 0; u < kPrefixRun; ++u) {
            s += kc[u];
            sc += (kc[u] + 7) >> 3;
        }
        const int v = wave_incl_scan(s), vc = wave_incl_scan(sc);
        if (lane == 63) {
            wsum[0][wv] = v;
            wsum[1][wv] = vc;
        }
        __syncthreads();
        int run = v - s, runc = vc - sc;   // exclusive prefixes
        for (int u = 0; u < wv; ++u) {
            run += wsum[0][u];
            runc += wsum[1][u];
        }
#pragma unroll
        for (int u = 0; u < kPrefixRun; ++u) {
            if (lo + u < hi) {
                base[lo + u] = run;
                if (bid == 0) {
                    start[lo + u] = run;
                    cstart[lo + u] = runc;
                }
                run += kc[u];
                runc += (kc[u] + 7) >> 3;
            }
        }
        if (bid == 0 && t == 255) {
            start[ncol] = run;
            cstart[ncol] = runc;
        }
        if (bid == 0 && wv == 1) {
            double qa = 0.0, qb = 0.0;
            for (int k = lane; k < nqpart; k += 64) {
                qa += qpart[2 * k];
                qb += qpart[2 * k + 1];
            }
            qa = wave_sum_d(qa);
            qb = wave_sum_d(qb);
            if (lane == 0) {
                qstats[0] = qa;
                qstats[1] = qb;
            }
        }
    }
    __syncthreads();
    int r = 0;
    if (i < n) r = local ? atomicAdd(&hist[c], 1) : atomicAdd(&fill[c], 1);
    __syncthreads();
    if (local)
        for (int k = t; k < ncol; k += 256)
            if (hist[k] > 0) base[k] = (fused ? base[k] : start[k]) + atomicAdd(&fill[k], hist[k]);
    __syncthreads();
    if (i < n) {
        const int slot = (local ? base[c] : start[c]) + r;
        slots[slot] = i;
        sorted[slot] = rec;
    }
}

__global__ void __launch_bounds__(256) k_scatter(int fused, int nqpart,
                                                 const uint4* __restrict__ coord,
                                                 const int* __restrict__ count,
                                                 uint4* __restrict__ sorted,
                                                 int* __restrict__ start, int* __restrict__ cstart,
                                                 int* __restrict__ fill, int* __restrict__ slots,
                                                 const double* __restrict__ qpart,
                                                 double* __restrict__ qstats, BinArgs a) {
    scatter_body(a, blockIdx.x, fused != 0, coord, sorted, count, start, cstart, fill, slots,
                 qpart, nqpart, qstats);
}

__global__ void __launch_bounds__(256) k_scatter_batch(const BatchTable* __restrict__ tab,
                                                       const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_SCATTER, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        scatter_body(d.bin, item, false, d.coord, d.sorted, d.col_count, d.col_start,
                     d.clus_start, d.col_fill, d.slots, d.qpart, d.nq, d.qstats);
    });
}

// One block per column: sort the column's charges by the key (z, input
// index) -- unique, so the order is deterministic: up to 256 charges by
// counting each key's rank in LDS, up to kSortCap by a bitonic sort in LDS,
// beyond by ranking from global memory -- then write the permutation, the
// sorted positions, the column's clusters and its z-plane index.
constexpr int kSortCap = 1024;

__device__ __forceinline__ void colsort_body(int col, const int* __restrict__ start,
                                             const int* __restrict__ cstart,
                                             const int* __restrict__ slots,
                                             const uint4* __restrict__ coord,
                                             int* __restrict__ perm, uint4* __restrict__ sorted,
                                             int2* __restrict__ cl_info, int* __restrict__ cl_col,
                                             int ncx,
                                             uint2* __restrict__ cl_z, int gz,
                                             int* __restrict__ zbin, int* __restrict__ count,
                                             int* __restrict__ fill, int ncol, int npb) {
    __shared__ unsigned long long key[kSortCap];
    __shared__ uint32_t skz[kSortCap];         // z of the sorted charges
    const int t = threadIdx.x;
    const int lo = start[col], cnt = start[col + 1] - lo;
    if (t == 0) {   // the column's counters, cleared for the next evaluation
        count[col] = 0;
        fill[col] = 0;
    }
    if (col == ncol - 1)   // cluster numbers past the last cluster: no charges
        for (int k = cstart[ncol] + t; k < npb; k += 256) cl_info[k] = make_int2(start[ncol], 0);
    int* zrow = zbin + (size_t)col * (gz + 1);
    if (cnt == 0) {
        for (int b = t; b <= gz; b += 256) zrow[b] = lo;
        return;
    }
    if (cnt <= 256) {
        // one charge per thread, its rank counted against every key
        unsigned long long mine = ~0ull;
        uint4 c = make_uint4(0, 0, 0, 0);
        int i = 0;
        if (t < cnt) {   // the column's records as scatter left them (read before any write)
            i = slots[lo + t];
            c = sorted[lo + t];
            mine = ((unsigned long long)c.z << 32) | (unsigned)i;
            key[t] = mine;
        }
        __syncthreads();
        if (t < cnt) {
            // four independent counts, so that consecutive comparisons do not
            // wait on each other's sums (one wavefront per SIMD here)
            int r0 = 0, r1 = 0, r2 = 0, r3 = 0, m = 0;
#pragma unroll 4
            for (; m + 4 <= cnt; m += 4) {
                r0 += key[m] < mine;
                r1 += key[m + 1] < mine;
                r2 += key[m + 2] < mine;
                r3 += key[m + 3] < mine;
            }
            for (; m < cnt; ++m) r0 += key[m] < mine;
            const int r = (r0 + r1) + (r2 + r3);
            perm[lo + r] = i;
            sorted[lo + r] = c;
            skz[r] = c.z;
        }
    } else if (cnt <= kSortCap) {
        int m = 1;
        while (m < cnt) m <<= 1;
        for (int k = t; k < m; k += 256) {
            if (k < cnt) {
                const int i = slots[lo + k];
                key[k] = ((unsigned long long)coord[i].z << 32) | (unsigned)i;
            } else {
                key[k] = ~0ull;
            }
        }
        __syncthreads();
        for (int size = 2; size <= m; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = t; k < m; k += 256) {
                    const int o = k ^ stride;
                    if (o > k) {
                        const bool up = (k & size) == 0;
                        const unsigned long long x = key[k], y = key[o];
                        if ((x > y) == up) {
                            key[k] = y;
                            key[o] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int k = t; k < cnt; k += 256) {
            const int i = (int)(unsigned)(key[k] & 0xffffffffull);
            perm[lo + k] = i;
            sorted[lo + k] = coord[i];
            skz[k] = (uint32_t)(key[k] >> 32);
        }
    } else {
        // rank by counting (O(cnt^2) work spread over the block)
        for (int k = t; k < cnt; k += 256) {
            const int i = slots[lo + k];
            const unsigned long long ki = ((unsigned long long)coord[i].z << 32) | (unsigned)i;
            int rank = 0;
            for (int m = 0; m < cnt; ++m) {
                const int j = slots[lo + m];
                rank += (((unsigned long long)coord[j].z << 32) | (unsigned)j) < ki;
            }
            perm[lo + rank] = i;
            sorted[lo + rank] = coord[i];
        }
    }
    __syncthreads();
    const bool in_lds = cnt <= kSortCap;
    // z-plane index of the column: zrow[b] = first charge whose grid z index
    // is >= b (b = 0 .. gz), for the spreading and gathering windows
    for (int b = t; b <= gz; b += 256) {
        int l = 0, h = cnt;
        while (l < h) {
            const int mid = (l + h) >> 1;
            const uint32_t z = in_lds ? skz[mid] : sorted[lo + mid].z;
            if (cell_coord(z, gz) < b) l = mid + 1; else h = mid;
        }
        zrow[b] = lo + l;
    }
    // clusters: 8 consecutive charges of the column (the last may be short);
    // the column is stored as its coordinates cx | cy << 16
    const int c0 = cstart[col], nclus = (cnt + 7) >> 3;
    const int cyx = (col % ncx) | ((col / ncx) << 16);
    for (int k = t; k < nclus; k += 256) {
        const int b = lo + 8 * k;
        const int nk = min(8, cnt - 8 * k);
        cl_info[c0 + k] = make_int2(b, nk);
        cl_col[c0 + k] = cyx;
        cl_z[c0 + k] = in_lds ? make_uint2(skz[8 * k], skz[8 * k + nk - 1])
                              : make_uint2(sorted[b].z, sorted[b + nk - 1].z);
    }
}

__global__ void __launch_bounds__(256) k_colsort(const int* __restrict__ start,
                                                 const int* __restrict__ cstart,
                                                 const int* __restrict__ slots,
                                                 const uint4* __restrict__ coord,
                                                 int* __restrict__ perm,
                                                 uint4* __restrict__ sorted,
                                                 int2* __restrict__ cl_info,
                                                 int* __restrict__ cl_col, int ncx,
                                                 uint2* __restrict__ cl_z, int gz,
                                                 int* __restrict__ zbin, int* __restrict__ count,
                                                 int* __restrict__ fill, int npb) {
    colsort_body(blockIdx.x, start, cstart, slots, coord, perm, sorted, cl_info, cl_col, ncx, cl_z, gz,
                 zbin, count, fill, (int)gridDim.x, npb);
}

__global__ void __launch_bounds__(256) k_colsort_batch(const BatchTable* __restrict__ tab,
                                                       const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_COLSORT, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        colsort_body(item, d.col_start, d.clus_start, d.slots, d.coord, d.perm, d.sorted,
                     d.cl_info, d.cl_col, d.bin.nc[0], d.cl_z, d.grid.g[2], d.zbin, d.col_count,
                     d.col_fill, d.ncol, d.npb);
    });
}

// ------------------------------------------------------------ two-launch binning
constexpr int kLocalBlocks = 4096;   // bin_local blocks whose prefixes colbuild reads
constexpr int kLocalRun = kLocalBlocks / 256;

bool bin_local_ok(int n, int ncol) {
    const long long nb = ((long long)n + 255) / 256;
    return n > 0 && ncol <= kHistCols && nb <= kLocalBlocks && nb * (ncol + 1) <= (1ll << 22);
}

// Block b: the records (fixed-point position and charge bits) of charges
// 256 b .. 256 b + 255, grouped by column into coord[256 b ...] with their
// input indices in slots[...] (order within a column as the LDS atomics
// leave it), the block's exclusive column prefix in bpre[b][0 .. ncol]
// (bpre[b][ncol]: its charge count) and its charge sums in qpart.
__device__ __forceinline__ void bin_local_body(const BinArgs& a, int b, const float* __restrict__ xyz,
                                               const float* __restrict__ q,
                                               uint4* __restrict__ coord,
                                               int* __restrict__ slots, int* __restrict__ bpre,
                                               double* __restrict__ qpart) {
    __shared__ int hist[kHistCols];
    __shared__ int wsum[4];
    __shared__ double red[2][4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int ncol = a.nc[0] * a.nc[1];
    for (int k = t; k < ncol; k += 256) hist[k] = 0;
    __syncthreads();
    const int i = b * 256 + t;
    uint4 rec = make_uint4(0, 0, 0, 0);
    int c = 0, r = 0;
    double qs = 0.0, q2 = 0.0;
    if (i < a.n) {
        uint32_t u[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = to_fixed((double)xyz[3 * i + k], a.inv_box[k]);
        const float qi = q[i];
        c = cell_coord(u[1], a.nc[1]) * a.nc[0] + cell_coord(u[0], a.nc[0]);
        rec = make_uint4(u[0], u[1], u[2], __float_as_uint(qi));
        r = atomicAdd(&hist[c], 1);   // rank within the block's charges of column c
        qs = qi;
        q2 = (double)qi * (double)qi;
    }
    __syncthreads();
    // exclusive prefix of the block's column counts: thread t owns the run of
    // columns [t run, t run + run), run = ceil(ncol / 256) <= kPrefixRun
    const int run = (ncol + 255) / 256;
    const int lo = min(t * run, ncol), hi = min(lo + run, ncol);
    int kc[kPrefixRun];
    int s = 0;
#pragma unroll
    for (int u = 0; u < kPrefixRun; ++u) {
        kc[u] = lo + u < hi ? hist[lo + u] : 0;
        s += kc[u];
    }
    const int v = wave_incl_scan(s);
    if (lane == 63) wsum[wv] = v;
    __syncthreads();   // every count read before it is replaced by its prefix
    int pre = v - s;
    for (int u = 0; u < wv; ++u) pre += wsum[u];
    int* row = bpre + (size_t)b * (ncol + 1);
#pragma unroll
    for (int u = 0; u < kPrefixRun; ++u) {
        if (lo + u < hi) {
            hist[lo + u] = pre;
            row[lo + u] = pre;
            pre += kc[u];
        }
    }
    if (t == 255) row[ncol] = pre;   // the last run ends at ncol: pre is the block's total
    __syncthreads();
    if (i < a.n) {
        const int slot = b * 256 + hist[c] + r;
        coord[slot] = rec;
        slots[slot] = i;
    }
    // charge sums: wavefront sums, then the 4 wavefront sums in order
    qs = wave_sum_d(qs);
    q2 = wave_sum_d(q2);
    if (lane == 0) {
        red[0][wv] = qs;
        red[1][wv] = q2;
    }
    __syncthreads();
    if (t == 0) {
        qpart[2 * b] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        qpart[2 * b + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// Block c (column c): from P[b][c] and P[b][c + 1] of the nb bin_local blocks,
// the column's first sorted position lo = sum_b P[b][c], its count and the
// offset of each block's segment in the column's list; then its charges
// gathered (list position k lies in the segment b with segoff[b] <= k <
// segoff[b + 1]), sorted by (z, input index) -- up to 256 by counting ranks,
// up to kSortCap by a bitonic sort in LDS, beyond by ranking from global
// memory -- and written with the column's z-plane index and clusters.
// reduce_q: this block also reduces the charge sums (qstats_reduce).
__device__ __forceinline__ void qstats_reduce(int nb, const double* __restrict__ qpart,
                                              double* __restrict__ qstats) {
    const int lane = threadIdx.x & 63;
    double qa = 0.0, qb = 0.0;
    for (int k = lane; k < nb; k += 64) {
        qa += qpart[2 * k];
        qb += qpart[2 * k + 1];
    }
    qa = wave_sum_d(qa);
    qb = wave_sum_d(qb);
    if (lane == 0) {
        qstats[0] = qa;
        qstats[1] = qb;
    }
}

__device__ __forceinline__ void colbuild_body(int col, int nb, int ncol, int ncx, int gz, int npb,
                                              bool reduce_q,
                                              const int* __restrict__ bpre,
                                              const uint4* __restrict__ coord,
                                              const int* __restrict__ slots,
                                              int* __restrict__ perm, uint4* __restrict__ sorted,
                                              int2* __restrict__ cl_info, int* __restrict__ cl_col,
                                              uint2* __restrict__ cl_z, int* __restrict__ zbin,
                                              const double* __restrict__ qpart,
                                              double* __restrict__ qstats) {
    __shared__ int segoff[kLocalBlocks + 1];
    __shared__ int segbase[kLocalBlocks];      // slot of list position k: segbase[b] + k
    __shared__ unsigned long long key[kSortCap];
    __shared__ int pay[kSortCap];              // list position carried through the sort
    __shared__ uint4 lrec[kSortCap];
    __shared__ int lidx[kSortCap];
    __shared__ uint32_t skz[kSortCap];         // z of the sorted charges
    __shared__ int wsum[2][4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int stride = ncol + 1;

    // segment counts h_b = P[b][c + 1] - P[b][c] over a contiguous run of b
    // per thread; their exclusive scan (segment offsets) and the sum of P[b][c]
    const int run = (nb + 255) / 256;
    const int blo = min(t * run, nb), bhi = min(blo + run, nb);
    int h[kLocalRun], pc[kLocalRun];
    int s = 0, ps = 0;
#pragma unroll
    for (int u = 0; u < kLocalRun; ++u) {
        h[u] = pc[u] = 0;
        if (blo + u < bhi) {
            const int* rowp = bpre + (size_t)(blo + u) * stride + col;
            pc[u] = rowp[0];
            h[u] = rowp[1] - pc[u];
        }
        s += h[u];
        ps += pc[u];
    }
    const int v = wave_incl_scan(s), vp = wave_incl_scan(ps);
    if (lane == 63) {
        wsum[0][wv] = v;
        wsum[1][wv] = vp;
    }
    __syncthreads();
    int off = v - s;
    for (int u = 0; u < wv; ++u) off += wsum[0][u];
    const int cnt = ((wsum[0][0] + wsum[0][1]) + wsum[0][2]) + wsum[0][3];
    const int lo = ((wsum[1][0] + wsum[1][1]) + wsum[1][2]) + wsum[1][3];
#pragma unroll
    for (int u = 0; u < kLocalRun; ++u) {
        if (blo + u < bhi) {
            segoff[blo + u] = off;
            segbase[blo + u] = (blo + u) * 256 + pc[u] - off;
            off += h[u];
        }
    }
    if (t == 0) segoff[nb] = cnt;
    if (reduce_q && wv == 1) qstats_reduce(nb, qpart, qstats);

    // cluster numbers: this column's from floor(lo / 8) + col, the next
    // column's from floor((lo + cnt) / 8) + col + 1 (the last column's run to
    // npb); those between its clusters and the next column's hold no charge
    const int c0 = lo / 8 + col, nclus = (cnt + 7) >> 3;
    const int cend = col == ncol - 1 ? npb : (lo + cnt) / 8 + col + 1;
    for (int k = c0 + nclus + t; k < cend; k += 256) cl_info[k] = make_int2(lo + cnt, 0);
    int* zrow = zbin + (size_t)col * (gz + 1);
    if (cnt == 0) {
        for (int k = t; k <= gz; k += 256) zrow[k] = lo;
        return;
    }
    __syncthreads();
    // the slot of list position k
    auto slot_of = [&](int k) {
        int l = 0, hh = nb;                  // last b with segoff[b] <= k
        while (hh - l > 1) {
            const int mid = (l + hh) >> 1;
            if (segoff[mid] <= k) l = mid; else hh = mid;
        }
        return segbase[l] + k;
    };
    if (cnt <= 256) {
        // one charge per thread, its rank counted against every key
        unsigned long long mine = ~0ull;
        uint4 c = make_uint4(0, 0, 0, 0);
        int i = 0;
        if (t < cnt) {
            const int sl = slot_of(t);
            c = coord[sl];
            i = slots[sl];
            mine = ((unsigned long long)c.z << 32) | (unsigned)i;
            key[t] = mine;
        }
        __syncthreads();
        if (t < cnt) {
            int r0 = 0, r1 = 0, r2 = 0, r3 = 0, m = 0;
#pragma unroll 4
            for (; m + 4 <= cnt; m += 4) {
                r0 += key[m] < mine;
                r1 += key[m + 1] < mine;
                r2 += key[m + 2] < mine;
                r3 += key[m + 3] < mine;
            }
            for (; m < cnt; ++m) r0 += key[m] < mine;
            const int r = (r0 + r1) + (r2 + r3);
            perm[lo + r] = i;
            sorted[lo + r] = c;
            skz[r] = c.z;
        }
    } else if (cnt <= kSortCap) {
        int m = 1;
        while (m < cnt) m <<= 1;
        for (int k = t; k < m; k += 256) {
            if (k < cnt) {
                const int sl = slot_of(k);
                const uint4 c = coord[sl];
                const int i = slots[sl];
                lrec[k] = c;
                lidx[k] = i;
                key[k] = ((unsigned long long)c.z << 32) | (unsigned)i;
            } else {
                key[k] = ~0ull;
            }
            pay[k] = k;
        }
        __syncthreads();
        for (int size = 2; size <= m; size <<= 1) {
            for (int stride2 = size >> 1; stride2 > 0; stride2 >>= 1) {
                for (int k = t; k < m; k += 256) {
                    const int o = k ^ stride2;
                    if (o > k) {
                        const bool up = (k & size) == 0;
                        const unsigned long long x = key[k], y = key[o];
                        if ((x > y) == up) {
                            key[k] = y;
                            key[o] = x;
                            const int pk = pay[k];
                            pay[k] = pay[o];
                            pay[o] = pk;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int k = t; k < cnt; k += 256) {
            const int p = pay[k];
            perm[lo + k] = lidx[p];
            sorted[lo + k] = lrec[p];
            skz[k] = (uint32_t)(key[k] >> 32);
        }
    } else {
        // rank by counting over the column's segments (O(cnt^2) global reads)
        for (int k = t; k < cnt; k += 256) {
            const int sl = slot_of(k);
            const uint4 c = coord[sl];
            const int i = slots[sl];
            const unsigned long long ki = ((unsigned long long)c.z << 32) | (unsigned)i;
            int rank = 0;
            for (int bb = 0; bb < nb; ++bb) {
                const int e = segoff[bb + 1] - segoff[bb];
                for (int j = 0; j < e; ++j) {
                    const int sj = segbase[bb] + segoff[bb] + j;
                    rank += (((unsigned long long)coord[sj].z << 32) | (unsigned)slots[sj]) < ki;
                }
            }
            perm[lo + rank] = i;
            sorted[lo + rank] = c;
        }
    }
    __syncthreads();
    const bool in_lds = cnt <= kSortCap;
    // z-plane index: zrow[z] = first charge whose grid z index is >= z.  From
    // the LDS copy, sorted charge k writes the planes after its predecessor's
    // grid z index up to its own (the last charge also those up to gz);
    // otherwise a search per plane
    if (in_lds) {
        for (int k = t; k < cnt; k += 256) {
            const int zk = cell_coord(skz[k], gz);
            const int zp = k > 0 ? cell_coord(skz[k - 1], gz) : -1;
            for (int z = zp + 1; z <= zk; ++z) zrow[z] = lo + k;
            if (k == cnt - 1)
                for (int z = zk + 1; z <= gz; ++z) zrow[z] = lo + cnt;
        }
    } else {
        for (int z = t; z <= gz; z += 256) {
            int l = 0, hh = cnt;
            while (l < hh) {
                const int mid = (l + hh) >> 1;
                if (cell_coord(sorted[lo + mid].z, gz) < z) l = mid + 1; else hh = mid;
            }
            zrow[z] = lo + l;
        }
    }
    const int cyx = (col % ncx) | ((col / ncx) << 16);
    for (int k = t; k < nclus; k += 256) {
        const int b0 = lo + 8 * k;
        const int nk = min(8, cnt - 8 * k);
        cl_info[c0 + k] = make_int2(b0, nk);
        cl_col[c0 + k] = cyx;
        cl_z[c0 + k] = in_lds ? make_uint2(skz[8 * k], skz[8 * k + nk - 1])
                              : make_uint2(sorted[b0].z, sorted[b0 + nk - 1].z);
    }
}

__global__ void __launch_bounds__(256) k_bin_local(const float* __restrict__ xyz,
                                                   const float* __restrict__ q,
                                                   uint4* __restrict__ coord,
                                                   int* __restrict__ slots,
                                                   int* __restrict__ bpre,
                                                   double* __restrict__ qpart, BinArgs a) {
    bin_local_body(a, blockIdx.x, xyz, q, coord, slots, bpre, qpart);
}

__global__ void __launch_bounds__(256) k_colbuild(int nb, int ncol, int ncx, int gz, int npb,
                                                  const int* __restrict__ bpre,
                                                  const uint4* __restrict__ coord,
                                                  const int* __restrict__ slots,
                                                  int* __restrict__ perm,
                                                  uint4* __restrict__ sorted,
                                                  int2* __restrict__ cl_info,
                                                  int* __restrict__ cl_col,
                                                  uint2* __restrict__ cl_z,
                                                  int* __restrict__ zbin,
                                                  const double* __restrict__ qpart,
                                                  double* __restrict__ qstats) {
    // block ncol (one past the columns) reduces the charge sums, beside the columns
    if (blockIdx.x == ncol) {
        if (threadIdx.x < 64) qstats_reduce(nb, qpart, qstats);
        return;
    }
    colbuild_body(blockIdx.x, nb, ncol, ncx, gz, npb, false, bpre, coord, slots, perm, sorted,
                  cl_info, cl_col, cl_z, zbin, qpart, qstats);
}

__global__ void __launch_bounds__(256) k_bin_local_batch(const BatchTable* __restrict__ tab,
                                                         const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_BINLOCAL, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        bin_local_body(d.bin, item, d.xyz, d.q, d.coord, d.slots, d.bpre, d.qpart);
    });
}

__global__ void __launch_bounds__(256) k_colbuild_batch(const BatchTable* __restrict__ tab,
                                                        const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_COLBUILD, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        colbuild_body(item, d.nq, d.ncol, d.bin.nc[0], d.grid.g[2], d.npb, item == 0, d.bpre,
                      d.coord, d.slots, d.perm, d.sorted, d.cl_info, d.cl_col, d.cl_z, d.zbin,
                      d.qpart, d.qstats);
    });
}

hipError_t launch_bin_local_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_bin_local_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_colbuild_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_colbuild_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_bin_local(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                            int* slots, int* bpre, double* qpart, hipStream_t st) {
    const int nb = (a.n + 255) / 256;
    if (nb > 0)
        hipLaunchKernelGGL(k_bin_local, dim3(nb), dim3(256), 0, st, xyz, q, coord, slots, bpre,
                           qpart, a);
    return hipGetLastError();
}

hipError_t launch_colbuild(int n, int ncol, int ncx, int gz, int npb, const int* bpre,
                           const uint4* coord, const int* slots, int* perm, uint4* sorted,
                           int2* cl_info, int* cl_col, uint2* cl_z, int* zbin,
                           const double* qpart, double* qstats, hipStream_t st) {
    const int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_colbuild, dim3(ncol + 1), dim3(256), 0, st, nb, ncol, ncx, gz, npb, bpre,
                       coord, slots, perm, sorted, cl_info, cl_col, cl_z, zbin, qpart, qstats);
    return hipGetLastError();
}

hipError_t launch_encode(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                         int* col_count, double* qpart, int nqpart, hipStream_t st) {
    if (a.n > 0)
        hipLaunchKernelGGL(k_encode, dim3(nqpart), dim3(256), 0, st, xyz, q, coord, col_count,
                           qpart, a);
    return hipGetLastError();
}

hipError_t launch_scan(int ncol, int* col_count, int* col_start, int* clus_start,
                       int* col_fill, const double* qpart, int nqpart, double* qstats,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, ncol, col_count, col_start, clus_start,
                       col_fill, qpart, nqpart, qstats);
    return hipGetLastError();
}

bool scan_fused(int n, int ncol) {
    const long long nb = (n + 255) / 256;
    return ncol <= kHistCols && nb * ncol <= (1ll << 22);
}

hipError_t launch_scatter(const BinArgs& a, const uint4* coord, uint4* sorted, const int* col_count,
                          int* col_start, int* clus_start, int* col_fill, int* slots,
                          const double* qpart, int nqpart, double* qstats, hipStream_t st) {
    const int n = a.n, ncol = a.nc[0] * a.nc[1];
    const int fused = scan_fused(n, ncol) ? 1 : 0;
    // with no charges the fused prefix still has to run once (all columns empty)
    const int nb = std::max(1, (n + 255) / 256);
    if (n > 0 || fused)
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, st, fused, nqpart, coord, col_count,
                           sorted, col_start, clus_start, col_fill, slots, qpart, qstats, a);
    return hipGetLastError();
}

hipError_t launch_colsort(int ncol, int ncx, const int* col_start, const int* clus_start,
                          const int* slots, const uint4* coord, int* perm, uint4* sorted,
                          int2* cl_info, int* cl_col, uint2* cl_z, int gz, int* zbin,
                          int* col_count, int* col_fill, int npb, hipStream_t st) {
    hipLaunchKernelGGL(k_colsort, dim3(ncol), dim3(256), 0, st, col_start, clus_start, slots,
                       coord, perm, sorted, cl_info, cl_col, ncx, cl_z, gz, zbin, col_count,
                       col_fill, npb);
    return hipGetLastError();
}

hipError_t launch_encode_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_encode_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_scan_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_batch, dim3(grid), dim3(1024), 0, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_scatter_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_colsort_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_colsort_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

}  // namespace useries
