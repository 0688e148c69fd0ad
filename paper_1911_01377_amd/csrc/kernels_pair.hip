// Near part of the u-series (eq. 20): for every pair closer than r_c,
//   energy  q_i q_j (1/r - F(r)),
//   force   q_i q_j (1/r^3 + F'(r)/r) (r_i - r_j)  on charge i,
// where F is the infinite far series (eq. 24), represented inside the cutoff
// by a polynomial in x = r^2/r_c^2 fitted on the host in FP64.
//
// Layout: cluster-pair tiles.  Charges are binned into x-y columns, sorted
// by z, and cut into clusters of up to 8 (see kernels_bin.hip).  One
// wavefront takes one i-cluster: lane (a, b) = (lane / 8, lane % 8) holds
// i-charge a and, at each step, j-charge b of the current j-cluster, so every
// lane evaluates one pair per step and no lane waits on another's branch.
// The j-clusters are those of the columns within r_c of the i-column (x-y
// gap) whose z extent meets the i-cluster's z extent widened by the z reach
// sqrt(r_c^2 - gap^2): a contiguous range per column, found by binary search
// on the z-sorted clusters.  The candidate j-charges are staged in LDS in
// chunks with coalesced loads.  The force on charge a is summed over its 8
// lanes by shuffles at the end.
//
// Each ordered pair (i, j) is evaluated once, by i's wavefront (no
// Newton's-third-law sharing), so forces need no atomics and the result does
// not depend on scheduling.
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

namespace {

constexpr int kChunk = 32;            // staged j-clusters per pass (4 KB of LDS)

// Polynomial coefficients held in registers (compile-time degree, fully
// unrolled): F = c0 + x P(x) with c0 carried as hi + lo, and G = F'(r)/r,
// each fitted separately in FP64 on the host.
template <int DEG>
struct Poly {
    float c[DEG + 1];
    float c0lo;
    float d[DEG + 1];
    __device__ __forceinline__ explicit Poly(const PairArgs& a) {
#pragma unroll
        for (int m = 0; m <= DEG; ++m) {
            c[m] = a.c[m];
            d[m] = a.d[m];
        }
        c0lo = a.c0lo;
    }
};

// column k of an axis window around the i-column ci and its minimum-image
// distance (in columns) to ci; a full axis (few columns) is walked once
__device__ __forceinline__ void stencil_col(int k, int ci, int R, int nc, bool full, int* col,
                                            int* d) {
    if (full) {
        *col = k;
        int v = k - ci;
        if (2 * v > nc) v -= nc;
        if (2 * v < -nc) v += nc;
        *d = v;
    } else {
        *d = k - R;
        *col = wrapi(ci + k - R, nc);
    }
}

}  // namespace

template <int DEG>
__device__ __forceinline__ void pair_body(const PairArgs& a, int I, const uint4* __restrict__ sorted,
                                          const int* __restrict__ clus_start,
                                          const int2* __restrict__ cl_info,
                                          const int* __restrict__ cl_col,
                                          const uint2* __restrict__ cl_z,
                                          float4* __restrict__ fnear,
                                          double* __restrict__ epart) {
    __shared__ uint4 stage[kChunk * 8];
    __shared__ int rbeg[2 * kMaxStencilCols];
    __shared__ int roff[2 * kMaxStencilCols + 1];
    const int lane = threadIdx.x, ia = lane >> 3, ja = lane & 7;
    const int ncx = a.nc[0], ncy = a.nc[1];
    if (I >= clus_start[ncx * ncy]) {
        if (lane == 0) epart[I] = 0.0;
        return;
    }
    const Poly<DEG> P(a);
    const int2 ii = cl_info[I];
    const int C = cl_col[I];
    const uint2 zI = cl_z[I];
    const int cx = C % ncx, cy = C / ncx;
    const bool fullx = 2 * a.R[0] + 1 >= ncx, fully = 2 * a.R[1] + 1 >= ncy;
    const int nxs = fullx ? ncx : 2 * a.R[0] + 1, nys = fully ? ncy : 2 * a.R[1] + 1;
    const int NC = nxs * nys;

    // candidate j-cluster ranges, two slots per stencil column
    for (int k = lane; k < NC; k += 64) {
        int colx, coly, dx, dy;
        stencil_col(k % nxs, cx, a.R[0], ncx, fullx, &colx, &dx);
        stencil_col(k / nxs, cy, a.R[1], ncy, fully, &coly, &dy);
        const float gx = (float)max(0, abs(dx) - 1) * a.cw[0];
        const float gy = (float)max(0, abs(dy) - 1) * a.cw[1];
        const float d2 = gx * gx + gy * gy;
        int b0 = 0, l0 = 0, b1 = 0, l1 = 0;
        if (d2 < a.rc2) {
            const long long rz = (long long)(sqrtf(a.rc2 - d2) * a.zinv) + 2;
            const int col = coly * ncx + colx;
            column_zrange(cl_z, clus_start[col], clus_start[col + 1], (long long)zI.x - rz,
                          (long long)zI.y + rz, &b0, &l0, &b1, &l1);
        }
        rbeg[2 * k] = b0;
        rbeg[2 * k + 1] = b1;
        roff[2 * k + 1] = l0;
        roff[2 * k + 2] = l1;
    }
    wave_sync();
    // prefix offsets of the 2 NC ranges (4 per lane, wavefront scan)
    const int nr = 2 * NC;
    {
        int v[4], s = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = 4 * lane + u;
            v[u] = r < nr ? roff[r + 1] : 0;
            s += v[u];
        }
        int incl = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        int run = incl - s;
        wave_sync();
        if (lane == 0) roff[0] = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = 4 * lane + u;
            run += v[u];
            if (r < nr) roff[r + 1] = run;
        }
    }
    wave_sync();
    const int total = roff[nr];

    const bool ivalid = ia < ii.y;
    const uint4 ci = ivalid ? sorted[ii.x + ia] : make_uint4(0, 0, 0, 0);   // q = 0 if invalid
    const float qi = __uint_as_float(ci.w);
    const float sx = a.scale[0], sy = a.scale[1], sz = a.scale[2], rc2 = a.rc2, irc2 = a.inv_rc2;
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    double e = 0.0;                      // FP32 pair energies, flushed to FP64 per chunk
    for (int base = 0; base < total; base += kChunk) {
        float ec = 0.0f;
        const int nch = min(kChunk, total - base);
        for (int t = lane; t < nch * 8; t += 64) {
            const int p = base + (t >> 3), k = t & 7;
            int lo = 0, hi = nr;                 // range r with roff[r] <= p < roff[r + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (roff[mid] <= p) lo = mid; else hi = mid;
            }
            const int J = rbeg[lo] + (p - roff[lo]);
            const int2 jj = cl_info[J];
            stage[t] = k < jj.y ? sorted[jj.x + k] : make_uint4(0, 0, 0, 0);
        }
        wave_sync();
        for (int s = 0; s < nch; ++s) {
            const uint4 cj = stage[s * 8 + ja];
            const float dx = (float)(int)(ci.x - cj.x) * sx;
            const float dy = (float)(int)(ci.y - cj.y) * sy;
            const float dz = (float)(int)(ci.z - cj.z) * sz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float qq = qi * __uint_as_float(cj.w);
            if (r2 < rc2 && r2 > 0.0f && qq != 0.0f) {
                const float rinv = __builtin_amdgcn_rsqf(r2);   // r2 is a normal number here
                const float x = r2 * irc2;
                float Pp = P.c[DEG];
#pragma unroll
                for (int m = DEG - 1; m >= 1; --m) Pp = fmaf(Pp, x, P.c[m]);
                const float Flo = fmaf(Pp, x, P.c0lo);
                float G = P.d[DEG];
#pragma unroll
                for (int m = DEG - 1; m >= 0; --m) G = fmaf(G, x, P.d[m]);
                ec = fmaf(qq, (rinv - P.c[0]) - Flo, ec);
                const float fs = qq * fmaf(rinv * rinv, rinv, G);
                fx = fmaf(fs, dx, fx);
                fy = fmaf(fs, dy, fy);
                fz = fmaf(fs, dz, fz);
            }
        }
        e += (double)ec;
        wave_sync();
    }
    // force on i-charge a: sum over its 8 lanes
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        fx += __shfl_xor(fx, off, 64);
        fy += __shfl_xor(fy, off, 64);
        fz += __shfl_xor(fz, off, 64);
    }
    if (ja == 0 && ivalid) fnear[ii.x + ia] = make_float4(fx, fy, fz, 0.0f);
    // each pair was seen from both ends: half of the summed pair energies
    const double es = wave_sum_d(e);
    if (lane == 0) epart[I] = 0.5 * es;
}

template <int DEG>
__global__ void __launch_bounds__(64) k_pair(PairArgs a, const uint4* __restrict__ sorted,
                                             const int* __restrict__ clus_start,
                                             const int2* __restrict__ cl_info,
                                             const int* __restrict__ cl_col,
                                             const uint2* __restrict__ cl_z,
                                             float4* __restrict__ fnear,
                                             double* __restrict__ epart) {
    pair_body<DEG>(a, blockIdx.x, sorted, clus_start, cl_info, cl_col, cl_z, fnear, epart);
}

template <int DEG>
__global__ void __launch_bounds__(64) k_pair_batch(const BatchTable* __restrict__ tab,
                                                   const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_PAIR, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        pair_body<DEG>(d.pair, item, d.sorted, d.clus_start, d.cl_info, d.cl_col, d.cl_z,
                       d.fnear, d.pair_parts);
    });
}

hipError_t launch_pair(const PairArgs& a, int nblocks, const uint4* sorted, const int* clus_start,
                       const int2* cl_info, const int* cl_col, const uint2* cl_z, float4* fnear,
                       double* epart, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid(nblocks), block(64);
    switch (a.deg) {
#define USERIES_PAIR_DEG(D)                                                                   \
    case D:                                                                                   \
        hipLaunchKernelGGL(k_pair<D>, grid, block, 0, st, a, sorted, clus_start, cl_info,     \
                           cl_col, cl_z, fnear, epart);                                       \
        break;
        USERIES_PAIR_DEG(4) USERIES_PAIR_DEG(5) USERIES_PAIR_DEG(6) USERIES_PAIR_DEG(7)
        USERIES_PAIR_DEG(8) USERIES_PAIR_DEG(9) USERIES_PAIR_DEG(10) USERIES_PAIR_DEG(11)
        USERIES_PAIR_DEG(12) USERIES_PAIR_DEG(13) USERIES_PAIR_DEG(14)
#undef USERIES_PAIR_DEG
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pair_batch(const BatchTable* tab, const BoxDesc* desc, int deg, int grid,
                             hipStream_t st) {
    switch (deg) {
#define USERIES_PAIR_DEG(D)                                                                   \
    case D:                                                                                   \
        hipLaunchKernelGGL(k_pair_batch<D>, dim3(grid), dim3(64), 0, st, tab, desc);          \
        break;
        USERIES_PAIR_DEG(4) USERIES_PAIR_DEG(5) USERIES_PAIR_DEG(6) USERIES_PAIR_DEG(7)
        USERIES_PAIR_DEG(8) USERIES_PAIR_DEG(9) USERIES_PAIR_DEG(10) USERIES_PAIR_DEG(11)
        USERIES_PAIR_DEG(12) USERIES_PAIR_DEG(13) USERIES_PAIR_DEG(14)
#undef USERIES_PAIR_DEG
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace useries
