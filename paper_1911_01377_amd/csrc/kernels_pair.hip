// Near part of the u-series (eq. 20): for every pair closer than r_c,
//   energy  q_i q_j (1/r - F(r)),
//   force   q_i q_j (1/r^3 + F'(r)/r) (r_i - r_j)  on charge i,
// where F is the infinite far series (eq. 24), represented inside the cutoff
// by a polynomial in x = r^2/r_c^2 fitted on the host in FP64.
//
// Layout.  Cells are at least r_c/2 wide and sorted x-fastest, so the
// neighbours of a charge lie in the 5x5x5 cells around its own (all cells of
// an axis with fewer than 5), and along x those cells are contiguous in the
// sorted stream.  A group of G consecutive cells of one x-row gives the i
// charges (one lane each, 64 per pass).  Its 25 stencil rows (y, z offsets)
// are dealt to five single-wavefront blocks, five rows each, mixing central
// and outer rows so the blocks carry similar work.  A block stages the union
// of the x-windows of its rows (G + 4 cells per row) from HBM into LDS with
// coalesced loads; then every lane walks, for each row, the cells that
// intersect its cutoff sphere (a row out of reach is skipped).  The five
// partial forces of a charge go to separate slices and are summed, in a fixed
// order, by the gather step.
//
// Inside a window the candidates are taken 32 at a time: a cheap distance
// test builds a bit mask per lane, then only in-range pairs are evaluated, so
// a lane's pair arithmetic is not serialised behind the tests of its
// neighbours.
//
// Each pair is evaluated from both ends (no Newton's-third-law sharing), so
// forces need no atomics and the result does not depend on scheduling.
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

namespace {

constexpr int kRowSets = 5;      // blocks per cell group, each taking a fifth of the 25 rows
constexpr int kRowsPerSet = 5;
constexpr int kStageCap = 512;   // staged charges per block (five rows)
constexpr int kMaxUnion = kMaxPairGroup + 4;

struct PairAcc {
    float fx, fy, fz;
    double e;
};

// Polynomial coefficients held in registers (compile-time degree, fully
// unrolled): F = c0 + x (c1 + x P(x)) with c0 and c1 as hi + lo pairs, and
// G = F'(r)/r.
template <int DEG>
struct Poly {
    float c[DEG + 1];
    float c0lo, c1lo;
    float d[DEG];
    __device__ __forceinline__ explicit Poly(const PairArgs& a) {
#pragma unroll
        for (int m = 0; m <= DEG; ++m) c[m] = a.c[m];
#pragma unroll
        for (int m = 0; m < DEG; ++m) d[m] = a.d[m];
        c0lo = a.c0lo;
        c1lo = a.c1lo;
    }
};

template <int DEG, class Load>
__device__ __forceinline__ void pair_window(const PairArgs& a, const Poly<DEG>& P, Load load,
                                            const uint4& ci, float qi, int j0, int j1,
                                            PairAcc& acc) {
    const float sx = a.scale[0], sy = a.scale[1], sz = a.scale[2], rc2 = a.rc2,
                irc2 = a.inv_rc2;
    for (int base = j0; base < j1; base += 32) {
        const int cnt = min(32, j1 - base);
        uint32_t mask = 0;
        // distance tests four at a time, loads issued together; indices past
        // the window end re-read its last charge and their bits are dropped
        for (int k = 0; k < cnt; k += 4) {
            uint4 cj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) cj[u] = load(base + min(k + u, cnt - 1));
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float dx = (float)(int)(ci.x - cj[u].x) * sx;
                const float dy = (float)(int)(ci.y - cj[u].y) * sy;
                const float dz = (float)(int)(ci.z - cj[u].z) * sz;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                if (r2 < rc2 && r2 > 0.0f) mask |= 1u << (k + u);
            }
        }
        mask &= cnt == 32 ? 0xffffffffu : ((1u << cnt) - 1u);
        while (mask) {
            const int k = __builtin_ctz(mask);
            mask &= mask - 1;
            const uint4 cj = load(base + k);
            const float dx = (float)(int)(ci.x - cj.x) * sx;
            const float dy = (float)(int)(ci.y - cj.y) * sy;
            const float dz = (float)(int)(ci.z - cj.z) * sz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float qq = qi * __uint_as_float(cj.w);
            const float rinv = __builtin_amdgcn_rsqf(r2);   // r2 is a normal number here
            const float x = r2 * irc2;
            float Pp = P.c[DEG];
#pragma unroll
            for (int m = DEG - 1; m >= 2; --m) Pp = fmaf(Pp, x, P.c[m]);
            const float t1 = fmaf(Pp, x, P.c1lo) + P.c[1];
            const float Flo = fmaf(t1, x, P.c0lo);
            float G = P.d[DEG - 1];
#pragma unroll
            for (int m = DEG - 2; m >= 0; --m) G = fmaf(G, x, P.d[m]);
            acc.e += (double)(qq * ((rinv - P.c[0]) - Flo));
            const float fs = qq * fmaf(rinv * rinv, rinv, G);
            acc.fx = fmaf(fs, dx, acc.fx);
            acc.fy = fmaf(fs, dy, acc.fy);
            acc.fz = fmaf(fs, dz, acc.fz);
        }
    }
}

}  // namespace

template <int DEG>
__global__ void __launch_bounds__(64) k_pair(PairArgs a, const uint4* __restrict__ sorted,
                                             const int* __restrict__ cell_start,
                                             float4* __restrict__ fpart,
                                             double* __restrict__ epart) {
    const Poly<DEG> P(a);
    __shared__ uint4 stage[kStageCap];
    __shared__ int soff[kRowsPerSet * kMaxUnion + 1];
    __shared__ int sbeg[kRowsPerSet * kMaxUnion];
    const int lane = threadIdx.x;
    const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
    const int G = a.group;
    const int ngx = (nc0 + G - 1) / G;
    const int set = blockIdx.x % kRowSets;           // which fifth of the stencil rows
    const int grp = blockIdx.x / kRowSets;
    const int gx = grp % ngx;
    const int cy = (grp / ngx) % nc1;
    const int cz = grp / (ngx * nc1);
    const int cx0 = gx * G;
    const int Gc = min(G, nc0 - cx0);
    const int Wn = min(5, nc0);                      // x-window length (cells)
    const int s0 = nc0 >= 5 ? cx0 - 2 : cx0;         // first cell of a staged union
    const int U = Gc + Wn - 1;                       // staged cells per row (may repeat if nc0 small)
    const int nyr = min(5, nc1), nzr = min(5, nc2);
    const int nrows = nyr * nzr;
    const int nmine = nrows > set ? (nrows - set + kRowSets - 1) / kRowSets : 0;
    const int NU = nmine * U;                        // staged cells of this block
    const int row_i = (cz * nc1 + cy) * nc0;
    const int i0 = cell_start[row_i + cx0], i1 = cell_start[row_i + cx0 + Gc];

    // stencil rows r = set, set + 5, ... of the (y, z) offsets; their union
    // cells: first charge and count, prefix offsets, one coalesced LDS copy
    for (int k = lane; k < NU; k += 64) {
        const int m = k / U, u = k - m * U;
        const int r = set + kRowSets * m;
        const int ky = r % nyr, kz = r / nyr;
        const int yy = nc1 >= 5 ? wrapi(cy - 2 + ky, nc1) : ky;
        const int zz = nc2 >= 5 ? wrapi(cz - 2 + kz, nc2) : kz;
        const int c = (zz * nc1 + yy) * nc0 + wrapi(s0 + u, nc0);
        sbeg[k] = cell_start[c];
        soff[k + 1] = cell_start[c + 1] - cell_start[c];
    }
    wave_sync();
    if (lane == 0) {
        soff[0] = 0;
        for (int u = 1; u <= NU; ++u) soff[u] += soff[u - 1];
    }
    wave_sync();
    const int total = soff[NU];
    if (total <= kStageCap) {
        for (int t = lane; t < total; t += 64) {
            int lo = 0, hi = NU;                       // the cell holding slot t
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= t) lo = mid; else hi = mid;
            }
            stage[t] = sorted[sbeg[lo] + (t - soff[lo])];
        }
    }
    wave_sync();

    double eblock = 0.0;
    for (int ibase = i0; ibase < i1; ibase += 64) {
        const int i = ibase + lane;
        if (i >= i1) break;
        const uint4 ci = sorted[i];
        const float qi = __uint_as_float(ci.w);
        int cxi, cyi, czi;
        float fx, fy, fz;                      // position inside the own cell, in cell widths
        grid_coord(ci.x, nc0, &cxi, &fx);
        grid_coord(ci.y, nc1, &cyi, &fy);
        grid_coord(ci.z, nc2, &czi, &fz);
        const int p = wrapi(cxi - cx0, nc0);   // 0..Gc-1
        // distance from the charge to the slab of cells at offset k (0 for
        // k = 0, and 0 when an axis has fewer than 5 cells: offsets unused)
        auto slab_gap = [](int k, float f, float wd) {
            return k > 0 ? (k - f) * wd : (k < 0 ? (f - k - 1) * wd : 0.0f);
        };
        PairAcc acc = {0.0f, 0.0f, 0.0f, 0.0};
        for (int m = 0; m < nmine; ++m) {
            const int r = set + kRowSets * m;
            const int ky = r % nyr, kz = r / nyr;
            const float gy = nc1 >= 5 ? slab_gap(ky - 2, fy, a.cw[1]) : 0.0f;
            const float gz = nc2 >= 5 ? slab_gap(kz - 2, fz, a.cw[2]) : 0.0f;
            const float rx2 = a.rc2 - gy * gy - gz * gz;
            if (rx2 <= 0.0f) continue;         // the whole row is out of reach
            // x-cells of the row that intersect [x_i - dx, x_i + dx]
            int lo = 0, hi = Wn - 1;
            if (nc0 >= 5) {
                const float dxc = sqrtf(rx2) / a.cw[0];
                lo = max(0, (int)floorf(fx - dxc) + 2);
                hi = min(4, (int)floorf(fx + dxc) + 2);
            }
            const int c0 = m * U + p;
            if (total <= kStageCap) {
                pair_window<DEG>(a, P, [&](int j) { return stage[j]; }, ci, qi, soff[c0 + lo],
                                 soff[c0 + hi + 1], acc);
            } else {
                // more charges than LDS holds: read the window from HBM, cell by cell
                for (int u = c0 + lo; u <= c0 + hi; ++u)
                    pair_window<DEG>(a, P, [&](int j) { return sorted[j]; }, ci, qi, sbeg[u],
                                     sbeg[u] + (soff[u + 1] - soff[u]), acc);
            }
        }
        fpart[(size_t)set * a.n + i] = make_float4(acc.fx, acc.fy, acc.fz, 0.0f);
        eblock += acc.e;
    }
    // each pair was seen from both ends: half of the summed pair energies
    const double e = wave_sum_d(eblock);
    if (lane == 0) epart[blockIdx.x] = 0.5 * e;
}

int pair_blocks(const PairArgs& a) {
    return ((a.nc[0] + a.group - 1) / a.group) * a.nc[1] * a.nc[2] * kRowSets;
}

hipError_t launch_pair(const PairArgs& a, const uint4* sorted, const int* cell_start,
                       float4* fpart, double* epart, hipStream_t st) {
    const dim3 grid(pair_blocks(a)), block(64);
    switch (a.deg) {
#define USERIES_PAIR_DEG(D)                                                                  \
    case D:                                                                                  \
        hipLaunchKernelGGL(k_pair<D>, grid, block, 0, st, a, sorted, cell_start, fpart, epart); \
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
