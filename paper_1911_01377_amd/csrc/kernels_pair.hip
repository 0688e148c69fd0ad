// Near part of the u-series (eq. 20): for every pair closer than r_c,
//   energy  q_i q_j (1/r - F(r)),
//   force   q_i q_j (1/r^3 + F'(r)/r) (r_i - r_j)  on charge i,
// where F is the infinite far series (eq. 24), represented inside the cutoff
// by a polynomial in x = r^2/r_c^2 fitted on the host in FP64.
//
// Layout.  Cells are at least r_c/2 wide and sorted x-fastest, so the
// neighbours of a charge lie in the 5x5x5 cells around its own (all cells of
// an axis with fewer than 5), and along x those cells are contiguous in the
// sorted stream.  One block handles a group of G consecutive cells of one
// x-row (the i charges, one lane each, 64 per pass).  Its five wavefronts
// take the five z-offsets of the stencil; for each y-offset a wavefront
// stages the union of the x-windows of the group (G + 4 cells) from HBM into
// LDS with coalesced loads, then every lane walks its own 5-cell window out of
// LDS.  The partial forces of the five wavefronts are summed in a fixed order.
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

constexpr int kWaves = 5;        // one per z-offset of the stencil
constexpr int kStageCap = 512;   // staged charges per wavefront
constexpr int kMaxUnion = kMaxPairGroup + 4;

struct PairAcc {
    float fx, fy, fz;
    double e;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
        for (int k = 0; k < cnt; ++k) {
            const uint4 cj = load(base + k);
            const float dx = (float)(int)(ci.x - cj.x) * sx;
            const float dy = (float)(int)(ci.y - cj.y) * sy;
            const float dz = (float)(int)(ci.z - cj.z) * sz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (r2 < rc2 && r2 > 0.0f) mask |= 1u << k;
        }
        while (mask) {
            const int k = __builtin_ctz(mask);
            mask &= mask - 1;
            const uint4 cj = load(base + k);
            const float dx = (float)(int)(ci.x - cj.x) * sx;
            const float dy = (float)(int)(ci.y - cj.y) * sy;
            const float dz = (float)(int)(ci.z - cj.z) * sz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float qq = qi * __uint_as_float(cj.w);
            const float rinv = rsqrtf(r2);
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
__global__ void __launch_bounds__(64 * kWaves) k_pair(PairArgs a, const uint4* __restrict__ sorted,
                                                      const int* __restrict__ cell_start,
                                                      float4* __restrict__ fnear,
                                                      double* __restrict__ epart) {
    const Poly<DEG> P(a);
    __shared__ uint4 stage[kWaves][kStageCap];
    __shared__ int soff[kWaves][kMaxUnion + 1];
    __shared__ int sbeg[kWaves][kMaxUnion];
    __shared__ float4 fred[kWaves][64];
    __shared__ double ered[kWaves][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
    const int G = a.group;
    const int ngx = (nc0 + G - 1) / G;
    const int gx = blockIdx.x % ngx;
    const int cy = (blockIdx.x / ngx) % nc1;
    const int cz = blockIdx.x / (ngx * nc1);
    const int cx0 = gx * G;
    const int Gc = min(G, nc0 - cx0);
    const int Wn = min(5, nc0);                      // x-window length (cells)
    const int s0 = nc0 >= 5 ? cx0 - 2 : cx0;         // first cell of the staged union
    const int U = Gc + Wn - 1;                       // staged cells (may repeat if nc0 small)
    const int nyr = min(5, nc1), nzr = min(5, nc2);
    const int row_i = (cz * nc1 + cy) * nc0;
    const int i0 = cell_start[row_i + cx0], i1 = cell_start[row_i + cx0 + Gc];
    const bool active = w < nzr;
    const int zz = nc2 >= 5 ? wrapi(cz - 2 + w, nc2) : w;
    double eblock = 0.0;

    for (int ibase = i0; ibase < i1; ibase += 64) {
        const int i = ibase + lane;
        const bool valid = i < i1;
        uint4 ci = make_uint4(0, 0, 0, 0);
        if (valid) ci = sorted[i];
        const float qi = __uint_as_float(ci.w);
        const int p = valid ? wrapi(cell_coord(ci.x, nc0) - cx0, nc0) : 0;   // 0..Gc-1
        PairAcc acc = {0.0f, 0.0f, 0.0f, 0.0};
        if (active) {
            for (int ky = 0; ky < nyr; ++ky) {
                const int yy = nc1 >= 5 ? wrapi(cy - 2 + ky, nc1) : ky;
                const int row = (zz * nc1 + yy) * nc0;
                // per staged cell: first charge and count -> LDS offsets
                if (lane < U) {
                    const int c = row + wrapi(s0 + lane, nc0);
                    sbeg[w][lane] = cell_start[c];
                    soff[w][lane + 1] = cell_start[c + 1] - cell_start[c];
                }
                wave_sync();
                if (lane == 0) {
                    soff[w][0] = 0;
                    for (int u = 1; u <= U; ++u) soff[w][u] += soff[w][u - 1];
                }
                wave_sync();
                const int total = soff[w][U];
                if (total <= kStageCap) {
                    for (int t = lane; t < total; t += 64) {
                        int u = 0;
                        while (soff[w][u + 1] <= t) ++u;
                        stage[w][t] = sorted[sbeg[w][u] + (t - soff[w][u])];
                    }
                    wave_sync();
                    if (valid)
                        pair_window<DEG>(a, P, [&](int j) { return stage[w][j]; }, ci, qi, soff[w][p],
                                    soff[w][p + Wn], acc);
                } else if (valid) {
                    // more charges than LDS holds: read the window from HBM, cell by cell
                    for (int u = p; u < p + Wn; ++u)
                        pair_window<DEG>(a, P, [&](int j) { return sorted[j]; }, ci, qi, sbeg[w][u],
                                    sbeg[w][u] + (soff[w][u + 1] - soff[w][u]), acc);
                }
                wave_sync();
            }
        }
        fred[w][lane] = make_float4(acc.fx, acc.fy, acc.fz, 0.0f);
        ered[w][lane] = acc.e;
        __syncthreads();
        if (w == 0 && valid) {
            float4 f = fred[0][lane];
            double e = ered[0][lane];
            for (int v = 1; v < kWaves; ++v) {
                f.x += fred[v][lane].x;
                f.y += fred[v][lane].y;
                f.z += fred[v][lane].z;
                e += ered[v][lane];
            }
            fnear[i] = make_float4(f.x, f.y, f.z, 0.0f);
            eblock += e;
        }
        __syncthreads();
    }
    if (w == 0) {
        // each pair was seen from both ends: half of the summed pair energies
        const double e = wave_sum_d(eblock);
        if (lane == 0) epart[blockIdx.x] = 0.5 * e;
    }
}

int pair_blocks(const PairArgs& a) {
    return ((a.nc[0] + a.group - 1) / a.group) * a.nc[1] * a.nc[2];
}

hipError_t launch_pair(const PairArgs& a, const uint4* sorted, const int* cell_start,
                       float4* fnear, double* epart, hipStream_t st) {
    const dim3 grid(pair_blocks(a)), block(64 * kWaves);
    switch (a.deg) {
#define USERIES_PAIR_DEG(D)                                                                  \
    case D:                                                                                  \
        hipLaunchKernelGGL(k_pair<D>, grid, block, 0, st, a, sorted, cell_start, fnear, epart); \
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
