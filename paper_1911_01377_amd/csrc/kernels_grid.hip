// Spreading and gathering of the far part (Sec. IV.A mesh evaluation, Sec. V
// grid convolution).  Each charge is smeared on the grid by a normalised,
// separable Gaussian of width sigma_s (per axis), sampled on a cube stencil
// of 2P points per axis around it:
//   rho_g = sum_i q_i prod_a W_a(g_a h_a - x_ia),
//   W_a(d) = h_a / (sqrt(2 pi) sigma_s,a) exp(-d^2 / (2 sigma_s,a^2)),
// and potentials and forces are read back with the same weights:
//   phi_i = sum_g phi_g prod_a W_a,   F_i = -q_i grad_i phi_i.
// The mean of rho (its k = 0 mode, the net charge) is removed on the grid.
//
// spread: one block per 8x8x8 brick of the grid.  Candidates come from the
//   x-y columns that can hold a charge touching the brick, each contributing
//   the charges of the brick's z-planes (per-column z-plane index); the block
//   keeps those that touch it, stages their weights in LDS and accumulates the
//   brick in registers by x halves, four wavefronts per half, a lane owning a
//   4-point x row of it; each wavefront takes a share of the charges that
//   touch its half, and the partial sums are added in a fixed order.  No
//   atomics.
// gather: one block per brick with the potential on the brick and its halo in
//   LDS; each charge is evaluated by the block whose brick holds its stencil
//   anchor, 8 or 16 lanes per charge.  One more block forms the energy total.
#include <algorithm>

#include "useries_internal.h"
#include "device_common.h"
#include "energy_total.h"

namespace useries {

namespace {

constexpr int kBrick = 8;
constexpr int kSpreadWaves = 8;                  // wavefronts per brick
constexpr int kSpreadChunk = 64 * kSpreadWaves;  // candidates loaded per pass, one per thread

__device__ __forceinline__ int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int ceildiv(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }
__device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}
__device__ __forceinline__ long long ceildiv_ll(long long a, long long b) {
    return a >= 0 ? (a + b - 1) / b : -((-a) / b);
}

// columns along one axis that can hold charges touching grid points
// [X0, X0 + bn): charges whose stencil start lies in [X0 - P, X0 + bn + P - 1)
__device__ __forceinline__ void cell_window(int X0, int bn, int P, int g, int nc, int* lo,
                                            int* cnt) {
    const int l = floordiv((X0 - P) * nc, g);
    const int h = ceildiv((X0 + bn + P - 1) * nc, g) - 1;
    if (h - l + 1 >= nc) {
        *lo = 0;
        *cnt = nc;
    } else {
        *lo = wrapi(l, nc);
        *cnt = h - l + 1;
    }
}

}  // namespace

// One block per 8x8x8 brick.  The window of a brick: in x and y the columns
// that can hold a charge whose stencil touches it, in z the grid planes
// [Z0 - P, Z0 + B2 + P - 2] (periodic), read from each column's z-plane index
// as at most two contiguous charge ranges.  The block loads the candidates in
// chunks of one per thread, keeps those whose stencil touches the brick
// (compacted in thread order within three classes: those meeting only the x
// half 0 (x 0..3), both halves, only half 1 -- so the order is deterministic
// and each half's charges are one contiguous run), stages their 3 x 8 weights
// in LDS, and wavefront 4 h + u accumulates every fourth of half h's charges
// from the u-th into its partial half brick (a dense 4 x 8 x 8 product per
// charge; a charge whose stencil ends at brick position d meets both halves
// only for 4 <= d <= 2P + 2, so at P = 3 about 60% of the charges are
// accumulated by one half only); the four partials of each point are summed
// in a fixed order at the end.
// PT > 0: the stencil half width as a compile-time constant; PT = 0 takes it
// from a.P.
template <int PT>
__device__ __forceinline__ void spread_body(const GridArgs& a, int bid,
                                            const uint4* __restrict__ sorted,
                                            const int* __restrict__ zbin,
                                            const double* __restrict__ qstats,
                                            float* __restrict__ rho) {
    __shared__ __align__(16) float sw[kSpreadChunk][3 * kBrick];   // rows of 96 B (16-byte stores)
    static_assert(kSpreadWaves == 8 && kBrick == 8, "four wavefronts per half brick; 8-wide rows");
    // the wavefronts' partial half bricks, summed after the last chunk (reuses
    // sw; rows of 65 so that the 8 partials a thread group reads lie in
    // different banks)
    float (*red)[4][65] = reinterpret_cast<float (*)[4][65]>(&sw[0][0]);
    static_assert(kSpreadWaves * 4 * 65 <= kSpreadChunk * 3 * kBrick, "red fits in sw");
    __shared__ int pbeg[2 * kMaxWindowCols];       // first charge of each column piece
    __shared__ int poff[2 * kMaxWindowCols + 1];   // prefix sums of the piece lengths
    __shared__ int wtot[kSpreadWaves];
    __shared__ int wcat[3][kSpreadWaves];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    // wavefronts 4 h .. 4 h + 3 accumulate the x half h of the brick
    // (x 4 h .. 4 h + 3); lane (y, z) owns the four points of that row,
    // partial sums acc[x - 4 h]
    const int hx = w >> 2, ly = lane & 7, lz = lane >> 3;
    // the grid mean of the charge (removed at the end), loaded first
    const float mean = (float)(qstats[0] * a.inv_ngrid);
    const int nbx = (a.g[0] + kBrick - 1) / kBrick, nby = (a.g[1] + kBrick - 1) / kBrick;
    const int X0 = (bid % nbx) * kBrick, Y0 = ((bid / nbx) % nby) * kBrick,
              Z0 = (bid / (nbx * nby)) * kBrick;
    const int B0 = min(kBrick, a.g[0] - X0), B1 = min(kBrick, a.g[1] - Y0),
              B2 = min(kBrick, a.g[2] - Z0);
    const int P = PT > 0 ? PT : a.P, gz = a.g[2];
    constexpr int KMAX = PT > 0 ? 2 * PT : 2 * kMaxStencilHalf;   // stencil points per axis
    int lo[2], cnt[2];
    cell_window(X0, B0, P, a.g[0], a.nc[0], &lo[0], &cnt[0]);
    cell_window(Y0, B1, P, a.g[1], a.nc[1], &lo[1], &cnt[1]);
    const int ncw = cnt[0] * cnt[1];
    const int np = 2 * ncw;
    // z planes of the window: [zs, zs + zl) modulo gz
    const int zl = B2 + 2 * P - 1;
    const int zs = wrapi(Z0 - P, gz);
    for (int k = tid; k < ncw; k += 64 * kSpreadWaves) {
        const int col = wrapi(lo[1] + k / cnt[0], a.nc[1]) * a.nc[0] + wrapi(lo[0] + k % cnt[0], a.nc[0]);
        const int* zr = zbin + (size_t)col * (gz + 1);
        int b0, e0, b1 = 0, e1 = 0;
        if (zl >= gz) {
            b0 = zr[0];
            e0 = zr[gz];
        } else if (zs + zl <= gz) {
            b0 = zr[zs];
            e0 = zr[zs + zl];
        } else {
            b0 = zr[zs];
            e0 = zr[gz];
            b1 = zr[0];
            e1 = zr[zs + zl - gz];
        }
        pbeg[2 * k] = b0;
        pbeg[2 * k + 1] = b1;
        poff[2 * k + 1] = e0 - b0;
        poff[2 * k + 2] = e1 - b1;
    }
    __syncthreads();
    // inclusive prefix of the np <= 512 piece lengths: two per thread
    {
        const int r0 = 2 * tid, r1 = 2 * tid + 1;
        const int v0 = r0 < np ? poff[r0 + 1] : 0, v1 = r1 < np ? poff[r1 + 1] : 0;
        const int incl = wave_incl_scan(v0 + v1);
        if (lane == 63) wtot[w] = incl;
        __syncthreads();
        int wbase = 0;
        for (int v = 0; v < w; ++v) wbase += wtot[v];
        const int excl = wbase + incl - v0 - v1;
        if (r0 < np) poff[r0 + 1] = excl + v0;
        if (r1 < np) poff[r1 + 1] = excl + v0 + v1;
        if (tid == 0) poff[0] = 0;
        __syncthreads();
    }
    const int total = poff[np];
    const int X0s[3] = {X0, Y0, Z0};
    const int Bs[3] = {B0, B1, B2};

    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};

    // candidate t of the window (loads are issued one chunk ahead)
    auto fetch = [&](int t) {
        uint4 c = make_uint4(0, 0, 0, 0);
        if (t < total) {
            int l = 0, h = np;                 // piece r with poff[r] <= t < poff[r + 1]
            while (h - l > 1) {
                const int mid = (l + h) >> 1;
                if (poff[mid] <= t) l = mid; else h = mid;
            }
            c = sorted[pbeg[l] + (t - poff[l])];
        }
        return c;
    };
    uint4 next = fetch(tid);
    for (int base = 0; base < total; base += kSpreadChunk) {
        const int t = base + tid;
        bool touch = false;
        int cat = 0;
        int gi[3];
        float f[3];
        float qj = 0.0f;
        const uint4 c = next;
        if (base + kSpreadChunk < total) next = fetch(t + kSpreadChunk);
        if (t < total) {
            grid_coord(c.x, a.g[0], &gi[0], &f[0]);
            grid_coord(c.y, a.g[1], &gi[1], &f[1]);
            grid_coord(c.z, a.g[2], &gi[2], &f[2]);
            qj = __uint_as_float(c.w);
            touch = true;
            int d[3];   // last stencil point's brick position (first: d - 2P + 1)
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                d[ax] = wrap1(gi[ax] - (X0s[ax] - P), a.g[ax]);
                touch = touch && d[ax] <= Bs[ax] + 2 * P - 2;
            }
            // x halves met: 0 (x 0..3) only, both, 1 (x 4 .. B0 - 1) only
            const bool h0 = d[0] - 2 * P + 1 <= 3, h1 = d[0] >= 4 && B0 > 4;
            cat = h0 ? (h1 ? 1 : 0) : 2;
        }
        // compaction in thread order within each x-half class, the classes
        // one after the other: half 0's charges are rows [0, n0 + n01), half
        // 1's rows [n0, nst)
        const uint64_t mc[3] = {__ballot(touch && cat == 0), __ballot(touch && cat == 1),
                                __ballot(touch && cat == 2)};
        if (lane < 3) wcat[lane][w] = __popcll(lane == 0 ? mc[0] : lane == 1 ? mc[1] : mc[2]);
        __syncthreads();
        int ncat[3] = {0, 0, 0}, bcat[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < kSpreadWaves; ++v) {
                bcat[k] += v < w ? wcat[k][v] : 0;
                ncat[k] += wcat[k][v];
            }
        const int nst = ncat[0] + ncat[1] + ncat[2];
        // the touching charges' records: record s in the first 16 bytes of
        // weight row s
        if (touch) {
            const int cb = cat == 0 ? 0 : cat == 1 ? ncat[0] : ncat[0] + ncat[1];
            const uint64_t mm = cat == 0 ? mc[0] : cat == 1 ? mc[1] : mc[2];
            *reinterpret_cast<uint4*>(sw[cb + bcat[cat] + lanes_below(mm)]) = c;
        }
        __syncthreads();
        if (tid < nst) {
            // thread s: the 3 x 8 brick weights of staged charge s (row s is
            // its own until the next barrier): zero, then the 2P stencil points
            // of each axis at their brick positions (k - k0) mod g
            float* row = sw[tid];
            const uint4 cs = *reinterpret_cast<const uint4*>(row);
            grid_coord(cs.x, a.g[0], &gi[0], &f[0]);
            grid_coord(cs.y, a.g[1], &gi[1], &f[1]);
            grid_coord(cs.z, a.g[2], &gi[2], &f[2]);
            qj = __uint_as_float(cs.w);
#pragma unroll
            for (int b = 0; b < 3 * kBrick; b += 4)
                *reinterpret_cast<float4*>(row + b) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int k0 = wrap1(X0s[ax] - gi[ax] + P - 1, a.g[ax]);
                const float c = (float)(P - 1) + f[ax];
                const float sc = ax == 1 ? a.cw[ax] * qj : a.cw[ax];
                const float e2 = -a.hs[ax] * 1.44269504f;   // exp(-t^2 hs) = 2^(t^2 e2)
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (PT > 0 || k < 2 * P) {
                        int b = k - k0;
                        if (b < 0) b += a.g[ax];
                        if (b < Bs[ax]) {
                            const float t = (float)k - c;
                            row[ax * kBrick + b] = sc * __builtin_amdgcn_exp2f(t * t * e2);
                        }
                    }
                }
            }
        }
        __syncthreads();
        // the staged charges of this wavefront's x half, every fourth one, in
        // staged order, two at a time with their LDS reads issued together;
        // per charge the half's four x weights (one 16-byte read, the same
        // address on every lane), the lane's y and z weights, one y z product
        // and four FMAs
        auto wts = [&](int sidx, float4& X, float& Y, float& Z) {
            const float* row = sw[sidx];
            X = *reinterpret_cast<const float4*>(row + 4 * hx);
            Y = row[kBrick + ly];
            Z = row[2 * kBrick + lz];
        };
        auto add = [&](const float4 X, const float Y, const float Z) {
            const float yz = Y * Z;
            acc[0] = fmaf(X.x, yz, acc[0]);
            acc[1] = fmaf(X.y, yz, acc[1]);
            acc[2] = fmaf(X.z, yz, acc[2]);
            acc[3] = fmaf(X.w, yz, acc[3]);
        };
        // (uniform per wavefront: loop control in scalar registers)
        const int hend = __builtin_amdgcn_readfirstlane(hx == 0 ? ncat[0] + ncat[1] : nst);
        int sidx = __builtin_amdgcn_readfirstlane((hx == 0 ? 0 : ncat[0]) + (w & 3));
        for (; sidx + 4 < hend; sidx += 8) {
            float4 X0w, X1w;
            float Y0w, Z0w, Y1w, Z1w;
            wts(sidx, X0w, Y0w, Z0w);
            wts(sidx + 4, X1w, Y1w, Z1w);
            add(X0w, Y0w, Z0w);
            add(X1w, Y1w, Z1w);
        }
        if (sidx < hend) {
            float4 Xw;
            float Yw, Zw;
            wts(sidx, Xw, Yw, Zw);
            add(Xw, Yw, Zw);
        }
        __syncthreads();
    }

    // fixed-order sum of the four partials of each point (those of its half's
    // wavefronts, in wavefront order): all partials to LDS, then thread
    // (x, y, z) = (tid % 8, tid / 8 % 8, tid / 64) adds those of its point,
    // lane (y, z)'s partial x % 4 of wavefronts 4 (x / 4) + u
#pragma unroll
    for (int k = 0; k < 4; ++k) red[w][k][lane] = acc[k];
    __syncthreads();
    const int px = tid & 7, py = (tid >> 3) & 7, pz = tid >> 6;
    const int h = px >> 2, k = px & 3, l = py + 8 * pz;
    float v = red[4 * h][k][l];
#pragma unroll
    for (int u = 1; u < 4; ++u) v += red[4 * h + u][k][l];
    if (px < B0 && py < B1 && pz < B2)
        rho[((size_t)(Z0 + pz) * a.g[1] + (Y0 + py)) * a.g[0] + X0 + px] = v - mean;
}

template <int PT>
__global__ void __launch_bounds__(64 * kSpreadWaves) k_spread(int nb,
                                                              const int* __restrict__ zbin,
                                                              const double* __restrict__ qstats,
                                                              const uint4* __restrict__ sorted,
                                                              float* __restrict__ rho, GridArgs a) {
    const int item = xcd_item(blockIdx.x, nb);
    if (item < nb) spread_body<PT>(a, item, sorted, zbin, qstats, rho);
}

// PT > 0 only when every box of the batch has stencil half width PT
template <int PT>
__global__ void __launch_bounds__(64 * kSpreadWaves) k_spread_batch(
        const BatchTable* __restrict__ tab, const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_SPREAD, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        spread_body<PT>(d.grid, item, d.sorted, d.zbin, d.qstats, d.rho);
    });
}

// gather: one block per brick of the grid (8^3 for P <= 5, 4^3 beyond).  The
// block stages the potential on the brick and its stencil halo (edge
// brick + 2P - 1) in LDS with coalesced row loads, then takes the charges
// whose stencil anchor (grid cell) lies in the brick: per overlapping column
// the z-plane index gives one contiguous range; candidates are loaded one per
// thread and the owners compacted in thread order.  A wavefront evaluates
// eight owners at a time with 8 lanes each (stencils of up to 8 points per
// axis, compiled for that width) or four with 16: a lane owns stencil rows
// (y, z) and reads the 2P x points of each from LDS; the groups then reduce.
constexpr int kGatherMaxPieces = 256;     // columns overlapping a brick
constexpr int kGatherWaves = 8;           // wavefronts per brick
constexpr int kGatherThreads = 64 * kGatherWaves;
constexpr int kGatherBatch = 8;           // halo loads issued together per thread
constexpr int kGatherOwners = 8;          // owners per wavefront pass, at most

__host__ __device__ constexpr int gather_brick(int P) { return P <= 5 ? 8 : 4; }

// Dynamic LDS of a gather block for stencil half width P (byte offsets): the
// halo of edge brick + 2P - 1 and the per-owner weights are sized by P.
struct GatherLds {
    int own, ownf, ownp, sphi, sw, rowtab, pbeg, poff, wtot, total;
};
__host__ __device__ inline GatherLds gather_lds(int P) {
    const int E = gather_brick(P) + 2 * P - 1;
    GatherLds L{};
    int o = 0;
    auto take = [&](int bytes) {
        const int r = o;
        o += (bytes + 15) & ~15;
        return r;
    };
    L.own = take(16 * kGatherThreads);                 // owner records
    L.ownf = take(16 * kGatherThreads);                // owners' near forces
    L.ownp = take(4 * kGatherThreads);                 // owners' input indices
    L.sphi = take(4 * E * E * E);                      // potential on brick + halo
    L.sw = take(4 * kGatherWaves * kGatherOwners * 6 * 2 * P);   // weights, derivatives [wave][owner][6][2P]
    L.rowtab = take(8 * 4 * P * P);                    // stencil rows {offset, ky | kz << 16}
    L.pbeg = take(4 * kGatherMaxPieces);
    L.poff = take(4 * (kGatherMaxPieces + 1));
    L.wtot = take(4 * kGatherWaves);
    L.total = o;
    return L;
}

// PT > 0: the stencil half width as a compile-time constant (fully unrolled
// stencil rows, weights held in registers); PT = 0 takes it from a.P.
template <int PT>
__device__ __forceinline__ void gather_body(const GridArgs& a, int bid,
                                            const uint4* __restrict__ sorted,
                                            const int* __restrict__ perm,
                                            const int* __restrict__ zbin,
                                            const float* __restrict__ phi,
                                            const float4* __restrict__ fnear,
                                            float* __restrict__ forces, char* lds) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // LPO lanes per owner charge (8 for a compile-time stencil of at most 8
    // points per axis, else 16), OPW owners per wavefront pass
    constexpr int LPO = (PT > 0 && 2 * PT <= 8) ? 8 : 16, OPW = 64 / LPO;
    const int g = lane / LPO, lg = lane % LPO;
    const int P = PT > 0 ? PT : a.P, P2 = 2 * P, GB = gather_brick(P);
    constexpr int KMAX = PT > 0 ? 2 * PT : 2 * kMaxStencilHalf;   // x points per stencil row
    const GatherLds LL = gather_lds(P);
    uint4* own = reinterpret_cast<uint4*>(lds + LL.own);
    float4* ownf = reinterpret_cast<float4*>(lds + LL.ownf);
    int* ownp = reinterpret_cast<int*>(lds + LL.ownp);
    float* sphi = reinterpret_cast<float*>(lds + LL.sphi);
    float* swb = reinterpret_cast<float*>(lds + LL.sw);
    int2* rowtab = reinterpret_cast<int2*>(lds + LL.rowtab);
    int* pbeg = reinterpret_cast<int*>(lds + LL.pbeg);
    int* poff = reinterpret_cast<int*>(lds + LL.poff);
    int* wtot = reinterpret_cast<int*>(lds + LL.wtot);
    const int nbx = (a.g[0] + GB - 1) / GB, nby = (a.g[1] + GB - 1) / GB;
    const int X0 = (bid % nbx) * GB, Y0 = ((bid / nbx) % nby) * GB, Z0 = (bid / (nbx * nby)) * GB;
    const int B0 = min(GB, a.g[0] - X0), B1 = min(GB, a.g[1] - Y0), B2 = min(GB, a.g[2] - Z0);
    const int E0 = B0 + P2 - 1, E1 = B1 + P2 - 1, E2 = B2 + P2 - 1;
    // potential on the brick and halo: local (hx, hy, hz) = global (X0 - P + 1 + hx, ...)
    // approximate reciprocals: (idx + 1/2) / E stays 1 / (2E) from an integer
    const float inv0 = __builtin_amdgcn_rcpf((float)E0), inv1 = __builtin_amdgcn_rcpf((float)E1);
    const int nh = E0 * E1 * E2;
    // columns overlapping the brick's cells in x and y (at most one per
    // thread): the charge range of the brick's z-planes in each, loaded first
    // so that these loads are in flight with the halo's
    static_assert(kGatherMaxPieces <= kGatherThreads, "one column per thread");
    const int cxl = X0 * a.nc[0] / a.g[0], cxh = ((X0 + B0) * a.nc[0] + a.g[0] - 1) / a.g[0] - 1;
    const int cyl = Y0 * a.nc[1] / a.g[1], cyh = ((Y0 + B1) * a.nc[1] + a.g[1] - 1) / a.g[1] - 1;
    const int cxn = cxh - cxl + 1, np = cxn * (cyh - cyl + 1);
    int zb = 0, ze = 0;
    if (tid < np) {
        const int col = (cyl + tid / cxn) * a.nc[0] + cxl + tid % cxn;
        const int* zr = zbin + (size_t)col * (a.g[2] + 1);
        zb = zr[Z0];
        ze = zr[Z0 + B2];
    }
    // the loads of a pass are issued together, then stored; a compile-time
    // stencil gives a fixed number of passes (unrolled, so the column loads
    // above stay in flight with the first pass's)
    auto halo_pass = [&](int base) {
        float v[kGatherBatch];
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
            const int idx = base + kGatherThreads * u;
            const int r = small_div(idx, inv0), hx = idx - r * E0;
            const int hz = small_div(r, inv1), hy = r - hz * E1;
            const int gx = wrap1(X0 - P + 1 + hx, a.g[0]);
            const int gy = wrap1(Y0 - P + 1 + hy, a.g[1]);
            const int gz = wrap1(Z0 - P + 1 + hz, a.g[2]);
            v[u] = idx < nh ? phi[((size_t)gz * a.g[1] + gy) * a.g[0] + gx] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
            const int idx = base + kGatherThreads * u;
            if (idx < nh) sphi[idx] = v[u];
        }
    };
    constexpr int kPass = kGatherThreads * kGatherBatch;
    if constexpr (PT > 0) {
        constexpr int EM = gather_brick(PT) + 2 * PT - 1;   // edge of a whole brick's halo
#pragma unroll
        for (int ps = 0; ps < (EM * EM * EM + kPass - 1) / kPass; ++ps) halo_pass(tid + ps * kPass);
    } else {
        for (int base = tid; base < nh; base += kPass) halo_pass(base);
    }
    // stencil rows (ky, kz) of a charge and their offsets in the halo, once per block
    for (int r = tid; r < P2 * P2; r += kGatherThreads) {
        const int ky = r % P2, kz = r / P2;
        rowtab[r] = make_int2((kz * E1 + ky) * E0, ky | (kz << 16));
    }
    if (tid < np) {
        pbeg[tid] = zb;
        poff[tid + 1] = ze - zb;
    }
    __syncthreads();
    {
        const int v = tid < np ? poff[tid + 1] : 0;
        const int incl = wave_incl_scan(v);
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < wave; ++w) wbase += wtot[w];
        if (tid < np) poff[tid + 1] = wbase + incl;
        if (tid == 0) poff[0] = 0;
        __syncthreads();
    }
    const int total = poff[np];
    for (int base = 0; base < total; base += kGatherThreads) {
        const int t = base + tid;
        bool mine = false;
        uint4 c = make_uint4(0, 0, 0, 0);
        float4 fn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int pj = 0;
        if (t < total) {
            int l = 0, h = np;
            while (h - l > 1) {
                const int mid = (l + h) >> 1;
                if (poff[mid] <= t) l = mid; else h = mid;
            }
            const int j = pbeg[l] + (t - poff[l]);
            // the near force and input index load with the record (most
            // candidates are owners), saving a round trip after the ballot
            c = sorted[j];
            fn = fnear[j];
            pj = perm[j];
            const int gx = cell_coord(c.x, a.g[0]), gy = cell_coord(c.y, a.g[1]);
            mine = gx >= X0 && gx < X0 + B0 && gy >= Y0 && gy < Y0 + B1;
        }
        const uint64_t m = __ballot(mine);
        if (lane == 0) wtot[wave] = __popcll(m);
        __syncthreads();
        int before = 0, nown = 0;
#pragma unroll
        for (int w = 0; w < kGatherWaves; ++w) {
            before += w < wave ? wtot[w] : 0;
            nown += wtot[w];
        }
        if (mine) {
            const int slot = before + __popcll(m & ((1ull << lane) - 1ull));
            own[slot] = c;
            ownf[slot] = fn;
            ownp[slot] = pj;
        }
        __syncthreads();
        // OPW owners per wavefront pass, groups dealt round-robin to the wavefronts
        static_assert(OPW <= kGatherOwners, "weights sized for kGatherOwners per wavefront");
        for (int o0 = wave * OPW; o0 < nown; o0 += OPW * kGatherWaves) {
            const int o = o0 + g;
            const bool valid = o < nown;
            int gi[3] = {0, 0, 0};
            float f[3] = {0.0f, 0.0f, 0.0f};
            float qi = 0.0f;
            if (valid) {
                const uint4 cc = own[o];
                grid_coord(cc.x, a.g[0], &gi[0], &f[0]);
                grid_coord(cc.y, a.g[1], &gi[1], &f[1]);
                grid_coord(cc.z, a.g[2], &gi[2], &f[2]);
                qi = __uint_as_float(cc.w);
                // lane lg < 2P: weights and derivatives of stencil point lg, all axes
                if (lg < P2) {
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const float tt = (float)(lg - P + 1) - f[ax];
                        const float w = a.cw[ax] * __expf(-tt * tt * a.hs[ax]);
                        swb[((wave * kGatherOwners + g) * 6 + ax) * P2 + lg] = w;
                        swb[((wave * kGatherOwners + g) * 6 + 3 + ax) * P2 + lg] = w * tt * a.dws[ax];
                    }
                }
            }
            wave_sync();
            float px = 0.0f, py = 0.0f, pz = 0.0f;
            if (valid) {
                const float* W = swb + (wave * kGatherOwners + g) * 6 * P2;   // [6][2P]
                // stencil point k of the charge is halo point (gi - brick origin) + k
                const int lx = gi[0] - X0, ly = gi[1] - Y0, lz = gi[2] - Z0;
                const float* obase = sphi + (lz * E1 + ly) * E0 + lx;
                for (int r = lg; r < P2 * P2; r += LPO) {
                    const int2 rt = rowtab[r];
                    const int ky = rt.y & 0xffff, kz = rt.y >> 16;
                    const float* rowp = obase + rt.x;
                    float sx = 0.0f, dsx = 0.0f;
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        if (PT > 0 || k < P2) {
                            const float v = rowp[k];
                            sx = fmaf(W[k], v, sx);
                            dsx = fmaf(W[3 * P2 + k], v, dsx);
                        }
                    }
                    const float wy = W[P2 + ky], wz = W[2 * P2 + kz];
                    px = fmaf(wy * wz, dsx, px);
                    py = fmaf(W[4 * P2 + ky] * wz, sx, py);
                    pz = fmaf(wy * W[5 * P2 + kz], sx, pz);
                }
            }
            px = LPO == 8 ? sum8(px) : row_sum16(px);
            py = LPO == 8 ? sum8(py) : row_sum16(py);
            pz = LPO == 8 ? sum8(pz) : row_sum16(pz);
            if (valid && lg == 0) {
                const float4 fn = ownf[o];    // near force from the pair kernel
                const int oi = ownp[o];
                forces[3 * oi + 0] = fn.x - qi * px;
                forces[3 * oi + 1] = fn.y - qi * py;
                forces[3 * oi + 2] = fn.z - qi * pz;
            }
            wave_sync();
        }
        __syncthreads();
    }
}

// Block xcd_blocks(nb) (one past the bricks' blocks) forms the energy total:
// it reads only what earlier launches wrote, so it runs beside the bricks.
template <int PT>
__global__ void __launch_bounds__(kGatherThreads) k_gather(int nb,
                                                const int* __restrict__ zbin,
                                                const float* __restrict__ phi,
                                                const uint4* __restrict__ sorted,
                                                const float4* __restrict__ fnear,
                                                const int* __restrict__ perm,
                                                float* __restrict__ forces,
                                                const double* __restrict__ pair_parts,
                                                const double* __restrict__ far_parts,
                                                const double* __restrict__ qstats,
                                                double* __restrict__ energy,
                                                double* __restrict__ parts, GridArgs a,
                                                FinalArgs fa) {
    extern __shared__ char dyn[];
    if ((int)blockIdx.x == xcd_blocks(nb)) {
        energy_total<kGatherThreads>(fa, pair_parts, far_parts, qstats, energy, parts,
                                     reinterpret_cast<double*>(dyn));
        return;
    }
    const int item = xcd_item(blockIdx.x, nb);
    if (item < nb) gather_body<PT>(a, item, sorted, perm, zbin, phi, fnear, forces, dyn);
}

// PT > 0 only when every box of the batch has stencil half width PT
template <int PT>
__global__ void __launch_bounds__(kGatherThreads) k_gather_batch(const BatchTable* __restrict__ tab,
                                                      const BoxDesc* __restrict__ desc) {
    extern __shared__ char dyn[];
    batch_for(tab, BK_GATHER, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        if (item == d.ngb)   // the box's energy total, after its bricks
            energy_total<kGatherThreads>(d.fin, d.pair_parts, d.far_parts, d.qstats,
                                         d.energies + tab->step[i], nullptr,
                                         reinterpret_cast<double*>(dyn));
        else
            gather_body<PT>(d.grid, item, d.sorted, d.perm, d.zbin, d.phi, d.fnear, d.forces,
                            dyn);
    });
}

hipError_t launch_spread(const GridArgs& a, const uint4* sorted, const int* zbin,
                         const double* qstats, float* rho, hipStream_t st) {
    const int nb = ((a.g[0] + kBrick - 1) / kBrick) * ((a.g[1] + kBrick - 1) / kBrick) *
                   ((a.g[2] + kBrick - 1) / kBrick);
    const dim3 grid(xcd_blocks(nb)), block(64 * kSpreadWaves);
    if (a.P == 3)
        hipLaunchKernelGGL(k_spread<3>, grid, block, 0, st, nb, zbin, qstats, sorted, rho, a);
    else if (a.P == 5)
        hipLaunchKernelGGL(k_spread<5>, grid, block, 0, st, nb, zbin, qstats, sorted, rho, a);
    else
        hipLaunchKernelGGL(k_spread<0>, grid, block, 0, st, nb, zbin, qstats, sorted, rho, a);
    return hipGetLastError();
}

int gather_blocks(const GridArgs& a) {
    const int GB = gather_brick(a.P);
    return ((a.g[0] + GB - 1) / GB) * ((a.g[1] + GB - 1) / GB) * ((a.g[2] + GB - 1) / GB);
}

hipError_t launch_gather(const GridArgs& a, const uint4* sorted, const int* perm, const int* zbin,
                         const float* phi, const float4* fnear, float* forces,
                         const FinalArgs& fa, const double* pair_parts, const double* far_parts,
                         const double* qstats, double* energy, double* parts, hipStream_t st) {
    const int nb = gather_blocks(a);
    const dim3 grid(xcd_blocks(nb) + 1), block(kGatherThreads);
    const size_t lds = gather_lds(a.P).total;
    // the default stencils of the two forms (P = 3, 5) have their own code
#define USERIES_GATHER_LAUNCH(PT)                                                            \
    hipLaunchKernelGGL(k_gather<PT>, grid, block, lds, st, nb, zbin, phi, sorted, fnear,     \
                       perm, forces, pair_parts, far_parts, qstats, energy, parts, a, fa)
    if (a.P == 3)
        USERIES_GATHER_LAUNCH(3);
    else if (a.P == 5)
        USERIES_GATHER_LAUNCH(5);
    else
        USERIES_GATHER_LAUNCH(0);
#undef USERIES_GATHER_LAUNCH
    return hipGetLastError();
}

hipError_t launch_spread_batch(const BatchTable* tab, const BoxDesc* desc, int P, int grid,
                               hipStream_t st) {
    const dim3 g(grid), b(64 * kSpreadWaves);
    if (P == 3)
        hipLaunchKernelGGL(k_spread_batch<3>, g, b, 0, st, tab, desc);
    else if (P == 5)
        hipLaunchKernelGGL(k_spread_batch<5>, g, b, 0, st, tab, desc);
    else
        hipLaunchKernelGGL(k_spread_batch<0>, g, b, 0, st, tab, desc);
    return hipGetLastError();
}

size_t gather_lds_bytes(int P) { return (size_t)gather_lds(P).total; }

hipError_t launch_gather_batch(const BatchTable* tab, const BoxDesc* desc, int P, size_t lds,
                               int grid, hipStream_t st) {
    const dim3 g(grid), b(kGatherThreads);
    if (P == 3)
        hipLaunchKernelGGL(k_gather_batch<3>, g, b, lds, st, tab, desc);
    else if (P == 5)
        hipLaunchKernelGGL(k_gather_batch<5>, g, b, lds, st, tab, desc);
    else
        hipLaunchKernelGGL(k_gather_batch<0>, g, b, lds, st, tab, desc);
    return hipGetLastError();
}

}  // namespace useries
