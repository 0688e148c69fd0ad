// Near part of the u-series (eq. 20): for every pair closer than r_c,
//   energy  q_i q_j (1/r - F(r)),
//   force   q_i q_j (1/r^3 + F'(r)/r) (r_i - r_j)  on charge i,
// where F is the infinite far series (eq. 24), represented inside the cutoff
// by a polynomial in x = r^2/r_c^2 fitted on the host in FP64.  For the
// kernels 1/r^6 and 1/r^12 (App. A) the same with 1/r^alpha - F(r) and
// alpha/r^(alpha + 2) + F'(r)/r.
//
// Layout: cluster-pair tiles.  Charges are binned into x-y columns, sorted
// by z, and cut into clusters of up to 8 (see kernels_bin.hip).  One block of
// two wavefronts takes one i-cluster.  Its candidate j-charges are those of
// the columns within r_c of the i-column (x-y gap) lying in the grid z-planes
// that meet the i-cluster's z extent widened by the z reach
// sqrt(r_c^2 - gap^2): per column at most two contiguous ranges of sorted
// charges, read from the column's z-plane index (kernels_bin.hip).  The
// concatenated ranges are walked 8 charges per step: lane (a, b) =
// (lane / 8, lane % 8) holds i-charge a and j-charge b of the step, so every
// lane evaluates one pair per step and no lane waits on another's branch.
// The two wavefronts take alternate chunks of 256 candidates, each loading
// its chunk one chunk ahead (4 consecutive candidates per lane; the range
// of a lane's first one from a per-cluster table of candidate groups, or a
// search when the candidates are many) and staging in LDS only the
// candidates within r_c of the i-cluster's bounding box (about 58% of them
// in water), so the steps skip most pairs that cannot be in range.  The force on
// charge a is summed over its 8 lanes by shuffles, then over the two
// wavefronts in a fixed order.  The one-box kernel is compiled separately for
// cubic cells (where the box test and the pair steps stay in fixed-point
// units) and for other cells; the batched kernel decides per box.
//
// Each ordered pair (i, j) is evaluated once, by i's block (no
// Newton's-third-law sharing), so forces need no atomics and the result does
// not depend on scheduling.
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

namespace {

constexpr int kPairWaves = 2;         // wavefronts per i-cluster
constexpr int kChunk = 32;            // steps of 8 j-charges staged per pass (4 KB of LDS)
constexpr int kChunkCharges = 8 * kChunk;
constexpr int kPerLane = kChunkCharges / 64;   // consecutive candidates loaded per lane
// groups of kPerLane candidates with a range table entry; the block's LDS
// (about 11 KB with it) must stay within 160 KB / 14 blocks, or the kernel
// loses its 7th wavefront per SIMD (a 1024-entry table did: 2.3 us slower)
constexpr int kPairTab = 512;

// a loop-invariant value held in a vector register (lets a polynomial step
// take its two coefficients from one scalar and one vector operand)
__device__ __forceinline__ float to_vgpr(float s) {
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// Polynomial coefficients held in registers (compile-time degree, fully
// unrolled): F = c0 + x P(x) and G = F'(r)/r, each fitted separately in
// FP64 on the host and rounded to FP32.  EXACT: the ne (<= kMaxExact)
// narrowest far terms are not in the polynomials but evaluated as
// Gaussians, a_j 2^(x ex_j) in F and -a_j/s_j^2 2^(x ex_j) in G (small b puts
// them deep inside r_c, where no polynomial of modest degree follows them).
template <int DEG, bool EXACT>
struct Poly {
    float c[DEG + 1];
    float d[DEG + 1];
    int ne;
    float ex[EXACT ? kMaxExact : 1], ea[EXACT ? kMaxExact : 1], eg[EXACT ? kMaxExact : 1];
    // units: the coefficients for distances in fixed-point units u (F u and
    // G u^3, the 1/r kernel in cubic cells)
    __device__ __forceinline__ Poly(const PairArgs& a, bool units) {
#pragma unroll
        for (int m = 0; m <= DEG; ++m) {
            c[m] = units ? a.cu[m] : a.c[m];
            d[m] = units ? a.du[m] : a.d[m];
        }
        ne = a.ne;
        if (EXACT) {
#pragma unroll
            for (int j = 0; j < kMaxExact; ++j) {
                ex[j] = a.ex[j];
                ea[j] = units ? a.eau[j] : a.ea[j];
                eg[j] = units ? a.egu[j] : a.eg[j];
            }
        }
    }
};

// column k of an axis window around the i-column ci and its minimum-image
// distance (in columns) to ci; a full axis (few columns) is walked once, else
// the window has 2R + 1 < nc columns, so one wrap suffices
struct StencilCol {
    int col, d;
};
__device__ __forceinline__ StencilCol stencil_col(int k, int ci, int R, int nc, bool full) {
    if (full) {
        int v = k - ci;
        if (2 * v > nc) v -= nc;
        if (2 * v < -nc) v += nc;
        return {k, v};
    }
    return {wrap1(ci + k - R, nc), k - R};
}

}  // namespace

// Scale terms of the 1/r^6 and 1/r^12 kernels.  A power p of 1/r carries p
// times the relative error of the unit scale, and an FP32 scale is off by up
// to 2^-24: a bias of a few 1e-7 in every pair at p = 12.  These kernels take
// the scale as an FP32 pair (hi + lo) instead: per axis for components in A,
// and (1/u)^2 for distances in fixed-point units.
struct PowScale {
    float lo[3];          // scale_lo per axis (components scaled to A)
    float is2h, is2l;     // (1/u)^2 = is2h + is2l (distances kept in units)
};

// 1/r2 to about half an ulp: the hardware reciprocal and one Newton step
__device__ __forceinline__ float recip_nr(float r2) {
    const float y = __builtin_amdgcn_rcpf(r2);
    return fmaf(y, fmaf(-r2, y, 1.0f), y);
}

// nsteps steps of 8 staged j-charges (st8[s * 8 + ja]) against i-charge ci,
// accumulating sum_j q_j (...) (q_i is applied once, at the end).  CUBIC:
// distance components in fixed-point units u (one scale for all axes), rc2
// and irc2 in those units; for 1/r the polynomials P are those for units
// too (1/r, F in 1/u, G in 1/u^3), for the powers 1/r^2 is taken back to A.
// Otherwise components in A.
template <int DEG, bool CUBIC, bool EXACT, int ALPHA, bool PIPE>
__device__ __forceinline__ void pair_steps(const Poly<DEG, EXACT>& P, const uint4* st8, int ja,
                                           int nsteps,
                                           uint4 ci, float sx, float sy, float sz,
                                           float rc2, float irc2, const PowScale& ps,
                                           float ctop, float dtop,
                                           float& fx, float& fy, float& fz, float& ec) {
    // PIPE: the next step's j-charge is read while this step computes (the
    // stage has 8 spare slots, so the read past the last step stays in
    // bounds); it costs four registers
    uint4 cn = st8[ja];
    for (int s = 0; s < nsteps; ++s) {
        const uint4 cj = PIPE ? cn : st8[s * 8 + ja];
        if (PIPE) cn = st8[(s + 1) * 8 + ja];
        float dx = (float)(int)(ci.x - cj.x), dy = (float)(int)(ci.y - cj.y),
              dz = (float)(int)(ci.z - cj.z);
        if (!CUBIC) {
            if (ALPHA == 1) {
                dx *= sx;
                dy *= sy;
                dz *= sz;
            } else {
                dx = fmaf(dx, sx, dx * ps.lo[0]);
                dy = fmaf(dy, sy, dy * ps.lo[1]);
                dz = fmaf(dz, sz, dz * ps.lo[2]);
            }
        }
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        // a charge of 0 (padding) contributes exactly 0; r2 is then still
        // >= (L / 2^32)^2 (>= 1 in fixed-point units) or 0, never subnormal
        if (r2 < rc2 && r2 > 0.0f) {
            const float qj = __uint_as_float(cj.w);
            const float x = r2 * irc2;
            float Pp = fmaf(ctop, x, P.c[DEG - 1]);
#pragma unroll
            for (int m = DEG - 2; m >= 1; --m) Pp = fmaf(Pp, x, P.c[m]);
            const float Flo = fmaf(Pp, x, P.c[0]);
            float G = fmaf(dtop, x, P.d[DEG - 1]);
#pragma unroll
            for (int m = DEG - 2; m >= 0; --m) G = fmaf(G, x, P.d[m]);
            float Fe = 0.0f;
            if (EXACT) {
#pragma unroll
                for (int j = 0; j < kMaxExact; ++j) {
                    if (j < P.ne) {   // uniform: a scalar branch
                        const float e = __builtin_amdgcn_exp2f(x * P.ex[j]);
                        Fe = fmaf(P.ea[j], e, Fe);
                        G = fmaf(P.eg[j], e, G);
                    }
                }
            }
            float fs;
            if (ALPHA == 1) {
                const float rinv = __builtin_amdgcn_rsqf(r2);
                ec = fmaf(qj, (rinv - Flo) - Fe, ec);
                fs = qj * fmaf(rinv * rinv, rinv, G);
            } else {
                float i2 = recip_nr(r2);                     // 1/r^2 in 1/A^2
                if (CUBIC) i2 = fmaf(i2, ps.is2h, i2 * ps.is2l);
                const float i6 = i2 * i2 * i2;
                const float ip = ALPHA == 12 ? i6 * i6 : i6;
                ec = fmaf(qj, (ip - Flo) - Fe, ec);
                fs = qj * fmaf((float)ALPHA * ip, i2, G);
            }
            fx = fmaf(fs, dx, fx);
            fy = fmaf(fs, dy, fy);
            fz = fmaf(fs, dz, fz);
        }
    }
}

// CM: the cell shape, 1 cubic, 2 other, 0 decided per box at run time (the
// batched kernel); a one-box kernel compiled for one shape holds one chunk loop
template <int DEG, bool EXACT, int ALPHA, bool PIPE, int CM>
__device__ __forceinline__ void pair_body(const PairArgs& a, int I, const uint4* __restrict__ sorted,
                                          const int2* __restrict__ cl_info,
                                          const int* __restrict__ cl_col,
                                          const uint2* __restrict__ cl_z,
                                          const int* __restrict__ zbin,
                                          float4* __restrict__ fnear,
                                          double* __restrict__ epart) {
    __shared__ uint4 stage[kPairWaves][kChunkCharges + 8];
    __shared__ int rbeg[2 * kMaxStencilCols];       // first sorted charge of each non-empty range
    __shared__ int roff[2 * kMaxStencilCols + 1];   // prefix sums of the range lengths
    __shared__ unsigned char rtab[kPairTab];         // range of candidate kPerLane g
    static_assert(2 * kMaxStencilCols <= 256, "range indices fit in a byte");
    __shared__ int wtot[kPairWaves][2];
    __shared__ float4 fother[8];
    __shared__ double eother;
    __shared__ int ibox[6];                          // the i-cluster's box: centre, half extents
    static_assert(kMaxStencilCols <= 64 * kPairWaves, "one stencil column per thread");
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int ia = lane >> 3, ja = lane & 7;
    const int ncx = a.nc[0], ncy = a.nc[1], gz = a.gz;
    // the cluster's records, loaded together (those of a cluster number
    // with no charges are not used); the empty asm takes all three, so that
    // none of the loads is moved past the test below and waited for alone
    const int2 ii = cl_info[I];
    const int C = cl_col[I];                  // cx | cy << 16
    const uint2 zI = cl_z[I];
    asm volatile("" ::"s"(ii.x), "s"(ii.y), "s"(C), "s"(zI.x), "s"(zI.y));
    if (ii.y == 0) {
        if (tid == 0) epart[I] = 0.0;
        return;
    }
    // the i-charges and the cluster's first charge, in flight with the
    // stencil columns' loads below
    const bool ivalid = ia < ii.y;
    const uint4 ci = ivalid ? sorted[ii.x + ia] : make_uint4(0, 0, 0, 0);   // q = 0 if invalid
    const uint4 c0 = sorted[ii.x];
    const int cx = C & 0xffff, cy = C >> 16;
    const bool fullx = 2 * a.R[0] + 1 >= ncx, fully = 2 * a.R[1] + 1 >= ncy;
    const int nxs = fullx ? ncx : 2 * a.R[0] + 1, nys = fully ? ncy : 2 * a.R[1] + 1;
    const int NC = nxs * nys;

    // candidate charge ranges of stencil column k = tid: at most two (the
    // second only where the z window wraps)
    int rb0 = 0, n0 = 0, rb1 = 0, n1 = 0;
    if (tid < NC) {
        // tid < 128, nxs <= 128: (tid + 1/2) / nxs stays 1/256 from an integer,
        // far beyond the reciprocal's error
        const int ky = small_div(tid, __builtin_amdgcn_rcpf((float)nxs));
        const StencilCol sx = stencil_col(tid - ky * nxs, cx, a.R[0], ncx, fullx);
        const StencilCol sy = stencil_col(ky, cy, a.R[1], ncy, fully);
        const int colx = sx.col, coly = sy.col, dx = sx.d, dy = sy.d;
        const float gx = (float)max(0, abs(dx) - 1) * a.cw[0];
        const float gy = (float)max(0, abs(dy) - 1) * a.cw[1];
        const float d2 = gx * gx + gy * gy;
        if (d2 < a.rc2) {
            // grid z-planes of the window [zI.x - rz, zI.y + rz] (fixed point,
            // periodic; rz < 2^31 as r_c < L/2, widened by 1e-6 relative to
            // cover the rounding of the square root and product), then the
            // column's charges of those planes
            const uint32_t rz =
                (uint32_t)(__builtin_amdgcn_sqrtf(a.rc2 - d2) * a.zinv * 1.000001f) + 2u;
            const uint32_t zlo = zI.x - rz, zhi = zI.y + rz;   // modulo 2^32: periodic
            const int zs = (int)__umulhi(zlo, (uint32_t)gz);
            const int zhp = (int)__umulhi(zhi, (uint32_t)gz);
            const bool whole = (uint64_t)(zI.y - zI.x) + 2ull * rz >= (1ull << 32);
            const int len = (zhi >= zlo ? zhp - zs : zhp + gz - zs) + 1;
            const int* zr = zbin + (size_t)(coly * ncx + colx) * (gz + 1);
            if (whole || len >= gz) {
                rb0 = zr[0];
                n0 = zr[gz] - rb0;
            } else {
                const int ze = zs + len;
                rb0 = zr[zs];
                if (ze <= gz) {
                    n0 = zr[ze] - rb0;
                } else {
                    n0 = zr[gz] - rb0;
                    rb1 = zr[0];
                    n1 = zr[ze - gz] - rb1;
                }
            }
        }
    }
    // non-empty ranges stored compactly: exclusive scans over the threads of
    // (ranges, charges), then each thread writes its ranges
    {
        const int m = (n0 > 0) + (n1 > 0), len = n0 + n1;
        const int im = wave_incl_scan(m), il = wave_incl_scan(len);
        if (lane == 63) {
            wtot[w][0] = im;
            wtot[w][1] = il;
        }
        __syncthreads();
        int M = im - m, O = il - len;
        for (int v = 0; v < w; ++v) {
            M += wtot[v][0];
            O += wtot[v][1];
        }
        if (n0 > 0) {
            rbeg[M] = rb0;
            roff[M] = O;
        }
        if (n1 > 0) {
            rbeg[M + (n0 > 0)] = rb1;
            roff[M + (n0 > 0)] = O + n0;
        }
    }
    // bounding box of the i-cluster (fixed point, offsets from its first
    // charge), as a centre and half extents.  Per axis the periodic distance
    // of a candidate from any i-charge is at least its periodic distance from
    // the centre minus the half extent, so a candidate whose such distances
    // put it r_c or more from the box meets no i-charge within r_c and is
    // dropped before the pair steps (the margin covers the FP32 rounding of
    // the test: the pair set is unchanged).  Both wavefronts hold the same
    // i-charges: wavefront 0 forms the box and leaves it in LDS for the
    // barrier below
    if (w == 0) {
        int bl[3], bh[3];
        bl[0] = bh[0] = ivalid ? (int)(ci.x - c0.x) : 0;
        bl[1] = bh[1] = ivalid ? (int)(ci.y - c0.y) : 0;
        bl[2] = bh[2] = ivalid ? (int)(ci.z - c0.z) : 0;
        // extremes over the i-charges (lanes l, l ^ 8, l ^ 16, l ^ 32): the
        // xor-8 partner by a DPP row rotation, the other two by permutes
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            bl[k] = min(bl[k], dpp_move<0x128>(bl[k]));
            bh[k] = max(bh[k], dpp_move<0x128>(bh[k]));
        }
#pragma unroll
        for (int off = 16; off < 64; off <<= 1)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bl[k] = min(bl[k], __shfl_xor(bl[k], off, 64));
                bh[k] = max(bh[k], __shfl_xor(bh[k], off, 64));
            }
        if (lane == 0) {
            ibox[0] = (int)(c0.x + (uint32_t)((bl[0] + bh[0]) / 2));
            ibox[1] = (int)(c0.y + (uint32_t)((bl[1] + bh[1]) / 2));
            ibox[2] = (int)(c0.z + (uint32_t)((bl[2] + bh[2]) / 2));
            ibox[3] = (bh[0] - bl[0]) / 2 + 1;
            ibox[4] = (bh[1] - bl[1]) / 2 + 1;
            ibox[5] = (bh[2] - bl[2]) / 2 + 1;
        }
    }
    int nr = 0, tot = 0;
#pragma unroll
    for (int v = 0; v < kPairWaves; ++v) {
        nr += wtot[v][0];
        tot += wtot[v][1];
    }
    if (tid == 0) roff[nr] = tot;
    __syncthreads();
    const int total = __builtin_amdgcn_readfirstlane(tot);   // uniform: loop bounds in SGPRs
    // the range of each lane's first candidate in a chunk from a table when
    // the candidates are few enough (one LDS read instead of a search)
    const bool tabbed = total <= kPerLane * kPairTab;
    if (tabbed) {
        for (int r = tid; r < nr; r += 64 * kPairWaves) {
            const int g1 = (roff[r + 1] + kPerLane - 1) / kPerLane;
            for (int g = (roff[r] + kPerLane - 1) / kPerLane; g < g1; ++g) rtab[g] = (unsigned char)r;
        }
        __syncthreads();
    }

    // candidates p0 .. p0 + 3 of a chunk (p0 = chunk start + 4 lane), loaded by
    // this lane: one search for the range of p0, then at most one range
    // boundary per step (ranges are non-empty); q = 0 and position 0 past the end
    auto fetch = [&](int c, uint4* out) {
        const int p0 = c * kChunkCharges + kPerLane * lane;
        int r = 0;
        if (p0 < total) {
            if (tabbed) {
                r = rtab[p0 / kPerLane];
            } else {
                int lo = 0, hi = nr;             // range r with roff[r] <= p0 < roff[r + 1]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (roff[mid] <= p0) lo = mid; else hi = mid;
                }
                r = lo;
            }
        }
        int end = roff[r + 1];
        int b = rbeg[r] - roff[r];
#pragma unroll
        for (int u = 0; u < kPerLane; ++u) {
            const int p = p0 + u;
            out[u] = make_uint4(0, 0, 0, 0);
            if (p < total) {
                if (p >= end) {
                    ++r;
                    b = rbeg[r] - roff[r];
                    end = roff[r + 1];
                }
                out[u] = sorted[b + p];
            }
        }
    };

    const float qi = __uint_as_float(ci.w);
    const float sx = a.scale[0], sy = a.scale[1], sz = a.scale[2];
    // cubic cells: distance components stay in fixed-point units u = L / 2^32
    // (the scale folded into r_c^2, x = r^2 / r_c^2, for 1/r into the
    // polynomials, and into the factors applied at the end); otherwise each
    // component is scaled to A
    const bool cubic = CM == 1 || (CM == 0 && sx == sy && sx == sz);
    const bool units = cubic && ALPHA == 1;
    const float isx = a.inv_scale;
    const float rc2w = cubic ? a.rc2 * isx * isx : a.rc2;
    const float irc2w = cubic ? a.inv_rc2 * sx * sx : a.inv_rc2;
    // q_i and the scale of the sums over j: force sum_j q_j (1/r^3 + G) d in
    // 1/u^2 (units), A / u (cubic powers) or A; energy in 1/u or 1/A
    const float ffac = units ? qi * (isx * isx) : (cubic ? qi * sx : qi);
    const double efac = units ? (double)qi * a.inv_scale_d : (double)qi;
    const Poly<DEG, EXACT> P(a, false), Pu(a, ALPHA == 1);
    PowScale ps = {};
    if (ALPHA != 1) {
        ps.lo[0] = a.scale_lo[0];
        ps.lo[1] = a.scale_lo[1];
        ps.lo[2] = a.scale_lo[2];
        ps.is2h = a.is2h;
        ps.is2l = a.is2l;
    }
    const float ctop = to_vgpr(cubic ? Pu.c[DEG] : P.c[DEG]);
    const float dtop = to_vgpr(cubic ? Pu.d[DEG] : P.d[DEG]);

    // the i-cluster's box (formed by wavefront 0 before the range barrier):
    // half extents in fixed-point units; for a kernel compiled for cubic cells
    // the test runs in those units (the reach r_c + margin scaled to them, no
    // per-candidate scaling), otherwise in A per axis
    const uint32_t cenx = (uint32_t)ibox[0], ceny = (uint32_t)ibox[1], cenz = (uint32_t)ibox[2];
    const float hxu = (float)ibox[3], hyu = (float)ibox[4], hzu = (float)ibox[5];
    const float hx = CM == 1 ? hxu : hxu * sx, hy = CM == 1 ? hyu : hyu * sy,
                hz = CM == 1 ? hzu : hzu * sz;
    const float rcm2 = CM == 1 ? a.rcm2 * isx * isx : a.rcm2;
    auto near_box = [&](const uint4& cj) {
        float dx = (float)(int)(cj.x - cenx), dy = (float)(int)(cj.y - ceny),
              dz = (float)(int)(cj.z - cenz);
        if constexpr (CM != 1) {
            dx *= sx;
            dy *= sy;
            dz *= sz;
        }
        const float ex = fmaxf(0.0f, fabsf(dx) - hx);
        const float ey = fmaxf(0.0f, fabsf(dy) - hy);
        const float ez = fmaxf(0.0f, fabsf(dz) - hz);
        return fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rcm2;
    };

    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    double e = 0.0;                      // FP32 pair energies, flushed to FP64 per chunk
    const int nchunks = (total + kChunkCharges - 1) / kChunkCharges;
    uint4 pre[kPerLane];
    if (w < nchunks) fetch(w, pre);
    for (int c = w; c < nchunks; c += kPairWaves) {
        // keep the candidates near the box, compacted in candidate order,
        // padded with zero charges to whole steps of 8
        int kept = 0;
        // candidates from this chunk's start (uniform: the masks below in scalar registers)
        const int rem = __builtin_amdgcn_readfirstlane(total - c * kChunkCharges);
#pragma unroll
        for (int u = 0; u < kPerLane; ++u) {
            // candidate u of lane l (position 4 l + u in the chunk) exists for
            // the first ceil((rem - u) / 4) lanes: a mask in scalar registers;
            // a candidate past the end is the zero record fetch left, tested
            // (no branch) and dropped by the mask.  The ballot of the single
            // compare is the compare's own lane mask, and the store's branch
            // takes the mask back as the lane condition
            const int ru = rem - u;
            const int nl = ru <= 0 ? 0 : min(64, (ru + kPerLane - 1) / kPerLane);
            const uint64_t live = nl >= 64 ? ~0ull : ((1ull << nl) - 1ull);
            const uint64_t m = __builtin_amdgcn_ballot_w64(near_box(pre[u])) & live;
            if (__builtin_amdgcn_inverse_ballot_w64(m)) stage[w][kept + lanes_below(m)] = pre[u];
            kept += __popcll(m);
        }
        if (lane < ((kept + 7) & ~7) - kept) stage[w][kept + lane] = make_uint4(0, 0, 0, 0);
        wave_sync();
        if (c + kPairWaves < nchunks) fetch(c + kPairWaves, pre);   // in flight during the steps
        const int nsteps = (kept + 7) >> 3;
        float ec = 0.0f;
        if (cubic)
            pair_steps<DEG, true, EXACT, ALPHA, PIPE>(Pu, stage[w], ja, nsteps, ci, sx, sx, sx, rc2w,
                                                irc2w, ps, ctop, dtop, fx, fy, fz, ec);
        else
            pair_steps<DEG, false, EXACT, ALPHA, PIPE>(P, stage[w], ja, nsteps, ci, sx, sy, sz, rc2w,
                                                 irc2w, ps, ctop, dtop, fx, fy, fz, ec);
        e += (double)ec;
        wave_sync();
    }
    // force on i-charge a: sum over its 8 lanes, then over the wavefronts
    fx = ffac * sum8(fx);
    fy = ffac * sum8(fy);
    fz = ffac * sum8(fz);
    const double es = wave_sum_d(e * efac);
    if (w == 1) {
        if (ja == 0) fother[ia] = make_float4(fx, fy, fz, 0.0f);
        if (lane == 0) eother = es;
    }
    __syncthreads();
    if (w == 0) {
        if (ja == 0 && ivalid) {
            const float4 o = fother[ia];
            fnear[ii.x + ia] = make_float4(fx + o.x, fy + o.y, fz + o.z, 0.0f);
        }
        // each pair was seen from both ends: half of the summed pair energies
        if (lane == 0) epart[I] = 0.5 * (es + eother);
    }
}

// Held to 72 registers without exact Gaussians (7 wavefronts per SIMD, no
// spill), 80 with them.
template <int DEG, bool EXACT, int ALPHA, bool CUB>
__global__ void __launch_bounds__(64 * kPairWaves)
__attribute__((amdgpu_waves_per_eu(EXACT ? 6 : 7)))
k_pair(int nb, const int2* __restrict__ cl_info, const int* __restrict__ cl_col,
       const uint2* __restrict__ cl_z, const int* __restrict__ zbin,
       const uint4* __restrict__ sorted, float4* __restrict__ fnear, double* __restrict__ epart,
       PairArgs a) {
    const int item = xcd_item(blockIdx.x, nb);
    if (item < nb)
        pair_body<DEG, EXACT, ALPHA, true, CUB ? 1 : 2>(a, item, sorted, cl_info, cl_col, cl_z, zbin,
                                                      fnear, epart);
}

// Held to 80 registers (6 wavefronts per SIMD instead of 5; the variant with
// exact Gaussians then spills about 24 bytes per lane), without the step
// pipelining (its four registers would spill here).
template <int DEG, bool EXACT>
__global__ void __launch_bounds__(64 * kPairWaves) __attribute__((amdgpu_waves_per_eu(6)))
k_pair_batch(const BatchTable* __restrict__ tab,
                                                   const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_PAIR, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        pair_body<DEG, EXACT, 1, false, 0>(d.pair, item, d.sorted, d.cl_info, d.cl_col, d.cl_z, d.zbin,
                                 d.fnear, d.pair_parts);
    });
}

hipError_t launch_pair(const PairArgs& a, int nblocks, const uint4* sorted,
                       const int2* cl_info, const int* cl_col, const uint2* cl_z, const int* zbin,
                       float4* fnear, double* epart, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid(xcd_blocks(nblocks)), block(64 * kPairWaves);
    const bool exact = a.ne > 0;
    // the kernel's test of a cubic cell, made here (the same FP32 comparison)
    const bool cubic = a.scale[0] == a.scale[1] && a.scale[0] == a.scale[2];
    if (a.alpha != 1 && a.alpha != 6 && a.alpha != 12) return hipErrorInvalidValue;
    switch (a.deg) {
#define USERIES_PAIR_LAUNCH(D, E, A)                                                          \
    if (cubic)                                                                                \
        hipLaunchKernelGGL((k_pair<D, E, A, true>), grid, block, 0, st, nblocks, cl_info,     \
                           cl_col, cl_z, zbin, sorted, fnear, epart, a);                      \
    else                                                                                      \
        hipLaunchKernelGGL((k_pair<D, E, A, false>), grid, block, 0, st, nblocks, cl_info,    \
                           cl_col, cl_z, zbin, sorted, fnear, epart, a)
#define USERIES_PAIR_DEG(D)                                                                   \
    case D:                                                                                   \
        if (a.alpha == 6) {                                                                   \
            if (exact) USERIES_PAIR_LAUNCH(D, true, 6);                                       \
            else USERIES_PAIR_LAUNCH(D, false, 6);                                            \
        } else if (a.alpha == 12) {                                                           \
            if (exact) USERIES_PAIR_LAUNCH(D, true, 12);                                      \
            else USERIES_PAIR_LAUNCH(D, false, 12);                                           \
        } else if (exact) {                                                                   \
            USERIES_PAIR_LAUNCH(D, true, 1);                                                  \
        } else {                                                                              \
            USERIES_PAIR_LAUNCH(D, false, 1);                                                 \
        }                                                                                     \
        break;
        USERIES_PAIR_DEG(4) USERIES_PAIR_DEG(5) USERIES_PAIR_DEG(6) USERIES_PAIR_DEG(7)
        USERIES_PAIR_DEG(8) USERIES_PAIR_DEG(9) USERIES_PAIR_DEG(10) USERIES_PAIR_DEG(11)
        USERIES_PAIR_DEG(12) USERIES_PAIR_DEG(13) USERIES_PAIR_DEG(14)
#undef USERIES_PAIR_DEG
#undef USERIES_PAIR_LAUNCH
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pair_batch(const BatchTable* tab, const BoxDesc* desc, int deg, bool exact,
                             int grid, hipStream_t st) {
    switch (deg) {
#define USERIES_PAIR_DEG(D)                                                                   \
    case D:                                                                                   \
        if (exact)                                                                            \
            hipLaunchKernelGGL((k_pair_batch<D, true>), dim3(grid), dim3(64 * kPairWaves), 0, \
                               st, tab, desc);                                                \
        else                                                                                  \
            hipLaunchKernelGGL((k_pair_batch<D, false>), dim3(grid), dim3(64 * kPairWaves),   \
                               0, st, tab, desc);                                             \
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
