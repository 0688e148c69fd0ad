// Separable periodic convolutions of the far part (Sec. V, eqs. 31-32):
//   phi = sum_t K_t^z K_t^y K_t^x rho,
// where K_t^a is the n_a x n_a symmetric circulant of the periodised 1D
// Gaussian of term t (built on the host, amplitude folded into K_t^x).  Each
// 1D convolution is a dense matrix product on the matrix cores (MFMA).
//
// conv_xy: one block per (z plane, term): the plane rho[z] (n_y x n_x) is
//   staged in LDS, U = rho[z] K_t^x, then T_t[z] = K_t^y U is written out.
// conv_z:  one block per 16 grid columns (x, y): phi[:, c] = sum_t K_t^z T_t[:, c],
//   the sum over terms being part of the contraction.
//
// Two arithmetic forms share the structure:
//   FP32   v_mfma_f32_16x16x4_f32;
//   BF16X3 v_mfma_f32_16x16x32_bf16 with both operands split as hi + lo
//          (hi = bf16(v), lo = bf16(v - hi)) and the three products
//          hi*hi + hi*lo + lo*hi accumulated in FP32.
//
// MFMA lane layouts (wave64): for a 16 x 16 output tile, lane l supplies
// A[l % 16][k] and B[k][l % 16], with k = l / 16 (16x16x4 f32) or
// k = 8 (l / 16) + 0..7 (16x16x32 bf16); it receives D[4 (l / 16) + r][l % 16],
// r = 0..3.
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));


__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// round-to-nearest-even float -> bf16 bits (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
    return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ void split(float v, unsigned short* hi, unsigned short* lo) {
    *hi = bf16_bits(v);
    *lo = bf16_bits(v - bf16_val(*hi));
}

__device__ __forceinline__ f32x4 mfma3(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x4 c) {
    c = mfma32(al, bh, c);
    c = mfma32(ah, bl, c);
    return mfma32(ah, bh, c);
}

typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// Staging works on runs of 8 consecutive values of a row (an "octet"): one
// split and one 16-byte LDS store per run.  row[x0 .. x0 + 7], 0 at and past
// n (two 16-byte loads when the run is inside the row and aligned).
__device__ __forceinline__ void load8(const float* __restrict__ row, int x0, int n, float v[8]) {
    if (x0 + 8 <= n && (reinterpret_cast<uintptr_t>(row + x0) & 15) == 0) {
        const float4 a = *reinterpret_cast<const float4*>(row + x0);
        const float4 b = *reinterpret_cast<const float4*>(row + x0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x0 + u < n ? row[x0 + u] : 0.0f;
    }
}

__device__ __forceinline__ void split8(const float v[8], u16x8* hi, u16x8* lo) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        unsigned short h, l;
        split(v[u], &h, &l);
        (*hi)[u] = h;
        (*lo)[u] = l;
    }
}

}  // namespace

// Both forms run blocks of eight wavefronts.  In each product wavefront w owns
// the output tile column w mod n_tiles (and, when n_tiles divides 8, every
// G-th of its strips, G = 8 / n_tiles) and keeps the matching fragments of
// the constant matrix in registers for the whole item, loaded together with
// the staging of the grid operand, so the MFMA loops read only LDS and
// registers.
constexpr int kConvWaves = 8;
constexpr int kConvThreads = 64 * kConvWaves;

// wavefronts sharing one output tile column when `tiles` divides kConvWaves
// (they split that column's strips), else 1
__host__ __device__ inline int tile_groups(int tiles) {
    return (tiles <= kConvWaves && kConvWaves % tiles == 0) ? kConvWaves / tiles : 1;
}

// ------------------------------------------------------------------ FP32

// The contraction index of a 16x16x4 step is permuted so that every operand
// is read as a float4: in k-chunk j (16 values) lane group lk supplies
// k = 16 j + 4 lk + e at the chunk's step e = 0..3.
constexpr int kMaxChunks = kMaxGrid / 16;

struct Frag32 {
    f32x4 v[kMaxChunks];
};

// rows tile*16 + li of the row-major gp x gp matrix m, in the chunk order above
__device__ __forceinline__ void load_frag32(Frag32& f, const float* __restrict__ m, int gp,
                                            int tile, int li, int lk) {
#pragma unroll
    for (int j = 0; j < kMaxChunks; ++j)
        if (16 * j < gp)
            f.v[j] = *reinterpret_cast<const f32x4*>(m + (size_t)(tile * 16 + li) * gp + 16 * j +
                                                     4 * lk);
}

__device__ __forceinline__ f32x4 mfma_chunk(f32x4 a, f32x4 b, f32x4 c) {
    c = mfma4(a[0], b[0], c);
    c = mfma4(a[1], b[1], c);
    c = mfma4(a[2], b[2], c);
    return mfma4(a[3], b[3], c);
}

// plane z, term t; smem: the dynamic LDS (conv_xy_lds_bytes).  The plane is
// staged as [y][x]; U = rho Kx is kept transposed ([x][y]) so that both
// products read their LDS operand along the contraction index.
__device__ __forceinline__ void conv_xy_f32_body(const ConvArgs& a, int z, int t, float* smem,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ kx,
                                                 const float* __restrict__ ky,
                                                 float* __restrict__ tgrid) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int g0 = a.g[0], g1 = a.g[1], p0 = a.gp[0], p1 = a.gp[1];
    const int ld = (p0 > p1 ? p0 : p1) + 4;     // floats per LDS row
    float* rp = smem;                            // [p1][ld] rho plane
    float* ut = rp + p1 * ld;                    // [p0][ld] U^T
    const int tx_n = p0 / 16, ty_n = p1 / 16;
    const int G1 = tile_groups(tx_n), G2 = tile_groups(ty_n);
    const bool act1 = w < tx_n * G1, act2 = w < ty_n * G2;
    const int tx = w % tx_n, s0 = w / tx_n;      // U = rho Kx: column tile, first strip
    const int ty = w % ty_n, c0 = w / ty_n;      // T = Ky U: row tile, first column strip
    // B of U = rho Kx: Kx[j][k] (Kx symmetric); A of T = Ky U: Ky rows
    Frag32 bx, ay;
    if (act1) load_frag32(bx, kx + (size_t)p0 * p0 * t, p0, tx, li, lk);
    if (act2) load_frag32(ay, ky + (size_t)p1 * p1 * t, p1, ty, li, lk);
    const float* src = rho + (size_t)z * g1 * g0;
    // octets of the padded plane, two per thread per pass (loads first)
    const int no = p1 * (p0 / 8);
    const float iq = __builtin_amdgcn_rcpf((float)(p0 / 8));   // small_div: ample margin
    for (int o0 = threadIdx.x; o0 < no; o0 += 2 * kConvThreads) {
        float v[2][8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = o0 + u * kConvThreads;
            const int y = small_div(o, iq), x0 = 8 * (o - y * (p0 / 8));
            if (o < no && y < g1) load8(src + (size_t)y * g0, x0, g0, v[u]);
            else
#pragma unroll
                for (int e = 0; e < 8; ++e) v[u][e] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = o0 + u * kConvThreads;
            const int y = small_div(o, iq), x0 = 8 * (o - y * (p0 / 8));
            if (o < no) {
                float* d = rp + y * ld + x0;
                *reinterpret_cast<float4*>(d) = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
                *reinterpret_cast<float4*>(d + 4) = make_float4(v[u][4], v[u][5], v[u][6], v[u][7]);
            }
        }
    }
    __syncthreads();
    if (act1)
        for (int s = s0; s < ty_n; s += G1) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* ar = rp + (s * 16 + li) * ld + 4 * lk;
#pragma unroll
            for (int j = 0; j < kMaxChunks; ++j)
                if (16 * j < p0)
                    acc = mfma_chunk(*reinterpret_cast<const f32x4*>(ar + 16 * j), bx.v[j], acc);
            // acc[r] = U[s*16 + 4 lk + r][tx*16 + li]
            *reinterpret_cast<f32x4*>(ut + (tx * 16 + li) * ld + s * 16 + 4 * lk) = acc;
        }
    __syncthreads();
    float* dst = tgrid + ((size_t)t * a.g[2] + z) * g1 * g0;
    if (act2)
        for (int c = c0; c < tx_n; c += G2) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* br = ut + (c * 16 + li) * ld + 4 * lk;
#pragma unroll
            for (int j = 0; j < kMaxChunks; ++j)
                if (16 * j < p1)
                    acc = mfma_chunk(ay.v[j], *reinterpret_cast<const f32x4*>(br + 16 * j), acc);
            const int x = c * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = ty * 16 + 4 * lk + r;
                if (y < g1 && x < g0) dst[y * g0 + x] = acc[r];
            }
        }
}

// wavefront groups of a conv_z block (each takes every G-th term)
__host__ __device__ inline int conv_z_groups(const ConvArgs& a) {
    return tile_groups(a.gp[2] / 16);
}

// Terms whose 16 columns a conv_z block stages in LDS at once: all of them
// when they fit in 20 KiB, else the largest multiple of the group count that
// does (at least one).  A staged column takes 4 bytes per z' in both forms
// (FP32, or BF16 hi + lo), rows padded by 4 (FP32) or 8 (BF16) values.
__host__ __device__ inline int conv_z_chunk(const ConvArgs& a) {
    const int per = 16 * (a.gp[2] + (a.bf16x3 ? 8 : 4)) * 4;
    const int G = conv_z_groups(a);
    int tc = (20 * 1024) / per;
    if (tc >= a.nterms) return a.nterms;
    tc -= tc % G;
    return tc > 0 ? tc : 1;
}

// wavefront partial sums of groups 1 .. G-1 added to group 0's, in group order
__device__ __forceinline__ f32x4 conv_z_reduce(f32x4 acc, float* smem, bool act, int grp, int G,
                                               int tz, int tz_n, int l) {
    __syncthreads();
    f32x4* red = reinterpret_cast<f32x4*>(smem);
    if (act && grp > 0) red[((grp - 1) * tz_n + tz) * 64 + l] = acc;
    __syncthreads();
    if (act && grp == 0)
        for (int g = 1; g < G; ++g) {
            const f32x4 o = red[((g - 1) * tz_n + tz) * 64 + l];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] += o[r];
        }
    return acc;
}

// Output of a conv_z wavefront of group 0: phi at rows tz 16 + 4 lk + r of
// columns c0 + li (the spectral part ps added), written to the grid, and the
// wavefront's share of the far energy, sum rho phi over those points in FP64
// (products of FP32 values, exact in FP64), to fpart[bid tz_n + tz].
// rho at the points a wavefront of group 0 writes, loaded when the block
// starts (off the end of the block's dependency chain)
__device__ __forceinline__ f32x4 conv_z_rho(const ConvArgs& a, int tz, int li, int lk, int c0,
                                            const float* __restrict__ rho) {
    const int g2 = a.g[2], ncol = a.g[0] * a.g[1];
    const int col = c0 + li;
    f32x4 v = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int zz = tz * 16 + 4 * lk + r;
        if (zz < g2 && col < ncol) v[r] = rho[(size_t)zz * ncol + col];
    }
    return v;
}

__device__ __forceinline__ void conv_z_store(const ConvArgs& a, int bid, int tz, int li, int lk,
                                             int c0, f32x4 acc, const float* ps, f32x4 rv,
                                             float* __restrict__ phi, double* __restrict__ fpart) {
    const int g2 = a.g[2], ncol = a.g[0] * a.g[1];
    const int col = c0 + li;
    double e = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int zz = tz * 16 + 4 * lk + r;
        if (zz < g2 && col < ncol) {
            const size_t o = (size_t)zz * ncol + col;
            const float v = ps ? acc[r] + ps[li * g2 + zz] : acc[r];
            phi[o] = v;
            e = fma((double)rv[r], (double)v, e);
        }
    }
    e = wave_sum_d(e);
    if (fpart && threadIdx.x % 64 == 0) fpart[bid * (a.gp[2] / 16) + tz] = e;
}

// phi[:, c] = sum_t Kz_t T_t[:, c] for the block's 16 grid columns c.  The
// columns of a chunk of terms are staged transposed ([t][col][z']); the
// wavefronts form G groups, in a group wavefront w owns row tile w mod n_tiles
// and the group takes the chunk's terms grp, grp + G, ..., loading the Kz
// fragment of its next term while it multiplies the current one.
__device__ __forceinline__ void conv_z_f32_body(const ConvArgs& a, int bid, float* smem,
                                                const float* __restrict__ tgrid,
                                                const float* __restrict__ kz,
                                                float* __restrict__ phi,
                                                const float* __restrict__ rho,
                                                double* __restrict__ fpart,
                                                const float* ps = nullptr,
                                                bool straight = true) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int g2 = a.g[2], p2 = a.gp[2], ld = p2 + 4;
    const int ncol = a.g[0] * a.g[1];
    const int tz_n = p2 / 16, G = conv_z_groups(a);
    const int cb = bid * 16;
    const bool act = w < tz_n * G;
    const int tz = w % tz_n, grp = w / tz_n;
    const size_t mz = (size_t)p2 * p2;
    const int tc = conv_z_chunk(a);
    const float iq8 = __builtin_amdgcn_rcpf((float)(p2 / 8));   // small_div: ample margin
    const f32x4 rv = (act && grp == 0) ? conv_z_rho(a, tz, li, lk, cb, rho)
                                       : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // one chunk of terms; with a single chunk and a single staging pass (the
    // usual case) and `straight`, no loop is emitted, so that the loads of
    // rho, of the Kz fragments and of the columns are all in flight together
    // (the batched kernel keeps the loops: the straight copy would cost it
    // registers and a resident block per CU)
    auto chunk = [&](int t0) {
        const int nt = (a.nterms - t0 < tc) ? a.nterms - t0 : tc;
        Frag32 cur, nxt;
        if (act && grp < nt) load_frag32(cur, kz + mz * (t0 + grp), p2, tz, li, lk);
        if (t0 > 0) __syncthreads();     // the previous chunk's columns are consumed
        // octets (t, column c, z' = 8 zb .. 8 zb + 7): 8 loads down the
        // column (each coalesced over the 16 columns), two 16-byte stores
        auto stage = [&](int o) {
            const int c = o & 15, q8 = o >> 4;
            const int t = small_div(q8, iq8), zb = q8 - t * (p2 / 8);
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int zp = 8 * zb + u;
                v[u] = (zp < g2 && cb + c < ncol)
                           ? tgrid[((size_t)(t0 + t) * g2 + zp) * ncol + cb + c]
                           : 0.0f;
            }
            float* d = smem + (t * 16 + c) * ld + 8 * zb;
            *reinterpret_cast<float4*>(d) = make_float4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<float4*>(d + 4) = make_float4(v[4], v[5], v[6], v[7]);
        };
        const int no = nt * 16 * (p2 / 8);
        if (straight && no <= kConvThreads) {
            if ((int)threadIdx.x < no) stage(threadIdx.x);
        } else {
            for (int o = threadIdx.x; o < no; o += kConvThreads) stage(o);
        }
        __syncthreads();
        if (act)
            for (int t = grp; t < nt; t += G) {
                if (t + G < nt) load_frag32(nxt, kz + mz * (t0 + t + G), p2, tz, li, lk);
                const float* br = smem + (t * 16 + li) * ld + 4 * lk;
#pragma unroll
                for (int j = 0; j < kMaxChunks; ++j)
                    if (16 * j < p2)
                        acc = mfma_chunk(cur.v[j], *reinterpret_cast<const f32x4*>(br + 16 * j), acc);
                cur = nxt;
            }
    };
    if (straight && a.nterms <= tc) {
        chunk(0);
    } else {
        for (int t0 = 0; t0 < a.nterms; t0 += tc) chunk(t0);
    }
    if (G > 1) acc = conv_z_reduce(acc, smem, act, grp, G, tz, tz_n, l);
    if (!act || grp != 0) return;
    conv_z_store(a, bid, tz, li, lk, cb, acc, ps, rv, phi, fpart);
}

// ------------------------------------------------------------------ BF16X3

// kx/ky/kz hold, per term, the hi matrix followed by the lo matrix (bf16 bits).
//
constexpr int kMaxKSteps = kMaxGrid / 32;   // K steps of 32 (BF16 MFMA)

struct Frag {
    u16x8 h[kMaxKSteps], l[kMaxKSteps];
};

// fragment of rows tile*16 + li, k = 32 ks + 8 lk .. + 7, of the gp x gp
// matrices mh / ml (row-major)
__device__ __forceinline__ void load_frag(Frag& f, const unsigned short* __restrict__ mh,
                                          const unsigned short* __restrict__ ml, int gp, int tile,
                                          int li, int lk) {
#pragma unroll
    for (int ks = 0; ks < kMaxKSteps; ++ks) {
        if (32 * ks < gp) {
            const size_t o = (size_t)(tile * 16 + li) * gp + 32 * ks + 8 * lk;
            f.h[ks] = *reinterpret_cast<const u16x8*>(mh + o);
            f.l[ks] = *reinterpret_cast<const u16x8*>(ml + o);
        }
    }
}

__device__ __forceinline__ void conv_xy_bf16_body(const ConvArgs& a, int z, int t, float* smem,
                                                  const float* __restrict__ rho,
                                                  const unsigned short* __restrict__ kx,
                                                  const unsigned short* __restrict__ ky,
                                                  float* __restrict__ tgrid) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int g0 = a.g[0], g1 = a.g[1], p0 = a.gp[0], p1 = a.gp[1];
    const int ldb = (p0 > p1 ? p0 : p1) + 8;            // bf16 elements per LDS row
    unsigned short* ph = reinterpret_cast<unsigned short*>(smem);   // [p1][ldb] rho hi
    unsigned short* pl = ph + p1 * ldb;                              // rho lo
    unsigned short* uh = pl + p1 * ldb;                              // [p0][ldb] U^T hi
    unsigned short* ul = uh + p0 * ldb;                              // U^T lo
    const size_t mx = (size_t)p0 * p0, my = (size_t)p1 * p1;
    const int tx_n = p0 / 16, ty_n = p1 / 16;
    const int G1 = tile_groups(tx_n), G2 = tile_groups(ty_n);
    const bool act1 = w < tx_n * G1, act2 = w < ty_n * G2;
    const int tx = w % tx_n, s0 = w / tx_n;      // U = rho Kx: column tile, first strip
    const int ty = w % ty_n, c0 = w / ty_n;      // T = Ky U: row tile, first column strip
    // B of U = rho Kx: Kx[j][k] (Kx symmetric); A of T = Ky U: Ky rows
    Frag bx, ay;
    if (act1) load_frag(bx, kx + 2 * mx * t, kx + 2 * mx * t + mx, p0, tx, li, lk);
    if (act2) load_frag(ay, ky + 2 * my * t, ky + 2 * my * t + my, p1, ty, li, lk);
    const float* src = rho + (size_t)z * g1 * g0;
    // octets of the padded plane, two per thread per pass (loads first)
    const int no = p1 * (p0 / 8);
    const float iq = __builtin_amdgcn_rcpf((float)(p0 / 8));   // small_div: ample margin
    for (int o0 = threadIdx.x; o0 < no; o0 += 2 * kConvThreads) {
        float v[2][8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = o0 + u * kConvThreads;
            const int y = small_div(o, iq), x0 = 8 * (o - y * (p0 / 8));
            if (o < no && y < g1) load8(src + (size_t)y * g0, x0, g0, v[u]);
            else
#pragma unroll
                for (int e = 0; e < 8; ++e) v[u][e] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = o0 + u * kConvThreads;
            const int y = small_div(o, iq), x0 = 8 * (o - y * (p0 / 8));
            if (o < no) {
                u16x8 h, lo;
                split8(v[u], &h, &lo);
                *reinterpret_cast<u16x8*>(ph + y * ldb + x0) = h;
                *reinterpret_cast<u16x8*>(pl + y * ldb + x0) = lo;
            }
        }
    }
    __syncthreads();
    // U = rho Kx: tiles (strip s, column tile tx); U stored transposed, split
    if (act1)
        for (int s = s0; s < ty_n; s += G1) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < kMaxKSteps; ++ks) {
                if (32 * ks < p0) {
                    const int ao = (s * 16 + li) * ldb + 32 * ks + 8 * lk;
                    const u16x8 ah = *reinterpret_cast<const u16x8*>(ph + ao);
                    const u16x8 al = *reinterpret_cast<const u16x8*>(pl + ao);
                    acc = mfma3(ah, al, bx.h[ks], bx.l[ks], acc);
                }
            }
            u16x4 h4, l4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                unsigned short h, lo;
                split(acc[r], &h, &lo);
                h4[r] = h;
                l4[r] = lo;
            }
            const int o = (tx * 16 + li) * ldb + s * 16 + 4 * lk;
            *reinterpret_cast<u16x4*>(uh + o) = h4;
            *reinterpret_cast<u16x4*>(ul + o) = l4;
        }
    __syncthreads();
    // T = Ky U: tiles (row tile ty, column strip c); B[k][j] = U^T[x][y']
    float* dst = tgrid + ((size_t)t * a.g[2] + z) * g1 * g0;
    if (act2)
        for (int c = c0; c < tx_n; c += G2) {
            const int x = c * 16 + li;
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < kMaxKSteps; ++ks) {
                if (32 * ks < p1) {
                    const int bo = (c * 16 + li) * ldb + 32 * ks + 8 * lk;
                    const u16x8 bh = *reinterpret_cast<const u16x8*>(uh + bo);
                    const u16x8 bl = *reinterpret_cast<const u16x8*>(ul + bo);
                    acc = mfma3(ay.h[ks], ay.l[ks], bh, bl, acc);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int y = ty * 16 + 4 * lk + r;
                if (y < g1 && x < g0) dst[y * g0 + x] = acc[r];
            }
        }
}

// phi[:, c] = sum_t Kz_t T_t[:, c] for the block's 16 grid columns c, as in
// the FP32 form: the columns of a chunk of terms are staged (transposed to
// [col][z'], split); the wavefronts form G groups, in a group wavefront w owns
// row tile w mod n_tiles and the group takes the chunk's terms grp, grp + G,
// ..., loading the Kz fragment of its next term while it multiplies the
// current one.  The groups' partial sums are added in group order through LDS.
__device__ __forceinline__ void conv_z_bf16_body(const ConvArgs& a, int bid, float* smem,
                                                 const float* __restrict__ tgrid,
                                                 const unsigned short* __restrict__ kz,
                                                 float* __restrict__ phi,
                                                 const float* __restrict__ rho,
                                                 double* __restrict__ fpart,
                                                 const float* ps = nullptr,
                                                 bool straight = true) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 15, lk = l >> 4;
    const int g2 = a.g[2], p2 = a.gp[2], ld = p2 + 8;
    const int ncol = a.g[0] * a.g[1];
    const int tz_n = p2 / 16, G = tile_groups(tz_n);
    const int c0 = bid * 16;
    const bool act = w < tz_n * G;
    const int tz = w % tz_n, grp = w / tz_n;
    const size_t mz = (size_t)p2 * p2;
    const int tc = conv_z_chunk(a);
    const float iq8 = __builtin_amdgcn_rcpf((float)(p2 / 8));   // small_div: ample margin
    unsigned short* th = reinterpret_cast<unsigned short*>(smem);   // [t][16][ld] hi
    unsigned short* tl = th + (size_t)tc * 16 * ld;                 // lo
    const f32x4 rv = (act && grp == 0) ? conv_z_rho(a, tz, li, lk, c0, rho)
                                       : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // one chunk of terms; with a single chunk and a single staging pass (the
    // usual case) and `straight`, no loop is emitted, so that the loads of
    // rho, of the Kz fragments and of the columns are all in flight together
    // (the batched kernel keeps the loops: the straight copy would cost it
    // registers and a resident block per CU)
    auto chunk = [&](int t0) {
        const int nt = (a.nterms - t0 < tc) ? a.nterms - t0 : tc;
        Frag cur, nxt;
        if (act && grp < nt)
            load_frag(cur, kz + 2 * mz * (t0 + grp), kz + 2 * mz * (t0 + grp) + mz, p2, tz, li, lk);
        if (t0 > 0) __syncthreads();     // the previous chunk's columns are consumed
        // octets (t, column c, z' = 8 zb .. 8 zb + 7): 8 loads down the
        // column (each coalesced over the 16 columns), one split, two
        // 16-byte stores
        auto stage = [&](int o) {
            const int c = o & 15, q8 = o >> 4;
            const int t = small_div(q8, iq8), zb = q8 - t * (p2 / 8);
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int zp = 8 * zb + u;
                v[u] = (zp < g2 && c0 + c < ncol)
                           ? tgrid[((size_t)(t0 + t) * g2 + zp) * ncol + c0 + c]
                           : 0.0f;
            }
            u16x8 h, lo;
            split8(v, &h, &lo);
            *reinterpret_cast<u16x8*>(th + (t * 16 + c) * ld + 8 * zb) = h;
            *reinterpret_cast<u16x8*>(tl + (t * 16 + c) * ld + 8 * zb) = lo;
        };
        const int no = nt * 16 * (p2 / 8);
        if (straight && no <= kConvThreads) {
            if ((int)threadIdx.x < no) stage(threadIdx.x);
        } else {
            for (int o = threadIdx.x; o < no; o += kConvThreads) stage(o);
        }
        __syncthreads();
        if (act)
            for (int t = grp; t < nt; t += G) {
                if (t + G < nt)
                    load_frag(nxt, kz + 2 * mz * (t0 + t + G), kz + 2 * mz * (t0 + t + G) + mz, p2,
                              tz, li, lk);
                const unsigned short* bhp = th + (t * 16 + li) * ld + 8 * lk;
                const unsigned short* blp = tl + (t * 16 + li) * ld + 8 * lk;
#pragma unroll
                for (int ks = 0; ks < kMaxKSteps; ++ks) {
                    if (32 * ks < p2) {
                        const u16x8 bh = *reinterpret_cast<const u16x8*>(bhp + 32 * ks);
                        const u16x8 bl = *reinterpret_cast<const u16x8*>(blp + 32 * ks);
                        acc = mfma3(cur.h[ks], cur.l[ks], bh, bl, acc);
                    }
                }
                cur = nxt;
            }
    };
    if (straight && a.nterms <= tc) {
        chunk(0);
    } else {
        for (int t0 = 0; t0 < a.nterms; t0 += tc) chunk(t0);
    }
    if (G > 1) acc = conv_z_reduce(acc, smem, act, grp, G, tz, tz_n, l);
    if (!act || grp != 0) return;
    conv_z_store(a, bid, tz, li, lk, c0, acc, ps, rv, phi, fpart);
}

// ------------------------------------------------------------------ spectral wide terms
// The widest terms together as (U_z x U_y x U_x) diag(W) (U_z x U_y x U_x)^T rho
// (ConvArgs::spec), in three steps, FP32 FMAs (a few hundred thousand per
// step: no matrix cores needed):
//   conv_xy, one extra block per plane:  C[z] = U_y^T rho[z] U_x        (r_y x r_x)
//   spec_core, once:                     G = W o (sum_z U_z[z] C[z])     (r_z x r_y x r_x)
//   conv_z, in each column block:        phi[z, c] += sum U_z[z] U_y[y_c] U_x[x_c] G

// C[z] from the plane rho[z]; smem holds g_y g_x + g_y r_x + g_x r_x + g_y r_y floats
__device__ __forceinline__ void spec_fwd_plane(const ConvArgs& a, int z, float* smem,
                                               const float* __restrict__ rho, const SpecPtrs& sp) {
    const int g0 = a.g[0], g1 = a.g[1], r0 = a.rk[0], r1 = a.rk[1];
    const int t = threadIdx.x;
    float* sr = smem;              // rho[z] as [y][x]
    float* pp = sr + g1 * g0;      // P = rho[z] U_x as [y][ix]
    float* ux = pp + g1 * r0;      // U_x [x][ix]
    float* uy = ux + g0 * r0;      // U_y [y][iy]
    const float* src = rho + (size_t)z * g1 * g0;
    for (int i = t; i < g1 * g0; i += kConvThreads) sr[i] = src[i];
    for (int i = t; i < g0 * r0; i += kConvThreads) ux[i] = sp.ux[i];
    for (int i = t; i < g1 * r1; i += kConvThreads) uy[i] = sp.uy[i];
    __syncthreads();
    for (int o = t; o < g1 * r0; o += kConvThreads) {
        const int y = o / r0, ix = o - y * r0;
        const float* row = sr + y * g0;
        float acc0 = 0.0f, acc1 = 0.0f;
        int x = 0;
        for (; x + 1 < g0; x += 2) {
            acc0 = fmaf(row[x], ux[x * r0 + ix], acc0);
            acc1 = fmaf(row[x + 1], ux[(x + 1) * r0 + ix], acc1);
        }
        if (x < g0) acc0 = fmaf(row[x], ux[x * r0 + ix], acc0);
        pp[o] = acc0 + acc1;
    }
    __syncthreads();
    for (int o = t; o < r1 * r0; o += kConvThreads) {
        const int iy = o / r0, ix = o - iy * r0;
        float acc0 = 0.0f, acc1 = 0.0f;
        int y = 0;
        for (; y + 1 < g1; y += 2) {
            acc0 = fmaf(uy[y * r1 + iy], pp[y * r0 + ix], acc0);
            acc1 = fmaf(uy[(y + 1) * r1 + iy], pp[(y + 1) * r0 + ix], acc1);
        }
        if (y < g1) acc0 = fmaf(uy[y * r1 + iy], pp[y * r0 + ix], acc0);
        sp.c[(size_t)z * r1 * r0 + o] = acc0 + acc1;
    }
}

// G = W o (U_z^T C).  A block takes 16 consecutive outputs (iz, o): thread
// (slice, j) adds the planes z = slice, slice + 16, ... of output j (one
// round of independent loads, 16 consecutive o per row of lanes), and the 16
// slices are then summed in a fixed order.
constexpr int kSpecCoreThreads = 256;
__global__ void __launch_bounds__(kSpecCoreThreads) k_spec_core(float* __restrict__ g, ConvArgs a,
                                                               SpecPtrs sp) {
    __shared__ float red[16][17];
    const int R = a.rk[1] * a.rk[0], r2 = a.rk[2], g2 = a.g[2];
    const int j = threadIdx.x & 15, slice = threadIdx.x >> 4;
    const int idx = blockIdx.x * 16 + j;
    const bool valid = idx < r2 * R;
    const int iz = valid ? idx / R : 0, o = valid ? idx - iz * R : 0;
    constexpr int kMaxPer = kMaxGrid / 16;
    float c[kMaxPer], u[kMaxPer];
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const int z = slice + 16 * k;
        const bool in = valid && z < g2;
        c[k] = in ? sp.c[(size_t)z * R + o] : 0.0f;
        u[k] = in ? sp.uz[z * r2 + iz] : 0.0f;
    }
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) acc = fmaf(u[k], c[k], acc);
    red[slice][j] = acc;
    __syncthreads();
    if (threadIdx.x < 16 && valid) {
        float sum = 0.0f;
        for (int sl = 0; sl < 16; ++sl) sum += red[sl][threadIdx.x];
        g[idx] = sp.w[idx] * sum;
    }
}

// rows of the block's 16 columns (consecutive, x fastest) for grid rows of g_x points
__host__ __device__ inline int spec_rows(int gx) { return 15 / gx + 2; }

// floats of LDS a conv_z block needs for the spectral part (0 without it)
__host__ __device__ inline int spec_z_lds_floats(const ConvArgs& a) {
    if (!a.spec) return 0;
    const int r0 = a.rk[0], r1 = a.rk[1], r2 = a.rk[2];
    return r2 * r1 * r0 + spec_rows(a.g[0]) * r2 * r0 + r2 * 16 + 16 * a.g[2] + a.g[0] * r0 +
           a.g[2] * r2;
}

// the spectral terms' potential on the block's 16 columns, left in LDS as
// ps[c][z] (returned); ls: spec_z_lds_floats(a) floats.  The columns share
// at most spec_rows(g_x) grid rows y, so G is first contracted with U_y for
// those rows only.
__device__ __forceinline__ const float* spec_z_part(const ConvArgs& a, int bid, float* ls,
                                                    const float* __restrict__ g,
                                                    const SpecPtrs& sp) {
    const int g0 = a.g[0], g2 = a.g[2], r0 = a.rk[0], r1 = a.rk[1], r2 = a.rk[2];
    const int ncol = a.g[0] * a.g[1], cb = bid * 16, t = threadIdx.x;
    const int nG = r2 * r1 * r0;
    const int y0 = cb / g0, cl = min(cb + 15, ncol - 1), ny = cl / g0 - y0 + 1;
    float* sg = ls;                                  // G [iz][iy][ix]
    float* gy = sg + nG;                             // [jy][iz][ix], y = y0 + jy
    float* sh = gy + spec_rows(g0) * r2 * r0;        // H [iz][c]
    float* ps = sh + r2 * 16;                        // [c][z]
    float* ux = ps + 16 * g2;                        // U_x [x][ix]
    float* uz = ux + g0 * r0;                        // U_z [z][iz]
    for (int i = t; i < nG; i += kConvThreads) sg[i] = g[i];
    for (int i = t; i < g0 * r0; i += kConvThreads) ux[i] = sp.ux[i];
    for (int i = t; i < g2 * r2; i += kConvThreads) uz[i] = sp.uz[i];
    __syncthreads();
    for (int o = t; o < ny * r2 * r0; o += kConvThreads) {
        const int jy = o / (r2 * r0), rem = o - jy * r2 * r0;
        const int iz = rem / r0, ix = rem - iz * r0;
        const float* uyr = sp.uy + (size_t)(y0 + jy) * r1;
        float acc = 0.0f;
        for (int iy = 0; iy < r1; ++iy) acc = fmaf(uyr[iy], sg[(iz * r1 + iy) * r0 + ix], acc);
        gy[o] = acc;
    }
    __syncthreads();
    for (int o = t; o < r2 * 16; o += kConvThreads) {
        const int iz = o >> 4, cc = o & 15, col = cb + cc;
        float acc = 0.0f;
        if (col < ncol) {
            const int y = col / g0, x = col - y * g0;
            const float* gr = gy + ((y - y0) * r2 + iz) * r0;
            for (int ix = 0; ix < r0; ++ix) acc = fmaf(ux[x * r0 + ix], gr[ix], acc);
        }
        sh[o] = acc;
    }
    __syncthreads();
    for (int o = t; o < 16 * g2; o += kConvThreads) {
        const int cc = o / g2, z = o - cc * g2;
        float acc = 0.0f;
        for (int iz = 0; iz < r2; ++iz) acc = fmaf(uz[z * r2 + iz], sh[iz * 16 + cc], acc);
        ps[o] = acc;
    }
    __syncthreads();
    return ps;
}

// ------------------------------------------------------------------ kernels

// blockIdx.y == a.nterms (only with spectral terms): the plane's projection
__global__ void __launch_bounds__(kConvThreads) k_conv_xy_f32(const float* __restrict__ rho,
                                                     const float* __restrict__ kx,
                                                     const float* __restrict__ ky,
                                                     float* __restrict__ tgrid, ConvArgs a,
                                                     SpecPtrs sp) {
    extern __shared__ float dyn_lds[];
    if ((int)blockIdx.y == a.nterms) {
        spec_fwd_plane(a, blockIdx.x, dyn_lds, rho, sp);
        return;
    }
    conv_xy_f32_body(a, blockIdx.x, blockIdx.y, dyn_lds, rho, kx, ky, tgrid);
}

// conv_z launches take xcd_blocks(nb) blocks: neighbouring column groups,
// which share 128-byte lines of T, then run on one XCD and share its L2.
// With spectral terms the dynamic LDS holds the dense staging and then the
// spectral part (from float offset spec_off).
__global__ void __launch_bounds__(kConvThreads) k_conv_z_f32(int nb, int spec_off,
                                                             const float* __restrict__ tgrid,
                                                             const float* __restrict__ kz,
                                                             float* __restrict__ phi,
                                                             const float* __restrict__ rho,
                                                             double* __restrict__ fpart,
                                                             const float* __restrict__ g,
                                                             ConvArgs a, SpecPtrs sp) {
    extern __shared__ float dyn_lds[];
    const int item = xcd_item(blockIdx.x, nb);
    if (item >= nb) return;
    const float* ps = a.spec ? spec_z_part(a, item, dyn_lds + spec_off, g, sp) : nullptr;
    conv_z_f32_body(a, item, dyn_lds, tgrid, kz, phi, rho, fpart, ps);
}

__global__ void __launch_bounds__(kConvThreads) k_conv_xy_bf16(const float* __restrict__ rho,
                                                      const unsigned short* __restrict__ kx,
                                                      const unsigned short* __restrict__ ky,
                                                      float* __restrict__ tgrid, ConvArgs a,
                                                      SpecPtrs sp) {
    extern __shared__ float dyn_lds[];
    if ((int)blockIdx.y == a.nterms) {
        spec_fwd_plane(a, blockIdx.x, dyn_lds, rho, sp);
        return;
    }
    conv_xy_bf16_body(a, blockIdx.x, blockIdx.y, dyn_lds, rho, kx, ky, tgrid);
}

__global__ void __launch_bounds__(kConvThreads) k_conv_z_bf16(int nb, int spec_off,
                                                              const float* __restrict__ tgrid,
                                                              const unsigned short* __restrict__ kz,
                                                              float* __restrict__ phi,
                                                              const float* __restrict__ rho,
                                                              double* __restrict__ fpart,
                                                              const float* __restrict__ g,
                                                              ConvArgs a, SpecPtrs sp) {
    extern __shared__ float dyn_lds[];
    const int item = xcd_item(blockIdx.x, nb);
    if (item >= nb) return;
    const float* ps = a.spec ? spec_z_part(a, item, dyn_lds + spec_off, g, sp) : nullptr;
    conv_z_bf16_body(a, item, dyn_lds, tgrid, kz, phi, rho, fpart, ps);
}

// batched: item = t * g_z + z (conv_xy), 16-column group (conv_z)
template <int BF16>
__global__ void __launch_bounds__(kConvThreads) k_conv_xy_batch(const BatchTable* __restrict__ tab,
                                                       const BoxDesc* __restrict__ desc) {
    extern __shared__ float dyn_lds[];
    batch_for(tab, BK_CONV_XY, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        const int gz = d.conv.g[2];
        const int t = item / gz, z = item - t * gz;
        if constexpr (BF16 != 0)
            conv_xy_bf16_body(d.conv, z, t, dyn_lds, d.rho,
                              reinterpret_cast<const unsigned short*>(d.kx),
                              reinterpret_cast<const unsigned short*>(d.ky), d.tgrid);
        else
            conv_xy_f32_body(d.conv, z, t, dyn_lds, d.rho, d.kx, d.ky, d.tgrid);
    });
}

template <int BF16>
__global__ void __launch_bounds__(kConvThreads) k_conv_z_batch(const BatchTable* __restrict__ tab,
                                                      const BoxDesc* __restrict__ desc) {
    extern __shared__ float dyn_lds[];
    batch_for(tab, BK_CONV_Z, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        if constexpr (BF16 != 0)
            conv_z_bf16_body(d.conv, item, dyn_lds, d.tgrid,
                             reinterpret_cast<const unsigned short*>(d.kz), d.phi, d.rho,
                             d.far_parts, nullptr, false);
        else
            conv_z_f32_body(d.conv, item, dyn_lds, d.tgrid, d.kz, d.phi, d.rho, d.far_parts,
                            nullptr, false);
    });
}

// ------------------------------------------------------------------ launch

size_t conv_xy_lds_bytes(const ConvArgs& a) {
    size_t dense;
    if (a.bf16x3) {
        const int ldb = (a.gp[0] > a.gp[1] ? a.gp[0] : a.gp[1]) + 8;
        dense = (size_t)2 * ldb * (a.gp[0] + a.gp[1]) * sizeof(unsigned short);
    } else {
        const int ld = (a.gp[0] > a.gp[1] ? a.gp[0] : a.gp[1]) + 4;
        dense = (size_t)ld * (a.gp[0] + a.gp[1]) * sizeof(float);
    }
    if (!a.spec) return dense;
    // the plane projection: rho[z], P, U_x, U_y
    const size_t spec = sizeof(float) * ((size_t)a.g[1] * a.g[0] + (size_t)a.g[1] * a.rk[0] +
                                         (size_t)a.g[0] * a.rk[0] + (size_t)a.g[1] * a.rk[1]);
    return dense > spec ? dense : spec;
}

// the dense part's LDS (staging of the terms' columns, partial sums)
static size_t conv_z_dense_lds_bytes(const ConvArgs& a) {
    const size_t stage = (size_t)conv_z_chunk(a) * 16 * (a.gp[2] + (a.bf16x3 ? 8 : 4)) * 4;
    const size_t red = (size_t)(conv_z_groups(a) - 1) * (a.gp[2] / 16) * 64 * 4 * sizeof(float);
    return ((stage > red ? stage : red) + 15) & ~(size_t)15;
}

size_t conv_z_lds_bytes(const ConvArgs& a) {
    return conv_z_dense_lds_bytes(a) + sizeof(float) * (size_t)spec_z_lds_floats(a);
}

int conv_z_blocks(const ConvArgs& a) { return (a.g[0] * a.g[1] + 15) / 16; }

int far_parts(const ConvArgs& a) { return conv_z_blocks(a) * (a.gp[2] / 16); }

hipError_t launch_conv_xy(const ConvArgs& a, const float* rho, const float* kx, const float* ky,
                          float* tgrid, const SpecPtrs& sp, hipStream_t st) {
    const size_t lds = conv_xy_lds_bytes(a);
    const dim3 grid(a.g[2], a.nterms + (a.spec ? 1 : 0));
    if (a.bf16x3)
        hipLaunchKernelGGL(k_conv_xy_bf16, grid, dim3(kConvThreads), lds, st, rho,
                           reinterpret_cast<const unsigned short*>(kx),
                           reinterpret_cast<const unsigned short*>(ky), tgrid, a, sp);
    else
        hipLaunchKernelGGL(k_conv_xy_f32, grid, dim3(kConvThreads), lds, st, rho, kx, ky, tgrid, a,
                           sp);
    return hipGetLastError();
}

hipError_t launch_conv_z(const ConvArgs& a, const float* tgrid, const float* kz, float* phi,
                         const float* rho, double* fpart, const SpecPtrs& sp, hipStream_t st) {
    const int nb = conv_z_blocks(a);
    // the spectral core G goes to the plane-projection buffer's tail
    float* g = a.spec ? sp.c + (size_t)a.g[2] * a.rk[1] * a.rk[0] : nullptr;
    if (a.spec) {
        const int n = a.rk[2] * a.rk[1] * a.rk[0];
        hipLaunchKernelGGL(k_spec_core, dim3((n + 15) / 16), dim3(kSpecCoreThreads), 0, st, g, a,
                           sp);
    }
    const int off = (int)(conv_z_dense_lds_bytes(a) / sizeof(float));
    if (a.bf16x3)
        hipLaunchKernelGGL(k_conv_z_bf16, dim3(xcd_blocks(nb)), dim3(kConvThreads),
                           conv_z_lds_bytes(a), st, nb, off, tgrid,
                           reinterpret_cast<const unsigned short*>(kz), phi, rho, fpart, g, a,
                           sp);
    else
        hipLaunchKernelGGL(k_conv_z_f32, dim3(xcd_blocks(nb)), dim3(kConvThreads),
                           conv_z_lds_bytes(a), st, nb, off, tgrid, kz, phi, rho, fpart, g, a, sp);
    return hipGetLastError();
}

hipError_t launch_conv_xy_batch(const BatchTable* tab, const BoxDesc* desc, int bf16x3,
                                size_t lds, int grid, hipStream_t st) {
    if (bf16x3)
        hipLaunchKernelGGL(k_conv_xy_batch<1>, dim3(grid), dim3(kConvThreads), lds, st, tab, desc);
    else
        hipLaunchKernelGGL(k_conv_xy_batch<0>, dim3(grid), dim3(kConvThreads), lds, st, tab, desc);
    return hipGetLastError();
}

hipError_t launch_conv_z_batch(const BatchTable* tab, const BoxDesc* desc, int bf16x3, size_t lds,
                               int grid, hipStream_t st) {
    if (bf16x3)
        hipLaunchKernelGGL(k_conv_z_batch<1>, dim3(grid), dim3(kConvThreads), lds, st, tab, desc);
    else
        hipLaunchKernelGGL(k_conv_z_batch<0>, dim3(grid), dim3(kConvThreads), lds, st, tab, desc);
    return hipGetLastError();
}

}  // namespace useries
