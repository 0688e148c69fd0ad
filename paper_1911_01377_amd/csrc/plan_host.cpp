// Host part of a plan (no device calls): parameters of the series for the
// requested construction, the near polynomial, the column bounds, the grid
// and spreading arguments, and the convolution matrices in the device format.
// Shared by useries_plan and the serving loop.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "useries_internal.h"

namespace useries {

namespace {

uint16_t host_bf16(float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

float host_bf16_val(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

int fail(std::string* err, int code, const char* msg) {
    if (err) *err = msg;
    return code;
}

}  // namespace

int build_host_plan(HostPlan* hp, const double box[3], double r_c, double b, double sigma,
                    int n_terms, const int grid[3], const useries_opts* opts, std::string* err) {
    useries_opts o;
    useries_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != USERIES_PLAIN_FP32 && o.precision != USERIES_BF16X3)
        return fail(err, USERIES_EINVAL, "unknown precision");
    const bool bf = o.precision == USERIES_BF16X3;
    const double ratio = o.sigma_s_over_h > 0 ? o.sigma_s_over_h : (bf ? 0.74 : 0.9);
    const int P = o.stencil_half > 0 ? o.stencil_half : (bf ? 3 : 5);
    const int deg = o.poly_degree > 0 ? o.poly_degree : (bf ? 5 : 7);
    if (P < 1 || P > kMaxStencilHalf) return fail(err, USERIES_EINVAL, "stencil_half out of [1, 8]");
    if (deg < 4 || deg > kMaxPolyDeg) return fail(err, USERIES_EINVAL, "poly_degree out of [4, 14]");
    if (!(o.nterms_tol > 0)) return fail(err, USERIES_EINVAL, "nterms_tol must be > 0");
    double lmin = 1e300, lmax = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(box[a] > 0) || !std::isfinite(box[a]))
            return fail(err, USERIES_EINVAL, "box edges must be > 0");
        lmin = std::min(lmin, box[a]);
        lmax = std::max(lmax, box[a]);
        if (grid[a] < 2 * P || grid[a] > kMaxGrid)
            return fail(err, USERIES_EINVAL, "grid points per axis must lie in [2P, 128]");
    }
    if (!(r_c > 0) || !(r_c < 0.5 * lmin))
        return fail(err, USERIES_EINVAL, "need 0 < r_c < min(L)/2");
    if (n_terms > kMaxTerms) return fail(err, USERIES_EINVAL, "n_terms > 32");
    const int alpha = o.alpha > 0 ? o.alpha : 1;
    if (alpha != 1 && alpha != 6 && alpha != 12)
        return fail(err, USERIES_EINVAL, "alpha must be 1, 6 or 12");
    if (alpha != 1 && o.construction != USERIES_C1)
        return fail(err, USERIES_EINVAL, "1/r^6 supports the C1 construction only");

    double bb, r0c, w0c, s0c;
    std::string e2;
    const int rc = alpha == 1 ? solve_construction(o.construction, b, &bb, &r0c, &w0c, &s0c, &e2)
                              : solve_c1_alpha(b, alpha, &r0c, &w0c, &e2);
    if (alpha != 1) {
        bb = b;
        s0c = 1.0;
    }
    if (rc) {
        if (err) *err = e2;
        return rc;
    }
    HostPlan& p = *hp;
    p = HostPlan();
    std::memcpy(p.box, box, sizeof(p.box));
    std::memcpy(p.grid, grid, sizeof(p.grid));
    p.rc = r_c;
    p.b = bb;
    p.s0 = s0c;
    p.construction = o.construction;
    p.precision = o.precision;
    p.alpha = alpha;
    p.P = P;
    p.deg = deg;
    const bool preset = o.construction != USERIES_C0 && o.construction != USERIES_C1;
    if (sigma <= 0) {
        p.r0 = r0c;
        p.w0 = w0c;
        p.sigma = r_c / r0c;
    } else if (preset) {
        if (std::fabs(sigma * r0c / r_c - 1.0) > 1e-12)
            return fail(err, USERIES_EINVAL, "preset constructions fix sigma = r_c / r0");
        p.r0 = r0c;
        p.w0 = w0c;
        p.sigma = sigma;
    } else {
        // continuity correction: keep r_c, re-solve w0 of eq. 25 at r0 = r_c / sigma
        p.sigma = sigma;
        p.r0 = r_c / sigma;
        p.w0 = alpha == 1 ? c1_w0_of_r0(bb, p.r0) : c1_w0_of_r0_alpha(bb, alpha, p.r0);
    }
    p.nterms = n_terms > 0 ? n_terms : choose_nterms_alpha(bb, alpha, p.sigma, lmax, o.nterms_tol);
    p.eq33 = trunc_bound(p.nterms, bb, alpha, p.sigma, lmax);

    Series s;
    s.b = bb;
    s.sigma = p.sigma;
    s.w0 = p.w0;
    s.s0 = p.s0;
    s.alpha = alpha;
    p.f_inf0 = s.f_inf0();
    double dF;
    s.f_inf(r_c, &dF);
    p.c1_slope = -(double)alpha * std::pow(r_c, -(double)alpha - 1.0) - dF;

    // near part: F_inf and F_inf'/r inside the cutoff as polynomials in
    // r^2 / r_c^2 after the narrowest `ne` terms, which the pair kernel
    // evaluates as Gaussians.  Small b puts the narrowest Gaussians deep
    // inside r_c (u = r_c / s_j up to 5.6 for Table 1 row 3), where a
    // polynomial of modest degree cannot follow them; ne is the smallest count
    // whose remainder fits within the form's budget relative to max |F|
    // (FP32 level 1e-7 for the plain path, 2e-5 for BF16X3, whose force
    // budget is 1e-3).
    const double budget = bf ? 2e-5 : 1e-7;
    double coef[kMaxPolyDeg + 1], gcoef[kMaxPolyDeg + 1];
    int ne = 0;
    for (;; ++ne) {
        p.poly_maxerr = fit_near_poly(s, r_c, deg, ne, coef, gcoef);
        if (p.poly_maxerr <= budget) break;
        if (ne == kMaxExact)
            return fail(err, USERIES_EINVAL,
                        "near part: the polynomial of this degree misses the form's accuracy "
                        "even with the 8 narrowest Gaussians evaluated exactly (raise "
                        "poly_degree or b)");
    }
    p.near_exact = ne;
    PairArgs& pa = p.pair;
    pa.deg = deg;
    pa.alpha = alpha;
    pa.ne = ne;
    const double u = (double)(float)(box[0] / 4294967296.0), u3 = u * u * u;
    for (int k = 0; k <= deg; ++k) {
        pa.c[k] = (float)coef[k];
        pa.d[k] = (float)gcoef[k];
        pa.cu[k] = (float)(coef[k] * u);
        pa.du[k] = (float)(gcoef[k] * u3);
    }
    for (int j = 0; j < kMaxExact; ++j) {
        double aj = 0.0, sj = 1.0;
        if (j < ne) s.term(j, &aj, &sj);
        pa.ex[j] = (float)(-1.4426950408889634 * r_c * r_c / (2.0 * sj * sj));
        pa.ea[j] = (float)aj;
        pa.eg[j] = (float)(-aj / (sj * sj));
        pa.eau[j] = (float)(aj * u);
        pa.egu[j] = (float)(-aj / (sj * sj) * u3);
    }
    pa.gz = grid[2];
    pa.rc2 = (float)(r_c * r_c);
    pa.inv_rc2 = (float)(1.0 / (r_c * r_c));

    // x-y columns: at least r_c / 4 wide (so the pair stencil stays within
    // 9 x 9 columns), and wide enough that a spreading brick touches at most
    // 16 columns per axis; the grid used is chosen per evaluation from n
    for (int a = 0; a < 2; ++a) {
        const double h = box[a] / grid[a];
        const double wmin = std::max(0.25 * r_c, (8 + 2 * P - 1) * h / 14.0);
        // at most 65535 per axis: a cluster's column is stored as cx | cy << 16
        p.ncmax[a] = std::max(1, (int)std::min(65535.0, std::floor(box[a] / wmin)));
    }
    while ((int64_t)p.ncmax[0] * p.ncmax[1] > (1 << 20)) {
        const int am = p.ncmax[1] > p.ncmax[0] ? 1 : 0;
        p.ncmax[am] = std::max(1, p.ncmax[am] * 3 / 4);
    }
    p.ncol_max = p.ncmax[0] * p.ncmax[1];
    for (int a = 0; a < 3; ++a) {
        p.bin.inv_box[a] = 1.0 / box[a];
        pa.scale[a] = (float)(box[a] / 4294967296.0);
        pa.scale_lo[a] = (float)(box[a] / 4294967296.0 - (double)pa.scale[a]);
    }
    pa.zinv = (float)(4294967296.0 / box[2]);
    pa.inv_scale = 1.0f / pa.scale[0];
    pa.inv_scale_d = 1.0 / (double)pa.scale[0];
    {
        const double ux = (double)pa.scale[0] + (double)pa.scale_lo[0];
        const double is2 = 1.0 / (ux * ux);
        pa.is2h = (float)is2;
        pa.is2l = (float)(is2 - (double)pa.is2h);
        const float rcm = std::sqrt(pa.rc2) + 1e-3f;
        pa.rcm2 = rcm * rcm;
    }

    // far part.  A term so wide that every non-zero Fourier mode of its
    // periodised Gaussian lies below 2^-60 of the k = 0 mode equals, to double
    // precision, that mode alone, which the far part removes (uniform
    // background): it would add nothing but rounding, so the grid evaluates
    // only the leading terms narrower than that (terms widen with t).
    const double pi = 3.14159265358979323846;
    int ngrid = 0;
    for (int t = 0; t < p.nterms; ++t) {
        double at, st;
        s.term(t, &at, &st);
        const double u = 2.0 * pi * st / lmax;
        if (0.5 * u * u > 60.0 * std::log(2.0)) break;
        ngrid = t + 1;
    }
    p.nterms_grid = std::max(1, ngrid);
    GridArgs& ga = p.gridargs;
    ga.P = P;
    ga.inv_ngrid = 1.0 / ((double)grid[0] * grid[1] * grid[2]);
    ConvArgs& ca = p.conv;
    ca.bf16x3 = bf ? 1 : 0;
    // every grid term's circulant column per axis (term amplitude folded into x)
    std::vector<std::vector<double>> cols[3];
    for (int a = 0; a < 3; ++a) {
        const double h = box[a] / grid[a];
        const double ss = ratio * h;
        cols[a].resize(p.nterms_grid);
        for (int t = 0; t < p.nterms_grid; ++t) {
            double at, st;
            s.term(t, &at, &st);
            const double sk2 = st * st - 2.0 * ss * ss;
            if (!(sk2 > 0))
                return fail(err, USERIES_EINVAL,
                            "grid too coarse: the spreading Gaussian must be narrower than "
                            "s_0 / sqrt(2)");
            const double sk = std::sqrt(sk2);
            cols[a][t].resize(grid[a]);
            circulant_column(grid[a], h, sk, (st / sk) * (a == 0 ? at : 1.0), cols[a][t].data());
        }
    }
    // Spectral form of the wide terms (Sec. V leaves the wide terms' cost open;
    // this is a low-rank form of their circulants).  A symmetric circulant is
    // diagonal in the real Fourier basis: K = sum_k lambda(k) (c_k c_k^T +
    // s_k s_k^T), lambda(k) = sum_m col[m] cos(2 pi k m / n).  A wide term's
    // lambda(k) falls like exp(-2 pi^2 k^2 s^2 / L^2), so its modes k > K are
    // below 1e-9 of its first mode for a small K.  From the first term t_d
    // whose modes fit in r = 2K + 1 <= min(kMaxSpecRank, n/4) on every axis,
    // all wider terms are applied together through that basis (at least two
    // of them, else the dense form is kept).
    int td = p.nterms_grid;
    int rk[3] = {0, 0, 0};
    std::vector<std::vector<double>> lam[3];
    if (o.spectral) {
        for (int a = 0; a < 3; ++a) {
            const int g = grid[a], kh = g / 2;
            lam[a].assign(p.nterms_grid, std::vector<double>(kh + 1, 0.0));
            for (int t = 0; t < p.nterms_grid; ++t)
                for (int k = 0; k <= kh; ++k) {
                    double acc = 0.0;
                    for (int m = 0; m < g; ++m)
                        acc += cols[a][t][m] * std::cos(2.0 * pi * (double)k * m / g);
                    lam[a][t][k] = acc;
                }
        }
        auto rank_of = [&](int t, int a) {
            const int kh = grid[a] / 2;
            // modes below 1e-9 of the first one, or at the FP64 rounding level
            // of the transform (1e-13 of the k = 0 gain; the dense circulants
            // carry FP32 rounding of 1e-7 of it), are dropped
            const double tau = std::max(1e-9 * std::fabs(lam[a][t][std::min(1, kh)]),
                                        1e-13 * std::fabs(lam[a][t][0]));
            int K = kh;
            while (K > 0 && std::fabs(lam[a][t][K]) <= tau) --K;
            return 2 * K + 1;
        };
        auto fits = [&](int t) {
            for (int a = 0; a < 3; ++a) {
                const int r = rank_of(t, a);
                if (r > kMaxSpecRank || 4 * r > grid[a]) return false;
            }
            return true;
        };
        while (td > 1 && fits(td - 1)) --td;
        // forced (spectral > 0): from two terms on; automatic (< 0): from six,
        // below which the dense matrix-core convolutions of those few terms
        // cost less than the spectral steps (measured on the 64 A water box)
        if (p.nterms_grid - td < (o.spectral > 0 ? 2 : 6)) td = p.nterms_grid;
        if (td < p.nterms_grid)
            for (int a = 0; a < 3; ++a)
                for (int t = td; t < p.nterms_grid; ++t) rk[a] = std::max(rk[a], rank_of(t, a));
    }
    p.nterms_spec = p.nterms_grid - td;
    ca.nterms = td;
    ca.spec = p.nterms_spec > 0 ? 1 : 0;
    for (int a = 0; a < 3; ++a) ca.rk[a] = ca.spec ? rk[a] : 0;
    if (ca.spec) {
        for (int a = 0; a < 3; ++a) {
            const int g = grid[a], r = rk[a];
            auto& U = p.ubasis[a];
            U.assign((size_t)g * r, 0.0f);
            for (int i = 0; i < g; ++i) {
                U[(size_t)i * r] = (float)(1.0 / std::sqrt((double)g));
                for (int k = 1; 2 * k < r; ++k) {
                    const double ph = 2.0 * pi * (double)k * i / g;
                    U[(size_t)i * r + 2 * k - 1] = (float)(std::sqrt(2.0 / g) * std::cos(ph));
                    U[(size_t)i * r + 2 * k] = (float)(std::sqrt(2.0 / g) * std::sin(ph));
                }
            }
        }
        // W[iz][iy][ix] = sum over the spectral terms of the products of their
        // eigenvalues (basis column i carries mode (i + 1) / 2); k = 0 removed
        p.wspec.assign((size_t)rk[0] * rk[1] * rk[2], 0.0f);
        for (int iz = 0; iz < rk[2]; ++iz)
            for (int iy = 0; iy < rk[1]; ++iy)
                for (int ix = 0; ix < rk[0]; ++ix) {
                    double acc = 0.0;
                    if (iz || iy || ix)
                        for (int t = td; t < p.nterms_grid; ++t)
                            acc += lam[2][t][(iz + 1) / 2] * lam[1][t][(iy + 1) / 2] *
                                   lam[0][t][(ix + 1) / 2];
                    p.wspec[((size_t)iz * rk[1] + iy) * rk[0] + ix] = (float)acc;
                }
    }
    for (int a = 0; a < 3; ++a) {
        const double h = box[a] / grid[a];
        const double ss = ratio * h;
        p.sigma_s[a] = ss;
        ga.g[a] = ca.g[a] = grid[a];
        // padded to the MFMA K step: 4 (FP32, tiles of 16) or 32 (BF16)
        ca.gp[a] = bf ? (grid[a] + 31) / 32 * 32 : (grid[a] + 15) / 16 * 16;
        ga.hs[a] = (float)(h * h / (2.0 * ss * ss));
        ga.cw[a] = (float)(h / (std::sqrt(2.0 * pi) * ss));
        ga.dws[a] = (float)(h / (ss * ss));
        const int g = grid[a], gp = ca.gp[a];
        const size_t m = (size_t)gp * gp;
        // per dense term the circulant M[i][j] = col[(i - j) mod g], zero-padded to gp x gp
        if (bf)
            p.mats[a].assign(2 * m * ca.nterms * sizeof(uint16_t), 0);
        else
            p.mats[a].assign(m * ca.nterms * sizeof(float), 0);
        std::vector<float> colf(g);
        std::vector<uint16_t> chi(g), clo(g);
        for (int t = 0; t < ca.nterms; ++t) {
            const std::vector<double>& col = cols[a][t];
            for (int k = 0; k < g; ++k) {
                colf[k] = (float)col[k];
                chi[k] = host_bf16(colf[k]);
                clo[k] = host_bf16(colf[k] - host_bf16_val(chi[k]));
            }
            if (bf) {
                uint16_t* hi = reinterpret_cast<uint16_t*>(p.mats[a].data()) + 2 * m * t;
                uint16_t* lo = hi + m;
                for (int i = 0; i < g; ++i)
                    for (int j = 0; j < g; ++j) {
                        const int k = i >= j ? i - j : i - j + g;
                        hi[(size_t)i * gp + j] = chi[k];
                        lo[(size_t)i * gp + j] = clo[k];
                    }
            } else {
                float* M = reinterpret_cast<float*>(p.mats[a].data()) + m * t;
                for (int i = 0; i < g; ++i)
                    for (int j = 0; j < g; ++j) M[(size_t)i * gp + j] = colf[i >= j ? i - j : i - j + g];
            }
        }
    }
    const double V = box[0] * box[1] * box[2];
    p.fin.f_inf0 = p.f_inf0;
    // Coulomb: the neutralising background of a net charge (k = 0 dropped);
    // 1/r^6: no background, but the far terms' k = 0 components, which the
    // grid removes, are added back for the net "charge" Q = sum c_i
    p.fin.near_int_over_v = alpha == 1 ? s.near_integral(r_c) / V : 0.0;
    p.fin.k0_far = alpha == 1 ? 0.0 : s.kzero_sum(V);
    return USERIES_OK;
}

int columns_per_axis(const HostPlan& p, int n, int a) {
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double w = n > 0 ? std::cbrt(8.0 * V / n) : 1e300;
    return std::max(1, std::min(p.ncmax[a], (int)std::floor(p.box[a] / w)));
}

void choose_columns(HostPlan* hp, int n) {
    HostPlan& p = *hp;
    for (int a = 0; a < 2; ++a) {
        const int nc = columns_per_axis(p, n, a);
        p.bin.nc[a] = p.pair.nc[a] = p.gridargs.nc[a] = nc;
        p.pair.cw[a] = (float)(p.box[a] / nc);
        p.pair.R[a] = (int)std::ceil(p.rc * nc / p.box[a]);
    }
    p.bin.n = p.pair.n = p.gridargs.n = n;
    const int ncol = p.bin.nc[0] * p.bin.nc[1];
    p.fin.n_pair_parts = pair_blocks(n, ncol);
    p.fin.n_far_parts = far_parts(p.conv);
}

}  // namespace useries
