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

    double bb, r0c, w0c, s0c;
    std::string e2;
    const int rc = solve_construction(o.construction, b, &bb, &r0c, &w0c, &s0c, &e2);
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
        p.w0 = c1_w0_of_r0(bb, p.r0);
    }
    p.nterms = n_terms > 0 ? n_terms : choose_nterms(bb, p.sigma, lmax, o.nterms_tol);
    p.eq33 = eq33_bound(p.nterms, bb, p.sigma, lmax);

    Series s;
    s.b = bb;
    s.sigma = p.sigma;
    s.w0 = p.w0;
    s.s0 = p.s0;
    p.f_inf0 = s.f_inf0();
    double dF;
    s.f_inf(r_c, &dF);
    p.c1_slope = -1.0 / (r_c * r_c) - dF;

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
    pa.ne = ne;
    for (int k = 0; k <= deg; ++k) pa.c[k] = (float)coef[k];
    pa.c0lo = (float)(coef[0] - (double)pa.c[0]);
    for (int k = 0; k <= deg; ++k) pa.d[k] = (float)gcoef[k];
    for (int j = 0; j < kMaxExact; ++j) {
        double aj = 0.0, sj = 1.0;
        if (j < ne) s.term(j, &aj, &sj);
        pa.ex[j] = (float)(-1.4426950408889634 * r_c * r_c / (2.0 * sj * sj));
        pa.ea[j] = (float)aj;
        pa.eg[j] = (float)(-aj / (sj * sj));
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
    }
    pa.zinv = (float)(4294967296.0 / box[2]);

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
    ca.nterms = p.nterms_grid;
    ca.bf16x3 = bf ? 1 : 0;
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
        // per term the circulant M[i][j] = col[(i - j) mod g], zero-padded to gp x gp
        if (bf)
            p.mats[a].assign(2 * m * p.nterms_grid * sizeof(uint16_t), 0);
        else
            p.mats[a].assign(m * p.nterms_grid * sizeof(float), 0);
        std::vector<double> col(g);
        std::vector<float> colf(g);
        std::vector<uint16_t> chi(g), clo(g);
        for (int t = 0; t < p.nterms_grid; ++t) {
            double at, st;
            s.term(t, &at, &st);
            const double sk2 = st * st - 2.0 * ss * ss;
            if (!(sk2 > 0))
                return fail(err, USERIES_EINVAL,
                            "grid too coarse: the spreading Gaussian must be narrower than "
                            "s_0 / sqrt(2)");
            const double sk = std::sqrt(sk2);
            circulant_column(g, h, sk, (st / sk) * (a == 0 ? at : 1.0), col.data());
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
    p.fin.near_int_over_v = s.near_integral(r_c) / V;
    p.fin.inv_ngrid = ga.inv_ngrid;
    return USERIES_OK;
}

void choose_columns(HostPlan* hp, int n) {
    HostPlan& p = *hp;
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double w = n > 0 ? std::cbrt(8.0 * V / n) : 1e300;
    for (int a = 0; a < 2; ++a) {
        const int nc = std::max(1, std::min(p.ncmax[a], (int)std::floor(p.box[a] / w)));
        p.bin.nc[a] = p.pair.nc[a] = p.gridargs.nc[a] = nc;
        p.pair.cw[a] = (float)(p.box[a] / nc);
        p.pair.R[a] = (int)std::ceil(p.rc * nc / p.box[a]);
    }
    p.bin.n = p.pair.n = p.gridargs.n = n;
    const int ncol = p.bin.nc[0] * p.bin.nc[1];
    p.fin.n_pair_parts = pair_blocks(n, ncol);
    p.fin.n_gather_parts = gather_blocks(p.gridargs);
}

}  // namespace useries
