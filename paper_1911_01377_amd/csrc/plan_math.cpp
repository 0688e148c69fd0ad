// FP64 host math of a plan: the u-series coefficients, the construction
// roots, the eq. 33 term count, the near-part polynomial and the periodic 1D
// convolution kernels of the far part.
//
// Paper: Predescu et al., "The u-series" (arXiv:1911.01377).
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "useries_internal.h"

namespace useries {

namespace {
constexpr double kPi = 3.14159265358979323846;

// Table 1 (C2 points of the C1 construction) and Table 2 (b = 2), as printed.
struct Preset {
    double b, r0, w0, s0;
};
constexpr Preset kTable1[3] = {
    {1.62976708826776469, 2.75200266680234223, 1.00780697934380681, 1.0},
    {1.32070036405934420, 4.39145547116383425, 1.00188914114811980, 1.0},
    {1.21812525709410644, 5.63552881512711037, 1.00090146156033341, 1.0},
};
constexpr Preset kTable2C2 = {2.0, 2.39427106444012661, 0.892857784448501290,
                              1.02474173246377476};
}  // namespace

// ---------------------------------------------------------------- series

double Series::pref() const {
    // alpha = 1: eq. 11's 2 ln b / (sqrt(2 pi) sigma).  Otherwise eq. A2 with
    // the Gaussian exp(-u^2/2) as scaling function: ln b / (phi~(alpha)
    // sigma^alpha), phi~(alpha) = 2^(alpha/2 - 1) Gamma(alpha/2) its Mellin
    // transform (eq. A1); phi~(1) = sqrt(pi/2) gives eq. 11 again.
    if (alpha == 1) return 2.0 * std::log(b) / (std::sqrt(2.0 * kPi) * sigma);
    const double mellin = std::pow(2.0, 0.5 * alpha - 1.0) * std::tgamma(0.5 * alpha);
    return std::log(b) / (mellin * std::pow(sigma, alpha));
}

void Series::term(int j, double* a, double* s) const {
    // eq. 11 / 24 / 28 (A2): a_j exp(-r^2/(2 s_j^2)), a_j = pref w_j b^(-alpha j)
    const double p = pref();
    if (j == 0) {
        *a = p * w0;
        *s = sigma * s0;
    } else {
        *a = p * std::pow(b, -(double)alpha * j);
        *s = sigma * std::pow(b, j);
    }
}

int Series::length() const {
    return (int)std::ceil(18.0 * std::log(10.0) / (alpha * std::log(b))) + 1;
}

double Series::kzero_sum(double V) const {
    // sum over all terms of a_j (2 pi s_j^2)^(3/2) / V; from j = 1 on a
    // geometric series of ratio b^(3 - alpha), summed in closed form
    double a0, s0_, a1, s1;
    term(0, &a0, &s0_);
    term(1, &a1, &s1);
    const double m0 = a0 * std::pow(2.0 * kPi * s0_ * s0_, 1.5) / V;
    const double m1 = a1 * std::pow(2.0 * kPi * s1 * s1, 1.5) / V;
    return m0 + m1 / (1.0 - std::pow(b, 3.0 - alpha));
}

double Series::f_inf(double r, double* df) const {
    double v = 0.0, d = 0.0;
    for (int j = length() - 1; j >= 0; --j) {
        double a, s;
        term(j, &a, &s);
        const double e = a * std::exp(-r * r / (2.0 * s * s));
        v += e;
        d -= r / (s * s) * e;
    }
    if (df) *df = d;
    return v;
}

double Series::f_inf0() const {
    // sum_j a_j = pref (w0 + sum_{j>=1} b^(-alpha j))
    return pref() * (w0 + 1.0 / (std::pow(b, (double)alpha) - 1.0));
}

double Series::near_integral(double rc) const {
    // int_{r<rc} (1/r - sum_j a_j exp(-r^2/2s_j^2)) 4 pi r^2 dr; per term
    // int_0^rc r^2 exp(-r^2/2s^2) dr = s^3 m(rc/s), m(u) = int_0^u v^2 exp(-v^2/2) dv.
    // Wide terms have u << 1, where m is summed as a power series (the
    // erf form cancels catastrophically there).
    double g = 0.0;
    for (int j = length() - 1; j >= 0; --j) {
        double a, s;
        term(j, &a, &s);
        const double u = rc / s;
        double m;
        if (u > 1.0) {
            m = std::sqrt(kPi / 2.0) * std::erf(u / std::sqrt(2.0)) - u * std::exp(-u * u / 2.0);
        } else {
            // m(u) = u^3 sum_k (-u^2/2)^k / (k! (2k + 3))
            double c = 1.0, acc = 0.0;
            for (int k = 0; k < 40; ++k) {
                acc += c / (2 * k + 3);
                c *= -u * u / (2.0 * (k + 1));
            }
            m = u * u * u * acc;
        }
        g += a * s * s * s * m;
    }
    return 4.0 * kPi * (rc * rc / 2.0 - g);
}

double bsa_bound(double b) { return std::pow(2.0, 1.5) * std::exp(-kPi * kPi / (2.0 * std::log(b))); }

double eq33_bound(int n, double b, double sigma, double lmax) {
    return std::exp(2.0 * n * std::log(b) -
                    2.0 * (std::pow(b, 2.0 * n) - 1.0) * kPi * kPi * sigma * sigma / (lmax * lmax));
}

int choose_nterms(double b, double sigma, double lmax, double tol) {
    for (int n = 1; n <= kMaxTerms; ++n)
        if (eq33_bound(n, b, sigma, lmax) <= tol) return n;
    return kMaxTerms;
}

double trunc_bound(int n, double b, int alpha, double sigma, double lmax) {
    // the k-space weight a_t (2 pi s_t^2)^(3/2) exp(-s_t^2 k^2/2) of the first
    // dropped term relative to term 0's at k = 2 pi / L (eq. 33 at alpha = 1)
    if (alpha == 1) return eq33_bound(n, b, sigma, lmax);
    return std::exp((3.0 - alpha) * n * std::log(b) -
                    2.0 * (std::pow(b, 2.0 * n) - 1.0) * kPi * kPi * sigma * sigma / (lmax * lmax));
}

int choose_nterms_alpha(double b, int alpha, double sigma, double lmax, double tol) {
    for (int n = 1; n <= kMaxTerms; ++n)
        if (trunc_bound(n, b, alpha, sigma, lmax) <= tol) return n;
    return kMaxTerms;
}

// ---------------------------------------------------------------- roots

namespace {

// G_1(r) and the tail sum_{j>=1} b^-j G_1(b^-j r) with its r-derivative
void tail_sum(double b, double r, double* t, double* dt) {
    Series s;
    s.b = b;
    s.sigma = 1.0;
    double v = 0.0, d = 0.0;
    for (int j = s.length() - 1; j >= 1; --j) {
        const double bj = std::pow(b, -j);
        const double x = bj * r;
        const double g = std::exp(-x * x / 2.0) / std::sqrt(2.0 * kPi);
        v += bj * g;
        d += bj * (-x * bj) * g;
    }
    *t = v;
    *dt = d;
}

// C0: g(r) = r F(r) - 1 with w0 = 1, sigma = 1 (eq. 21)
double c0_resid(double b, double r) {
    Series s;
    s.b = b;
    return r * s.f_inf(r) - 1.0;
}

// C1: eq. 26 residual r^2 F'(r) + 1 with w0 = w0(r) of eq. 25
double c1_resid(double b, double r) {
    double t, dt;
    tail_sum(b, r, &t, &dt);
    const double g0 = std::exp(-r * r / 2.0) / std::sqrt(2.0 * kPi);
    const double w0 = (1.0 / (2.0 * std::log(b) * r) - t) / g0;
    const double fp = 2.0 * std::log(b) * (w0 * (-r) * g0 + dt);
    return r * r * fp + 1.0;
}

template <class F>
double refine_sign_change(F f, double lo, double hi) {
    double flo = f(lo);
    for (int it = 0; it < 300; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = f(mid);
        if (fm == 0.0) return mid;
        if ((fm < 0.0) == (flo < 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

// golden-section minimum of |f| on [lo, hi]
template <class F>
double refine_min_abs(F f, double lo, double hi, double* fmin) {
    const double gr = (std::sqrt(5.0) - 1.0) / 2.0;
    double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
    double fc = std::fabs(f(c)), fd = std::fabs(f(d));
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        if (fc < fd) {
            hi = d;
            d = c;
            fd = fc;
            c = hi - gr * (hi - lo);
            fc = std::fabs(f(c));
        } else {
            lo = c;
            c = d;
            fc = fd;
            d = lo + gr * (hi - lo);
            fd = std::fabs(f(d));
        }
    }
    const double x = 0.5 * (lo + hi);
    *fmin = std::fabs(f(x));
    return x;
}

// Smallest root of f on [0.3, 50): scan, then bisect a sign change or, for a
// tangential (double) root with no sign change, minimise |f| and accept the
// minimum if it is below tang_tol.
template <class F>
bool smallest_root(F f, double tang_tol, double* root) {
    const double h = 2e-3;
    double r_prev = 0.3, f_prev = f(r_prev), r_prev2 = r_prev, f_prev2 = f_prev;
    for (double r = r_prev + h; r < 50.0; r += h) {
        const double fr = f(r);
        if ((fr < 0.0) != (f_prev < 0.0) || fr == 0.0) {
            *root = refine_sign_change(f, r_prev, r);
            return true;
        }
        // |f| has a local minimum at r_prev without a sign change
        if (std::fabs(f_prev) < std::fabs(f_prev2) && std::fabs(f_prev) < std::fabs(fr)) {
            double fm;
            double x = refine_min_abs(f, r_prev2, r, &fm);
            if (fm <= tang_tol) {
                // a double root is an extremum of f: sharpen it as the simple
                // root of the central difference f(r + d) - f(r - d).  Where f
                // is so flat that this difference is rounding noise (the third
                // C2 point of Table 1), the sharpened point wanders off; it is
                // kept only if it stays within 1e-5 of the minimum of |f|.
                const double d = 1e-4;
                auto slope = [&](double t) { return f(t + d) - f(t - d); };
                const double lo = x - 1e-3, hi = x + 1e-3;
                if ((slope(lo) < 0.0) != (slope(hi) < 0.0)) {
                    const double xs = refine_sign_change(slope, lo, hi);
                    if (std::fabs(xs - x) < 1e-5) x = xs;
                }
                *root = x;
                return true;
            }
        }
        r_prev2 = r_prev;
        f_prev2 = f_prev;
        r_prev = r;
        f_prev = fr;
    }
    return false;
}

}  // namespace

double c1_w0_of_r0_alpha(double b, int alpha, double r0) {
    // continuity of the near part at r0 (sigma = 1): r0^alpha F(r0) = 1
    if (alpha == 1) return c1_w0_of_r0(b, r0);
    Series s;
    s.b = b;
    s.alpha = alpha;
    double tail = 0.0;
    for (int j = s.length() - 1; j >= 1; --j) {
        double a, w;
        s.term(j, &a, &w);
        tail += a * std::exp(-r0 * r0 / (2.0 * w * w));
    }
    return (std::pow(r0, -(double)alpha) - tail) / (s.pref() * std::exp(-r0 * r0 / 2.0));
}

int solve_c1_alpha(double b, int alpha, double* r0, double* w0, std::string* err) {
    if (alpha == 1) {
        double bb, s0;
        return solve_construction(USERIES_C1, b, &bb, r0, w0, &s0, err);
    }
    if (!(b > 1.0) || !std::isfinite(b)) {
        if (err) *err = "base b must be > 1";
        return USERIES_EINVAL;
    }
    // slope condition r^(alpha+1) F'(r) + alpha = 0 with w0 from continuity
    auto resid = [b, alpha](double r) {
        Series s;
        s.b = b;
        s.alpha = alpha;
        s.w0 = c1_w0_of_r0_alpha(b, alpha, r);
        double df;
        s.f_inf(r, &df);
        return std::pow(r, alpha + 1.0) * df + alpha;
    };
    double root;
    if (!smallest_root(resid, 1e-12, &root)) {
        if (err) *err = "no C1 root below r = 50";
        return USERIES_EINVAL;
    }
    *r0 = root;
    *w0 = c1_w0_of_r0_alpha(b, alpha, root);
    return USERIES_OK;
}

double c1_w0_of_r0(double b, double r0) {
    double t, dt;
    tail_sum(b, r0, &t, &dt);
    const double g0 = std::exp(-r0 * r0 / 2.0) / std::sqrt(2.0 * kPi);
    return (1.0 / (2.0 * std::log(b) * r0) - t) / g0;
}

namespace {
int solve_construction_uncached(int construction, double b, double* r0, double* w0,
                                std::string* err);
}  // namespace

int solve_construction(int construction, double b, double* b_out, double* r0, double* w0,
                       double* s0, std::string* err) {
    switch (construction) {
    case USERIES_TABLE1_ROW1:
    case USERIES_TABLE1_ROW2:
    case USERIES_TABLE1_ROW3: {
        const Preset& p = kTable1[construction - USERIES_TABLE1_ROW1];
        *b_out = p.b;
        *r0 = p.r0;
        *w0 = p.w0;
        *s0 = p.s0;
        return USERIES_OK;
    }
    case USERIES_C2_B2:
        *b_out = kTable2C2.b;
        *r0 = kTable2C2.r0;
        *w0 = kTable2C2.w0;
        *s0 = kTable2C2.s0;
        return USERIES_OK;
    case USERIES_C0:
    case USERIES_C1:
        break;
    default:
        if (err) *err = "unknown construction";
        return USERIES_EINVAL;
    }
    if (!(b > 1.0) || !std::isfinite(b)) {
        if (err) *err = "base b must be > 1";
        return USERIES_EINVAL;
    }
    *b_out = b;
    *s0 = 1.0;
    // the roots depend on (construction, b) only: solved once per process
    static std::mutex cache_mu;
    static std::map<std::pair<int, double>, std::pair<double, double>> cache;
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        auto it = cache.find({construction, b});
        if (it != cache.end()) {
            *r0 = it->second.first;
            *w0 = it->second.second;
            return USERIES_OK;
        }
    }
    const int rc = solve_construction_uncached(construction, b, r0, w0, err);
    if (rc == USERIES_OK) {
        std::lock_guard<std::mutex> lk(cache_mu);
        cache[{construction, b}] = {*r0, *w0};
    }
    return rc;
}

namespace {
int solve_construction_uncached(int construction, double b, double* r0, double* w0,
                                std::string* err) {
    double root;
    if (construction == USERIES_C0) {
        if (!smallest_root([b](double r) { return c0_resid(b, r); }, 1e-12, &root)) {
            if (err) *err = "no C0 root below r = 50";
            return USERIES_EINVAL;
        }
        *r0 = root;
        *w0 = 1.0;
        return USERIES_OK;
    }
    if (!smallest_root([b](double r) { return c1_resid(b, r); }, 1e-12, &root)) {
        if (err) *err = "no C1 root below r = 50";
        return USERIES_EINVAL;
    }
    *r0 = root;
    *w0 = c1_w0_of_r0(b, root);
    return USERIES_OK;
}
}  // namespace

// ---------------------------------------------------------------- near polynomial

double Series::g_inf(double r) const {
    // F'(r) / r = -sum_j a_j / s_j^2 exp(-r^2 / (2 s_j^2)), regular at r = 0
    double v = 0.0;
    for (int j = length() - 1; j >= 0; --j) {
        double a, s;
        term(j, &a, &s);
        v -= a / (s * s) * std::exp(-r * r / (2.0 * s * s));
    }
    return v;
}

namespace {

// Chebyshev interpolation of f on x in [0, 1] at degree+1 Chebyshev nodes,
// converted to monomial coefficients in x; returns the max absolute error on
// a fine sample.
template <class Fn>
double fit_poly01(Fn f, int degree, double* coef) {
    const int m = degree + 1;
    double cheb[kMaxPolyDeg + 1] = {0};
    double fv[kMaxPolyDeg + 1];
    double tn[kMaxPolyDeg + 1];
    for (int k = 0; k < m; ++k) {
        const double t = std::cos(kPi * (k + 0.5) / m);
        fv[k] = f((t + 1.0) / 2.0);
        tn[k] = t;
    }
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc += fv[k] * std::cos(j * std::acos(tn[k]));
        cheb[j] = acc * 2.0 / m;
    }
    cheb[0] *= 0.5;
    // T_j(2x - 1) as monomials in x
    double tp[kMaxPolyDeg + 1] = {0}, tc[kMaxPolyDeg + 1] = {0}, tnx[kMaxPolyDeg + 1];
    for (int k = 0; k <= degree; ++k) coef[k] = 0.0;
    tp[0] = 1.0;                        // T_0
    tc[0] = -1.0;                       // T_1 = 2x - 1
    tc[1] = 2.0;
    coef[0] += cheb[0];
    if (degree >= 1)
        for (int k = 0; k <= 1; ++k) coef[k] += cheb[1] * tc[k];
    for (int j = 2; j <= degree; ++j) {
        // T_j = 2 (2x - 1) T_{j-1} - T_{j-2}
        for (int k = 0; k <= degree; ++k) {
            double v = -2.0 * tc[k] - tp[k];
            if (k > 0) v += 4.0 * tc[k - 1];
            tnx[k] = v;
        }
        for (int k = 0; k <= degree; ++k) {
            tp[k] = tc[k];
            tc[k] = tnx[k];
            coef[k] += cheb[j] * tc[k];
        }
    }
    double maxerr = 0.0;
    for (int i = 0; i <= 4000; ++i) {
        const double x = i / 4000.0;
        double p = 0.0;
        for (int k = degree; k >= 0; --k) p = p * x + coef[k];
        maxerr = std::fmax(maxerr, std::fabs(p - f(x)));
    }
    return maxerr;
}

}  // namespace

namespace {

// The fit of the series with sigma = 1 on [0, u] (u = r_c / sigma): F_inf(r)
// and F_inf'(r)/r minus their first `nexact` terms, as polynomials in
// x = r^2 / rc^2, fitted separately.  The terms are tabulated once; the sums
// run in the same order and with the same expressions as Series::f_inf and
// Series::g_inf.  The errors are relative to the full functions' maxima,
// F_inf(0) and |F_inf'/r|(0) (all terms decrease with r).
double fit_near_poly_unit(const Series& s, double rc, int degree, int nexact, double* fcoef,
                          double* gcoef) {
    const int len = s.length();
    std::vector<double> ta(len), ts(len);
    for (int j = 0; j < len; ++j) s.term(j, &ta[j], &ts[j]);
    auto f = [&](double x) {
        const double r = rc * std::sqrt(x);
        double v = 0.0;
        for (int j = len - 1; j >= nexact; --j) v += ta[j] * std::exp(-r * r / (2.0 * ts[j] * ts[j]));
        return v;
    };
    auto g = [&](double x) {
        const double r = rc * std::sqrt(x);
        double v = 0.0;
        for (int j = len - 1; j >= nexact; --j)
            v -= ta[j] / (ts[j] * ts[j]) * std::exp(-r * r / (2.0 * ts[j] * ts[j]));
        return v;
    };
    double fmax = 0.0, gmax = 0.0;
    for (int j = len - 1; j >= 0; --j) {
        fmax += ta[j];
        gmax += ta[j] / (ts[j] * ts[j]);
    }
    const double ef = fit_poly01(f, degree, fcoef) / fmax;
    const double eg = fit_poly01(g, degree, gcoef) / gmax;
    return std::fmax(ef, eg);
}

}  // namespace

double fit_near_poly(const Series& s, double rc, int degree, int nexact, double* fcoef,
                     double* gcoef) {
    // Every term scales with sigma: F(r; sigma) = F(r / sigma; 1) / sigma^alpha
    // and F'(r; sigma)/r = (F'/r)(r / sigma; 1) / sigma^(alpha + 2).  The fit is
    // made once per (b, alpha, w0, s0, r_c / sigma, degree, nexact) at sigma = 1
    // and scaled.
    struct Key {
        double b, w0, s0, u;
        int alpha, degree, nexact;
        bool operator<(const Key& o) const {
            if (b != o.b) return b < o.b;
            if (alpha != o.alpha) return alpha < o.alpha;
            if (w0 != o.w0) return w0 < o.w0;
            if (s0 != o.s0) return s0 < o.s0;
            if (u != o.u) return u < o.u;
            if (degree != o.degree) return degree < o.degree;
            return nexact < o.nexact;
        }
    };
    struct Fit {
        double f[kMaxPolyDeg + 1], g[kMaxPolyDeg + 1], err;
    };
    static std::mutex mu;
    static std::map<Key, Fit> cache;
    const Key key{s.b, s.w0, s.s0, rc / s.sigma, s.alpha, degree, nexact};
    Fit fit;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            fit = it->second;
            have = true;
        }
    }
    if (!have) {
        Series unit = s;
        unit.sigma = 1.0;
        fit.err = fit_near_poly_unit(unit, key.u, degree, nexact, fit.f, fit.g);
        std::lock_guard<std::mutex> lk(mu);
        if (cache.size() > 4096) cache.clear();
        cache[key] = fit;
    }
    const double s1 = 1.0 / s.sigma;
    const double sf = s.alpha == 1 ? s1 : std::pow(s.sigma, -(double)s.alpha);
    const double sg = s.alpha == 1 ? s1 * s1 * s1 : sf * s1 * s1;
    for (int k = 0; k <= degree; ++k) {
        fcoef[k] = fit.f[k] * sf;
        gcoef[k] = fit.g[k] * sg;
    }
    return fit.err;
}

// ---------------------------------------------------------------- far kernels

void circulant_column(int n, double h, double sk, double scale, double* k) {
    const int pmax = (int)std::ceil(10.0 * sk / (n * h)) + 1;
    for (int m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int p = pmax; p >= -pmax; --p) {
            const double x = (m + (double)p * n) * h;
            acc += std::exp(-x * x / (2.0 * sk * sk));
        }
        k[m] = scale * acc;
    }
}

}  // namespace useries
