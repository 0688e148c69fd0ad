/*
 * useries_oracle.c -- FP64 CPU oracle for u-series electrostatics.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plainly written reference
 * that the GPU library is checked against.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or constant table with the GPU library.
 *
 * Everything is double precision, Gaussian units (Coulomb constant 1):
 * charges in e, lengths in Angstrom, energy in e^2/A, force in e^2/A^2.
 *
 * What is computed (paper: Predescu et al., "The u-series", arXiv:1911.01377):
 *
 *   Far series (Sec. III.A eq. 11 with the C1 weight of eq. 24 and the
 *   optional narrowest width s0 of eq. 28, unnormalised as Table 2 row 3
 *   requires):
 *       F(r) = sum_{j>=0} a_j exp(-r^2 / (2 s_j^2)),
 *       a_0 = 2 ln b w0 / (sqrt(2 pi) sigma),  s_0 = sigma s0,
 *       a_j = 2 ln b b^-j / (sqrt(2 pi) sigma), s_j = sigma b^j   (j >= 1).
 *   "Infinite" sums keep every term with b^-j > 1e-18 relative weight.
 *
 *   Near part (eq. 20): N(r) = 1/r - F_inf(r) for r < r_c, else 0, summed
 *   over all pairs and periodic images (the minimum image when r_c < L/2).
 *
 *   Far part (Sec. V): F truncated to its first N terms; each Gaussian is
 *   separable (eq. 31), so its periodic image sum is a product of three 1D
 *   theta sums.  The k = 0 (uniform) component is removed, i.e. tin-foil
 *   boundary conditions with a neutralising background for non-neutral input
 *   (eqs. 4, 9, 10 sum only k != 0).  The i = j pairs are included: they are
 *   the self-interaction of eq. 3 before its removal.
 *
 *   Self term: E_self = 1/2 F_inf(0) sum q_i^2 (the u-series analogue of the
 *   Ewald self term of eq. 10, Appendix F eq. F1 "before subtracting the
 *   self-interactions").  The infinite series is used: the dropped terms
 *   j >= N are nearly constant across the cell, so their periodic pair sum
 *   vanishes for a neutral cell (its remainder is what eq. 33 bounds) but their
 *   value at r = 0 does not.
 *
 *   Background: for a net charge Q the k = 0 component of the near kernel is
 *   removed as well, E_bg = -Q^2/(2V) int N d^3r (zero for neutral input),
 *   which is the u-series form of the usual Ewald background correction.
 *
 *   E = E_near + E_far - E_self + E_bg,  F_i = -dE/dr_i.
 *
 * Kernel 1/r^alpha (App. A; the paper's example is the dispersion 1/r^6):
 * the BSA of eq. A2 with the Gaussian as scaling function, whose Mellin
 * transform (eq. A1) is phi~(alpha) = 2^(alpha/2 - 1) Gamma(alpha/2), gives
 *       a_j = ln b w_j b^(-alpha j) / (phi~(alpha) sigma^alpha),  s_j = sigma b^j,
 * and the near part is 1/r^alpha - F_inf(r) below r_c.  The charges are then
 * the coefficients c_i of E = 1/2 sum' c_i c_j / r^alpha.  For alpha > 3 the
 * periodic lattice sum converges absolutely, so nothing is neutralised: the
 * far part keeps every term's k = 0 component (the dropped terms j >= N
 * contribute theirs analytically) and E_bg = 0.  Only alpha = 1 and
 * alpha > 3 are accepted.
 *
 * A second, independent form of E_far and its forces is the k-space sum of
 * Appendix F eq. F1 (equivalently eq. 32 with S^ = 1), related to the
 * real-space theta form by Poisson summation.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    double b;      /* base b > 1 */
    double sigma;  /* width sigma of the narrowest Gaussian (before s0) */
    double w0;     /* weight of the narrowest Gaussian, eq. 24 (1 for C0) */
    double s0;     /* width factor of the narrowest Gaussian, eq. 28 (1 for C0/C1) */
    double rc;     /* cutoff radius r_c of the near part, eq. 20 */
    int nterms;    /* N: terms kept in the far part, Sec. V */
    double alpha;  /* kernel 1/r^alpha (App. A); 0 or 1: Coulomb */
} uo_params;

/* the power alpha of the kernel (0 stands for the Coulomb default 1) */
static double kpow(const uo_params *p)
{
    return p->alpha > 0.0 ? p->alpha : 1.0;
}

/* Mellin transform of the unit Gaussian exp(-u^2/2), eq. A1:
 * int_0^inf exp(-u^2/2) u^(alpha-1) du = 2^(alpha/2 - 1) Gamma(alpha/2) */
double uo_mellin_gauss(double alpha)
{
    return pow(2.0, 0.5 * alpha - 1.0) * tgamma(0.5 * alpha);
}

/* ---------------------------------------------------------------- series */

/* number of terms for the "infinite" series: b^-J < 1e-18 */
int uo_series_len(double b)
{
    return (int)ceil(18.0 * log(10.0) / log(b)) + 1;
}

/* the same for the 1/r^alpha series, whose weights fall as b^(-alpha j) */
static int series_len_p(const uo_params *p)
{
    double al = kpow(p);
    if (al == 1.0) return uo_series_len(p->b);
    return (int)ceil(18.0 * log(10.0) / (al * log(p->b))) + 1;
}

/* amplitude a_j and width s_j of Gaussian term j (eqs. 11, 24, 28).
 * For 1/r^alpha the BSA of eq. A2 with the Gaussian scaling function gives
 * the prefactor ln b / (phi~(alpha) sigma^alpha) and weights b^(-alpha j);
 * at alpha = 1, phi~(1) = sqrt(pi/2) and this is eq. 11's 2 ln b/(sqrt(2 pi) sigma). */
void uo_term(const uo_params *p, int j, double *a, double *s)
{
    double al = kpow(p);
    double pref = al == 1.0 ? 2.0 * log(p->b) / (sqrt(2.0 * M_PI) * p->sigma)
                            : log(p->b) / (uo_mellin_gauss(al) * pow(p->sigma, al));
    if (j == 0) {
        *a = pref * p->w0;
        *s = p->sigma * p->s0;
    } else {
        *a = pref * pow(p->b, -al * (double)j);
        *s = p->sigma * pow(p->b, (double)j);
    }
}

/* F(r) over terms [j0, j1) and its first two r-derivatives */
static void far_sum(const uo_params *p, int j0, int j1, double r,
                    double *f, double *df, double *d2f)
{
    double v = 0.0, d1 = 0.0, d2 = 0.0;
    for (int j = j1 - 1; j >= j0; --j) {     /* small terms first */
        double a, s;
        uo_term(p, j, &a, &s);
        double s2 = s * s;
        double e = a * exp(-r * r / (2.0 * s2));
        v += e;
        d1 += -r / s2 * e;
        d2 += (r * r / (s2 * s2) - 1.0 / s2) * e;
    }
    if (f) *f = v;
    if (df) *df = d1;
    if (d2f) *d2f = d2;
}

/* F_inf(r), F_inf'(r), F_inf''(r) (eq. 19 / 24 / 28, all terms) */
void uo_far_inf(const uo_params *p, double r, double out[3])
{
    far_sum(p, 0, series_len_p(p), r, &out[0], &out[1], &out[2]);
}

/* near kernel N(r) of eq. 20 and its r-derivative: 1/r^alpha - F_inf(r)
 * below r_c */
void uo_near(const uo_params *p, double r, double out[2])
{
    if (r >= p->rc) { out[0] = 0.0; out[1] = 0.0; return; }
    double f[3], al = kpow(p);
    uo_far_inf(p, r, f);
    if (al == 1.0) {
        out[0] = 1.0 / r - f[0];
        out[1] = -1.0 / (r * r) - f[1];
    } else {
        out[0] = pow(r, -al) - f[0];
        out[1] = -al * pow(r, -al - 1.0) - f[1];
    }
}

/* BSA relative-error bound M_b, eq. 14 */
double uo_bsa_bound(double b)
{
    return pow(2.0, 1.5) * exp(-M_PI * M_PI / (2.0 * log(b)));
}

/* Truncation bound for 1/r^alpha: the k-space weight of the first dropped
 * term relative to that of term 0 at the smallest wavevector 2 pi / L, the
 * quantity that eq. 33 bounds for alpha = 1 (the k-space weight of term t
 * is a_t (2 pi s_t^2)^(3/2) exp(-s_t^2 k^2 / 2), proportional to
 * b^((3 - alpha) t) exp(-s_t^2 k^2 / 2)).  At alpha = 1 it is eq. 33. */
double uo_trunc_bound(int n, double b, double alpha, double sigma, double lmax)
{
    return exp((3.0 - alpha) * n * log(b)
               - 2.0 * (pow(b, 2.0 * n) - 1.0) * M_PI * M_PI * sigma * sigma / (lmax * lmax));
}

/* truncation bound for the far energy with N terms, eq. 33 (App. F, F4) */
double uo_eq33_bound(int n, double b, double sigma, double lmax)
{
    return exp(2.0 * n * log(b)
               - 2.0 * (pow(b, 2.0 * n) - 1.0) * M_PI * M_PI * sigma * sigma / (lmax * lmax));
}

/* ------------------------------------------------------- parameter roots */

/* C0 construction (eqs. 19-21) at sigma = 1: g(r) = r F(r) - 1 */
static double c0_resid(double b, double r)
{
    uo_params p = {b, 1.0, 1.0, 1.0, 0.0, 0};
    double f[3];
    uo_far_inf(&p, r, f);
    return r * f[0] - 1.0;
}

/* C1 construction: w0 from eq. 25 at sigma = 1 */
double uo_c1_w0(double b, double r)
{
    uo_params p = {b, 1.0, 1.0, 1.0, 0.0, 0};
    double tail, g0;
    far_sum(&p, 1, uo_series_len(b), r, &tail, NULL, NULL);     /* 2 ln b sum_{j>=1} ... */
    tail /= 2.0 * log(b);
    g0 = exp(-r * r / 2.0) / sqrt(2.0 * M_PI);                  /* G_1(r) */
    return (1.0 / (2.0 * log(b) * r) - tail) / g0;
}

/* eq. 26 residual with w0 = w0(r): F'(r) + 1/r^2 */
static double c1_resid(double b, double r)
{
    uo_params p = {b, 1.0, uo_c1_w0(b, r), 1.0, 0.0, 0};
    double f[3];
    uo_far_inf(&p, r, f);
    return f[1] + 1.0 / (r * r);
}

/* C1 construction for 1/r^alpha at sigma = 1 (the analogue of eqs. 24-26):
 * w0 makes the series equal r^-alpha at r (continuity of the near part), and
 * r0 is the smallest r at which the slopes agree as well,
 * r^(alpha+1) F'(r) + alpha = 0.  At alpha = 1 these are eqs. 25 and 26. */
double uo_c1_w0a(double b, double alpha, double r)
{
    uo_params p = {b, 1.0, 1.0, 1.0, 0.0, 0, alpha};
    double tail, a0, s0;
    far_sum(&p, 1, series_len_p(&p), r, &tail, NULL, NULL);
    uo_term(&p, 0, &a0, &s0);                                   /* a_0 at w0 = 1 */
    return (pow(r, -alpha) - tail) / (a0 * exp(-r * r / 2.0));
}

static double c1a_resid(double b, double alpha, double r)
{
    uo_params p = {b, 1.0, uo_c1_w0a(b, alpha, r), 1.0, 0.0, 0, alpha};
    double f[3];
    uo_far_inf(&p, r, f);
    return pow(r, alpha + 1.0) * f[1] + alpha;
}

/* (r0, w0) of the C1 construction for 1/r^alpha: smallest sign change of the
 * slope residual on (0.5, 50), scanned in steps of 1e-3 and bisected.
 * Returns 0 on success. */
int uo_solve_c1a(double b, double alpha, double *r0, double *w0)
{
    double h = 1e-3, r = 0.5, gp = c1a_resid(b, alpha, r);
    for (; r < 50.0; r += h) {
        double gn = c1a_resid(b, alpha, r + h);
        if ((gn < 0) != (gp < 0)) {
            double lo = r, hi = r + h, glo = gp;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double gm = c1a_resid(b, alpha, mid);
                if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; } else { hi = mid; }
            }
            *r0 = 0.5 * (lo + hi);
            *w0 = uo_c1_w0a(b, alpha, *r0);
            return 0;
        }
        gp = gn;
    }
    return -1;
}

static double bisect(double (*g)(double, double), double b, double lo, double hi)
{
    double glo = g(b, lo);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double gm = g(b, mid);
        if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; } else { hi = mid; }
    }
    return 0.5 * (lo + hi);
}

/* smallest sign change of g on (0.5, 50): scan in steps of 1e-3, then bisect.
 * Returns 0 on success. */
static int smallest_root(double (*g)(double, double), double b, double *root)
{
    double h = 1e-3, r = 0.5, gp = g(b, r);
    for (; r < 50.0; r += h) {
        double gn = g(b, r + h);
        if ((gn < 0) != (gp < 0)) { *root = bisect(g, b, r, r + h); return 0; }
        gp = gn;
    }
    return -1;
}

/* r0 of the C0 construction: smallest root of eq. 21 at sigma = 1 */
int uo_solve_c0(double b, double *r0)
{
    return smallest_root(c0_resid, b, r0);
}

/* (r0, w0) of the C1 construction: smallest root of eq. 26 with eq. 25 */
int uo_solve_c1(double b, double *r0, double *w0)
{
    if (smallest_root(c1_resid, b, r0)) return -1;
    *w0 = uo_c1_w0(b, *r0);
    return 0;
}

/* ------------------------------------------------------------ energies */

static double wrap_min(double d, double L)
{
    return d - L * nearbyint(d / L);
}

/* 1D periodic theta sum of one Gaussian: th = sum_m exp(-(d+mL)^2/(2s^2)),
 * dth = d th / d d.  Images up to |m| <= ceil(9 s / L) + 1. */
static void theta1(double d, double L, double s, double *th, double *dth)
{
    int M = (int)ceil(9.0 * s / L) + 1;
    double v = 0.0, dv = 0.0, s2 = s * s;
    for (int m = -M; m <= M; ++m) {
        double x = d + m * L;
        double e = exp(-x * x / (2.0 * s2));
        v += e;
        dv += -x / s2 * e;
    }
    *th = v;
    *dth = dv;
}

/* near energy/forces of eq. 20 over all pairs and images within r_c */
static double near_part(int n, const double *xyz, const double *q, const double L[3],
                        const uo_params *p, double *frc)
{
    int M[3];
    for (int a = 0; a < 3; ++a) M[a] = (int)floor(p->rc / L[a] + 0.5);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *fbuf = calloc((size_t)nth * n * 3, sizeof(double));
    double e = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+:e)
    for (int i = 0; i < n; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *f = fbuf + (size_t)tid * n * 3;
        for (int j = i; j < n; ++j) {
            double d0[3];
            for (int a = 0; a < 3; ++a) d0[a] = wrap_min(xyz[3 * i + a] - xyz[3 * j + a], L[a]);
            for (int mx = -M[0]; mx <= M[0]; ++mx)
            for (int my = -M[1]; my <= M[1]; ++my)
            for (int mz = -M[2]; mz <= M[2]; ++mz) {
                if (i == j && mx == 0 && my == 0 && mz == 0) continue;
                double d[3] = {d0[0] + mx * L[0], d0[1] + my * L[1], d0[2] + mz * L[2]};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r >= p->rc) continue;
                double nk[2];
                uo_near(p, r, nk);
                double qq = q[i] * q[j];
                /* pair (i,j) and (j,i) are the same image pair counted once here */
                double w = (i == j) ? 0.5 : 1.0;
                e += w * qq * nk[0];
                if (i != j) {
                    double g = -qq * nk[1] / r;     /* force on i along d */
                    for (int a = 0; a < 3; ++a) { f[3 * i + a] += g * d[a]; f[3 * j + a] -= g * d[a]; }
                }
            }
        }
    }
    for (int t = 0; t < nth; ++t)
        for (int k = 0; k < 3 * n; ++k) frc[k] += fbuf[(size_t)t * n * 3 + k];
    free(fbuf);
    return e;
}

/* k = 0 mean of term t's periodised Gaussian over the cell: a_t (2 pi s_t^2)^(3/2) / V */
static double term_mean(const uo_params *p, int t, double V)
{
    double a, s;
    uo_term(p, t, &a, &s);
    return a * pow(2.0 * M_PI * s * s, 1.5) / V;
}

/* sum_{j >= j0} of the terms' k = 0 means (alpha > 3).  For j >= 1 the means
 * a_j (2 pi s_j^2)^(3/2) / V form a geometric series of ratio b^(3 - alpha)
 * (a_j ~ b^(-alpha j), s_j^3 ~ b^(3 j)), summed here in closed form: it falls
 * only as b^(-(alpha - 3) j), far slower than the series itself. */
static double kzero_tail(const uo_params *p, int j0, double V)
{
    double m1 = term_mean(p, 1, V);                /* mean of term 1 */
    double ratio = pow(p->b, 3.0 - kpow(p));
    int j1 = j0 < 1 ? 1 : j0;
    double tail = m1 * pow(ratio, (double)(j1 - 1)) / (1.0 - ratio);
    return (j0 <= 0 ? term_mean(p, 0, V) : 0.0) + tail;
}

/* Far energy/forces: N separable Gaussians, periodic theta products (eq. 31).
 * Coulomb (alpha = 1): the k = 0 component of every term is removed (the
 * k != 0 sums of eqs. 4, 9, 10).  1/r^alpha with alpha > 3, whose lattice sum
 * converges absolutely: every term keeps its k = 0 component, and the terms
 * j >= N, dropped from the grid, still contribute theirs,
 * 1/2 Q^2 sum_{j>=N} a_j (2 pi s_j^2)^(3/2) / V (their k != 0 parts are what
 * the truncation bound measures). */
static double far_part(int n, const double *xyz, const double *q, const double L[3],
                       const uo_params *p, double *frc)
{
    double V = L[0] * L[1] * L[2];
    int keep_k0 = kpow(p) > 3.0;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *fbuf = calloc((size_t)nth * n * 3, sizeof(double));
    double e = 0.0, qsum = 0.0;
    for (int i = 0; i < n; ++i) qsum += q[i];
    if (keep_k0) e += 0.5 * qsum * qsum * kzero_tail(p, p->nterms, V);
    for (int t = 0; t < p->nterms; ++t) {
        double a, s;
        uo_term(p, t, &a, &s);
        /* k = 0 mean of the periodised Gaussian, removed (uniform background) */
        if (!keep_k0) e -= 0.5 * qsum * qsum * term_mean(p, t, V);
        double et = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+:et)
        for (int i = 0; i < n; ++i) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double *f = fbuf + (size_t)tid * n * 3;
            for (int j = i; j < n; ++j) {
                double th[3], dth[3];
                for (int c = 0; c < 3; ++c)
                    theta1(wrap_min(xyz[3 * i + c] - xyz[3 * j + c], L[c]), L[c], s, &th[c], &dth[c]);
                double P = a * th[0] * th[1] * th[2];
                double qq = q[i] * q[j];
                if (i == j) { et += 0.5 * qq * P; continue; }
                et += qq * P;
                double g[3] = {a * dth[0] * th[1] * th[2], a * th[0] * dth[1] * th[2],
                               a * th[0] * th[1] * dth[2]};
                for (int c = 0; c < 3; ++c) { f[3 * i + c] -= qq * g[c]; f[3 * j + c] += qq * g[c]; }
            }
        }
        e += et;
    }
    for (int t = 0; t < nth; ++t)
        for (int k = 0; k < 3 * n; ++k) frc[k] += fbuf[(size_t)t * n * 3 + k];
    free(fbuf);
    return e;
}

/* F_inf(0) by summing the series at r = 0 */
double uo_far_inf0(const uo_params *p)
{
    double f[3];
    uo_far_inf(p, 0.0, f);
    return f[0];
}

/* g(U) = int_0^U u^2 exp(-u^2/2) du
 *      = sqrt(pi/2) erf(U/sqrt2) - U exp(-U^2/2)       (integration by parts),
 * and for U < 1, where that difference cancels, its Taylor series
 *      sum_k (-1/2)^k U^(2k+3) / (k! (2k+3)). */
static double gauss_moment2(double U)
{
    if (U >= 1.0)
        return sqrt(M_PI / 2.0) * erf(U / sqrt(2.0)) - U * exp(-U * U / 2.0);
    double term = U * U * U, sum = 0.0;
    for (int k = 0; k < 40; ++k) {
        sum += term / (2 * k + 3);
        term *= -U * U / (2.0 * (k + 1));
    }
    return sum;
}

/*
 * Volume integral of the near kernel, int N(|r|) d^3r over the ball r < r_c:
 *   4 pi int_0^rc (r - r^2 F_inf(r)) dr,  with, for each Gaussian term,
 *   int_0^R r^2 exp(-r^2/(2s^2)) dr = s^3 g(R/s).
 */
double uo_near_integral(const uo_params *p)
{
    double R = p->rc, acc = 0.0;
    int J = uo_series_len(p->b);
    for (int j = J - 1; j >= 0; --j) {
        double a, s;
        uo_term(p, j, &a, &s);
        acc += a * s * s * s * gauss_moment2(R / s);
    }
    return 4.0 * M_PI * (R * R / 2.0 - acc);
}

/*
 * Full u-series evaluation.
 *   xyz   [n][3] positions (any image), q [n] charges, box [3] edge lengths.
 *   forces [n][3] output (overwritten);
 *   parts [5] = E_near, E_far, E_self, E_bg, E.
 * E_bg is the energy of a net charge Q = sum q against the uniform
 * neutralising background (the k = 0 component of the near kernel, which the
 * k != 0 convention of eqs. 4, 9, 10 drops): -Q^2/(2V) int N d^3r.  It is
 * exactly zero for neutral input and carries no force.
 * Returns 0, or -1 on invalid parameters.
 */
int uo_eval(int n, const double *xyz, const double *q, const double box[3],
            const uo_params *p, double *forces, double parts[5])
{
    if (n < 0 || p->b <= 1.0 || p->sigma <= 0.0 || p->nterms < 0) return -1;
    if (kpow(p) != 1.0 && !(kpow(p) > 3.0)) return -1;   /* Coulomb or alpha > 3 */
    memset(forces, 0, sizeof(double) * 3 * (size_t)n);
    double en = near_part(n, xyz, q, box, p, forces);
    double ef = far_part(n, xyz, q, box, p, forces);
    double q2 = 0.0, qs = 0.0;
    for (int i = 0; i < n; ++i) { q2 += q[i] * q[i]; qs += q[i]; }
    double es = 0.5 * uo_far_inf0(p) * q2;
    double V = box[0] * box[1] * box[2];
    /* the neutralising background is a Coulomb matter; for alpha > 3 the
     * far part keeps its k = 0 components instead */
    double eb = kpow(p) == 1.0 ? -0.5 * qs * qs * uo_near_integral(p) / V : 0.0;
    parts[0] = en;
    parts[1] = ef;
    parts[2] = es;
    parts[3] = eb;
    parts[4] = en + ef - es + eb;
    return 0;
}

/* near and far parts separately (either output pointer may be NULL) */
int uo_eval_near(int n, const double *xyz, const double *q, const double box[3],
                 const uo_params *p, double *forces, double *energy)
{
    memset(forces, 0, sizeof(double) * 3 * (size_t)n);
    *energy = near_part(n, xyz, q, box, p, forces);
    return 0;
}

int uo_eval_far(int n, const double *xyz, const double *q, const double box[3],
                const uo_params *p, double *forces, double *energy)
{
    memset(forces, 0, sizeof(double) * 3 * (size_t)n);
    *energy = far_part(n, xyz, q, box, p, forces);
    return 0;
}

/*
 * Forces on a subset of atoms only (idx[0..m)), each by its own O(n) sum of
 * near and far contributions, written to out[m][3].  Used for sampled checks
 * at sizes where the full O(n^2) evaluation is too slow.
 */
int uo_forces_subset(int n, const double *xyz, const double *q, const double box[3],
                     const uo_params *p, int m, const int *idx, double *out)
{
    int M[3];
    for (int a = 0; a < 3; ++a) M[a] = (int)floor(p->rc / box[a] + 0.5);
    double at[64], st[64];
    if (p->nterms > 64) return -1;
    for (int t = 0; t < p->nterms; ++t) uo_term(p, t, &at[t], &st[t]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < m; ++k) {
        int i = idx[k];
        double f[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j) {
            double d0[3];
            for (int a = 0; a < 3; ++a) d0[a] = wrap_min(xyz[3 * i + a] - xyz[3 * j + a], box[a]);
            double qq = q[i] * q[j];
            /* near */
            for (int mx = -M[0]; mx <= M[0]; ++mx)
            for (int my = -M[1]; my <= M[1]; ++my)
            for (int mz = -M[2]; mz <= M[2]; ++mz) {
                if (i == j && mx == 0 && my == 0 && mz == 0) continue;
                double d[3] = {d0[0] + mx * box[0], d0[1] + my * box[1], d0[2] + mz * box[2]};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r >= p->rc) continue;
                double nk[2];
                uo_near(p, r, nk);
                double g = -qq * nk[1] / r;
                for (int a = 0; a < 3; ++a) f[a] += g * d[a];
            }
            if (i == j) continue;
            /* far */
            for (int t = 0; t < p->nterms; ++t) {
                double th[3], dth[3];
                for (int c = 0; c < 3; ++c) theta1(d0[c], box[c], st[t], &th[c], &dth[c]);
                f[0] -= qq * at[t] * dth[0] * th[1] * th[2];
                f[1] -= qq * at[t] * th[0] * dth[1] * th[2];
                f[2] -= qq * at[t] * th[0] * th[1] * dth[2];
            }
        }
        for (int a = 0; a < 3; ++a) out[3 * k + a] = f[a];
    }
    return 0;
}

/*
 * k-space form of the far part (App. F eq. F1; eq. 32 with S^ = 1):
 *   E_far = 1/(2V) sum_{k != 0} c(k) |S(k)|^2  (+ for alpha > 3 the k = 0
 *           components of all terms, 1/2 Q^2 sum_j a_j (2 pi s_j^2)^(3/2) / V),
 *   c(k) = sum_{t<N} a_t (2 pi s_t^2)^{3/2} exp(-s_t^2 k^2 / 2),
 *   S(k) = sum_j q_j exp(i k.r_j),
 *   F_i  = (q_i / V) sum_{k != 0} c(k) k Im(exp(i k.r_i) conj(S(k))).
 * All k with exp(-s_min^2 k^2/2) > 1e-18 are kept.
 */
int uo_far_kspace(int n, const double *xyz, const double *q, const double box[3],
                  const uo_params *p, double *forces, double *energy)
{
    double V = box[0] * box[1] * box[2];
    double smin = 1e300, at[64], st[64];
    if (p->nterms > 64 || p->nterms < 1) return -1;
    for (int t = 0; t < p->nterms; ++t) {
        uo_term(p, t, &at[t], &st[t]);
        if (st[t] < smin) smin = st[t];
    }
    double kmax = sqrt(2.0 * 18.0 * log(10.0)) / smin;
    int mm[3];
    for (int a = 0; a < 3; ++a) mm[a] = (int)ceil(kmax * box[a] / (2.0 * M_PI));
    memset(forces, 0, sizeof(double) * 3 * (size_t)n);
    double e = 0.0;
    int nx = 2 * mm[0] + 1, ny = 2 * mm[1] + 1, nz = 2 * mm[2] + 1;
    long nk = (long)nx * ny * nz;
    double *fr = calloc((size_t)n * 3, sizeof(double));
#pragma omp parallel
    {
        double *fl = calloc((size_t)n * 3, sizeof(double));
        double el = 0.0;
#pragma omp for schedule(dynamic, 8)
        for (long kk = 0; kk < nk; ++kk) {
            int m0 = (int)(kk % nx) - mm[0];
            int m1 = (int)((kk / nx) % ny) - mm[1];
            int m2 = (int)(kk / ((long)nx * ny)) - mm[2];
            if (m0 == 0 && m1 == 0 && m2 == 0) continue;
            double k[3] = {2 * M_PI * m0 / box[0], 2 * M_PI * m1 / box[1], 2 * M_PI * m2 / box[2]};
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            if (k2 > kmax * kmax) continue;
            double c = 0.0;
            for (int t = 0; t < p->nterms; ++t)
                c += at[t] * pow(2.0 * M_PI * st[t] * st[t], 1.5) * exp(-st[t] * st[t] * k2 / 2.0);
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < n; ++j) {
                double ph = k[0] * xyz[3 * j] + k[1] * xyz[3 * j + 1] + k[2] * xyz[3 * j + 2];
                sr += q[j] * cos(ph);
                si += q[j] * sin(ph);
            }
            el += c * (sr * sr + si * si) / (2.0 * V);
            for (int i = 0; i < n; ++i) {
                double ph = k[0] * xyz[3 * i] + k[1] * xyz[3 * i + 1] + k[2] * xyz[3 * i + 2];
                /* Im(exp(i ph) * (sr - i si)) = sin(ph) sr - cos(ph) si */
                double im = sin(ph) * sr - cos(ph) * si;
                double g = q[i] * c * im / V;
                for (int a = 0; a < 3; ++a) fl[3 * i + a] += g * k[a];
            }
        }
#pragma omp critical
        {
            e += el;
            for (int x = 0; x < 3 * n; ++x) fr[x] += fl[x];
        }
        free(fl);
    }
    memcpy(forces, fr, sizeof(double) * 3 * (size_t)n);
    free(fr);
    if (kpow(p) > 3.0) {
        /* alpha > 3: the k = 0 components of all terms (no force) */
        double qs = 0.0;
        for (int j = 0; j < n; ++j) qs += q[j];
        e += 0.5 * qs * qs * kzero_tail(p, 0, V);
    }
    *energy = e;
    return 0;
}

int uo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
