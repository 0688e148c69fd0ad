// Internal declarations shared by the library's sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/useries.h"

namespace useries {

constexpr int kMaxTerms = 32;      // far Gaussians N
constexpr int kMaxGrid = 128;      // grid points per axis
constexpr int kMaxPolyDeg = 14;    // near polynomial degree
constexpr int kMaxStencilHalf = 8; // P
constexpr int kMaxStencilCols = 128;  // x-y columns within r_c of a column (pair kernel)
constexpr int kMaxWindowCols = 256;   // x-y columns touching a spreading brick
constexpr int kPairSlices = 1;        // near-force slices per charge

// ------------------------------------------------------------ host math
// FP64 parameter math of the u-series (plan_math.cpp).
struct Series {
    double b = 2.0, sigma = 1.0, w0 = 1.0, s0 = 1.0;
    // amplitude and width of term j (eqs. 11, 24, 28)
    void term(int j, double* a, double* s) const;
    int length() const;                         // terms with b^-j > 1e-18
    double f_inf(double r, double* df = nullptr) const;   // all terms
    double g_inf(double r) const;               // F_inf'(r) / r, all terms
    double f_inf0() const;                      // closed form (w0 + 1/(b-1)) 2ln b/(sqrt(2pi) sigma)
    double near_integral(double rc) const;      // int_{|r|<rc} (1/r - F_inf) d^3r
};

int solve_construction(int construction, double b, double* b_out, double* r0, double* w0,
                       double* s0, std::string* err);
double c1_w0_of_r0(double b, double r0);       // eq. 25 at sigma = 1
double eq33_bound(int n, double b, double sigma, double lmax);
int choose_nterms(double b, double sigma, double lmax, double tol);
double bsa_bound(double b);

// monomial coefficients in x = r^2/rc^2 on [0,1] of F_inf(r) (fcoef) and of
// F_inf'(r)/r (gcoef), each fitted separately; returns the larger of the two
// max errors relative to the function's max magnitude, on a fine sample.
double fit_near_poly(const Series& s, double rc, int degree, double* fcoef, double* gcoef);

// first column k[m], m = 0..n-1, of the periodic circulant that convolves the
// grid with a Gaussian of width sk (grid spacing h), scaled by `scale`.
void circulant_column(int n, double h, double sk, double scale, double* k);

// ------------------------------------------------------------ device args
struct BinArgs {
    int n;
    int nc[2];            // x-y columns per axis
    double inv_box[3];    // 1/L
};

struct PairArgs {
    int n;
    int nc[2];            // x-y columns per axis
    int R[2];             // columns within reach of r_c per axis: ceil(r_c / cw)
    float scale[3];       // L / 2^32: fixed-point units to A
    float cw[2];          // column widths L / nc
    float zinv;           // 2^32 / L_z: A to fixed-point units along z
    float rc2;            // r_c^2
    float inv_rc2;        // 1 / r_c^2
    int deg;              // polynomial degree
    float c[kMaxPolyDeg + 1];   // F_inf(r) = sum c_k x^k, x = r^2/rc^2
    float c0lo;                 // c_0 - (float)c_0
    float d[kMaxPolyDeg + 1];   // F_inf'(r)/r = sum d_k x^k
};

struct GridArgs {
    int n;
    int g[3];             // grid points per axis
    int nc[2];            // x-y columns per axis (candidate search for spreading)
    int P;                // stencil half width: 2P points per axis
    float hs[3];          // h^2 / (2 sigma_s^2) per axis
    float cw[3];          // h / (sqrt(2 pi) sigma_s): weight prefactor per axis
    float dws[3];         // 2 hs / h: derivative factor of the weights per axis
    double inv_ngrid;     // 1 / (gx gy gz)
};

struct ConvArgs {
    int g[3];
    int gp[3];            // padded: multiple of 16 (FP32) or 32 (BF16X3)
    int nterms;
    int bf16x3;
};

struct FinalArgs {
    int n_pair_parts;
    int n_gather_parts;
    double f_inf0;        // self-term coefficient
    double near_int_over_v;   // int N d^3r / V (background)
};

// ------------------------------------------------------------ kernel launchers
// All launchers enqueue on `st` and return hipGetLastError().
hipError_t launch_encode(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                         int* col_of, int* col_count, double* qpart, int nqpart, hipStream_t st);
hipError_t launch_scan(int ncol, const int* col_count, int* col_start, int* clus_start,
                       int* col_fill, const double* qpart, int nqpart, double* qstats,
                       hipStream_t st);
hipError_t launch_scatter(int n, int ncol, const int* col_of, const int* col_start, int* col_fill,
                          int* slots, hipStream_t st);
hipError_t launch_colsort(int ncol, const int* col_start, const int* clus_start, const int* slots,
                          const uint4* coord, int* perm, uint4* sorted, int2* cl_info,
                          int* cl_col, uint2* cl_z, hipStream_t st);
hipError_t launch_pair(const PairArgs& a, int nblocks, const uint4* sorted, const int* clus_start,
                       const int2* cl_info, const int* cl_col, const uint2* cl_z, float4* fnear,
                       double* epart, hipStream_t st);
hipError_t launch_spread(const GridArgs& a, const uint4* sorted, const int* clus_start,
                         const int2* cl_info, const uint2* cl_z, const double* qstats, float* rho,
                         hipStream_t st);
hipError_t launch_conv_xy(const ConvArgs& a, const float* rho, const float* kx,
                          const float* ky, float* tgrid, hipStream_t st);
hipError_t launch_conv_z(const ConvArgs& a, const float* tgrid, const float* kz, float* phi,
                         hipStream_t st);
hipError_t launch_gather(const GridArgs& a, const uint4* sorted, const int* perm,
                         const float* phi, const float4* fnear, int slice_stride, float* forces,
                         double* epart, int nblocks, hipStream_t st);
int gather_blocks(int n);
hipError_t launch_finalize(const FinalArgs& a, const double* pair_parts,
                           const double* gather_parts, const double* qstats, double* energy,
                           double* parts, hipStream_t st);

}  // namespace useries
