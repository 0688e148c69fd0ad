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
constexpr int kMaxExact = 8;       // narrowest far terms evaluated as Gaussians in the near part
constexpr int kMaxStencilHalf = 8; // P
constexpr int kMaxStencilCols = 128;  // x-y columns within r_c of a column (pair kernel)
constexpr int kMaxWindowCols = 256;   // x-y columns touching a spreading brick

// ------------------------------------------------------------ host math
// FP64 parameter math of the u-series (plan_math.cpp).
// The far series of the kernel 1/r^alpha (alpha = 1: Coulomb, eqs. 11, 24,
// 28; alpha = 6: the BSA of App. A, eq. A2, with the Gaussian scaling
// function).
struct Series {
    double b = 2.0, sigma = 1.0, w0 = 1.0, s0 = 1.0;
    int alpha = 1;
    double pref() const;                        // a_j = pref w_j b^(-alpha j)
    // amplitude and width of term j
    void term(int j, double* a, double* s) const;
    int length() const;                         // terms with b^(-alpha j) > 1e-18
    double f_inf(double r, double* df = nullptr) const;   // all terms
    double g_inf(double r) const;               // F_inf'(r) / r, all terms
    double f_inf0() const;                      // closed form pref (w0 + 1/(b^alpha - 1))
    double near_integral(double rc) const;      // int_{|r|<rc} (1/r - F_inf) d^3r (alpha = 1)
    double kzero_sum(double V) const;           // sum_j a_j (2 pi s_j^2)^(3/2) / V (alpha > 3)
};

int solve_construction(int construction, double b, double* b_out, double* r0, double* w0,
                       double* s0, std::string* err);
// (r0, w0) of the C1 construction for 1/r^alpha (alpha = 1: eqs. 25-26)
int solve_c1_alpha(double b, int alpha, double* r0, double* w0, std::string* err);
double c1_w0_of_r0(double b, double r0);       // eq. 25 at sigma = 1
double c1_w0_of_r0_alpha(double b, int alpha, double r0);
double eq33_bound(int n, double b, double sigma, double lmax);
// the kernel-power form of eq. 33: b^((3 - alpha) n) exp(-2 (b^(2n) - 1) pi^2 sigma^2 / L^2)
double trunc_bound(int n, double b, int alpha, double sigma, double lmax);
int choose_nterms(double b, double sigma, double lmax, double tol);
int choose_nterms_alpha(double b, int alpha, double sigma, double lmax, double tol);
double bsa_bound(double b);

// monomial coefficients in x = r^2/rc^2 on [0,1] of F_inf(r) (fcoef) and of
// F_inf'(r)/r (gcoef) without their first `nexact` terms (which the pair
// kernel evaluates as Gaussians), each fitted separately; returns the larger
// of the two max errors relative to the full function's max magnitude, on a
// fine sample.
double fit_near_poly(const Series& s, double rc, int degree, int nexact, double* fcoef,
                     double* gcoef);

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
    float scale_lo[3];    // L / 2^32 - scale: the FP32 rounding of the scale
    float inv_scale;      // 1 / scale[0] (FP32)
    double inv_scale_d;   // 1 / scale[0] (FP64)
    float is2h, is2l;     // (1 / (scale[0] + scale_lo[0]))^2 as FP32 hi + lo
    float rcm2;           // (r_c + 1e-3)^2: the bounding-box test's reach
    float cw[2];          // column widths L / nc
    float zinv;           // 2^32 / L_z: A to fixed-point units along z
    float rc2;            // r_c^2
    float inv_rc2;        // 1 / r_c^2
    int gz;               // grid points along z (planes of the z-plane index)
    int deg;              // polynomial degree
    int alpha;            // kernel power: 1 (1/r), 6 (1/r^6) or 12 (1/r^12)
    int ne;               // leading far terms evaluated as Gaussians (0..kMaxExact)
    float c[kMaxPolyDeg + 1];   // F_inf(r) = sum_{j<ne} ea_j 2^(x ex_j) + sum c_k x^k, x = r^2/rc^2
    float d[kMaxPolyDeg + 1];   // F_inf'(r)/r = sum_{j<ne} eg_j 2^(x ex_j) + sum d_k x^k
    float ex[kMaxExact];        // -log2(e) rc^2 / (2 s_j^2)
    float ea[kMaxExact];        // a_j
    float eg[kMaxExact];        // -a_j / s_j^2
    // the same for distances in fixed-point units u = scale[0] (cubic cells,
    // the 1/r kernel): F u and (F'/r) u^3
    float cu[kMaxPolyDeg + 1], du[kMaxPolyDeg + 1];
    float eau[kMaxExact], egu[kMaxExact];
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

constexpr int kMaxSpecRank = 17;   // Fourier modes per axis of the spectral wide terms

struct ConvArgs {
    int g[3];
    int gp[3];            // padded: multiple of 16 (FP32) or 32 (BF16X3)
    int nterms;           // terms convolved with dense circulants (the narrowest ones)
    int bf16x3;
    // The wider terms that follow, in spectral form (spec = 1): each of their
    // circulants is U diag(lambda_t) U^T up to modes below 1e-9 of its first
    // one, U the n x r real Fourier basis (1, cos, sin of modes 1..K, r =
    // 2K + 1), so together they are (U_z x U_y x U_x) diag(W) (...)^T with W the
    // summed products of their per-axis eigenvalues (k = 0 removed).
    int spec;
    int rk[3];            // r per axis (x, y, z)
};

struct FinalArgs {
    int n_pair_parts;
    int n_far_parts;      // far-energy partials: one per z tile of each conv_z column block
    double f_inf0;        // self-term coefficient
    double near_int_over_v;   // int N d^3r / V (Coulomb background)
    double k0_far;        // alpha > 3: sum of the far terms' k = 0 means (the grid drops them)
};

// ------------------------------------------------------------ host plan
// Everything a plan computes on the host for one cell shape: parameters,
// kernel arguments and the convolution matrices in the device format
// (FP32, or per term the BF16 hi matrix followed by the lo matrix).
struct HostPlan {
    double box[3] = {0, 0, 0};
    double rc = 0, b = 2, sigma = 1, r0 = 1, w0 = 1, s0 = 1;
    int construction = USERIES_C1, precision = USERIES_PLAIN_FP32, alpha = 1;
    int nterms = 0, P = 5, deg = 8;
    int near_exact = 0;    // leading far terms the pair kernel evaluates as Gaussians
    int nterms_grid = 0;   // leading terms evaluated on the grid (the rest: k = 0 only)
    int nterms_spec = 0;   // of those, the widest ones, in spectral form (ConvArgs::spec)
    int grid[3] = {0, 0, 0};
    double eq33 = 0, f_inf0 = 0, c1_slope = 0, poly_maxerr = 0, sigma_s[3] = {0, 0, 0};
    int ncmax[2] = {1, 1};   // bounds of the x-y column grid (chosen per evaluation)
    int ncol_max = 1;
    BinArgs bin{};
    PairArgs pair{};
    GridArgs gridargs{};
    ConvArgs conv{};
    FinalArgs fin{};
    std::vector<uint8_t> mats[3];   // device-format matrices per axis (dense terms)
    std::vector<float> ubasis[3];   // spectral terms: n_a x r_a Fourier bases, row-major
    std::vector<float> wspec;       // spectral terms: W [r_z][r_y][r_x]
};

// Record the message returned by useries_last_error() in this thread; returns code.
int set_last_error(int code, const std::string& msg);

// Host part of useries_plan (no device calls).  Returns USERIES_OK or an
// error code with *err set.
int build_host_plan(HostPlan* hp, const double box[3], double r_c, double b, double sigma,
                    int n_terms, const int grid[3], const useries_opts* opts, std::string* err);


// The x-y column grid for n charges (about 8 charges per cluster of one
// column cross-section and similar z extent, within the plan's bounds):
// sets nc, R, cw and n in the kernel arguments.
void choose_columns(HostPlan* hp, int n);
// the columns along x-y axis a that choose_columns takes for n charges (never
// fewer for more charges)
int columns_per_axis(const HostPlan& p, int n, int a);

// dynamic LDS bytes of the conv_xy and conv_z kernels for a grid shape
size_t conv_xy_lds_bytes(const ConvArgs& a);
size_t conv_z_lds_bytes(const ConvArgs& a);
// blocks of the conv_z kernel (grid columns per block depend on the form and n_z)
int conv_z_blocks(const ConvArgs& a);
// far-energy partials written by conv_z (one per 16-row z tile of each block)
int far_parts(const ConvArgs& a);

// Blocks of the pair kernel for n charges (an upper bound of the clusters)
// and of the gather kernel (its bricks)
inline int pair_blocks(int n, int ncol) { return n / 8 + 1 + ncol; }
int gather_blocks(const GridArgs& a);

// ------------------------------------------------------------ batched evaluation
// Several independent cells evaluated by the same launches: every kernel of
// the sequence takes a table of the boxes in the batch and, per kernel, the
// prefix sums of the work items (blocks) of each box; a block finds its box
// by binary search and runs the same body as the one-box launch.  Grids are
// fixed (persistent, grid-stride over the items) so that one captured graph
// serves every batch composition.
constexpr int kMaxBatch = 64;
enum BatchKernel {
    BK_BINLOCAL, BK_ENCODE, BK_SCAN, BK_SCATTER, BK_COLSORT, BK_COLBUILD, BK_PAIR, BK_SPREAD,
    BK_CONV_XY, BK_CONV_Z, BK_GATHER, BK_DISPLACE, BK_COUNT
};

// One cell's arguments and device buffers (resident while its request runs)
struct BoxDesc {
    BinArgs bin;
    PairArgs pair;
    GridArgs grid;
    ConvArgs conv;
    FinalArgs fin;
    int ncol, nq, npb, ngb;   // columns, blocks of 256 charges, pair blocks, gather bricks
    int n_evals;
    float disp_sigma;          // displacement per coordinate between evaluations (A)
    uint32_t key[2];           // Philox key of the request
    // state and outputs
    float* xyz;                // [n][3]
    const float* q;            // [n]
    float* forces;             // [n][3], input order
    double* energies;          // [n_evals]
    // workspace
    uint4 *coord, *sorted;
    int *perm, *slots, *cl_col;
    int2* cl_info;
    uint2* cl_z;
    float4* fnear;
    double *qpart, *pair_parts, *far_parts, *qstats;
    int *col_count, *col_start, *col_fill, *clus_start;
    int* bpre;                 // two-launch binning's block prefixes (NULL: four launches)
    int* zbin;                 // [ncol][g_z + 1]: first charge of each grid z-plane per column
    float *rho, *tgrid, *phi;
    const float *kx, *ky, *kz;
};

struct BatchTable {
    int nbox;
    int slot[kMaxBatch];               // descriptor index of batch entry i
    int step[kMaxBatch];               // evaluation index of batch entry i
    int off[BK_COUNT][kMaxBatch + 1];  // work-item prefix per kernel
};

// Batched launchers: `grid` blocks, grid-stride over the table's items.
hipError_t launch_encode_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st);
hipError_t launch_scan_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st);
hipError_t launch_scatter_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st);
hipError_t launch_colsort_batch(const BatchTable* tab, const BoxDesc* desc, int grid, hipStream_t st);
hipError_t launch_bin_local_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                  hipStream_t st);
hipError_t launch_colbuild_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                 hipStream_t st);
// exact: some box of the batch evaluates leading far terms as Gaussians (ne > 0)
hipError_t launch_pair_batch(const BatchTable* tab, const BoxDesc* desc, int deg, bool exact,
                             int grid, hipStream_t st);
// P: the stencil half width of every box in the batch (compiled code for 3
// and 5), or 0 when they differ
hipError_t launch_spread_batch(const BatchTable* tab, const BoxDesc* desc, int P, int grid,
                               hipStream_t st);
hipError_t launch_conv_xy_batch(const BatchTable* tab, const BoxDesc* desc, int bf16x3,
                                size_t lds, int grid, hipStream_t st);
hipError_t launch_conv_z_batch(const BatchTable* tab, const BoxDesc* desc, int bf16x3, size_t lds,
                               int grid, hipStream_t st);
// lds >= gather_lds_bytes(P) of every box in the batch; a box's items are
// its bricks and then one that writes its energy total to energies[step]
hipError_t launch_gather_batch(const BatchTable* tab, const BoxDesc* desc, int P, size_t lds,
                               int grid, hipStream_t st);
// dynamic LDS of one gather block for stencil half width P
size_t gather_lds_bytes(int P);
hipError_t launch_displace_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                 hipStream_t st);

// ------------------------------------------------------------ one-box evaluation
// The per-charge workspace of one evaluation (device pointers).
struct AtomWs {
    uint4 *coord = nullptr, *sorted = nullptr;
    int *perm = nullptr, *slots = nullptr;
    int2* cl_info = nullptr;
    int* cl_col = nullptr;
    uint2* cl_z = nullptr;
    double* pair_parts = nullptr;
    float4* fnear = nullptr;
    double* qpart = nullptr;
    int* bpre = nullptr;       // per-block column prefixes of two-launch binning
    int64_t bpre_cap = 0;      // ints available there (0: four-launch binning only)
};

// The evaluation sequence of useries_eval / useries_eval_parts.  ws == NULL:
// the plan's own per-charge workspace (grown with hipMalloc when n exceeds
// it); otherwise the given one, and nothing is allocated.
int plan_eval(useries_plan_t p, int64_t n, const float* xyz, const float* q, float* forces,
              double* energy, double* parts, void* stream, const AtomWs* ws);
// bytes of the per-charge workspace of n charges, and its arrays at `base`
// (device memory of that many bytes, 256-byte aligned)
size_t atom_workspace_bytes(useries_plan_t p, int64_t n);
AtomWs atom_workspace_at(useries_plan_t p, int64_t n, char* base);
int plan_device(useries_plan_t p);

// ------------------------------------------------------------ kernel launchers
// All launchers enqueue on `st` and return hipGetLastError().
hipError_t launch_encode(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                         int* col_count, double* qpart, int nqpart, hipStream_t st);
hipError_t launch_scan(int ncol, int* col_count, int* col_start, int* clus_start,
                       int* col_fill, const double* qpart, int nqpart, double* qstats,
                       hipStream_t st);
// true when scatter takes the column offsets itself (no scan launch): the
// counts fit in its LDS and every block can afford to read them
bool scan_fused(int n, int ncol);
// writes each charge's input index to `slots` and its record to `sorted`, in
// column order (colsort then sorts each column in place)
hipError_t launch_scatter(const BinArgs& a, const uint4* coord, uint4* sorted, const int* col_count,
                          int* col_start, int* clus_start, int* col_fill, int* slots,
                          const double* qpart, int nqpart, double* qstats, hipStream_t st);
// also clears col_count and col_fill of the ncol columns
// cl_col holds each cluster's column as cx | cy << 16 (ncx columns along x);
// cluster numbers from the last cluster to npb get a count of 0
hipError_t launch_colsort(int ncol, int ncx, const int* col_start, const int* clus_start,
                          const int* slots, const uint4* coord, int* perm, uint4* sorted,
                          int2* cl_info, int* cl_col, uint2* cl_z, int gz, int* zbin,
                          int* col_count, int* col_fill, int npb, hipStream_t st);
// Two-launch binning (in place of encode, scan, scatter, colsort) for n > 0
// charges when bin_local_ok(n, ncol); bpre holds ceil(n / 256) (ncol + 1) ints.
// coord and slots hold the records and input indices grouped by column per
// block of 256 charges; the outputs are those of colsort, except that column
// c's clusters are numbered from floor(lo_c / 8) + c (lo_c: its first sorted
// charge) and every other number below npb has a count of 0.
bool bin_local_ok(int n, int ncol);
hipError_t launch_bin_local(const BinArgs& a, const float* xyz, const float* q, uint4* coord,
                            int* slots, int* bpre, double* qpart, hipStream_t st);
hipError_t launch_colbuild(int n, int ncol, int ncx, int gz, int npb, const int* bpre,
                           const uint4* coord, const int* slots, int* perm, uint4* sorted,
                           int2* cl_info, int* cl_col, uint2* cl_z, int* zbin,
                           const double* qpart, double* qstats, hipStream_t st);
// one block per cluster number below nblocks (those with a count of 0 only
// write a zero energy part)
hipError_t launch_pair(const PairArgs& a, int nblocks, const uint4* sorted,
                       const int2* cl_info, const int* cl_col, const uint2* cl_z, const int* zbin,
                       float4* fnear, double* epart, hipStream_t st);
hipError_t launch_spread(const GridArgs& a, const uint4* sorted, const int* zbin,
                         const double* qstats, float* rho, hipStream_t st);
// device buffers of the spectral wide terms (ConvArgs::spec)
struct SpecPtrs {
    const float *ux = nullptr, *uy = nullptr, *uz = nullptr;   // [g_a][r_a] bases
    const float* w = nullptr;                                  // [r_z][r_y][r_x]
    float* c = nullptr;                                        // [g_z][r_y][r_x] plane projections
};
// conv_xy also projects each plane onto the spectral basis (one more block
// per plane); conv_z adds the spectral terms' potential to its columns
hipError_t launch_conv_xy(const ConvArgs& a, const float* rho, const float* kx,
                          const float* ky, float* tgrid, const SpecPtrs& sp, hipStream_t st);
// fpart: far_parts(a) doubles, the sums of rho phi over each z tile's grid
// points (FP64), for the far energy 1/2 sum_g rho_g phi_g
hipError_t launch_conv_z(const ConvArgs& a, const float* tgrid, const float* kz, float* phi,
                         const float* rho, double* fpart, const SpecPtrs& sp, hipStream_t st);
// forces in input order; one more block than the bricks forms the energy
// total from the pair and far partials and the charge sums (energy, parts)
hipError_t launch_gather(const GridArgs& a, const uint4* sorted, const int* perm, const int* zbin,
                         const float* phi, const float4* fnear, float* forces,
                         const FinalArgs& fa, const double* pair_parts, const double* far_parts,
                         const double* qstats, double* energy, double* parts, hipStream_t st);

}  // namespace useries
