/*
 * useries.h -- C ABI of the MI355X (gfx950) u-series electrostatics library.
 *
 * The library evaluates the electrostatic energy and forces of n point
 * charges in an orthorhombic periodic cell with the u-series decomposition
 * of Predescu et al., "The u-series: A separable decomposition for
 * electrostatics computation with improved accuracy" (arXiv:1911.01377):
 *
 *   near part  (Sec. III.C, eq. 20; C1 construction eqs. 24-26):
 *              1/r - F(r) for r < r_c, summed pairwise over a cell list;
 *   far part   (Sec. V, eqs. 31-33): F truncated to N Gaussians, evaluated by
 *              spreading the charges to a grid, three periodic 1D
 *              convolutions per Gaussian (x, y, z), summing the terms and
 *              gathering potentials and forces back to the charges;
 *   self term  1/2 F(0) sum q_i^2 (the analogue of the Ewald self term, eq. 10);
 *   background for a net charge Q, the uniform neutralising background of
 *              the k != 0 convention (eqs. 4, 9, 10); zero for neutral input.
 *
 * Units are Gaussian with Coulomb constant 1: charges in e, lengths in
 * Angstrom, energies in e^2/A, forces in e^2/A^2 (multiply by 332.0637 for
 * kcal/mol).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: USERIES_OK (0) or a negative
 *    USERIES_E* code; useries_strerror() gives its text, and
 *    useries_last_error() a message about the most recent failure.
 *  - Device pointers are HIP device memory of the current device (for
 *    example from torch.empty(..., device="cuda") on ROCm); host pointers are
 *    ordinary process memory.  The caller owns every buffer it passes; the
 *    library owns its plans and their device workspaces.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Evaluation is asynchronous on that stream.  One plan may be used by one
 *    stream at a time.
 */
#ifndef USERIES_H
#define USERIES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct useries_plan_s *useries_plan_t;

/* status codes */
enum {
    USERIES_OK = 0,
    USERIES_EINVAL = -1,     /* invalid argument */
    USERIES_ENOMEM = -2,     /* device or host allocation failed / budget exceeded */
    USERIES_EHIP = -3,       /* a HIP runtime call failed */
    USERIES_EBUSY = -4,      /* resource busy (serving: no slot) */
    USERIES_ENOTFOUND = -5,  /* unknown handle or ticket */
    USERIES_ESTATE = -6      /* call not valid in the object's current state */
};

/* far-series constructions (Sec. III.C, Tables 1 and 2) */
enum {
    USERIES_C0 = 0,             /* eq. 19: w0 = 1, r_c = smallest root of eq. 21 */
    USERIES_C1 = 1,             /* eq. 24: w0 from eq. 25, r0 = smallest root of eq. 26 */
    USERIES_C2_B2 = 2,          /* eq. 28 with the b = 2 parameters of Table 2 row 3 */
    USERIES_TABLE1_ROW1 = 11,   /* C1 construction at the C2 points of Table 1 */
    USERIES_TABLE1_ROW2 = 12,
    USERIES_TABLE1_ROW3 = 13
};

/* arithmetic of the far-part convolutions */
enum {
    USERIES_PLAIN_FP32 = 0,     /* FP32 MFMA convolutions, 10^3 spreading stencil,
                                   degree-7 near polynomials */
    USERIES_BF16X3 = 1          /* BF16 MFMA with 3-product split precision,
                                   6^3 spreading stencil, degree-5 near polynomials */
};

/*
 * Optional plan settings.  Fill with useries_default_opts() and override.
 *   construction     one of the USERIES_C* / USERIES_TABLE1_* values.
 *   precision        USERIES_PLAIN_FP32 or USERIES_BF16X3.
 *   sigma_s_over_h   width of the Gaussian that spreads charges to the grid,
 *                    in units of the grid spacing of each axis; <= 0 picks
 *                    the default of the precision (0.9 plain, 0.74 BF16X3).
 *   stencil_half     P: each charge touches 2P grid points per axis; <= 0
 *                    picks the default (5 plain, 3 BF16X3).  1 <= P <= 8.
 *   nterms_tol       relative far-energy truncation bound (eq. 33) used to
 *                    choose N when useries_plan gets n_terms <= 0.
 *   poly_degree      degree in r^2 of the polynomials that represent the
 *                    infinite far series F and F'(r)/r inside the cutoff
 *                    (near part); <= 0 picks the default of the precision:
 *                    7 plain (fit error ~7e-8 of max |F|, FP32 level), 5
 *                    BF16X3 (~2e-5, well inside that form's 1e-3 budget).
 *                    4 <= degree <= 14.  The narrowest far Gaussians are
 *                    taken out of the polynomial and evaluated exactly when
 *                    the fit would miss the form's budget (near_exact in
 *                    useries_plan_info); if even 8 of them do not suffice,
 *                    useries_plan fails with USERIES_EINVAL.
 *   max_atoms        workspace capacity in charges; <= 0 grows on demand
 *                    (a growth reallocates and synchronises the device).
 *   alpha            kernel power: 1 (Coulomb 1/r, the default), 6 (1/r^6,
 *                    e.g. London dispersion) or 12 (1/r^12, the repulsive
 *                    Lennard-Jones power); App. A.  With alpha > 1 the series
 *                    is the BSA of eq. A2 with a Gaussian scaling function
 *                    (a_j = ln b w_j b^(-alpha j) / (phi~(alpha) sigma^alpha),
 *                    phi~(alpha) = 2^(alpha/2 - 1) Gamma(alpha/2): 8 for 6,
 *                    3840 for 12), the construction must be USERIES_C1
 *                    (solved for 1/r^alpha at any b > 1: continuity and zero
 *                    slope at r_c), the "charges" are the coefficients c_i of
 *                    E = 1/2 sum'_{i,j,images} c_i c_j / r^alpha (no
 *                    neutrality: the lattice sum converges absolutely, and
 *                    every far term's k = 0 component is kept), and n_terms
 *                    <= 0 takes the smallest N with b^((3 - alpha) N)
 *                    exp(-2 (b^(2N) - 1) pi^2 sigma^2 / L^2) <= nterms_tol
 *                    (eq. 33's form for 1/r^alpha).  The Table 1 and 2
 *                    presets are Coulomb series.
 *   spectral         apply the widest far terms together in spectral form
 *                    (a low-rank form of their circulants: the real Fourier
 *                    modes each needs down to 1e-9 of its first mode, at most
 *                    17 per axis and a quarter of the axis), so that the
 *                    convolution cost stops growing with them.  < 0 (the
 *                    default): when at least six terms qualify (fewer cost
 *                    less as dense matrix-core convolutions); > 0: when at
 *                    least two do; 0: every term as a dense circulant.  The
 *                    count is n_terms_spectral in useries_plan_info.
 */
typedef struct {
    int construction;
    int precision;
    double sigma_s_over_h;
    int stencil_half;
    double nterms_tol;
    int poly_degree;
    int64_t max_atoms;
    int alpha;
    int spectral;
} useries_opts;

/* Fill *opts with the defaults: C1, PLAIN_FP32, nterms_tol 1e-8, the rest
 * "pick the default".  Returns USERIES_EINVAL for NULL. */
int useries_default_opts(useries_opts *opts);

/*
 * Build a plan for one cell shape (host work, then one upload).
 *   out      receives the plan handle.
 *   box      host [3]: edge lengths Lx, Ly, Lz > 0 of the orthorhombic cell.
 *   r_c      cutoff radius; 0 < r_c < min(L)/2.
 *   b        base of the series (> 1).  Ignored by the presets
 *            USERIES_C2_B2 and USERIES_TABLE1_*, which fix b.
 *   sigma    <= 0: sigma = r_c / r0 (Sec. III.C, eq. 23), the construction's
 *            own r0.  > 0: for C0 and C1 the cutoff stays r_c and w0 is
 *            re-solved from eq. 25 at r0 = r_c / sigma, which keeps the near
 *            part continuous at r_c (its slope then need not vanish).  The
 *            presets require sigma <= 0 or sigma = r_c / r0 within 1e-12.
 *   n_terms  N, the far Gaussians kept (Sec. V); <= 0 picks the smallest N
 *            whose eq. 33 bound is <= opts->nterms_tol.  At most 32.  Terms
 *            that are constant on the cell to 2^-60 besides their k = 0 mode
 *            are not evaluated on the grid (n_terms_grid, useries_plan_info).
 *   grid     host [3]: far-part grid points per axis, 2P <= n <= 128.
 *            Each axis needs its grid spacing h with
 *            s_0^2 > 2 (sigma_s_over_h * h)^2 (the spreading Gaussians must
 *            be narrower than the narrowest far Gaussian, Sec. IV.A).  For
 *            the plain form's accuracy keep h at or below about s_0 / 2
 *            (s_0 = sigma s0): the grid carries s_0 through narrower
 *            Gaussians still, and at h = 0.6 s_0 the far part already errs
 *            by about 1e-5 of the total energy.  Small b (Table 1) makes
 *            sigma = r_c / r0 small and so needs finer grids.
 *   opts     NULL for the defaults.
 * Errors: USERIES_EINVAL (bad argument or unsatisfiable constraint),
 * USERIES_ENOMEM, USERIES_EHIP.  The plan uses the current HIP device.
 */
int useries_plan(useries_plan_t *out, const double box[3], double r_c, double b,
                 double sigma, int n_terms, const int grid[3], const useries_opts *opts);

/*
 * Energy and forces of n charges (asynchronous on `stream`).
 *   xyz      device float [n][3]: positions in A, any periodic image.
 *   q        device float [n]: charges in e.
 *   forces   device float [n][3]: OVERWRITTEN with the forces, in the order
 *            of the inputs; never read.
 *   energy   device double [1]: OVERWRITTEN with the total energy.
 * n may be 0 (energy 0).  Coincident charges (r = 0 between two different
 * charges) are outside the contract.  Errors: USERIES_EINVAL (n < 0, NULL
 * pointers with n > 0, n above a fixed max_atoms), USERIES_ENOMEM,
 * USERIES_EHIP.
 */
int useries_eval(useries_plan_t plan, int64_t n, const float *xyz, const float *q,
                 float *forces, double *energy, void *stream);

/*
 * As useries_eval, and also writes the parts of the energy to
 *   parts    device double [5]: E_near, E_far (grid, k = 0 removed), E_self,
 *            E_background, E_total (= E_near + E_far - E_self + E_background).
 * `energy` may be NULL.
 */
int useries_eval_parts(useries_plan_t plan, int64_t n, const float *xyz, const float *q,
                       float *forces, double *energy, double *parts, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * useries_eval_parts (energy and parts may each be NULL, not both), with
 * the per-charge workspace (encoded and sorted positions, permutation,
 * cluster table, near forces, energy partials) in a fixed 16 MiB device
 * array of the library instead of memory the plan allocates on demand; the
 * call allocates nothing.  Enough for about 270,000 charges (the exact limit
 * depends on the plan's column grid); a larger n fails with USERIES_EINVAL
 * before anything is launched.  Each GPU holds one such array for the whole
 * process, shared by every plan on it: calls that overlap on one GPU (other
 * streams, other threads) race on it and must be ordered by the caller.
 * Errors: as useries_eval_parts, and USERIES_EHIP if the array's device
 * address cannot be obtained.
 */
int useries_eval_static(useries_plan_t plan, int64_t n, const float *xyz, const float *q,
                        float *forces, double *energy, double *parts, void *stream);

/*
 * Host copies of the plan's parameters (any pointer may be NULL):
 *   b, sigma, r0 (= r_c / sigma), w0, s0, n_terms, eq33 (the eq. 33 bound at
 *   n_terms with L = max edge), f_inf0 (F(0) of the infinite series, the
 *   self-term coefficient), c1_slope (N'(r_c) of the near part; 0 for C1),
 *   sigma_s (spreading width along x, A), stencil_half, ncell[3] (the x-y
 *   column grid used by the latest evaluation, chosen per evaluation from
 *   the number of charges; third entry 1; zeros before the first
 *   evaluation), poly_maxerr (max relative error of the near polynomial on
 *   [0, r_c], measured in FP64 on the host), n_terms_grid (the leading far
 *   terms evaluated on the grid: a term whose periodised Gaussian has every
 *   non-zero Fourier mode below 2^-60 of its k = 0 mode is, to double
 *   precision, only that mode, which the far part removes, so it is skipped),
 *   near_exact (the narrowest far Gaussians that the near part evaluates as
 *   exponentials instead of through the polynomial: the plan takes the
 *   fewest, 0 to 8, that bring the polynomial's fit error within the form's
 *   budget, 1e-7 of max |F| plain and 2e-5 BF16X3; small b, as in Table 1,
 *   needs them because its narrowest Gaussians lie deep inside r_c),
 *   n_terms_spectral (of the n_terms_grid terms, the widest ones applied in
 *   spectral form; 0 unless opts->spectral) and spectral_rank[3] (the real
 *   Fourier modes per axis they use; zeros when none).
 */
int useries_plan_info(useries_plan_t plan, double *b, double *sigma, double *r0, double *w0,
                      double *s0, int *n_terms, double *eq33, double *f_inf0,
                      double *c1_slope, double *sigma_s, int *stencil_half, int ncell[3],
                      double *poly_maxerr, int *n_terms_grid, int *near_exact,
                      int *n_terms_spectral, int spectral_rank[3]);

/* Release a plan and its device memory.  The caller must ensure that no
 * evaluation on it is still running. */
int useries_destroy(useries_plan_t plan);

/*
 * Per-kernel timing.  When enabled, each evaluation records HIP events
 * around each kernel on the evaluation stream; useries_timing_read (after the
 * stream has been synchronised) returns, for kernel k of the sequence
 * (bin_local, encode, scan, scatter, colsort, colbuild, pair, spread, conv_xy,
 * conv_z, gather: the binning runs either bin_local and colbuild or the four
 * kernels between them), its name, the summed duration in ms and the number
 * of launches timed (0 for kernels not run).
 * Enabling resets the sums.  Returns USERIES_ENOTFOUND when k is out of range.
 */
int useries_timing_enable(useries_plan_t plan, int enable);
int useries_timing_read(useries_plan_t plan, int k, const char **name, double *total_ms,
                        int64_t *launches);

/* ----------------------------------------------------------- serving */
/*
 * A server evaluates a stream of independent requests.  Each request is one
 * periodic cell (its own box, cutoff, grid and charges) evaluated n_evals
 * times; between two evaluations every coordinate moves by a normal deviate
 * of standard deviation disp_sigma drawn on the device from Philox4x32-10
 * (counter: charge index, evaluation index; key: the request's seed), so a
 * request's trajectory depends on nothing but the request.
 *
 * Continuous batching: a worker thread owns one HIP stream.  All running
 * requests advance together, one evaluation per step, in one sequence of
 * batched kernels, launched one by one by default (or, with the use_graph
 * option, as one captured HIP graph replay per step): every kernel takes a
 * table of the boxes in the batch and the per-box work-item offsets.
 * Between steps finished requests leave and waiting ones are admitted, as
 * batch slots and device memory allow.  Each request's positions, cell
 * lists, grids and convolution matrices stay resident in a device arena of
 * hbm_budget bytes, allocated once; a request is admitted when a slot is
 * free and its workspace fits in the arena (first fit, in arrival order,
 * with later requests allowed ahead of a waiting one for a bounded number of
 * rounds).  The arithmetic of a box does not depend on the rest of the batch:
 * each result is bitwise the same alone and in any mix.
 *
 * Parameters of every request: the construction and b of the server options,
 * sigma = r_c / r0, the eq. 33 term count at the options' tolerance, and the
 * precision form of the server.
 */
typedef struct useries_server_s *useries_server_t;

/* request states */
enum {
    USERIES_PENDING = 0,   /* queued, not yet admitted */
    USERIES_RUNNING = 1,   /* admitted: resident on the device, evaluations in progress */
    USERIES_DONE = 2,      /* outputs written to the request's host buffers */
    USERIES_ERROR = 3      /* failed; useries_poll sets the message of useries_last_error() */
};

/*
 * One request.  Every pointer is host memory owned by the caller and must
 * stay valid until useries_poll reports DONE or ERROR.
 *   n          charges, >= 1.
 *   xyz, q     [n][3] positions (A, any image) and [n] charges (e).
 *   box        cell edges; r_c cutoff (0 < r_c < min(L)/2); grid points per
 *              axis (2P <= n_a <= 128).
 *   n_evals    evaluations, >= 1.
 *   disp_sigma displacement per coordinate between evaluations (A), >= 0.
 *   seed       Philox key of the request's displacements.
 *   energies   [n_evals] out: total energy of each evaluation.
 *   forces     [n][3] out: forces of the last evaluation, input order.
 *   xyz_final  [n][3] out, or NULL: positions of the last evaluation.
 */
typedef struct {
    int64_t n;
    const float *xyz;
    const float *q;
    double box[3];
    double r_c;
    int grid[3];
    int n_evals;
    double disp_sigma;
    uint64_t seed;
    double *energies;
    float *forces;
    float *xyz_final;
} useries_request;

/*
 * Server options (useries_server_default_opts fills the defaults).
 *   construction, b, nterms_tol, poly_degree: as in useries_opts / useries_plan
 *              (defaults C1, b = 2, 1e-8, 0 = the precision's degree).
 *   use_graph  0: the step's kernels launched one by one (default); 1: one
 *              captured HIP graph per step (a graph is captured per set of
 *              dynamic LDS sizes and stencil width).  Launching a graph whose
 *              previous launch is still running blocks the host here, so the
 *              default keeps the worker free for admissions and retirements.
 *   inflight   steps enqueued ahead of the device (1..4, default 2).
 */
typedef struct {
    int construction;
    double b;
    double nterms_tol;
    int poly_degree;
    int use_graph;
    int inflight;
} useries_server_opts;

int useries_server_default_opts(useries_server_opts *opts);

/*
 * Create a server on the current HIP device.
 *   hbm_budget_bytes  device memory for the resident request workspaces
 *                     (allocated at once; >= 1 MiB).
 *   max_slots         requests in flight together, 1..64.
 *   precision         USERIES_PLAIN_FP32 or USERIES_BF16X3.
 *   opts              NULL for the defaults.
 * Errors: USERIES_EINVAL, USERIES_ENOMEM (budget not available), USERIES_EHIP.
 */
int useries_server_create(useries_server_t *out, size_t hbm_budget_bytes, int max_slots,
                          int precision, const useries_server_opts *opts);

/*
 * Queue a request (non-blocking apart from the host FP64 plan math of the
 * request's cell).  *ticket receives its handle.  A request that can never
 * fit (workspace above the budget, grid beyond the device's LDS) fails here
 * with USERIES_ENOMEM / USERIES_EINVAL and gets no ticket.
 */
int useries_submit(useries_server_t server, const useries_request *req, uint64_t *ticket);

/* hold != 0: admit no further requests (running ones go on); hold = 0:
 * resume.  Lets a caller queue a group that is then admitted together. */
int useries_server_hold(useries_server_t server, int hold);

/* Current state of a ticket (USERIES_PENDING .. USERIES_ERROR).
 * USERIES_ENOTFOUND for an unknown ticket. */
int useries_poll(useries_server_t server, uint64_t ticket, int *state);

/* Block until the ticket is DONE or ERROR; *state receives the final state. */
int useries_wait(useries_server_t server, uint64_t ticket, int *state);

/* Host wall-clock times (s, since the server's creation) of a ticket's
 * submission, admission to the device and completion (negative if not yet). */
int useries_request_times(useries_server_t server, uint64_t ticket, double *t_submit,
                          double *t_admit, double *t_done);

/*
 * Counters: out[0] steps launched, out[1] evaluations completed,
 * out[2] requests completed, out[3] largest batch, out[4] summed batch size
 * over steps, out[5] graphs instantiated.
 */
int useries_server_stats(useries_server_t server, int64_t out[6]);

/* Finish every queued request, stop the worker and free the server. */
int useries_server_destroy(useries_server_t server);

/* Host copy of the Philox4x32-10 bijection the displacements use
 * (counter[4], key[2] -> out[4]); for known-answer tests. */
void useries_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4]);

/* ----------------------------------------------------------- host math */
/* These touch no device and may be called without a GPU. */

/* (r0, w0, s0) of a construction at base b (b is ignored by the presets).
 * C0: eqs. 19-21; C1: eqs. 24-26, smallest root, including tangential
 * (double) roots at the C2 points of eq. 27; presets: Tables 1 and 2.
 * Writes *b_out with the base actually used.  USERIES_EINVAL if b <= 1 or no
 * root is found below r = 50. */
int useries_solve_construction(int construction, double b, double *b_out, double *r0,
                               double *w0, double *s0);

/* eq. 33: relative bound on the far energy truncated to n terms. */
double useries_eq33_bound(int n, double b, double sigma, double lmax);

/* smallest n in [1, 32] with useries_eq33_bound(n, ...) <= tol (32 if none) */
int useries_choose_nterms(double b, double sigma, double lmax, double tol);

/* eq. 14: asymptotic bound M_b of the relative error of the series */
double useries_bsa_bound(double b);

/* text of a status code, and a message about the latest failure in this thread */
const char *useries_strerror(int code);
const char *useries_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* USERIES_H */
