// C ABI of the library: plan construction (host FP64 math + one upload),
// device workspace, and the evaluation sequence
//   encode -> scan -> scatter -> colsort -> pair (near part)
//   -> spread -> conv_xy -> conv_z -> gather (far part, + near forces)
//   -> finalize (FP64 energy).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "useries_internal.h"

using namespace useries;

namespace useries {
size_t conv_xy_lds_bytes(const ConvArgs& a);
}

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(USERIES_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr const char* kKernelNames[] = {"encode", "scan",   "scatter", "colsort", "pair",
                                        "spread", "conv_xy", "conv_z", "gather",  "finalize"};
constexpr int kNumKernels = sizeof(kKernelNames) / sizeof(kKernelNames[0]);

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

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

struct useries_plan_s {
    int device = 0;
    // parameters
    double box[3] = {0, 0, 0};
    double rc = 0, b = 2, sigma = 1, r0 = 1, w0 = 1, s0 = 1;
    int construction = USERIES_C1, precision = USERIES_PLAIN_FP32;
    int nterms = 0;
    double eq33 = 0, f_inf0 = 0, c1_slope = 0, poly_maxerr = 0, sigma_s[3] = {0, 0, 0};
    int P = 5;
    int grid[3] = {0, 0, 0};
    int ncmax[2] = {1, 1};   // x-y column grid bounds (the grid itself is chosen per evaluation)
    int ncol_max = 1;
    int nc_used[2] = {0, 0};
    // kernel arguments
    BinArgs bin{};
    PairArgs pair{};
    GridArgs gridargs{};
    ConvArgs conv{};
    FinalArgs fin{};
    // device constants
    float *kx = nullptr, *ky = nullptr, *kz = nullptr;
    // fixed workspace
    int *col_count = nullptr, *col_start = nullptr, *col_fill = nullptr, *clus_start = nullptr;
    double *qstats = nullptr, *parts_tmp = nullptr;
    float *rho = nullptr, *tgrid = nullptr, *phi = nullptr;
    // per-atom workspace
    int64_t cap = 0;
    bool fixed_cap = false;
    uint4 *coord = nullptr, *sorted = nullptr;
    int *col_of = nullptr, *perm = nullptr, *slots = nullptr;
    int2* cl_info = nullptr;
    int* cl_col = nullptr;
    uint2* cl_z = nullptr;
    int64_t clmax = 0;
    float4* fnear = nullptr;
    double *qpart = nullptr, *pair_parts = nullptr, *gather_parts = nullptr;
    // timing
    bool timing = false;
    double tsum[kNumKernels] = {0};
    int64_t tcount[kNumKernels] = {0};
    struct Pending {
        int k;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;

    void free_atoms() {
        hipFree(coord);
        hipFree(sorted);
        hipFree(col_of);
        hipFree(cl_info);
        hipFree(cl_col);
        hipFree(cl_z);
        hipFree(pair_parts);
        hipFree(perm);
        hipFree(slots);
        hipFree(fnear);
        hipFree(qpart);
        hipFree(gather_parts);
        coord = sorted = nullptr;
        col_of = perm = slots = cl_col = nullptr;
        cl_info = nullptr;
        cl_z = nullptr;
        pair_parts = nullptr;
        fnear = nullptr;
        qpart = gather_parts = nullptr;
        cap = 0;
    }

    int alloc_atoms(int64_t n) {
        free_atoms();
        const int64_t c = std::max<int64_t>(n, 256);
        hipError_t e;
        clmax = c / 8 + 1 + ncol_max;   // clusters: sum over columns of ceil(count / 8)
        if ((e = dalloc(&coord, c)) || (e = dalloc(&sorted, c)) || (e = dalloc(&col_of, c)) ||
            (e = dalloc(&perm, c)) || (e = dalloc(&slots, c)) || (e = dalloc(&cl_info, clmax)) ||
            (e = dalloc(&cl_col, clmax)) || (e = dalloc(&cl_z, clmax)) ||
            (e = dalloc(&pair_parts, clmax)) ||
            (e = dalloc(&fnear, (size_t)kPairSlices * c)) ||
            (e = dalloc(&qpart, 2 * (size_t)((c + 255) / 256))) ||
            (e = dalloc(&gather_parts, (size_t)gather_blocks((int)c)))) {
            free_atoms();
            return fail(USERIES_ENOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
        }
        cap = c;
        return USERIES_OK;
    }

    hipEvent_t get_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hipEventCreate(&e);
        return e;
    }

    void harvest() {
        for (auto& p : pending) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                tsum[p.k] += ms;
                tcount[p.k] += 1;
            }
            event_pool.push_back(p.a);
            event_pool.push_back(p.b);
        }
        pending.clear();
    }

    ~useries_plan_s() {
        harvest();
        for (auto e : event_pool) hipEventDestroy(e);
        free_atoms();
        hipFree(kx);
        hipFree(ky);
        hipFree(kz);
        hipFree(col_count);
        hipFree(col_start);
        hipFree(col_fill);
        hipFree(clus_start);
        hipFree(qstats);
        hipFree(parts_tmp);
        hipFree(rho);
        hipFree(tgrid);
        hipFree(phi);
    }
};

namespace {

// RAII: make the plan's device current for the duration of a call
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

int upload_matrices(useries_plan_s* p, const std::vector<double> (&mats)[3]) {
    // mats[a] holds nterms padded gp x gp matrices (row-major) per axis
    float** dst[3] = {&p->kx, &p->ky, &p->kz};
    for (int a = 0; a < 3; ++a) {
        const size_t m = (size_t)p->conv.gp[a] * p->conv.gp[a];
        hipError_t e;
        if (p->precision == USERIES_BF16X3) {
            std::vector<uint16_t> h(2 * m * p->nterms);
            for (int t = 0; t < p->nterms; ++t)
                for (size_t k = 0; k < m; ++k) {
                    const float v = (float)mats[a][t * m + k];
                    const uint16_t hi = host_bf16(v);
                    const uint16_t lo = host_bf16(v - host_bf16_val(hi));
                    h[2 * m * t + k] = hi;
                    h[2 * m * t + m + k] = lo;
                }
            if ((e = hipMalloc((void**)dst[a], h.size() * sizeof(uint16_t))))
                return fail(USERIES_ENOMEM, "convolution matrices");
            if ((e = hipMemcpy(*dst[a], h.data(), h.size() * sizeof(uint16_t),
                               hipMemcpyHostToDevice)))
                return hip_fail(e, "upload");
        } else {
            std::vector<float> h(m * p->nterms);
            for (size_t k = 0; k < h.size(); ++k) h[k] = (float)mats[a][k];
            if ((e = hipMalloc((void**)dst[a], h.size() * sizeof(float))))
                return fail(USERIES_ENOMEM, "convolution matrices");
            if ((e = hipMemcpy(*dst[a], h.data(), h.size() * sizeof(float),
                               hipMemcpyHostToDevice)))
                return hip_fail(e, "upload");
        }
    }
    return USERIES_OK;
}

}  // namespace

extern "C" {

int useries_default_opts(useries_opts* o) {
    if (!o) return fail(USERIES_EINVAL, "NULL opts");
    o->construction = USERIES_C1;
    o->precision = USERIES_PLAIN_FP32;
    o->sigma_s_over_h = 0.0;
    o->stencil_half = 0;
    o->nterms_tol = 1e-8;
    o->poly_degree = 0;
    o->max_atoms = 0;
    return USERIES_OK;
}

int useries_plan(useries_plan_t* out, const double box[3], double r_c, double b, double sigma,
                 int n_terms, const int grid[3], const useries_opts* opts) {
    if (!out || !box || !grid) return fail(USERIES_EINVAL, "NULL argument");
    *out = nullptr;
    useries_opts o;
    useries_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != USERIES_PLAIN_FP32 && o.precision != USERIES_BF16X3)
        return fail(USERIES_EINVAL, "unknown precision");
    const bool bf = o.precision == USERIES_BF16X3;
    const double ratio = o.sigma_s_over_h > 0 ? o.sigma_s_over_h : (bf ? 0.83 : 0.9);
    const int P = o.stencil_half > 0 ? o.stencil_half : (bf ? 4 : 5);
    const int deg = o.poly_degree > 0 ? o.poly_degree : 8;
    if (P < 1 || P > kMaxStencilHalf) return fail(USERIES_EINVAL, "stencil_half out of [1, 8]");
    if (deg < 4 || deg > kMaxPolyDeg) return fail(USERIES_EINVAL, "poly_degree out of [4, 14]");
    if (!(o.nterms_tol > 0)) return fail(USERIES_EINVAL, "nterms_tol must be > 0");
    double lmin = 1e300, lmax = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(box[a] > 0) || !std::isfinite(box[a])) return fail(USERIES_EINVAL, "box edges must be > 0");
        lmin = std::min(lmin, box[a]);
        lmax = std::max(lmax, box[a]);
        if (grid[a] < 2 * P || grid[a] > kMaxGrid)
            return fail(USERIES_EINVAL, "grid points per axis must lie in [2P, 128]");
    }
    if (!(r_c > 0) || !(r_c < 0.5 * lmin)) return fail(USERIES_EINVAL, "need 0 < r_c < min(L)/2");
    if (n_terms > kMaxTerms) return fail(USERIES_EINVAL, "n_terms > 32");

    double bb, r0c, w0c, s0c;
    std::string err;
    int rc = solve_construction(o.construction, b, &bb, &r0c, &w0c, &s0c, &err);
    if (rc) return fail(rc, err);

    auto* p = new useries_plan_s();
    hipGetDevice(&p->device);
    std::memcpy(p->box, box, sizeof(p->box));
    std::memcpy(p->grid, grid, sizeof(p->grid));
    p->rc = r_c;
    p->b = bb;
    p->s0 = s0c;
    p->construction = o.construction;
    p->precision = o.precision;
    p->P = P;
    const bool preset = o.construction != USERIES_C0 && o.construction != USERIES_C1;
    if (sigma <= 0) {
        p->r0 = r0c;
        p->w0 = w0c;
        p->sigma = r_c / r0c;
    } else if (preset) {
        if (std::fabs(sigma * r0c / r_c - 1.0) > 1e-12) {
            delete p;
            return fail(USERIES_EINVAL, "preset constructions fix sigma = r_c / r0");
        }
        p->r0 = r0c;
        p->w0 = w0c;
        p->sigma = sigma;
    } else {
        // continuity correction: keep r_c, re-solve w0 of eq. 25 at r0 = r_c / sigma
        p->sigma = sigma;
        p->r0 = r_c / sigma;
        p->w0 = c1_w0_of_r0(bb, p->r0);
    }
    p->nterms = n_terms > 0 ? n_terms : choose_nterms(bb, p->sigma, lmax, o.nterms_tol);
    p->eq33 = eq33_bound(p->nterms, bb, p->sigma, lmax);

    Series s;
    s.b = bb;
    s.sigma = p->sigma;
    s.w0 = p->w0;
    s.s0 = p->s0;
    p->f_inf0 = s.f_inf0();
    double dF;
    s.f_inf(r_c, &dF);
    p->c1_slope = -1.0 / (r_c * r_c) - dF;

    // near part
    double coef[kMaxPolyDeg + 1], gcoef[kMaxPolyDeg + 1];
    p->poly_maxerr = fit_near_poly(s, r_c, deg, coef, gcoef);
    PairArgs& pa = p->pair;
    pa.deg = deg;
    for (int k = 0; k <= deg; ++k) pa.c[k] = (float)coef[k];
    pa.c0lo = (float)(coef[0] - (double)pa.c[0]);
    for (int k = 0; k <= deg; ++k) pa.d[k] = (float)gcoef[k];
    pa.rc2 = (float)(r_c * r_c);
    pa.inv_rc2 = (float)(1.0 / (r_c * r_c));

    // x-y columns: at least r_c / 4 wide (so the pair stencil stays within
    // 9 x 9 columns), and wide enough that a spreading brick touches at most
    // 16 columns per axis; the grid used is chosen per evaluation from n
    for (int a = 0; a < 2; ++a) {
        const double h = box[a] / grid[a];
        const double wmin = std::max(0.25 * r_c, (8 + 2 * P - 1) * h / 14.0);
        p->ncmax[a] = std::max(1, (int)std::floor(box[a] / wmin));
    }
    while ((int64_t)p->ncmax[0] * p->ncmax[1] > (1 << 20)) {
        const int am = p->ncmax[1] > p->ncmax[0] ? 1 : 0;
        p->ncmax[am] = std::max(1, p->ncmax[am] * 3 / 4);
    }
    p->ncol_max = p->ncmax[0] * p->ncmax[1];
    for (int a = 0; a < 3; ++a) {
        p->bin.inv_box[a] = 1.0 / box[a];
        pa.scale[a] = (float)(box[a] / 4294967296.0);
    }
    pa.zinv = (float)(4294967296.0 / box[2]);

    // far part
    GridArgs& ga = p->gridargs;
    ga.P = P;
    ga.inv_ngrid = 1.0 / ((double)grid[0] * grid[1] * grid[2]);
    ConvArgs& ca = p->conv;
    ca.nterms = p->nterms;
    ca.bf16x3 = bf ? 1 : 0;
    const double pi = 3.14159265358979323846;
    std::vector<double> mats[3];
    for (int a = 0; a < 3; ++a) {
        const double h = box[a] / grid[a];
        const double ss = ratio * h;
        p->sigma_s[a] = ss;
        ga.g[a] = ca.g[a] = grid[a];
        // padded to the MFMA K step: 4 (FP32, tiles of 16) or 32 (BF16)
        ca.gp[a] = bf ? (grid[a] + 31) / 32 * 32 : (grid[a] + 15) / 16 * 16;
        ga.hs[a] = (float)(h * h / (2.0 * ss * ss));
        ga.cw[a] = (float)(h / (std::sqrt(2.0 * pi) * ss));
        ga.dws[a] = (float)(h / (ss * ss));
        const int g = grid[a], gp = ca.gp[a];
        mats[a].assign((size_t)p->nterms * gp * gp, 0.0);
        std::vector<double> col(g);
        for (int t = 0; t < p->nterms; ++t) {
            double at, st;
            s.term(t, &at, &st);
            const double sk2 = st * st - 2.0 * ss * ss;
            if (!(sk2 > 0)) {
                delete p;
                return fail(USERIES_EINVAL,
                            "grid too coarse: the spreading Gaussian must be narrower than "
                            "s_0 / sqrt(2)");
            }
            const double sk = std::sqrt(sk2);
            circulant_column(g, h, sk, (st / sk) * (a == 0 ? at : 1.0), col.data());
            double* M = mats[a].data() + (size_t)t * gp * gp;
            for (int i = 0; i < g; ++i)
                for (int j = 0; j < g; ++j) M[(size_t)i * gp + j] = col[((i - j) % g + g) % g];
        }
    }
    const double V = box[0] * box[1] * box[2];
    p->fin.f_inf0 = p->f_inf0;
    p->fin.near_int_over_v = s.near_integral(r_c) / V;

    // device limits
    int lds_max = 0;
    hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    if (lds_max > 0 && conv_xy_lds_bytes(ca) > (size_t)lds_max) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "grid plane needs %zu bytes of LDS, device allows %d",
                      conv_xy_lds_bytes(ca), lds_max);
        delete p;
        return fail(USERIES_EINVAL, buf);
    }

    // device memory
    int r = upload_matrices(p, mats);
    if (r) {
        delete p;
        return r;
    }
    const size_t ng = (size_t)grid[0] * grid[1] * grid[2];
    hipError_t e;
    if ((e = dalloc(&p->col_count, p->ncol_max)) || (e = dalloc(&p->col_fill, p->ncol_max)) ||
        (e = dalloc(&p->col_start, p->ncol_max + 1)) ||
        (e = dalloc(&p->clus_start, p->ncol_max + 1)) || (e = dalloc(&p->qstats, 2)) ||
        (e = dalloc(&p->parts_tmp, 5)) || (e = dalloc(&p->rho, ng)) ||
        (e = dalloc(&p->tgrid, ng * p->nterms)) || (e = dalloc(&p->phi, ng))) {
        delete p;
        return fail(USERIES_ENOMEM, std::string("plan allocation: ") + hipGetErrorString(e));
    }
    if (o.max_atoms > 0) {
        if (o.max_atoms > INT_MAX / 4) {
            delete p;
            return fail(USERIES_EINVAL, "max_atoms too large");
        }
        r = p->alloc_atoms(o.max_atoms);
        if (r) {
            delete p;
            return r;
        }
        p->fixed_cap = true;
    }
    *out = p;
    return USERIES_OK;
}

static int eval_impl(useries_plan_t p, int64_t n, const float* xyz, const float* q, float* forces,
                     double* energy, double* parts, void* stream) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    if (n < 0 || n > INT_MAX / 4) return fail(USERIES_EINVAL, "n out of range");
    if (n > 0 && (!xyz || !q || !forces)) return fail(USERIES_EINVAL, "NULL buffer");
    DeviceGuard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    if (n > p->cap || !p->coord) {
        if (p->fixed_cap) return fail(USERIES_EINVAL, "n exceeds max_atoms");
        hipStreamSynchronize(st);
        int r = p->alloc_atoms(n);
        if (r) return r;
    }
    const int ni = (int)n;
    const int nq = (ni + 255) / 256;
    // x-y columns for this n: about 8 charges per cluster of one column
    // cross-section and similar z extent, within the plan's bounds
    {
        const double V = p->box[0] * p->box[1] * p->box[2];
        const double w = ni > 0 ? std::cbrt(8.0 * V / ni) : 1e300;
        for (int a = 0; a < 2; ++a) {
            const int nc = std::max(1, std::min(p->ncmax[a], (int)std::floor(p->box[a] / w)));
            p->bin.nc[a] = p->pair.nc[a] = p->gridargs.nc[a] = p->nc_used[a] = nc;
            p->pair.cw[a] = (float)(p->box[a] / nc);
            p->pair.R[a] = (int)std::ceil(p->rc * nc / p->box[a]);
        }
    }
    const int ncol = p->bin.nc[0] * p->bin.nc[1];
    const int npb = ni / 8 + 1 + ncol, ngb = gather_blocks(ni);
    p->bin.n = p->pair.n = p->gridargs.n = ni;
    p->fin.n_pair_parts = npb;
    p->fin.n_gather_parts = ngb;
    if (!parts && !energy) parts = p->parts_tmp;

    hipError_t e = hipMemsetAsync(p->col_count, 0, sizeof(int) * ncol, st);
    if (e) return hip_fail(e, "memset");
    int k = 0;
    hipEvent_t ev0 = nullptr;
    auto pre = [&]() {
        if (p->timing) {
            ev0 = p->get_event();
            hipEventRecord(ev0, st);
        }
    };
    auto post = [&](hipError_t err) -> hipError_t {
        if (p->timing) {
            hipEvent_t ev1 = p->get_event();
            hipEventRecord(ev1, st);
            p->pending.push_back({k, ev0, ev1});
        }
        ++k;
        return err;
    };
#define USERIES_STEP(call)                                             \
    do {                                                               \
        pre();                                                         \
        hipError_t err_ = post(call);                                  \
        if (err_ != hipSuccess) return hip_fail(err_, kKernelNames[k - 1]); \
    } while (0)
    USERIES_STEP(launch_encode(p->bin, xyz, q, p->coord, p->col_of, p->col_count, p->qpart, nq, st));
    USERIES_STEP(launch_scan(ncol, p->col_count, p->col_start, p->clus_start, p->col_fill, p->qpart,
                             nq, p->qstats, st));
    USERIES_STEP(launch_scatter(ni, ncol, p->col_of, p->col_start, p->col_fill, p->slots, st));
    USERIES_STEP(launch_colsort(ncol, p->col_start, p->clus_start, p->slots, p->coord, p->perm,
                                p->sorted, p->cl_info, p->cl_col, p->cl_z, st));
    USERIES_STEP(launch_pair(p->pair, npb, p->sorted, p->clus_start, p->cl_info, p->cl_col, p->cl_z,
                             p->fnear, p->pair_parts, st));
    USERIES_STEP(launch_spread(p->gridargs, p->sorted, p->clus_start, p->cl_info, p->cl_z,
                               p->qstats, p->rho, st));
    USERIES_STEP(launch_conv_xy(p->conv, p->rho, p->kx, p->ky, p->tgrid, st));
    USERIES_STEP(launch_conv_z(p->conv, p->tgrid, p->kz, p->phi, st));
    USERIES_STEP(launch_gather(p->gridargs, p->sorted, p->perm, p->phi, p->fnear, ni, forces,
                               p->gather_parts, ngb, st));
    USERIES_STEP(launch_finalize(p->fin, p->pair_parts, p->gather_parts, p->qstats, energy, parts, st));
#undef USERIES_STEP
    return USERIES_OK;
}

int useries_eval(useries_plan_t p, int64_t n, const float* xyz, const float* q, float* forces,
                 double* energy, void* stream) {
    if (!energy) return fail(USERIES_EINVAL, "NULL energy");
    return eval_impl(p, n, xyz, q, forces, energy, nullptr, stream);
}

int useries_eval_parts(useries_plan_t p, int64_t n, const float* xyz, const float* q,
                       float* forces, double* energy, double* parts, void* stream) {
    if (!parts) return fail(USERIES_EINVAL, "NULL parts");
    return eval_impl(p, n, xyz, q, forces, energy, parts, stream);
}

int useries_plan_info(useries_plan_t p, double* b, double* sigma, double* r0, double* w0,
                      double* s0, int* n_terms, double* eq33, double* f_inf0, double* c1_slope,
                      double* sigma_s, int* stencil_half, int ncell[3], double* poly_maxerr) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    if (b) *b = p->b;
    if (sigma) *sigma = p->sigma;
    if (r0) *r0 = p->r0;
    if (w0) *w0 = p->w0;
    if (s0) *s0 = p->s0;
    if (n_terms) *n_terms = p->nterms;
    if (eq33) *eq33 = p->eq33;
    if (f_inf0) *f_inf0 = p->f_inf0;
    if (c1_slope) *c1_slope = p->c1_slope;
    if (sigma_s) *sigma_s = p->sigma_s[0];
    if (stencil_half) *stencil_half = p->P;
    if (ncell) {
        ncell[0] = p->nc_used[0];
        ncell[1] = p->nc_used[1];
        ncell[2] = 1;
    }
    if (poly_maxerr) *poly_maxerr = p->poly_maxerr;
    return USERIES_OK;
}

int useries_destroy(useries_plan_t p) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    DeviceGuard guard(p->device);
    delete p;
    return USERIES_OK;
}

int useries_timing_enable(useries_plan_t p, int enable) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    p->harvest();
    p->timing = enable != 0;
    for (int k = 0; k < kNumKernels; ++k) {
        p->tsum[k] = 0;
        p->tcount[k] = 0;
    }
    return USERIES_OK;
}

int useries_timing_read(useries_plan_t p, int k, const char** name, double* total_ms,
                        int64_t* launches) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    if (k < 0 || k >= kNumKernels) return USERIES_ENOTFOUND;
    p->harvest();
    if (name) *name = kKernelNames[k];
    if (total_ms) *total_ms = p->tsum[k];
    if (launches) *launches = p->tcount[k];
    return USERIES_OK;
}

int useries_solve_construction(int construction, double b, double* b_out, double* r0, double* w0,
                               double* s0) {
    double bb, rr, ww, ss;
    std::string err;
    int rc = solve_construction(construction, b, &bb, &rr, &ww, &ss, &err);
    if (rc) return fail(rc, err);
    if (b_out) *b_out = bb;
    if (r0) *r0 = rr;
    if (w0) *w0 = ww;
    if (s0) *s0 = ss;
    return USERIES_OK;
}

double useries_eq33_bound(int n, double b, double sigma, double lmax) {
    return eq33_bound(n, b, sigma, lmax);
}

int useries_choose_nterms(double b, double sigma, double lmax, double tol) {
    return choose_nterms(b, sigma, lmax, tol);
}

double useries_bsa_bound(double b) { return bsa_bound(b); }

const char* useries_strerror(int code) {
    switch (code) {
    case USERIES_OK: return "ok";
    case USERIES_EINVAL: return "invalid argument";
    case USERIES_ENOMEM: return "out of memory";
    case USERIES_EHIP: return "HIP runtime error";
    case USERIES_EBUSY: return "busy";
    case USERIES_ENOTFOUND: return "not found";
    case USERIES_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

const char* useries_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
