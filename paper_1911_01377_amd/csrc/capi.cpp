// C ABI of the library: plan construction (host FP64 math + one upload),
// device workspace, and the evaluation sequence
//   bin_local -> colbuild (or, for very large inputs, encode -> [scan] -> scatter
//   -> colsort) -> pair (near part) -> spread -> conv_xy -> conv_z (far part,
//   far-energy partials) -> gather (far forces + near forces; one extra block
//   forms the FP64 energy total).
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

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(USERIES_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// the binning runs either bin_local, colbuild or encode, [scan,] scatter,
// colsort; gather's launch also forms the energy total
constexpr const char* kKernelNames[] = {"bin_local", "encode", "scan",    "scatter",
                                        "colsort",   "colbuild", "pair",  "spread",
                                        "conv_xy",   "conv_z",   "gather"};
constexpr int kNumKernels = sizeof(kKernelNames) / sizeof(kKernelNames[0]);

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

namespace useries {
int set_last_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace useries

// ints of the per-block column prefixes of two-launch binning for up to c
// charges (0: that binning is not used): fewer charges take no more blocks
// and no more columns
static int64_t bpre_ints(const useries::HostPlan& hp, int64_t c) {
    const int64_t nb = (c + 255) / 256;
    const int ncol = useries::columns_per_axis(hp, (int)c, 0) * useries::columns_per_axis(hp, (int)c, 1);
    return useries::bin_local_ok((int)c, ncol) ? nb * (ncol + 1) : 0;
}

struct useries_plan_s {
    int device = 0;
    HostPlan hp;
    int nc_used[2] = {0, 0};
    bool counts_dirty = false;   // column counters may be non-zero (an evaluation failed midway)
    // device constants
    void *kx = nullptr, *ky = nullptr, *kz = nullptr;
    float *ux = nullptr, *uy = nullptr, *uz = nullptr, *wspec = nullptr, *cspec = nullptr;
    // fixed workspace
    int *col_count = nullptr, *col_start = nullptr, *col_fill = nullptr, *clus_start = nullptr;
    int* zbin = nullptr;
    double *qstats = nullptr, *parts_tmp = nullptr;
    float *rho = nullptr, *tgrid = nullptr, *phi = nullptr;
    // per-atom workspace
    int64_t cap = 0;
    bool fixed_cap = false;
    uint4 *coord = nullptr, *sorted = nullptr;
    int *perm = nullptr, *slots = nullptr;
    int2* cl_info = nullptr;
    int* cl_col = nullptr;
    uint2* cl_z = nullptr;
    float4* fnear = nullptr;
    double *qpart = nullptr, *pair_parts = nullptr, *far_parts = nullptr;
    int* bpre = nullptr;
    int64_t bpre_cap = 0;
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
        hipFree(cl_info);
        hipFree(cl_col);
        hipFree(cl_z);
        hipFree(pair_parts);
        hipFree(perm);
        hipFree(slots);
        hipFree(fnear);
        hipFree(qpart);
        hipFree(bpre);
        bpre = nullptr;
        bpre_cap = 0;
        coord = sorted = nullptr;
        perm = slots = cl_col = nullptr;
        cl_info = nullptr;
        cl_z = nullptr;
        pair_parts = nullptr;
        fnear = nullptr;
        qpart = nullptr;
        cap = 0;
    }

    int alloc_atoms(int64_t n) {
        free_atoms();
        const int64_t c = std::max<int64_t>(n, 256);
        // clusters: at most sum over columns of ceil(count / 8)
        const int64_t clmax = pair_blocks((int)c, hp.ncol_max);
        hipError_t e;
        if ((e = dalloc(&coord, c)) || (e = dalloc(&sorted, c)) ||
            (e = dalloc(&perm, c)) || (e = dalloc(&slots, c)) || (e = dalloc(&cl_info, clmax)) ||
            (e = dalloc(&cl_col, clmax)) || (e = dalloc(&cl_z, clmax)) ||
            (e = dalloc(&pair_parts, clmax)) || (e = dalloc(&fnear, c)) ||
            (e = dalloc(&qpart, 2 * (size_t)((c + 255) / 256))) ||
            (bpre_ints(hp, c) > 0 && (e = dalloc(&bpre, (size_t)bpre_ints(hp, c))))) {
            free_atoms();
            return fail(USERIES_ENOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
        }
        bpre_cap = bpre_ints(hp, c);
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
        hipFree(ux);
        hipFree(uy);
        hipFree(uz);
        hipFree(wspec);
        hipFree(cspec);
        hipFree(col_count);
        hipFree(col_start);
        hipFree(col_fill);
        hipFree(clus_start);
        hipFree(zbin);
        hipFree(qstats);
        hipFree(far_parts);
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
    o->alpha = 1;
    o->spectral = -1;
    return USERIES_OK;
}

int useries_plan(useries_plan_t* out, const double box[3], double r_c, double b, double sigma,
                 int n_terms, const int grid[3], const useries_opts* opts) {
    if (!out || !box || !grid) return fail(USERIES_EINVAL, "NULL argument");
    *out = nullptr;
    if (opts && opts->max_atoms > INT_MAX / 4) return fail(USERIES_EINVAL, "max_atoms too large");
    auto* p = new useries_plan_s();
    std::string err;
    int r = build_host_plan(&p->hp, box, r_c, b, sigma, n_terms, grid, opts, &err);
    if (r) {
        delete p;
        return fail(r, err);
    }
    hipGetDevice(&p->device);
    const HostPlan& hp = p->hp;

    // device limits
    int lds_max = 0;
    hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
    const size_t lds_need = std::max(conv_xy_lds_bytes(hp.conv), conv_z_lds_bytes(hp.conv));
    if (lds_max > 0 && lds_need > (size_t)lds_max) {
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "grid and term count need %zu bytes of LDS per block, device allows %d",
                      lds_need, lds_max);
        delete p;
        return fail(USERIES_EINVAL, buf);
    }

    // device memory
    void** dst[3] = {&p->kx, &p->ky, &p->kz};
    hipError_t e;
    for (int a = 0; a < 3; ++a) {
        if ((e = hipMalloc(dst[a], hp.mats[a].size()))) {
            delete p;
            return fail(USERIES_ENOMEM, "convolution matrices");
        }
        if ((e = hipMemcpy(*dst[a], hp.mats[a].data(), hp.mats[a].size(), hipMemcpyHostToDevice))) {
            delete p;
            return hip_fail(e, "upload");
        }
    }
    if (hp.conv.spec) {
        // spectral wide terms: bases, weights and the planes' projections
        float** ub[3] = {&p->ux, &p->uy, &p->uz};
        for (int a = 0; a < 3; ++a) {
            const size_t bytes = hp.ubasis[a].size() * sizeof(float);
            if ((e = hipMalloc((void**)ub[a], bytes)) ||
                (e = hipMemcpy(*ub[a], hp.ubasis[a].data(), bytes, hipMemcpyHostToDevice))) {
                delete p;
                return hip_fail(e, "spectral bases");
            }
        }
        const size_t wb = hp.wspec.size() * sizeof(float);
        // plane projections [g_z][r_y][r_x], then the core G [r_z][r_y][r_x]
        const size_t cb = ((size_t)hp.grid[2] + hp.conv.rk[2]) * hp.conv.rk[1] * hp.conv.rk[0] *
                          sizeof(float);
        if ((e = hipMalloc((void**)&p->wspec, wb)) ||
            (e = hipMemcpy(p->wspec, hp.wspec.data(), wb, hipMemcpyHostToDevice)) ||
            (e = hipMalloc((void**)&p->cspec, cb))) {
            delete p;
            return hip_fail(e, "spectral weights");
        }
    }
    const size_t ng = (size_t)hp.grid[0] * hp.grid[1] * hp.grid[2];
    if ((e = dalloc(&p->col_count, hp.ncol_max)) || (e = dalloc(&p->col_fill, hp.ncol_max)) ||
        (e = dalloc(&p->col_start, hp.ncol_max + 1)) ||
        (e = dalloc(&p->clus_start, hp.ncol_max + 1)) ||
        (e = dalloc(&p->zbin, (size_t)hp.ncol_max * (hp.grid[2] + 1))) ||
        (e = dalloc(&p->qstats, 2)) ||
        (e = dalloc(&p->far_parts, (size_t)far_parts(hp.conv))) ||
        (e = dalloc(&p->parts_tmp, 5)) || (e = dalloc(&p->rho, ng)) ||
        (e = dalloc(&p->tgrid, ng * hp.conv.nterms)) || (e = dalloc(&p->phi, ng))) {
        delete p;
        return fail(USERIES_ENOMEM, std::string("plan allocation: ") + hipGetErrorString(e));
    }
    // the column counters start at zero; each evaluation's colsort clears them again
    if ((e = hipMemset(p->col_count, 0, sizeof(int) * hp.ncol_max)) ||
        (e = hipMemset(p->col_fill, 0, sizeof(int) * hp.ncol_max))) {
        delete p;
        return hip_fail(e, "memset");
    }
    if (opts && opts->max_atoms > 0) {
        r = p->alloc_atoms(opts->max_atoms);
        if (r) {
            delete p;
            return r;
        }
        p->fixed_cap = true;
    }
    *out = p;
    return USERIES_OK;
}

}  // extern "C"

namespace useries {

int plan_device(useries_plan_t p) { return p->device; }

// Byte offsets of the per-charge workspace of n charges in one contiguous
// buffer (each array 256-byte aligned).
struct AtomLayout {
    size_t coord, sorted, perm, slots, cl_info, cl_col, cl_z, pair_parts, fnear, qpart, bpre, total;
};

static AtomLayout atom_layout(const HostPlan& hp, int64_t n) {
    const int64_t c = std::max<int64_t>(n, 1);
    const int64_t clmax = pair_blocks((int)c, hp.ncol_max);
    AtomLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += (bytes + 255) & ~(size_t)255;
        return r;
    };
    L.coord = take(16 * (size_t)c);
    L.sorted = take(16 * (size_t)c);
    L.perm = take(4 * (size_t)c);
    L.slots = take(4 * (size_t)c);
    L.cl_info = take(8 * (size_t)clmax);
    L.cl_col = take(4 * (size_t)clmax);
    L.cl_z = take(8 * (size_t)clmax);
    L.pair_parts = take(8 * (size_t)clmax);
    L.fnear = take(16 * (size_t)c);
    L.qpart = take(16 * (size_t)((c + 255) / 256));
    L.bpre = take(4 * (size_t)bpre_ints(hp, c));
    L.total = o;
    return L;
}

size_t atom_workspace_bytes(useries_plan_t p, int64_t n) { return atom_layout(p->hp, n).total; }

AtomWs atom_workspace_at(useries_plan_t p, int64_t n, char* base) {
    const AtomLayout L = atom_layout(p->hp, n);
    AtomWs w;
    w.coord = (uint4*)(base + L.coord);
    w.sorted = (uint4*)(base + L.sorted);
    w.perm = (int*)(base + L.perm);
    w.slots = (int*)(base + L.slots);
    w.cl_info = (int2*)(base + L.cl_info);
    w.cl_col = (int*)(base + L.cl_col);
    w.cl_z = (uint2*)(base + L.cl_z);
    w.pair_parts = (double*)(base + L.pair_parts);
    w.fnear = (float4*)(base + L.fnear);
    w.qpart = (double*)(base + L.qpart);
    w.bpre_cap = bpre_ints(p->hp, std::max<int64_t>(n, 1));
    w.bpre = w.bpre_cap > 0 ? (int*)(base + L.bpre) : nullptr;
    return w;
}

int plan_eval(useries_plan_t p, int64_t n, const float* xyz, const float* q, float* forces,
              double* energy, double* parts, void* stream, const AtomWs* ext) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    if (n < 0 || n > INT_MAX / 4) return fail(USERIES_EINVAL, "n out of range");
    if (n > 0 && (!xyz || !q || !forces)) return fail(USERIES_EINVAL, "NULL buffer");
    DeviceGuard guard(p->device);
    hipStream_t st = (hipStream_t)stream;
    AtomWs own;
    if (!ext) {
        if (n > p->cap || !p->coord) {
            if (p->fixed_cap) return fail(USERIES_EINVAL, "n exceeds max_atoms");
            hipStreamSynchronize(st);
            int r = p->alloc_atoms(n);
            if (r) return r;
        }
        own.coord = p->coord;
        own.sorted = p->sorted;
        own.perm = p->perm;
        own.slots = p->slots;
        own.cl_info = p->cl_info;
        own.cl_col = p->cl_col;
        own.cl_z = p->cl_z;
        own.pair_parts = p->pair_parts;
        own.fnear = p->fnear;
        own.qpart = p->qpart;
        own.bpre = p->bpre;
        own.bpre_cap = p->bpre_cap;
    }
    const AtomWs& W = ext ? *ext : own;
    HostPlan& hp = p->hp;
    const int ni = (int)n;
    const int nq = (ni + 255) / 256;
    choose_columns(&hp, ni);
    p->nc_used[0] = hp.bin.nc[0];
    p->nc_used[1] = hp.bin.nc[1];
    const int ncol = hp.bin.nc[0] * hp.bin.nc[1];
    const int npb = hp.fin.n_pair_parts;
    if (!parts && !energy) parts = p->parts_tmp;

    if (p->counts_dirty) {
        hipError_t e = hipMemsetAsync(p->col_count, 0, sizeof(int) * hp.ncol_max, st);
        if (!e) e = hipMemsetAsync(p->col_fill, 0, sizeof(int) * hp.ncol_max, st);
        if (e) return hip_fail(e, "memset");
        p->counts_dirty = false;
    }
    // timing: HIP events around each kernel on the stream it runs on
    auto run = [&](int k, hipStream_t s, auto&& launch) -> hipError_t {
        hipEvent_t ev0 = nullptr;
        if (p->timing) {
            ev0 = p->get_event();
            hipEventRecord(ev0, s);
        }
        const hipError_t err = launch();
        if (p->timing) {
            hipEvent_t ev1 = p->get_event();
            hipEventRecord(ev1, s);
            p->pending.push_back({k, ev0, ev1});
        }
        if (err != hipSuccess) p->counts_dirty = true;
        return err;
    };
#define USERIES_STEP(k, s, call)                                               \
    do {                                                                       \
        const hipError_t err_ = run(k, s, [&]() { return (call); });          \
        if (err_ != hipSuccess) return hip_fail(err_, kKernelNames[k]);        \
    } while (0)
    const float* kx = (const float*)p->kx;
    const float* ky = (const float*)p->ky;
    const float* kz = (const float*)p->kz;
    if (W.bpre && bin_local_ok(ni, ncol) && (int64_t)nq * (ncol + 1) <= W.bpre_cap) {
        USERIES_STEP(0, st, launch_bin_local(hp.bin, xyz, q, W.coord, W.slots, W.bpre, W.qpart,
                                             st));
        USERIES_STEP(5, st, launch_colbuild(ni, ncol, hp.bin.nc[0], hp.grid[2], npb, W.bpre,
                                            W.coord, W.slots, W.perm, W.sorted, W.cl_info,
                                            W.cl_col, W.cl_z, p->zbin, W.qpart, p->qstats, st));
    } else {
        USERIES_STEP(1, st, launch_encode(hp.bin, xyz, q, W.coord, p->col_count, W.qpart,
                                          nq, st));
        if (!scan_fused(ni, ncol))
            USERIES_STEP(2, st, launch_scan(ncol, p->col_count, p->col_start, p->clus_start,
                                            p->col_fill, W.qpart, nq, p->qstats, st));
        USERIES_STEP(3, st, launch_scatter(hp.bin, W.coord, W.sorted, p->col_count,
                                           p->col_start, p->clus_start, p->col_fill, W.slots,
                                           W.qpart, nq, p->qstats, st));
        USERIES_STEP(4, st, launch_colsort(ncol, hp.bin.nc[0], p->col_start, p->clus_start,
                                           W.slots, W.coord, W.perm, W.sorted, W.cl_info,
                                           W.cl_col, W.cl_z, hp.grid[2], p->zbin, p->col_count,
                                           p->col_fill, npb, st));
    }
    USERIES_STEP(6, st, launch_pair(hp.pair, npb, W.sorted, W.cl_info, W.cl_col, W.cl_z,
                                    p->zbin, W.fnear, W.pair_parts, st));
    USERIES_STEP(7, st, launch_spread(hp.gridargs, W.sorted, p->zbin, p->qstats, p->rho, st));
    SpecPtrs sp;
    sp.ux = p->ux;
    sp.uy = p->uy;
    sp.uz = p->uz;
    sp.w = p->wspec;
    sp.c = p->cspec;
    USERIES_STEP(8, st, launch_conv_xy(hp.conv, p->rho, kx, ky, p->tgrid, sp, st));
    USERIES_STEP(9, st, launch_conv_z(hp.conv, p->tgrid, kz, p->phi, p->rho, p->far_parts, sp,
                                      st));
    USERIES_STEP(10, st, launch_gather(hp.gridargs, W.sorted, W.perm, p->zbin, p->phi, W.fnear,
                                       forces, hp.fin, W.pair_parts, p->far_parts, p->qstats,
                                       energy, parts, st));
#undef USERIES_STEP
    return USERIES_OK;
}

}  // namespace useries

extern "C" {

int useries_eval(useries_plan_t p, int64_t n, const float* xyz, const float* q, float* forces,
                 double* energy, void* stream) {
    if (!energy) return fail(USERIES_EINVAL, "NULL energy");
    return plan_eval(p, n, xyz, q, forces, energy, nullptr, stream, nullptr);
}

int useries_eval_parts(useries_plan_t p, int64_t n, const float* xyz, const float* q,
                       float* forces, double* energy, double* parts, void* stream) {
    if (!parts) return fail(USERIES_EINVAL, "NULL parts");
    return plan_eval(p, n, xyz, q, forces, energy, parts, stream, nullptr);
}

int useries_plan_info(useries_plan_t p, double* b, double* sigma, double* r0, double* w0,
                      double* s0, int* n_terms, double* eq33, double* f_inf0, double* c1_slope,
                      double* sigma_s, int* stencil_half, int ncell[3], double* poly_maxerr,
                      int* n_terms_grid, int* near_exact, int* n_terms_spectral,
                      int spectral_rank[3]) {
    if (!p) return fail(USERIES_EINVAL, "NULL plan");
    const HostPlan& hp = p->hp;
    if (b) *b = hp.b;
    if (sigma) *sigma = hp.sigma;
    if (r0) *r0 = hp.r0;
    if (w0) *w0 = hp.w0;
    if (s0) *s0 = hp.s0;
    if (n_terms) *n_terms = hp.nterms;
    if (eq33) *eq33 = hp.eq33;
    if (f_inf0) *f_inf0 = hp.f_inf0;
    if (c1_slope) *c1_slope = hp.c1_slope;
    if (sigma_s) *sigma_s = hp.sigma_s[0];
    if (stencil_half) *stencil_half = hp.P;
    if (ncell) {
        ncell[0] = p->nc_used[0];
        ncell[1] = p->nc_used[1];
        ncell[2] = 1;
    }
    if (poly_maxerr) *poly_maxerr = hp.poly_maxerr;
    if (n_terms_grid) *n_terms_grid = hp.nterms_grid;
    if (near_exact) *near_exact = hp.near_exact;
    if (n_terms_spectral) *n_terms_spectral = hp.nterms_spec;
    if (spectral_rank)
        for (int a = 0; a < 3; ++a) spectral_rank[a] = hp.conv.rk[a];
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
