// Total energy in FP64 (one block, fixed summation order):
//   E = E_near + E_far - E_self + E_bg,
//   E_self = 1/2 F(0) sum q^2            (u-series analogue of eq. 10's self term),
//   E_bg   = -Q^2/(2V) int N(r) d^3r     (uniform neutralising background; 0 if Q = 0).
#include "useries_internal.h"
#include "device_common.h"

namespace useries {

__device__ __forceinline__ void finalize_body(const FinalArgs& a, const double* __restrict__ pp,
                                              const double* __restrict__ gp,
                                              const double* __restrict__ qstats,
                                              double* __restrict__ energy,
                                              double* __restrict__ parts) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int k = threadIdx.x; k < a.n_pair_parts; k += 1024) s += pp[k];
    const double en = block_sum_d<1024>(s, red);
    __syncthreads();
    s = 0.0;
    for (int k = threadIdx.x; k < a.n_gather_parts; k += 1024) s += gp[k];
    const double ef = block_sum_d<1024>(s, red);
    if (threadIdx.x == 0) {
        const double Q = qstats[0], q2 = qstats[1];
        const double es = 0.5 * a.f_inf0 * q2;
        const double eb = -0.5 * Q * Q * a.near_int_over_v;
        const double e = en + ef - es + eb;
        if (energy) energy[0] = e;
        if (parts) {
            parts[0] = en;
            parts[1] = ef;
            parts[2] = es;
            parts[3] = eb;
            parts[4] = e;
        }
    }
}

__global__ void __launch_bounds__(1024) k_finalize(FinalArgs a, const double* __restrict__ pp,
                                                  const double* __restrict__ gp,
                                                  const double* __restrict__ qstats,
                                                  double* __restrict__ energy,
                                                  double* __restrict__ parts) {
    finalize_body(a, pp, gp, qstats, energy, parts);
}

// batched: the energy of evaluation `step` of each box goes to energies[step]
__global__ void __launch_bounds__(1024) k_finalize_batch(const BatchTable* __restrict__ tab,
                                                        const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_FINAL, [&](int i, int) {
        const BoxDesc& d = desc[tab->slot[i]];
        finalize_body(d.fin, d.pair_parts, d.gather_parts, d.qstats, d.energies + tab->step[i],
                      nullptr);
    });
}

hipError_t launch_finalize(const FinalArgs& a, const double* pair_parts,
                           const double* gather_parts, const double* qstats, double* energy,
                           double* parts, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, a, pair_parts, gather_parts, qstats,
                       energy, parts);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_batch, dim3(grid), dim3(1024), 0, st, tab, desc);
    return hipGetLastError();
}

}  // namespace useries
