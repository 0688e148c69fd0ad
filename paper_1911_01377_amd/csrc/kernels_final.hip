// Total energy in FP64 as its own launch after the gather kernel (one block
// per box).
#include "energy_total.h"

namespace useries {

__device__ __forceinline__ void finalize_body(const FinalArgs& a, const double* __restrict__ pp,
                                              const double* __restrict__ gp,
                                              const double* __restrict__ qstats,
                                              double* __restrict__ energy,
                                              double* __restrict__ parts) {
    __shared__ double wred[3 * 1024 / 64];
    energy_total<1024>(a, pp, gp, qstats, energy, parts, wred);
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
