// Total energy in FP64 from the per-block partial sums (fixed summation
// order, so the result does not depend on scheduling):
//   E = E_near + E_far - E_self + E_bg,
//   E_self = 1/2 F(0) sum q^2            (u-series analogue of eq. 10's self term),
//   E_bg   = -Q^2/(2V) int N(r) d^3r     (uniform neutralising background; 0 if Q = 0).
#pragma once

#include "useries_internal.h"
#include "device_common.h"

namespace useries {

// One block of NT threads: thread-strided sums of the pair and gather
// partials, wavefront sums (DPP), then the NT / 64 wavefront sums in
// order.  wred holds 2 NT / 64 doubles of LDS.
template <int NT>
__device__ __forceinline__ void energy_total(const FinalArgs& a, const double* __restrict__ pp,
                                             const double* __restrict__ gp,
                                             const double* __restrict__ qstats,
                                             double* __restrict__ energy,
                                             double* __restrict__ parts, double* wred) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double s = 0.0, g = 0.0;
    for (int k = t; k < a.n_pair_parts; k += NT) s += pp[k];
    for (int k = t; k < a.n_gather_parts; k += NT) g += gp[k];
    s = wave_sum_d(s);
    g = wave_sum_d(g);
    if (lane == 0) {
        wred[2 * w] = s;
        wred[2 * w + 1] = g;
    }
    __syncthreads();
    if (t == 0) {
        double en = 0.0, ef = 0.0;
        for (int v = 0; v < NT / 64; ++v) {
            en += wred[2 * v];
            ef += wred[2 * v + 1];
        }
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

}  // namespace useries
