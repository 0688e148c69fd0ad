// Total energy in FP64 from the per-block partial sums (fixed summation
// order, so the result does not depend on scheduling):
//   E = E_near + E_far - E_self + E_bg,
//   E_far  = 1/2 sum_g rho_g phi_g       (rho the grid with its mean removed),
//   E_self = 1/2 F(0) sum q^2            (u-series analogue of eq. 10's self term),
//   E_bg   = -Q^2/(2V) int N(r) d^3r     (uniform neutralising background; 0 if Q = 0).
// With the same spreading weights on both sides, sum_i q_i phi_i equals
// sum_g rho_g phi_g for the raw spread grid, so the grid form equals
// 1/2 sum_i q_i phi_i - 1/2 Q <phi>: the far part sums only k != 0 (eqs. 4,
// 9, 10), and a uniform offset of the grid potential (its k = 0 component,
// which the FP32 rounding of the widest terms leaves behind) meets the
// mean-free grid and drops out.
#pragma once

#include "useries_internal.h"
#include "device_common.h"

namespace useries {

// One block of NT threads: thread-strided sums of the pair and far
// partials, wavefront sums (DPP), then the NT / 64 wavefront sums in order.
// wred holds 2 NT / 64 doubles of LDS.
template <int NT>
__device__ __forceinline__ void energy_total(const FinalArgs& a, const double* __restrict__ pp,
                                             const double* __restrict__ fp,
                                             const double* __restrict__ qstats,
                                             double* __restrict__ energy,
                                             double* __restrict__ parts, double* wred) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double s = 0.0, g = 0.0;
    for (int k = t; k < a.n_pair_parts; k += NT) s += pp[k];
    for (int k = t; k < a.n_far_parts; k += NT) g += fp[k];
    s = wave_sum_d(s);
    g = wave_sum_d(g);
    if (lane == 0) {
        wred[2 * w] = s;
        wred[2 * w + 1] = g;
    }
    __syncthreads();
    if (t == 0) {
        double en = 0.0, gs = 0.0;
        for (int v = 0; v < NT / 64; ++v) {
            en += wred[2 * v];
            gs += wred[2 * v + 1];
        }
        const double Q = qstats[0], q2 = qstats[1];
        double ef = 0.5 * gs;
        ef += 0.5 * Q * Q * a.k0_far;        // 1/r^6: the k = 0 components (0 for 1/r)
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
