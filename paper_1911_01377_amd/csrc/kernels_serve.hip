// Serving: the move between two evaluations of one request.  Each coordinate
// of each charge is displaced by a normal deviate of standard deviation
// disp_sigma, drawn from Philox4x32-10 with the counter (charge, evaluation
// step, 0, 0) and the request's key; Box-Muller turns the four uniforms into
// normals (three are used, one per axis).  The deviates depend only on the
// request, the step and the charge, so a request moves the same way alone
// and in any batch.
#include "useries_internal.h"
#include "device_common.h"
#include "philox.h"

namespace useries {

__global__ void __launch_bounds__(256) k_displace_batch(const BatchTable* __restrict__ tab,
                                                        const BoxDesc* __restrict__ desc) {
    batch_for(tab, BK_DISPLACE, [&](int i, int item) {
        const BoxDesc& d = desc[tab->slot[i]];
        const int a = item * 256 + threadIdx.x;
        if (a >= d.bin.n) return;
        Philox4 c;
        c.v[0] = (uint32_t)a;
        c.v[1] = (uint32_t)tab->step[i];
        c.v[2] = 0u;
        c.v[3] = 0u;
        const Philox4 r = philox4x32_10(c, d.key[0], d.key[1]);
        const float u0 = philox_unit(r.v[0]), u1 = philox_unit(r.v[1]);
        const float u2 = philox_unit(r.v[2]), u3 = philox_unit(r.v[3]);
        const float twopi = 6.283185307179586f;
        const float m0 = sqrtf(-2.0f * logf(u0)), m1 = sqrtf(-2.0f * logf(u2));
        const float s = d.disp_sigma;
        float* x = d.xyz + 3 * (size_t)a;
        x[0] += s * (m0 * cosf(twopi * u1));
        x[1] += s * (m0 * sinf(twopi * u1));
        x[2] += s * (m1 * cosf(twopi * u3));
    });
}

hipError_t launch_displace_batch(const BatchTable* tab, const BoxDesc* desc, int grid,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_displace_batch, dim3(grid), dim3(256), 0, st, tab, desc);
    return hipGetLastError();
}

}  // namespace useries
