// kstep.h -- per-point pieces of the BDFk/EXTk step shared by the update kernels and
// the fused CP scatter kernel: right-hand side, level store, and the last-block
// finalization (energy log, health flag, step counter).
#pragma once

#include "kcommon.h"

namespace rom {

// Store y^n, form the right-hand side of eq. nse_d1 for point (b, i):
//   rhs = - sum_{q<=k} alpha_q y^{n+1-q} - (1/dt) sum_{q<=k} beta_q u^{n+1-q}.
__device__ __forceinline__ double bdf_rhs_point(const StepArgs& a, long long n, const BdfCoef& c,
                                                int k, int b, int i, double y) {
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N + i;
    a.yring[(size_t)slot_of(n) * BN + off] = y;
    double ylev[3], ulev[3];
    ylev[0] = y;
    ylev[1] = k >= 2 ? a.yring[(size_t)slot_of(n - 1) * BN + off] : 0.0;
    ylev[2] = k >= 3 ? a.yring[(size_t)slot_of(n - 2) * BN + off] : 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) ulev[q] = q < k ? a.uring[(size_t)slot_of(n - q) * BN + off] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) v -= c.alpha[q] * ylev[q];
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) v -= (c.beta[q + 1] * a.inv_dt) * ulev[q];
    return v;
}

// Coefficient copies for the batched contraction ([Bpad][Np] layout).
__device__ __forceinline__ void write_ucv(const StepArgs& a, int b, int i, double u) {
    const size_t o = (size_t)b * a.Np + i, oj = (size_t)i * a.Bpad + b;
    if (a.dtype == DT_F64) {
        reinterpret_cast<double*>(a.ucv)[o] = u;
        reinterpret_cast<double*>(a.uj)[oj] = u;
    } else {
        const float f = (float)u;
        float* uj = reinterpret_cast<float*>(a.uj);
        if (a.dtype == DT_F32) {
            reinterpret_cast<float*>(a.ucv)[o] = f;
            uj[oj] = f;
        } else if (a.dtype == DT_BF16) {
            const unsigned short h = bf16_bits(f);
            reinterpret_cast<unsigned short*>(a.ucv)[o] = h;
            uj[oj] = bf16_f(h);
        } else {
            const unsigned short h = bf16_bits(f);
            const unsigned short l = bf16_bits(f - bf16_f(h));
            reinterpret_cast<unsigned short*>(a.ucv)[o] = h;
            reinterpret_cast<unsigned short*>(a.ucv_lo)[o] = l;
            uj[oj] = f;
        }
    }
}

// Store level n+1 of trajectory b at row i, and its copies for the batched kernels.
__device__ __forceinline__ void write_level(const StepArgs& a, long long n1, int b, int i,
                                            double u) {
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N + i;
    a.uring[(size_t)slot_of(n1) * BN + off] = u;
    if (a.batched) write_ucv(a, b, i, u);
}

}  // namespace rom
