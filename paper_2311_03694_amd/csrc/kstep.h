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

// Last-arriving block of a grid of `nblk_total` blocks: sums the per-block energy
// partials epart[b][0..nblk) in a fixed order (deterministic), logs E^{n+1}, records the
// first non-finite level and advances the step counter.  Returns true in the block
// that finalized.  Must be called by every thread of every block (blockDim.x <= 1024,
// a multiple of 64).  One trajectory: the whole block reduces (strided partial sums,
// then the wavefront/LDS tree); a batch: one thread per trajectory, loads unrolled.
__device__ __forceinline__ bool finalize_step(const StepArgs& a, long long n, int nblk, unsigned nblk_total) {
    __shared__ int am_last;
    __shared__ double fred[16];
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(a.ticket, 1u);
        am_last = (prev == nblk_total - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
    if (a.B == 1) {
        double s = 0.0;
        for (int q = threadIdx.x; q < nblk; q += blockDim.x) s += a.epart[q];
        s = block_sum(s, fred);
        if (threadIdx.x == 0) {
            const double e = 0.5 * s;
            if (n + 1 < a.elog_cap) a.elog[n + 1] = e;
            if (!isfinite(e)) atomicMin(a.bad, n + 1);
        }
    } else {
        for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
            const double* ep = a.epart + (size_t)b * nblk;
            double s = 0.0;
#pragma unroll 8
            for (int q = 0; q < nblk; ++q) s += ep[q];
            const double e = 0.5 * s;
            if (n + 1 < a.elog_cap) a.elog[(size_t)(n + 1) * a.B + b] = e;
            if (!isfinite(e)) atomicMin(a.bad, n + 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *a.step = n + 1;
        *a.ticket = 0u;
        __threadfence();
    }
    return true;
}

}  // namespace rom
