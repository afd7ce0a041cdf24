// kstep.h -- per-point pieces of the BDFk/EXTk step shared by the update kernels and
// the fused CP scatter kernel: right-hand side, level store, and the step close
// (energy log, health flag, step counter).
#pragma once

#include "kcommon.h"

namespace rom {

// History of point (b, i) that the right-hand side of eq. nse_d1 at level n needs:
// y^{n-1}, y^{n-2} and u^n, u^{n-1}, u^{n-2} (zero beyond the order k).  Kernels whose
// contraction is long load it first, so that its latency hides behind the contraction.
struct BdfHist {
    double y1, y2, u[3];
};
__device__ __forceinline__ BdfHist bdf_hist_point(const StepArgs& a, long long n, int k, int b, int i) {
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N + i;
    BdfHist h;
    h.y1 = k >= 2 ? a.yring[(size_t)slot_of(n - 1) * BN + off] : 0.0;
    h.y2 = k >= 3 ? a.yring[(size_t)slot_of(n - 2) * BN + off] : 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) h.u[q] = q < k ? a.uring[(size_t)slot_of(n - q) * BN + off] : 0.0;
    return h;
}

// Store y^n, form the right-hand side of eq. nse_d1 for point (b, i) from its history:
//   rhs = - sum_{q<=k} alpha_q y^{n+1-q} - (1/dt) sum_{q<=k} beta_q u^{n+1-q}
//         [- zfull - (sum_q alpha_q) fz - nu a0],
// zfull = L uhat + (M - I) h carrying the zeroth-mode linear terms under the EXT sum and
// the mass matrix minus the identity times the history sum (full form).
// ZF: the caller formed the full form's G x of point (b, i) itself (zf_given); else it is
// read from a.zfull (summed over its partial products).
template <bool ZF = false>
__device__ __forceinline__ double bdf_rhs_hist(const StepArgs& a, long long n, const BdfCoef& c, int k, int b,
                                               int i, double y, const BdfHist& h, double zf_given = 0.0) {
    a.yring[(size_t)slot_of(n) * ((size_t)a.B * a.N) + (size_t)b * a.N + i] = y;
    const double ylev[3] = {y, h.y1, h.y2};
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) v -= c.alpha[q] * ylev[q];
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) v -= (c.beta[q + 1] * a.inv_dt) * h.u[q];
    if (a.zfull) {
        double sa = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (q < k) sa += c.alpha[q];
        double zf = zf_given;
        if constexpr (!ZF) {
            const size_t off = (size_t)b * a.N + i;
            zf = a.zfull[off];
            for (int q = 1; q < a.zsplit; ++q) zf += a.zfull[(size_t)q * a.zstride + off];
        }
        v -= zf + (sa * a.fz[i] + a.az[i]);
    }
    return v;
}

__device__ __forceinline__ double bdf_rhs_point(const StepArgs& a, long long n, const BdfCoef& c,
                                                int k, int b, int i, double y) {
    return bdf_rhs_hist(a, n, c, k, b, i, y, bdf_hist_point(a, n, k, b, i));
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

// ---------------------------------------------------------------- step close
//
// An update kernel writes level n+1.  Closing a step takes three things: advancing the
// device step counter, summing the per-block energy partials into E^{n+1} (eq.
// ene_fluc) and raising the health flag.  None of them needs a kernel of its own, nor
// a device-wide fence (on gfx950 such a fence writes back and invalidates the XCD's
// whole L2):
//  * Counter: the counter has two slots; the kernels of the step of level n read slot
//    n & 1 and one block of the update kernel stores n+1 into the other slot, which
//    no kernel of this step reads (the host, which knows every level's parity, passes
//    the slot pointers).  The next step reads it after the kernel boundary.
//  * Energy: the partials of level n+1 are summed one step later, by that same block
//    of the next update kernel, after the kernel boundary has made them visible.
//    Partials alternate between two slots by level parity, so that block reads one
//    slot while the kernel writes the other.  closep marks a level whose sum is still
//    pending; a closing kernel sums the last level of a sequence of steps.

// Energy partials of level n1: [B][enmax] in slot n1 & 1 (the first ecount[n1 & 1]
// of each trajectory are written).
__device__ __forceinline__ double* epart_of(const StepArgs& a, long long n1) {
    return a.epart + (size_t)(n1 & 1) * a.B * a.enmax;
}

// Whole block: if level n's energy is pending, sum its partials in a fixed order
// (deterministic), log E^n and record a non-finite level.
__device__ __forceinline__ void close_level(const StepArgs& a, long long n) {
    __shared__ double cred[4];
    if (*a.closep == 0) return;
    const double* ep = epart_of(a, n);
    const int cnt = a.ecount[n & 1];
    if (a.B == 1) {
        double s = 0.0;
        for (int q = threadIdx.x; q < cnt; q += blockDim.x) s += ep[q];
        s = block_sum(s, cred);
        if (threadIdx.x == 0) {
            const double e = 0.5 * s;
            if (n < a.elog_cap) a.elog[n] = e;
            if (!isfinite(e)) atomicMin(a.bad, n);
        }
    } else {
        for (int b = threadIdx.x; b < a.B; b += blockDim.x) {
            const double* eb = ep + (size_t)b * a.enmax;
            double s = 0.0;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) s += eb[q];
            const double e = 0.5 * s;
            if (n < a.elog_cap) a.elog[(size_t)n * a.B + b] = e;
            if (!isfinite(e)) atomicMin(a.bad, n);
        }
    }
}

// One block of each update kernel (whole block): closes level n, marks level n+1 as
// pending with the number of partials per trajectory its kernel writes, and advances
// the counter.
__device__ __forceinline__ void close_and_advance(const StepArgs& a, long long n, int nblk) {
    close_level(a, n);
    __syncthreads();                      // every thread has read closep
    if (threadIdx.x == 0) {
        a.ecount[(n + 1) & 1] = nblk;
        *a.closep = 1;
        *a.step_next = n + 1;
    }
}

// ---------------------------------------------------------------- Helmholtz apply rows

// Dense stiffness, one trajectory: u^{n+1}_i = sum_m Hinv_k[i][m] rhs_m, one wavefront
// per row.  Each lane issues its (up to 8) 16-byte loads of the row before rhs is
// staged in LDS; rows longer than 1024 elements loop.  Block blk of nblk covers rows
// 4 blk .. 4 blk + 3.
template <bool EVEN>
__device__ __forceinline__ void helm_gemv_body(const StepArgs& a, long long n, int blk) {
    extern __shared__ __attribute__((aligned(16))) double sm[];
    double* r = sm;                       // [N]
    __shared__ double red[4];
    constexpr int V = EVEN ? 2 : 1, U = 8;
    typedef typename RawT<8 * V>::T Raw;
    const int k = bdf_order(n);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int i = blk * 4 + w;
    const bool live = i < a.N;
    const double* h = a.hinv + ((size_t)(k - 1) * a.N + (live ? i : 0)) * a.Np;
    Raw hv[U];
    int m0 = lane * V;
    auto issue = [&](int mb) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int m = mb + q * kWave * V;
            if (live && m < a.N) hv[q] = ld_plain<8 * V>(h + m);
        }
    };
    issue(m0);
    staged_copy<8, double>(a.N, [&](int m) { return a.rhs[m]; }, [&](int m, double v) { r[m] = v; });
    __syncthreads();
    double e = 0.0;
    if (live) {
        double s = 0.0;
        while (m0 < a.N) {
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int m = m0 + q * kWave * V;
                if (m < a.N) {
                    const double* hd = reinterpret_cast<const double*>(&hv[q]);
#pragma unroll
                    for (int v = 0; v < V; ++v) s += hd[v] * r[m + v];
                }
            }
            m0 += kWave * V * U;
            if (m0 < a.N) issue(m0);
        }
        s = wave_sum(s);
        if (lane == 0) {
            write_level(a, n + 1, 0, i, s);
            e = s * s;
        }
    }
    const double es = block_sum(e, red);
    if (threadIdx.x == 0) epart_of(a, n + 1)[blk] = es;
}

}  // namespace rom
