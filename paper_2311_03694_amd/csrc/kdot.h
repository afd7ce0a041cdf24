// kdot.h -- the coefficient vector u staged in LDS in the contraction's number
// format, and the short dot product of V stored operator elements with V consecutive
// coefficients that the single-trajectory kernels are built from.
#pragma once

#include "kcommon.h"

namespace rom {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// LDS image of u.  The product operand `uh` is FP64 / FP32 values, or BF16 words
// (BF16X3: high words, with the low words in `ul`).  `uw` is the weight of a whole
// (j, .) row of the dense tensor: u_j as FP32 for FP32/BF16X3, the BF16 value of u_j
// for BF16, and uh itself for FP64/FP32.
template <int DT> struct LdsU {
    typedef typename Store<DT>::Acc Acc;
    typedef typename Store<DT>::T T;
    T* uh;
    unsigned short* ul;
    Acc* uw;

    // bytes needed for N (padded) coefficients (three 16-byte aligned regions)
    static __host__ __device__ size_t bytes(int N) { return lds_u_bytes(DT, N); }

    __device__ void bind(char* base, int N) {
        const size_t r = ((size_t)N * sizeof(T) + 15) & ~(size_t)15;
        uh = reinterpret_cast<T*>(base);
        if (DT == DT_F64 || DT == DT_F32) {
            ul = nullptr;
            uw = reinterpret_cast<Acc*>(base);
        } else {
            const size_t l = DT == DT_BF16X3 ? (((size_t)N * 2 + 15) & ~(size_t)15) : 0;
            ul = reinterpret_cast<unsigned short*>(base + r);
            uw = reinterpret_cast<Acc*>(base + r + l);
        }
    }

    // Entry q of the image from the FP64 value v.
    __device__ __forceinline__ void put(int q, double v) {
        if constexpr (DT == DT_F64) {
            uh[q] = v;
        } else if constexpr (DT == DT_F32) {
            uh[q] = (float)v;
        } else if constexpr (DT == DT_BF16) {
            const unsigned short h = bf16_bits((float)v);
            uh[q] = h;
            uw[q] = bf16_f(h);
        } else {
            const float f = (float)v;
            const unsigned short h = bf16_bits(f);
            uh[q] = h;
            ul[q] = bf16_bits(f - bf16_f(h));
            uw[q] = f;
        }
    }

    // Convert sgn * u (FP64, N values, sgn = +1 or -1) into an image of Np >= N entries,
    // zero beyond N; call with the whole block, then __syncthreads.
    __device__ void fill(const double* __restrict__ u, int N, int Np, double sgn = 1.0) {
        staged_copy<8, double>(
            Np, [&](int q) { return q < N ? sgn * u[q] : 0.0; }, [&](int q, double v) { put(q, v); });
    }
};

__device__ __forceinline__ float dot2_bf16(unsigned int a, unsigned int b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b),
                                           c, false);
}

// z = sum_{v<V} c[k+v] * u[k+v] for a raw vector of V stored elements (and the BF16X3
// low words `rl`); k is a multiple of V.  Stored rows are padded with zeros to a
// multiple of 8 elements, so V is always the full 16-byte width.  BF16 pairs use the packed dot2 instruction
// (exact products, FP32 accumulation); BF16X3 adds hi*hi + hi*lo + lo*hi.
template <int DT, int V, class R>
__device__ __forceinline__ typename Store<DT>::Acc dot_vec(const R& r, const R& rl, const LdsU<DT>& L,
                                                           int k) {
    typedef typename Store<DT>::Acc Acc;
    if constexpr ((DT == DT_BF16 || DT == DT_BF16X3) && V >= 2) {
        constexpr int W = V / 2;
        const unsigned int* cw = reinterpret_cast<const unsigned int*>(&r);
        const unsigned int* uhw = reinterpret_cast<const unsigned int*>(L.uh + k);
        float z = 0.0f;
        if constexpr (DT == DT_BF16) {
#pragma unroll
            for (int q = 0; q < W; ++q) z = dot2_bf16(cw[q], uhw[q], z);
        } else {
            const unsigned int* clw = reinterpret_cast<const unsigned int*>(&rl);
            const unsigned int* ulw = reinterpret_cast<const unsigned int*>(L.ul + k);
#pragma unroll
            for (int q = 0; q < W; ++q) {
                z = dot2_bf16(cw[q], uhw[q], z);
                z = dot2_bf16(cw[q], ulw[q], z);
                z = dot2_bf16(clw[q], uhw[q], z);
            }
        }
        return z;
    } else if constexpr (DT == DT_BF16 || DT == DT_BF16X3) {
        const float c = bf16_f(*reinterpret_cast<const unsigned short*>(&r));
        const float uhv = bf16_f(L.uh[k]);
        if constexpr (DT == DT_BF16) {
            return c * uhv;
        } else {
            const float cl = bf16_f(*reinterpret_cast<const unsigned short*>(&rl));
            return c * uhv + c * bf16_f(L.ul[k]) + cl * uhv;
        }
    } else {
        Acc cv[V];
        Decode<DT, V>::run(r, cv);
        Acc z = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) z += cv[v] * L.uh[k + v];
        return z;
    }
}

}  // namespace rom
