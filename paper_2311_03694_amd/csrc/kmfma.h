// kmfma.h -- matrix-core (MFMA) building blocks shared by the batched contraction
// kernels: operand formats per arithmetic kind, fragment loads and one k-step of
// MFMA issues.
//
// MFMA kinds: FP64 v_mfma_f64_16x16x4f64 (a lane holds 2 consecutive k, 2 issues per
// 16-byte lane vector), FP32 v_mfma_f32_16x16x4f32 (4 consecutive k, 4 issues), BF16
// v_mfma_f32_16x16x32_bf16 (8 consecutive k, 1 issue) and BF16X3 (three BF16 issues
// hi*hi + hi*lo + lo*hi).  In a 16x16 tile, lane l feeds row (A) or column (B) l%16 and
// the k group l/16.  Accumulator element v of lane l is column l%16 and row
// 4*(l/16) + v for the FP32-accumulating kinds, row l/16 + 4*v for FP64 (layouts
// measured on gfx950 with a one-hot probe).
#pragma once

#include "kcommon.h"

namespace rom {

enum MK { MK_F64 = 0, MK_F32 = 1, MK_BF16 = 2, MK_BF16X3 = 3 };

template <int MKD> struct MfmaT;
template <> struct MfmaT<MK_F64> {
    typedef double X;          // LDS element
    typedef f64x4 Acc4;
    typedef double Acc;
    typedef u32x4 Frag;        // double2 bit pattern
    static constexpr int KS = 8, VEC = 2;
};
template <> struct MfmaT<MK_F32> {
    typedef float X;
    typedef f32x4 Acc4;
    typedef float Acc;
    typedef u32x4 Frag;        // float4 bit pattern
    static constexpr int KS = 16, VEC = 4;
};
template <> struct MfmaT<MK_BF16> {
    typedef unsigned short X;
    typedef f32x4 Acc4;
    typedef float Acc;
    typedef u32x4 Frag;        // 8 bf16
    static constexpr int KS = 32, VEC = 8;
};
template <> struct MfmaT<MK_BF16X3> : MfmaT<MK_BF16> {};

// ---------------------------------------------------------------- fragment loads

// A fragment: VEC consecutive k of one row, converted to the MFMA operand format.
// ADT is the operator's storage format.  Loads are never predicated (the caller keeps
// every address inside the allocation), so the compiler can count them exactly.
// NT: non-temporal (streamed once) loads; plain loads when sibling blocks of other
// column tiles re-read the same rows through L2.
template <int BYTES, bool NT>
__device__ __forceinline__ typename RawT<BYTES>::T ld_a(const void* p) {
    if constexpr (NT) return ld_stream<BYTES>(p);
    else return ld_plain<BYTES>(p);
}

template <int ADT, int MKD, bool NT>
__device__ __forceinline__ void load_a(const void* A, const unsigned short* Alo, size_t off, u32x4& hi,
                                       u32x4& lo) {
    if constexpr (MKD == MK_F64 || (MKD == MK_F32 && ADT == DT_F32) || MKD == MK_BF16) {
        typedef typename Store<ADT>::T T;
        hi = ld_a<16, NT>(reinterpret_cast<const T*>(A) + off);
    } else if constexpr (MKD == MK_BF16X3) {
        hi = ld_a<16, NT>(reinterpret_cast<const unsigned short*>(A) + off);
        lo = ld_a<16, NT>(Alo + off);
    } else {
        // FP32 MFMA over a BF16 / BF16X3 operator: 4 words -> 4 floats (hi + lo exact)
        const u32x2 h = ld_a<8, NT>(reinterpret_cast<const unsigned short*>(A) + off);
        float f[4] = {bf16_lo_f(h[0]), bf16_hi_f(h[0]), bf16_lo_f(h[1]), bf16_hi_f(h[1])};
        if constexpr (ADT == DT_BF16X3) {
            const u32x2 l = ld_a<8, NT>(Alo + off);
            f[0] += bf16_lo_f(l[0]);
            f[1] += bf16_hi_f(l[0]);
            f[2] += bf16_lo_f(l[1]);
            f[3] += bf16_hi_f(l[1]);
        }
        hi[0] = __float_as_uint(f[0]);
        hi[1] = __float_as_uint(f[1]);
        hi[2] = __float_as_uint(f[2]);
        hi[3] = __float_as_uint(f[3]);
    }
}

template <int MKD>
__device__ __forceinline__ void mfma_step(typename MfmaT<MKD>::Acc4& acc, const u32x4& a, const u32x4& al,
                                          const u32x4& b, const u32x4& bl) {
    if constexpr (MKD == MK_F64) {
        const double* ad = reinterpret_cast<const double*>(&a);
        const double* bd = reinterpret_cast<const double*>(&b);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[0], bd[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[1], bd[1], acc, 0, 0, 0);
    } else if constexpr (MKD == MK_F32) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[e]), __uint_as_float(b[e]), acc, 0, 0, 0);
    } else if constexpr (MKD == MK_BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, bl),
                                                      acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
    }
}

}  // namespace rom
