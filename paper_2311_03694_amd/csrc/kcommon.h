// kcommon.h -- device helpers shared by the kernel sources: number-format
// conversions, vector loads and wavefront reductions.
#pragma once

#include "rom_dev.h"

namespace rom {

// ---------------------------------------------------------------- BF16 words

// FP32 -> BF16 word, round to nearest even (gfx950 has a hardware conversion).
__device__ __forceinline__ unsigned short bf16_bits(float f) {
    __bf16 h = (__bf16)f;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// ---------------------------------------------------------------- storage traits

// Per-dtype storage of the operator: element type, whether a low word stream exists,
// and the accumulation type of the contraction.
template <int DT> struct Store;
template <> struct Store<DT_F64> { typedef double T; typedef double Acc; static constexpr bool kLo = false; };
template <> struct Store<DT_F32> { typedef float T; typedef float Acc; static constexpr bool kLo = false; };
template <> struct Store<DT_BF16> { typedef unsigned short T; typedef float Acc; static constexpr bool kLo = false; };
template <> struct Store<DT_BF16X3> { typedef unsigned short T; typedef float Acc; static constexpr bool kLo = true; };

// ---------------------------------------------------------------- raw vector loads

template <int BYTES> struct RawT;
template <> struct RawT<16> { typedef u32x4 T; };
template <> struct RawT<8> { typedef u32x2 T; };
template <> struct RawT<4> { typedef unsigned int T; };
template <> struct RawT<2> { typedef unsigned short T; };

// Streaming (non-temporal) load of BYTES bytes; the address must be BYTES-aligned.
template <int BYTES>
__device__ __forceinline__ typename RawT<BYTES>::T ld_stream(const void* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename RawT<BYTES>::T*>(p));
}
template <int BYTES>
__device__ __forceinline__ typename RawT<BYTES>::T ld_plain(const void* p) {
    return *reinterpret_cast<const typename RawT<BYTES>::T*>(p);
}

// Decode V consecutive stored elements from a raw vector into the accumulation type.
template <int DT, int V> struct Decode;
template <int V> struct Decode<DT_F32, V> {
    template <class R> __device__ static void run(const R& r, float* out) {
        const unsigned int* w = reinterpret_cast<const unsigned int*>(&r);
#pragma unroll
        for (int q = 0; q < V; ++q) out[q] = __uint_as_float(w[q]);
    }
};
template <int V> struct Decode<DT_F64, V> {
    template <class R> __device__ static void run(const R& r, double* out) {
        const double* w = reinterpret_cast<const double*>(&r);
#pragma unroll
        for (int q = 0; q < V; ++q) out[q] = w[q];
    }
};
template <int V> struct DecodeBf16 {
    template <class R> __device__ static void run(const R& r, float* out) {
        if constexpr (V == 1) {
            out[0] = bf16_f(*reinterpret_cast<const unsigned short*>(&r));
        } else {
            const unsigned int* w = reinterpret_cast<const unsigned int*>(&r);
#pragma unroll
            for (int q = 0; q < V / 2; ++q) {
                out[2 * q] = bf16_lo_f(w[q]);
                out[2 * q + 1] = bf16_hi_f(w[q]);
            }
        }
    }
};
template <int V> struct Decode<DT_BF16, V> : DecodeBf16<V> {};
template <int V> struct Decode<DT_BF16X3, V> : DecodeBf16<V> {};

// ---------------------------------------------------------------- reductions

// Lane exchange within rows of 16 lanes (DPP row_ror:K, K = 1..15) and lane reads.
template <int K>
__device__ __forceinline__ float row_ror(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + K, 0xF, 0xF, false));
}
template <int K>
__device__ __forceinline__ double row_ror(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x120 + K, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x120 + K, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_read(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wavefront, the same value in every lane; every lane must be active.
// Within each row of 16 lanes, v += v rotated by 8, 4, 2, 1 lanes (after the rotation by
// k the row has period k, the two addends of every sum being the same pair in either
// order, so all 16 lanes hold the row's sum), then (row0 + row1) + (row2 + row3).  DPP
// moves and lane reads instead of LDS permutes: a few cycles a step.
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    v += row_ror<8>(v);
    v += row_ror<4>(v);
    v += row_ror<2>(v);
    v += row_ror<1>(v);
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// Sum over the block (blockDim.x a multiple of 64, at most 1024); result valid in
// thread 0.  `scratch` holds at least blockDim.x/64 values.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0) {
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) s += scratch[q];
    }
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- staging into LDS

// Block-cooperative loop over q in [0, n): out(q, in(q)), with U loads per thread
// issued before any store, so a staging pass costs one memory round trip per U
// elements instead of one per element.
template <int U, class T, class LoadF, class StoreF>
__device__ __forceinline__ void staged_copy(int n, LoadF load, StoreF store) {
    for (int base = threadIdx.x; base < n; base += U * (int)blockDim.x) {
        T v[U];
#pragma unroll
        for (int e = 0; e < U; ++e) {
            const int q = base + e * (int)blockDim.x;
            if (q < n) v[e] = load(q);
        }
#pragma unroll
        for (int e = 0; e < U; ++e) {
            const int q = base + e * (int)blockDim.x;
            if (q < n) store(q, v[e]);
        }
    }
}

// ---------------------------------------------------------------- grouped launches

// Job p with jobs[p].blk0 <= q < jobs[p+1].blk0 (jobs sorted by blk0, blk0[0] = 0).
template <class J>
__device__ __forceinline__ int find_job(const J* jobs, int n, int q) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk0 <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- BDFk/EXTk weights

// Row k-1 holds order k: beta0, beta_1..beta_3 (new level on the left, old levels
// on the right with a minus sign) and alpha_1..alpha_3 (extrapolation), eq. nse_d1.
struct BdfCoef { double beta[4]; double alpha[3]; };
__device__ __forceinline__ BdfCoef bdf_coef(int k) {
    BdfCoef c;
    if (k == 1) {
        c.beta[0] = 1.0; c.beta[1] = -1.0; c.beta[2] = 0.0; c.beta[3] = 0.0;
        c.alpha[0] = 1.0; c.alpha[1] = 0.0; c.alpha[2] = 0.0;
    } else if (k == 2) {
        c.beta[0] = 1.5; c.beta[1] = -2.0; c.beta[2] = 0.5; c.beta[3] = 0.0;
        c.alpha[0] = 2.0; c.alpha[1] = -1.0; c.alpha[2] = 0.0;
    } else {
        c.beta[0] = 11.0 / 6.0; c.beta[1] = -3.0; c.beta[2] = 1.5; c.beta[3] = -1.0 / 3.0;
        c.alpha[0] = 3.0; c.alpha[1] = -3.0; c.alpha[2] = 1.0;
    }
    return c;
}

__device__ __forceinline__ int bdf_order(long long n) { return n >= 2 ? 3 : (int)(n + 1); }
__device__ __forceinline__ int slot_of(long long level) { return (int)(((level % 3) + 3) % 3); }

}  // namespace rom
