// k_res.hip -- the one-trajectory CP step with its operator resident on chip.
//
// From level 2 on, every step of a one-trajectory CP state applies the same order-3
// operators (Sec. 3.1, eq. tc_ap, inside the BDF3/EXT3 step of eq. nse_d1): the rows of
// Af for the Hadamard-scatter, the projection rows (the pair form of Sec. 3.3 or
// [Bf|Cf]^T; with a dense stiffness their products with Hinv_3) and, with a dense
// stiffness, the rows of Hinv_3.  The per-step kernels stream those rows from memory
// twice a step.  Here one block per compute unit at most, all on the device at once (an
// otherwise idle device places every block of such a launch; the host orders the runs of
// one process across streams), copies its share of the rows into LDS once and then runs a
// whole sequence of steps on them: a step reads no operator bytes from memory.
//
// Between blocks only two vectors move per step: x (the right-hand side, N FP64 values;
// with a diagonal stiffness u^{n+1}) and w = lam .* s .* t (Rp values).  They travel as
// 64-bit words, a 32-bit payload beside a 32-bit tag (the message's sequence number),
// written and read with device-scope atomic stores and loads.  A block that needs a vector
// polls its words until every one carries the expected tag, so the wait and the transfer
// are one round trip and no grid barrier is needed.  One buffer per vector suffices: a
// block can only write the next version of a vector after reading every block's share
// of the other vector, which each block wrote after it had read the current version.
// Tags come from a per-state counter that only grows, so no stale word carries a tag
// that a later run waits for.  Every wait is bounded (spin_max rounds); a wait that gives
// up raises the error flag and every block then leaves at its next wait.
//
// Each dot product sums in the order of the per-step kernels (kbody.h, kstep.h), with the
// same reductions and the same per-block energy partials, so a run here equals the same
// steps through those kernels to the bit.
#include "kbody.h"

namespace rom {

namespace {

constexpr int kNT = 256;
constexpr int kWaitPer = kResWaitWords / kNT;   // message words per thread

__device__ __forceinline__ unsigned long long ld_msg(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_msg(unsigned long long* p, unsigned tag, unsigned payload) {
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_msg_f64(unsigned long long* p, unsigned tag, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    st_msg(p, tag, (unsigned)b);
    st_msg(p + 1, tag, (unsigned)(b >> 32));
}
template <class Acc>
__device__ __forceinline__ void st_msg_acc(unsigned long long* wmsg, int e, unsigned tag, Acc v) {
    if constexpr (sizeof(Acc) == 8) st_msg_f64(wmsg + 2 * e, tag, (double)v);
    else st_msg(wmsg + e, tag, __float_as_uint((float)v));
}

// Whole block: wait until every element e < ne of a message (WPE words each, 1 or 2)
// carries `tag` in all its words, handing each element's payload (the words' low halves,
// first word lowest) to put(e, bits) once.  Thread t polls elements t, t + 256, ...,
// reissuing in one round the loads of every element still stale.  Returns false in every
// thread if a wait of this block or of another gave up.  backoff: the block has just
// sent its share of the message it waits for (no other share can be there yet).
template <int WPE, class PutF>
__device__ bool res_wait(const ResJob& jb, const unsigned long long* src, int ne, unsigned tag, PutF put,
                         bool backoff) {
    constexpr int KE = kWaitPer / WPE;
    unsigned pend = 0;
#pragma unroll
    for (int t = 0; t < KE; ++t)
        if ((int)threadIdx.x + t * kNT < ne) pend |= 1u << t;
    unsigned spins = 0;
    bool ok = true;
    // right after a block's own message no other block's words can be there sooner than a
    // round trip to memory: polling at once would only load the memory side that the
    // writers' stores go through
    if (backoff) {
#pragma unroll
        for (int z = 0; z < 4; ++z) __builtin_amdgcn_s_sleep(8);
    }
    while (pend) {
        unsigned long long v[KE][WPE];
#pragma unroll
        for (int t = 0; t < KE; ++t)
#pragma unroll
            for (int q = 0; q < WPE; ++q)
                v[t][q] = (pend >> t) & 1u ? ld_msg(src + (size_t)(threadIdx.x + t * kNT) * WPE + q) : 0ull;
#pragma unroll
        for (int t = 0; t < KE; ++t) {
            bool here = (pend >> t) & 1u;
#pragma unroll
            for (int q = 0; q < WPE; ++q) here = here && (unsigned)(v[t][q] >> 32) == tag;
            if (here) {
                unsigned long long bits = (unsigned)v[t][0];
                if constexpr (WPE == 2) bits |= (unsigned long long)(unsigned)v[t][1] << 32;
                put((int)threadIdx.x + t * kNT, bits);
                pend &= ~(1u << t);
            }
        }
        if (pend) {
            ++spins;
            if (spins > jb.spin_max ||
                ((spins & 63u) == 0 && __hip_atomic_load(jb.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(jb.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return __syncthreads_or(ok ? 0 : 1) == 0;
}

// Whole block: copy nrows rows of row_bytes (a multiple of 16) to dst (rows
// back to back); src(r) is row r's address, or null for a row past the operator (zeros).
// nrows rows of row_bytes (a multiple of 16) into LDS at dst, a row whose src(r) is null as
// zeros.  16-byte direct loads from memory into LDS (no registers in between), all of the
// block's loads in flight at once: a wave's 64 lanes fill 1 KB of consecutive LDS per
// load.  The caller waits for them (lds_rows_done) before any wave reads the rows.
template <class SrcF>
__device__ void lds_rows(char* dst, int nrows, size_t row_bytes, SrcF src) {
    const int cpr = (int)(row_bytes / 16), n = nrows * cpr;
    const int lane = threadIdx.x % kWave;
    for (int base = (int)(threadIdx.x - lane); base < n; base += (int)blockDim.x) {   // wave-uniform
        const int q = base + lane, r = q / cpr, c = q - r * cpr;
        const char* s = q < n ? src(r) : nullptr;
        if (s) __builtin_amdgcn_global_load_lds(s + (size_t)c * 16, dst + (size_t)base * 16, 16, 0, 0);
        else if (q < n) *reinterpret_cast<u32x4*>(dst + (size_t)q * 16) = u32x4{0u, 0u, 0u, 0u};
    }
}

// The direct loads of lds_rows have landed (this wave's), then every wave's (barrier).
__device__ __forceinline__ void lds_rows_done() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Groups g = b, b + G, ... below n owned by block b.
__device__ __forceinline__ int owned(int n, int b, int G) { return b < n ? (n - b + G - 1) / G : 0; }

}  // namespace

template <int DT, bool EVEN>
__global__ __launch_bounds__(kNT) void k_cp_resident(ResJob jb) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(T);
    typedef typename RawT<16>::T Raw;
    constexpr bool X3 = (DT == DT_BF16X3);
    constexpr bool NEGU = (DT == DT_BF16 || DT == DT_BF16X3);
    constexpr int WPE = (int)sizeof(Acc) / 4;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ double red[4];

    const StepArgs& a = jb.a;
    const int N = a.N, Np = a.Np, Rp = jb.Rp, P = jb.P, R = jb.R;
    const bool pair = jb.layout != 0, dense_h = jb.dense_h != 0;
    const ResLayout lay = res_layout(DT, N, Np, Rp, jb.layout, jb.dense_h, jb.rg_per, jb.pg_per);
    Acc* W = reinterpret_cast<Acc*>(smem + lay.W);
    double* xr = reinterpret_cast<double*>(smem + lay.xr);
    LdsU<DT> L, Ln;
    L.bind(smem + lay.L, Np);
    Ln.bind(smem + lay.Ln, Np);
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int G = gridDim.x, b = blockIdx.x;
    const int nrg_b = owned(jb.nrg, b, G), npg_b = owned(jb.npg, b, G);
    const int PH = pair ? 3 : 2;
    const size_t eb = sizeof(T);

    // ---- the block's rows into LDS
    {
        const char* af = reinterpret_cast<const char*>(jb.Af);
        auto row_i = [&](int r) { return 4 * (b + (r / 4) * G) + r % 4; };
        lds_rows(smem + lay.af, 4 * nrg_b, (size_t)Rp * eb,
                 [&](int r) { const int i = row_i(r); return i < N ? af + (size_t)i * Rp * eb : nullptr; });
        if constexpr (X3) {
            const char* al = reinterpret_cast<const char*>(jb.Af_lo);
            lds_rows(smem + lay.aflo, 4 * nrg_b, (size_t)Rp * 2,
                     [&](int r) { const int i = row_i(r); return i < N ? al + (size_t)i * Rp * 2 : nullptr; });
        }
        if (dense_h) {
            const char* h3 = reinterpret_cast<const char*>(a.hinv + (size_t)2 * N * Np);
            lds_rows(smem + lay.hv, 4 * nrg_b, (size_t)Np * 8,
                     [&](int r) { const int i = row_i(r); return i < N ? h3 + (size_t)i * Np * 8 : nullptr; });
        }
        // projection row h of wave w in local group lp: pair form rows q, P + c0, P + c1
        // (q < P); general form rows r and Rp + r
        auto prow = [&](int r) -> long long {
            const int h = r % PH, slot = r / PH, w = slot % 4, lp = slot / 4;
            const int q = 4 * (b + lp * G) + w;
            if (pair) {
                if (q >= P) return -1;
                const int c0 = jb.layout == 1 ? 2 * q : q, c1 = jb.layout == 1 ? 2 * q + 1 : P + q;
                return h == 0 ? q : h == 1 ? P + c0 : P + c1;
            }
            if (q >= Rp) return -1;
            return h == 0 ? q : Rp + q;
        };
        const char* po = reinterpret_cast<const char*>(jb.Pop);
        lds_rows(smem + lay.pr, 4 * PH * npg_b, (size_t)Np * eb, [&](int r) {
            const long long k = prow(r);
            return k < 0 ? nullptr : po + (size_t)k * Np * eb;
        });
        if constexpr (X3) {
            const char* pl = reinterpret_cast<const char*>(jb.Pop_lo);
            lds_rows(smem + lay.prlo, 4 * PH * npg_b, (size_t)Np * 2, [&](int r) {
                const long long k = prow(r);
                return k < 0 ? nullptr : pl + (size_t)k * Np * 2;
            });
        }
    }
    lds_rows_done();

    const unsigned seq0 = *jb.seq;
    const BdfCoef cf = bdf_coef(3);
    const bool imgs = npg_b > 0, negu = NEGU && pair;
    // the images' padding entries (N <= q < Np) stay zero
    for (int q = N + (int)threadIdx.x; q < Np; q += kNT) {
        L.put(q, 0.0);
        if (negu) Ln.put(q, 0.0);
    }
    // element i of x: FP64 into xr, and into the images the projections read
    auto put_x = [&](int i, unsigned long long bits) {
        const double v = __longlong_as_double((long long)bits);
        xr[i] = v;
        if (imgs) {
            L.put(i, v);
            if (negu) Ln.put(i, -1.0 * v);
        }
    };
    auto put_w = [&](int e, unsigned long long bits) {
        if constexpr (WPE == 2) W[e] = (Acc)__longlong_as_double((long long)bits);
        else W[e] = (Acc)__uint_as_float((unsigned)bits);
    };

    // lam of the block's w entries (two per wave and projection group, pair form; one in
    // the general form), so that no global load sits between a projection and its message
    constexpr int kMaxPG = 8;                            // projection groups per block, at most
    __shared__ Acc lam_b[kMaxPG][4][2];
    {
        const Acc* lam = reinterpret_cast<const Acc*>(jb.lam);
        for (int q = threadIdx.x; q < npg_b * 8; q += kNT) {
            const int lp = q / 8, w = (q / 2) % 4, h = q % 2;
            const int qq = 4 * (b + lp * G) + w;
            Acc v = 0;
            if (pair && qq < P) v = lam[h == 0 ? (jb.layout == 1 ? 2 * qq : qq) : (jb.layout == 1 ? 2 * qq + 1 : P + qq)];
            else if (!pair && qq < Rp && h == 0) v = lam[qq];
            lam_b[lp][w][h] = v;
        }
        __syncthreads();
    }

    // projections of x (images L, Ln) for the block's groups: w entries as messages (and,
    // for the last level of a dense-stiffness run, into the state's w)
    auto projections = [&](unsigned tw, bool store_st) {
        constexpr int PU = 4;
        Acc* st = reinterpret_cast<Acc*>(a.st);
        for (int lp = 0; lp < npg_b; ++lp) {
            const int q = 4 * (b + lp * G) + wv;
            const T* rows = reinterpret_cast<const T*>(smem + lay.pr) + (size_t)(lp * 4 + wv) * PH * Np;
            const unsigned short* rlo =
                X3 ? reinterpret_cast<const unsigned short*>(smem + lay.prlo) + (size_t)(lp * 4 + wv) * PH * Np
                   : nullptr;
            if (pair) {
                if (q >= P) {
                    const int e = R + 2 * (q - P);               // zero padding of w past R
                    if (lane == 0 && e < Rp) {
                        st_msg_acc<Acc>(jb.wmsg, e, tw, (Acc)0);
                        if (store_st) st[e] = 0;
                        if (e + 1 < Rp) {
                            st_msg_acc<Acc>(jb.wmsg, e + 1, tw, (Acc)0);
                            if (store_st) st[e + 1] = 0;
                        }
                    }
                    continue;
                }
                Acc z[3] = {0, 0, 0};                            // beta, -alpha, gamma
                for (int k0 = lane * V; k0 < Np; k0 += kWave * V * PU) {
                    Raw rv[PU][3], rl[PU][3];
#pragma unroll
                    for (int t = 0; t < PU; ++t) {
                        const int k = k0 + t * kWave * V;
                        if (k < Np) {
#pragma unroll
                            for (int h = 0; h < 3; ++h) {
                                rv[t][h] = *reinterpret_cast<const Raw*>(rows + (size_t)h * Np + k);
                                if constexpr (X3) rl[t][h] = *reinterpret_cast<const Raw*>(rlo + (size_t)h * Np + k);
                                else rl[t][h] = rv[t][h];
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < PU; ++t) {
                        const int k = k0 + t * kWave * V;
                        if (k < Np) {
                            z[0] += dot_vec<DT, V>(rv[t][0], rl[t][0], L, k);
                            z[1] += dot_vec<DT, V>(rv[t][1], rl[t][1], NEGU ? Ln : L, k);
                            z[2] += dot_vec<DT, V>(rv[t][2], rl[t][2], L, k);
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < 3; ++h) z[h] = wave_sum(z[h]);
                if (lane == 0) {
                    const int c0 = jb.layout == 1 ? 2 * q : q, c1 = jb.layout == 1 ? 2 * q + 1 : P + q;
                    const Acc w0 = lam_b[lp][wv][0] * z[0] * z[2];
                    const Acc w1 = lam_b[lp][wv][1] * z[0] * (NEGU ? z[1] : -z[1]);
                    st_msg_acc<Acc>(jb.wmsg, c0, tw, w0);
                    st_msg_acc<Acc>(jb.wmsg, c1, tw, w1);
                    if (store_st) {
                        st[c0] = w0;
                        st[c1] = w1;
                    }
                }
            } else {
                if (q >= Rp) continue;
                Acc z[2] = {0, 0};
                for (int k0 = lane * V; k0 < Np; k0 += kWave * V * PU) {
                    Raw rv[PU][2], rl[PU][2];
#pragma unroll
                    for (int t = 0; t < PU; ++t) {
                        const int k = k0 + t * kWave * V;
                        if (k < Np) {
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                rv[t][h] = *reinterpret_cast<const Raw*>(rows + (size_t)h * Np + k);
                                if constexpr (X3) rl[t][h] = *reinterpret_cast<const Raw*>(rlo + (size_t)h * Np + k);
                                else rl[t][h] = rv[t][h];
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < PU; ++t) {
                        const int k = k0 + t * kWave * V;
                        if (k < Np) {
                            z[0] += dot_vec<DT, V>(rv[t][0], rl[t][0], L, k);
                            z[1] += dot_vec<DT, V>(rv[t][1], rl[t][1], L, k);
                        }
                    }
                }
                z[0] = wave_sum(z[0]);
                z[1] = wave_sum(z[1]);
                if (lane == 0) {
                    const Acc w0 = lam_b[lp][wv][0] * z[0] * z[1];
                    st_msg_acc<Acc>(jb.wmsg, q, tw, w0);
                    if (store_st) st[q] = w0;
                }
            }
        }
    };

    // the history of the block's rows (read by lane 0 of the wave that owns the row)
    constexpr int kMaxRG = 4;                            // row groups per block, at most
    __shared__ BdfHist hist[kMaxRG][4];
    __shared__ double hd[kMaxRG][4];

    // the block's scatter rows against W: y^n, the right-hand side and (diagonal
    // stiffness) u^{n+1} with its energy partials; x as messages
    auto scatter = [&](long long n, int j, unsigned tx) {
        constexpr int SU = 32 / V < 4 ? 4 : 32 / V;        // 32 weights per batch
        for (int lg = 0; lg < nrg_b; ++lg) {
            const int g = b + lg * G;
            const int i = 4 * g + wv;
            const bool live = i < N;
            const T* row = reinterpret_cast<const T*>(smem + lay.af) + (size_t)(lg * 4 + wv) * Rp;
            const unsigned short* rowlo =
                X3 ? reinterpret_cast<const unsigned short*>(smem + lay.aflo) + (size_t)(lg * 4 + wv) * Rp : nullptr;
            Acc z = 0;
            if (live) {
                for (int r0 = lane * V; r0 < Rp; r0 += kWave * V * SU) {
                    Raw rv[SU], rl[SU];
                    Acc wg[SU][V];
#pragma unroll
                    for (int t = 0; t < SU; ++t) {
                        const int r = r0 + t * kWave * V;
                        if (r < Rp) {
                            rv[t] = *reinterpret_cast<const Raw*>(row + r);
                            if constexpr (X3) rl[t] = *reinterpret_cast<const Raw*>(rowlo + r);
#pragma unroll
                            for (int v = 0; v < V; ++v) wg[t][v] = W[r + v];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < SU; ++t) {
                        const int r = r0 + t * kWave * V;
                        if (r < Rp) {
                            Acc cv[V];
                            Decode<DT, V>::run(rv[t], cv);
                            if constexpr (X3) {
                                float cl[V];
                                Decode<DT, V>::run(rl[t], cl);
#pragma unroll
                                for (int v = 0; v < V; ++v) z += (cv[v] + cl[v]) * wg[t][v];
                            } else {
#pragma unroll
                                for (int v = 0; v < V; ++v) z += cv[v] * wg[t][v];
                            }
                        }
                    }
                }
                z = wave_sum(z);
            }
            double e = 0.0;
            if (live && lane == 0) {
                const double rhs = bdf_rhs_hist(a, n, cf, 3, 0, i, (double)z, hist[lg][wv]);
                if (dense_h) {
                    st_msg_f64(jb.xmsg + 2 * i, tx, rhs);
                } else {
                    const double un = rhs * hd[lg][wv];
                    write_level(a, n + 1, 0, i, un);
                    e = un * un;
                    st_msg_f64(jb.xmsg + 2 * i, tx, un);
                }
            }
            if (!dense_h) {
                const double es = block_sum(e, red);
                if (threadIdx.x == 0) jb.epall[(size_t)j * jb.nrg + g] = es;
            }
        }
    };

    // the block's rows of Hinv_3 against xr: u^{n+1} and its energy partials
    auto helm_rows = [&](long long n, int j) {
        constexpr int HV = EVEN ? 2 : 1, HU = 8;
        for (int lg = 0; lg < nrg_b; ++lg) {
            const int g = b + lg * G;
            const int i = 4 * g + wv;
            const double* h = reinterpret_cast<const double*>(smem + lay.hv) + (size_t)(lg * 4 + wv) * Np;
            double e = 0.0;
            if (i < N) {
                double s = 0.0;
                for (int m0 = lane * HV; m0 < N; m0 += kWave * HV * HU) {
                    double hv[HU][HV], xv[HU][HV];
#pragma unroll
                    for (int t = 0; t < HU; ++t) {
                        const int m = m0 + t * kWave * HV;
                        if (m < N) {
#pragma unroll
                            for (int v = 0; v < HV; ++v) {
                                hv[t][v] = h[m + v];
                                xv[t][v] = xr[m + v];
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < HU; ++t) {
                        const int m = m0 + t * kWave * HV;
                        if (m < N) {
#pragma unroll
                            for (int v = 0; v < HV; ++v) s += hv[t][v] * xv[t][v];
                        }
                    }
                }
                s = wave_sum(s);
                if (lane == 0) {
                    write_level(a, n + 1, 0, i, s);
                    e = s * s;
                }
            }
            const double es = block_sum(e, red);
            if (threadIdx.x == 0) jb.epall[(size_t)j * jb.nrg + g] = es;
        }
    };

    for (int j = 0; j < jb.nsteps; ++j) {
        const long long n = jb.n0 + j;
        const unsigned tx = seq0 + 2u * (unsigned)j + 1u, tw = seq0 + 2u * (unsigned)j + 2u;
        // the history of the block's rows, behind the waits
        for (int lg = 0; lg < nrg_b; ++lg) {
            const int i = 4 * (b + lg * G) + wv;
            if (lane == 0 && i < N) {
                hist[lg][wv] = bdf_hist_point(a, n, 3, 0, i);
                hd[lg][wv] = dense_h ? 0.0 : a.hdiag[(size_t)2 * N + i];
            }
        }
        if (dense_h) {
            // scatter of level n against w^n, then w^{n+1} = lam .* s .* t of Hinv_3 rhs
            // (the next scatter waits for it) and u^{n+1} = Hinv_3 rhs (needed only by
            // this block's next right-hand sides, so it runs while w^{n+1} travels)
            if (nrg_b) {
                if (j == 0) {
                    const Acc* win = reinterpret_cast<const Acc*>(a.st);
                    staged_copy<8, Acc>(Rp, [&](int r) { return win[r]; }, [&](int r, Acc v) { W[r] = v; });
                    __syncthreads();
                } else if (!res_wait<WPE>(jb, jb.wmsg, Rp, tw - 2u, put_w, !imgs)) {
                    return;
                }
                scatter(n, j, tx);
            }
            if (!res_wait<2>(jb, jb.xmsg, N, tx, put_x, nrg_b > 0)) return;
            if (imgs) projections(tw, j + 1 == jb.nsteps);
            helm_rows(n, j);
        } else {
            // w^n from u^n, then the scatter of level n with the update to u^{n+1}
            if (imgs) {
                if (j == 0) {
                    const double* un = a.uring + (size_t)slot_of(n) * N;
                    for (int m = threadIdx.x; m < N; m += kNT)
                        put_x(m, (unsigned long long)__double_as_longlong(un[m]));
                    __syncthreads();
                } else if (!res_wait<2>(jb, jb.xmsg, N, tx - 2u, put_x, nrg_b > 0)) {
                    return;
                }
                projections(tw, false);
            }
            if (nrg_b) {
                if (!res_wait<WPE>(jb, jb.wmsg, Rp, tw, put_w, imgs)) return;
                scatter(n, j, tx);
            }
        }
    }
}

// Energies of the run's levels and the state's bookkeeping, after the run.  Block j < L - 1
// logs level n0 + 1 + j from the run's partials (summed in the order close_level sums);
// the last block closes level n0 if it is still pending, leaves level n0 + L pending in
// the parity slots the step kernels use, advances the counter and moves the tag base
// past the run's tags.  256 threads a block.
__global__ __launch_bounds__(kNT) void k_res_close(StepArgs a0, StepArgs aL, long long n0, int nsteps,
                                                   const double* __restrict__ epall, int nrg, unsigned* seq,
                                                   int close_last) {
    __shared__ double cred[4];
    const int j = blockIdx.x;
    if (j + 1 < nsteps) {
        const long long n = n0 + 1 + j;
        const double* ep = epall + (size_t)j * nrg;
        double s = 0.0;
        for (int q = threadIdx.x; q < nrg; q += blockDim.x) s += ep[q];
        s = block_sum(s, cred);
        if (threadIdx.x == 0) {
            const double e = 0.5 * s;
            if (n < a0.elog_cap) a0.elog[n] = e;
            if (!isfinite(e)) atomicMin(a0.bad, n);
        }
        return;
    }
    close_level(a0, n0);
    __syncthreads();
    const long long nl = n0 + nsteps;
    double* ep = epart_of(aL, nl);
    for (int q = threadIdx.x; q < nrg; q += blockDim.x) ep[q] = epall[(size_t)(nsteps - 1) * nrg + q];
    __syncthreads();
    if (threadIdx.x == 0) {
        aL.ecount[nl & 1] = nrg;
        *aL.closep = 1;
        *aL.step = nl;
        *seq += 2u * (unsigned)nsteps + 2u;
    }
    if (close_last) {
        // the run ends a sequence of steps: its last level is closed here, as a closing
        // kernel would close it
        __syncthreads();
        close_level(aL, nl);
        __syncthreads();
        if (threadIdx.x == 0) *aL.closep = 0;
    }
}

namespace {

template <int DT, bool EVEN>
hipError_t res_go(const ResJob& jb, int G, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_cp_resident<DT, EVEN>), dim3((unsigned)G), dim3(kNT), (unsigned)lds, s, jb);
    return hipGetLastError();
}

template <int DT, bool EVEN>
hipError_t res_attr_go(size_t cap, size_t lds, int* per_cu) {
    const void* f = reinterpret_cast<const void*>(&k_cp_resident<DT, EVEN>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, kNT, lds);
}

}  // namespace

hipError_t res_launch(int dt, const ResJob& jb, int G, size_t lds, hipStream_t s) {
    const bool even = jb.a.N % 2 == 0;
    switch (dt) {
        case DT_F64: return even ? res_go<DT_F64, true>(jb, G, lds, s) : res_go<DT_F64, false>(jb, G, lds, s);
        case DT_F32: return even ? res_go<DT_F32, true>(jb, G, lds, s) : res_go<DT_F32, false>(jb, G, lds, s);
        case DT_BF16: return even ? res_go<DT_BF16, true>(jb, G, lds, s) : res_go<DT_BF16, false>(jb, G, lds, s);
        default: return even ? res_go<DT_BF16X3, true>(jb, G, lds, s) : res_go<DT_BF16X3, false>(jb, G, lds, s);
    }
}

hipError_t res_attr(int dt, int N, size_t cap, size_t lds, int* per_cu) {
    const bool even = N % 2 == 0;
    switch (dt) {
        case DT_F64:
            return even ? res_attr_go<DT_F64, true>(cap, lds, per_cu) : res_attr_go<DT_F64, false>(cap, lds, per_cu);
        case DT_F32:
            return even ? res_attr_go<DT_F32, true>(cap, lds, per_cu) : res_attr_go<DT_F32, false>(cap, lds, per_cu);
        case DT_BF16:
            return even ? res_attr_go<DT_BF16, true>(cap, lds, per_cu) : res_attr_go<DT_BF16, false>(cap, lds, per_cu);
        default:
            return even ? res_attr_go<DT_BF16X3, true>(cap, lds, per_cu)
                        : res_attr_go<DT_BF16X3, false>(cap, lds, per_cu);
    }
}

void res_close_launch(const StepArgs& a0, const StepArgs& aL, long long n0, int nsteps, const double* epall,
                      int nrg, unsigned* seq, bool close_last, hipStream_t s) {
    hipLaunchKernelGGL(k_res_close, dim3((unsigned)nsteps), dim3(kNT), 0, s, a0, aL, n0, nsteps, epall, nrg, seq,
                       close_last ? 1 : 0);
}

}  // namespace rom
