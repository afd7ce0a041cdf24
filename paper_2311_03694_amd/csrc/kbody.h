// kbody.h -- the per-block bodies of the one-trajectory step kernels: the dense
// streaming contraction (and the SVD form's slab stream), the CP projections (general and
// pair form) and Hadamard-scatter, the Helmholtz apply with the next projections, the SVD
// form's first product, the BDF update from contraction partials and the full form's
// zeroth-mode and mass terms.  Each body runs one block's share of one state's work
// (block index blk), so the kernels of one state (k_dense1.hip, k_contract.hip,
// k_bdf.hip) and the mixed kernels over many states' work tables (k_multi.hip) run the
// same arithmetic.
#pragma once

#include "kdot.h"
#include "kstep.h"

namespace rom {

// ============================================================== dense contraction, one trajectory

template <int DT, int V, int UNR, int NT>
__device__ __forceinline__ void dense_gemv_body(const GemvJob& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    typedef typename RawT<V * (int)sizeof(T)>::T Raw;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ Acc red[NT / kWave];
    const int N = jb.N, Np = jb.Np, nchunk = jb.nchunk;
    const long long chunk_len = jb.chunk_len;
    const T* __restrict__ C = reinterpret_cast<const T*>(jb.C);
    LdsU<DT> L;
    L.bind(smem, Np);
    // slab weights: u itself (its accumulation-format image), or jb.wj staged behind it
    Acc* wl = reinterpret_cast<Acc*>(smem + LdsU<DT>::bytes(Np));
    const Acc* wsrc = jb.wj ? wl : L.uw;

    const int i = blk / nchunk;
    const int c = blk - i * nchunk;
    const long long NN = (long long)jb.J * Np;
    const long long m0 = (long long)c * chunk_len;
    const long long m1 = (m0 + chunk_len < NN) ? m0 + chunk_len : NN;
    const T* row = C + (size_t)i * NN;
    const unsigned short* rowlo = X3 ? jb.Clo + (size_t)i * NN : nullptr;

    constexpr int STEP = NT * V;
    const int dj = STEP / Np, dk = STEP - (STEP / Np) * Np;
    long long m = m0 + (long long)threadIdx.x * V;
    int j = (int)(m / Np), k = (int)(m - (long long)j * Np);

    Raw r[UNR], rl[UNR];
    int jj[UNR], kk[UNR];
    auto issue = [&](long long mb) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const long long mq = mb + (long long)q * STEP;
            jj[q] = j;
            kk[q] = k;
            if (mq < m1) {
                r[q] = ld_stream<BYTES>(row + mq);
                if constexpr (X3) rl[q] = ld_stream<BYTES>(rowlo + mq);
            }
            k += dk;
            j += dj;
            if (k >= Np) { k -= Np; ++j; }
        }
    };

    if (m < m1) issue(m);
    L.fill(jb.u_base + (jb.stepp ? (size_t)slot_of(*jb.stepp) * jb.slot_stride : 0), N, Np);
    if (jb.wj) {
        const Acc* wg = reinterpret_cast<const Acc*>(jb.wj);
        for (int q = threadIdx.x; q < jb.J; q += NT) wl[q] = wg[q];
    }
    __syncthreads();

    Acc acc = 0;
    while (m < m1) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            if (m + (long long)q * STEP < m1) acc += wsrc[jj[q]] * dot_vec<DT, V>(r[q], rl[q], L, kk[q]);
        }
        m += (long long)STEP * UNR;
        if (m < m1) issue(m);
    }
    const Acc s = block_sum(acc, red);
    if (threadIdx.x == 0) reinterpret_cast<Acc*>(jb.part)[(size_t)c * N + i] = s;
}


// ============================================================== full form terms

// Zeroth-mode and mass terms of the right-hand side of level n (eq. nse_d1), per
// trajectory b:
//   zfull = L uhat + (M - I) h,
//   uhat = sum_q alpha_q u^{n+1-q},  h = (1/dt) sum_q beta_q u^{n+1-q}
// (the EXT sum of the linear part of the bracket, and M minus the identity times the BDF
// history sum, which the rhs already carries; the constants are added with the rhs).
// Block blk of trajectory b (blockDim.x / 64 rows per block), one wavefront per row of G (2 Np doubles, read as
// 16-byte pairs in chunks of 16 per lane, a whole row up to N = 1024).  The first chunk of
// G and the history loads of the staging (up to 1024 coefficients per pass) are all issued
// before any of them is used, so the kernel waits for one round trip to memory instead of
// one per loop pass; eight rows per block share one staging of the history.
constexpr int kFullRows = 8, kFullChunk = 16, kFullStage = 2;

// The pieces of a row's term, shared by the terms kernel and the fused CP scatter so both
// sum in one order.  First chunk of row g2 (Np pairs) into gv, zero past Np or for an
// inactive row.
__device__ __forceinline__ void full_issue(const double2* __restrict__ g2, bool active, int lane, int Np,
                                           double2 (&gv)[kFullChunk]) {
#pragma unroll
    for (int u = 0; u < kFullChunk; ++u) {
        const int m = lane + u * kWave;
        gv[u] = (active && m < Np) ? g2[m] : make_double2(0.0, 0.0);
    }
}

// Element j of [uhat; h] from the element's history u[q] = u^{n-q}_j (q < k).
__device__ __forceinline__ void full_x_elem(const BdfCoef& c, int k, double inv_dt, const double (&u)[3], double& uh,
                                            double& h) {
    uh = 0.0;
    h = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        if (q < k) {
            uh += c.alpha[q] * u[q];
            h += (c.beta[q + 1] * inv_dt) * u[q];
        }
}

// Whole block: xs[0, Np) = uhat and xs[Np, 2 Np) = h of trajectory b at level n (zero past
// N); the caller synchronizes before reading.
__device__ __forceinline__ void full_stage_x(const StepArgs& a, long long n, int b, double* __restrict__ xs) {
    const int Np = a.Np, k = bdf_order(n);
    const BdfCoef c = bdf_coef(k);
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N;
    const double* lev[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) lev[q] = a.uring + (size_t)slot_of(n - q) * BN + off;
    for (int j0 = 0; j0 < Np; j0 += kFullStage * (int)blockDim.x) {
        double uv[3][kFullStage];
#pragma unroll
        for (int e = 0; e < kFullStage; ++e) {
            const int j = j0 + e * (int)blockDim.x + (int)threadIdx.x;
#pragma unroll
            for (int q = 0; q < 3; ++q) uv[q][e] = (q < k && j < a.N) ? lev[q][j] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < kFullStage; ++e) {
            const int j = j0 + e * (int)blockDim.x + (int)threadIdx.x;
            const double u3[3] = {uv[0][e], uv[1][e], uv[2][e]};
            double uh, h;
            full_x_elem(c, k, a.inv_dt, u3, uh, h);
            if (j < Np) {
                xs[j] = uh;
                xs[Np + j] = h;
            }
        }
    }
}

// The same staging in two halves for a block of 256 threads and Np <= 1024: the history
// loads (issued with the caller's other loads), then the elements into xs.
constexpr int kFullRegJ = 4;
struct FullHist { double u[3][kFullRegJ]; };
__device__ __forceinline__ void full_load_hist(const StepArgs& a, long long n, FullHist& fh) {
    const int k = bdf_order(n);
    const size_t BN = (size_t)a.B * a.N;
#pragma unroll
    for (int e = 0; e < kFullRegJ; ++e) {
        const int j = e * 256 + (int)threadIdx.x;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            fh.u[q][e] = (q < k && j < a.N) ? a.uring[(size_t)slot_of(n - q) * BN + j] : 0.0;
    }
}
__device__ __forceinline__ void full_store_x(const StepArgs& a, long long n, const FullHist& fh, double* __restrict__ xs) {
    const int Np = a.Np, k = bdf_order(n);
    const BdfCoef c = bdf_coef(k);
#pragma unroll
    for (int e = 0; e < kFullRegJ; ++e) {
        const int j = e * 256 + (int)threadIdx.x;
        const double u3[3] = {fh.u[0][e], fh.u[1][e], fh.u[2][e]};
        double uh, h;
        full_x_elem(c, k, a.inv_dt, u3, uh, h);
        if (j < Np) {
            xs[j] = uh;
            xs[Np + j] = h;
        }
    }
}

// The lane's part of row g2 . xs2 (chunks after the first loaded here), summed over its
// chunks in order; wave_sum of it is the row's term.
__device__ __forceinline__ double full_dot(const double2* __restrict__ g2, int lane, int Np,
                                           double2 (&gv)[kFullChunk], const double2* xs2) {
    double acc[kFullChunk];
#pragma unroll
    for (int u = 0; u < kFullChunk; ++u) acc[u] = 0.0;
    for (int base = 0; base < Np; base += kFullChunk * kWave) {
        if (base > 0) {
#pragma unroll
            for (int u = 0; u < kFullChunk; ++u) {
                const int m = base + lane + u * kWave;
                gv[u] = m < Np ? g2[m] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < kFullChunk; ++u) {
            const int m = base + lane + u * kWave;
            if (m < Np) {
                const double2 x = xs2[m];
                acc[u] += gv[u].x * x.x + gv[u].y * x.y;
            }
        }
    }
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < kFullChunk; ++u) t += acc[u];
    return t;
}

__device__ __forceinline__ void full_terms_body(const StepArgs& a, const double* __restrict__ G, int blk, int b) {
    extern __shared__ double2 xs2[];
    double* xs = reinterpret_cast<double*>(xs2);
    const int Np = a.Np;
    const int lane = threadIdx.x & (kWave - 1), i = blk * ((int)blockDim.x / kWave) + (threadIdx.x / kWave);
    const bool active = i < a.N;
    // row i of G as Np pairs (Np is a multiple of 8, rows 16-byte aligned)
    const double2* g2 = reinterpret_cast<const double2*>(G + (size_t)(active ? i : 0) * 2 * Np);
    double2 gv[kFullChunk];
    full_issue(g2, active, lane, Np, gv);
    full_stage_x(a, *a.step, b, xs);
    __syncthreads();
    if (!active) return;
    const double s = wave_sum(full_dot(g2, lane, Np, gv, xs2));
    if (lane == 0) a.zfull[(size_t)b * a.N + i] = s;
}


// ============================================================== CP, one trajectory

// Projections and Hadamard product: w[r] = lam_r (sum_k BCt[r][k] u_k)
// (sum_k BCt[Rp + r][k] u_k) for r < Rp (rows r < Rp are Bf^T, rows Rp + r are Cf^T).
// One wavefront per row pair, four per block; each lane issues its row loads before u
// is staged in LDS.  Each projection sums in the same order as a one-row dot product,
// and w = (lam s) t.
template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj1_body(const Proj1Job& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = jb.N, Np = jb.Np;
    LdsU<DT> L;
    L.bind(smem, Np);
    const int lane = threadIdx.x % kWave;
    const int r = blk * 4 + threadIdx.x / kWave;
    const bool live = r < jb.Rp;
    const size_t pair = (size_t)jb.Rp * Np;
    const T* row = reinterpret_cast<const T*>(jb.BCt) + (size_t)(live ? r : 0) * Np;
    const unsigned short* rowlo = X3 ? jb.BCt_lo + (size_t)(live ? r : 0) * Np : nullptr;
    Raw rv[2][U], rl[2][U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int k = kb + q * kWave * V;
                if (live && k < Np) {
                    rv[h][q] = ld_plain<BYTES>(row + (h ? pair : 0) + k);
                    if constexpr (X3) rl[h][q] = ld_plain<BYTES>(rowlo + (h ? pair : 0) + k);
                }
            }
    };
    issue(k0);
    L.fill(jb.u_base + (jb.stepp ? (size_t)slot_of(*jb.stepp) * jb.slot_stride : 0), N, Np);
    __syncthreads();
    if (!live) return;
    Acc z[2] = {0, 0};
    while (k0 < Np) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = k0 + q * kWave * V;
            if (k < Np) {
#pragma unroll
                for (int h = 0; h < 2; ++h) z[h] += dot_vec<DT, V>(rv[h][q], rl[h][q], L, k);
            }
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
    z[0] = wave_sum(z[0]);
    z[1] = wave_sum(z[1]);
    if (lane == 0) reinterpret_cast<Acc*>(jb.w)[r] = reinterpret_cast<const Acc*>(jb.lam)[r] * z[0] * z[1];
}

// The same for factors that keep the partial skew-symmetry (Sec. 3.3, eq.
// skew_abc_struct): column pair p = (c0, c1) has Bf[:,c1] = Bf[:,c0], Cf[:,c0] = Af[:,c1]
// and Cf[:,c1] = -Af[:,c0], so with beta = Bf[:,c0]^T u, alpha = Af[:,c0]^T u and
// gamma = Af[:,c1]^T u the pair's products are w[c0] = lam beta gamma and
// w[c1] = lam beta (-alpha).  The operator holds the P distinct columns of Bf and the R
// columns of Af as rows, [P + R][Np]: 1.5 R rows where the general form reads 2 R.  One
// wavefront per pair (three rows); pair slots past P write the zero padding of w.  Each
// dot product is computed as in cp_proj1_body.  In FP64 and FP32 the fused multiply-adds
// round symmetrically, so -alpha is the negated dot product; the packed BF16 dot
// instruction does not always give dot(-a, u) = -dot(a, u) to the bit, so the BF16
// formats form -alpha as Af[:,c0]^T (-u) against a second LDS image of -u, which
// presents it the same signed products as (-a) u.  So w is the general form's to the bit
// in every format.
template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj_skew_body(const Proj1Job& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = jb.N, Np = jb.Np, P = jb.P, R = jb.R;
    constexpr bool NEGU = (DT == DT_BF16 || DT == DT_BF16X3);
    LdsU<DT> L, Ln;                                      // u and (BF16 formats) -u
    L.bind(smem, Np);
    Ln.bind(smem + (NEGU ? LdsU<DT>::bytes(Np) : 0), Np);
    const int lane = threadIdx.x % kWave;
    const int q = blk * 4 + threadIdx.x / kWave;
    const bool live = q < P;
    const int c0 = jb.layout == 1 ? 2 * q : q, c1 = jb.layout == 1 ? 2 * q + 1 : P + q;
    const size_t rows[3] = {(size_t)(live ? q : 0), (size_t)(live ? P + c0 : 0), (size_t)(live ? P + c1 : 0)};
    const T* op = reinterpret_cast<const T*>(jb.BCt);
    Raw rv[3][U], rl[3][U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int h = 0; h < 3; ++h)
#pragma unroll
            for (int qq = 0; qq < U; ++qq) {
                const int k = kb + qq * kWave * V;
                if (live && k < Np) {
                    rv[h][qq] = ld_plain<BYTES>(op + rows[h] * Np + k);
                    if constexpr (X3) rl[h][qq] = ld_plain<BYTES>(jb.BCt_lo + rows[h] * Np + k);
                }
            }
    };
    issue(k0);
    const double* ub = jb.u_base + (jb.stepp ? (size_t)slot_of(*jb.stepp) * jb.slot_stride : 0);
    L.fill(ub, N, Np);
    if constexpr (NEGU) Ln.fill(ub, N, Np, -1.0);
    __syncthreads();
    Acc* w = reinterpret_cast<Acc*>(jb.w);
    if (!live) {
        const int e = R + 2 * (q - P);                  // zero padding of w past R
        if (lane == 0 && e < jb.Rp) {
            w[e] = 0;
            if (e + 1 < jb.Rp) w[e + 1] = 0;
        }
        return;
    }
    Acc z[3] = {0, 0, 0};                                // beta, -alpha, gamma
    while (k0 < Np) {
#pragma unroll
        for (int qq = 0; qq < U; ++qq) {
            const int k = k0 + qq * kWave * V;
            if (k < Np) {
                z[0] += dot_vec<DT, V>(rv[0][qq], rl[0][qq], L, k);
                z[1] += dot_vec<DT, V>(rv[1][qq], rl[1][qq], NEGU ? Ln : L, k);
                z[2] += dot_vec<DT, V>(rv[2][qq], rl[2][qq], L, k);
            }
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
#pragma unroll
    for (int h = 0; h < 3; ++h) z[h] = wave_sum(z[h]);
    if (lane == 0) {
        const Acc* lam = reinterpret_cast<const Acc*>(jb.lam);
        w[c0] = lam[c0] * z[0] * z[2];
        w[c1] = lam[c1] * z[0] * (NEGU ? z[1] : -z[1]);
    }
}

template <int DT, int V, int U>
__device__ __forceinline__ void cp_proj_any_body(const Proj1Job& jb, int blk) {
    if (jb.layout) cp_proj_skew_body<DT, V, U>(jb, blk);
    else cp_proj1_body<DT, V, U>(jb, blk);
}

// Scatter: W = lam .* s .* t staged in LDS, then y_i = sum_r Af[i][r] W_r, one
// wavefront per row (row loads issued before W is staged).  MODE 0 writes y (FP64,
// to y_out); MODE 1 applies the diagonal-stiffness BDF update with its energy
// partials; MODE 2 writes the right-hand side for the dense Helmholtz solve.  n is the
// state's level (MODE 1 and 2).  FULL (MODE 1 and 2, full form): the block also stages
// the level's [uhat; h] behind W and each wavefront forms its row's term G_i . x (the
// terms kernel's pieces, in its order) for the right-hand side, so a full-form step
// needs no kernel of its own for the terms.
template <int DT, int V, int U, int MODE, bool FULL = false>
__device__ __forceinline__ void cp_scatter1_body(const Scat1Job& jb, double* __restrict__ y_out, int blk,
                                                 long long n) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Acc* W = reinterpret_cast<Acc*>(smem);
    __shared__ double red[4];
    const int N = jb.N, R = jb.Rp;
    const StepArgs& a = jb.a;
    const Acc* __restrict__ win = reinterpret_cast<const Acc*>(jb.w);
    const int lane = threadIdx.x % kWave;
    const int i = blk * 4 + threadIdx.x / kWave;
    const bool live = i < N;
    const T* row = reinterpret_cast<const T*>(jb.Af) + (size_t)(live ? i : 0) * R;
    const unsigned short* rowlo = X3 ? jb.Af_lo + (size_t)(live ? i : 0) * R : nullptr;
    Raw rv[U], rl[U];
    int r0 = lane * V;
    auto issue = [&](int rb) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int r = rb + q * kWave * V;
            if (live && r < R) {
                rv[q] = ld_plain<BYTES>(row + r);
                if constexpr (X3) rl[q] = ld_plain<BYTES>(rowlo + r);
            }
        }
    };
    issue(r0);
    // full form: the first chunk of the row of G, behind the row loads
    const double2* g2 = nullptr;
    double2 gv[FULL ? kFullChunk : 1];
    FullHist fh;
    const bool full_regs = FULL && a.Np <= kFullRegJ * 256;      // block of 256 threads
    if constexpr (FULL) {
        g2 = reinterpret_cast<const double2*>(jb.G + (size_t)(live ? i : 0) * 2 * a.Np);
        full_issue(g2, live, lane, a.Np, gv);
        if (full_regs) full_load_hist(a, n, fh);
    }
    // the update's history (and diagonal inverse) behind the row loads
    BdfHist hist{};
    double hd = 0.0;
    int k = 0;
    if constexpr (MODE != 0) {
        k = bdf_order(n);
        if (live && lane == 0) {
            hist = bdf_hist_point(a, n, k, 0, i);
            if constexpr (MODE == 1) hd = a.hdiag[(size_t)(k - 1) * N + i];
        }
    }
    staged_copy<8, Acc>(R, [&](int r) { return win[r]; }, [&](int r, Acc v) { W[r] = v; });
    double* xs = reinterpret_cast<double*>(smem + ((sizeof(Acc) * (size_t)R + 15) & ~(size_t)15));
    if constexpr (FULL) {
        if (full_regs) full_store_x(a, n, fh, xs);
        else full_stage_x(a, n, 0, xs);
    }
    __syncthreads();
    Acc z = 0;
    if (live) {
        while (r0 < R) {
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int r = r0 + q * kWave * V;
                if (r < R) {
                    Acc cv[V];
                    Decode<DT, V>::run(rv[q], cv);
                    if constexpr (X3) {
                        float cl[V];
                        Decode<DT, V>::run(rl[q], cl);
#pragma unroll
                        for (int v = 0; v < V; ++v) z += (cv[v] + cl[v]) * W[r + v];
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) z += cv[v] * W[r + v];
                    }
                }
            }
            r0 += kWave * V * U;
            if (r0 < R) issue(r0);
        }
        z = wave_sum(z);
    }
    double zf = 0.0;
    if constexpr (FULL) {
        if (live) zf = wave_sum(full_dot(g2, lane, a.Np, gv, reinterpret_cast<const double2*>(xs)));
    }
    if constexpr (MODE == 0) {
        if (live && lane == 0) y_out[i] = (double)z;
    } else {
        const BdfCoef c = bdf_coef(k);
        double e = 0.0;
        if (live && lane == 0) {
            const double rhs = bdf_rhs_hist<FULL>(a, n, c, k, 0, i, (double)z, hist, zf);
            if constexpr (MODE == 1) {
                const double un = rhs * hd;
                write_level(a, n + 1, 0, i, un);
                e = un * un;
            } else {
                a.rhs[i] = rhs;
            }
        }
        if constexpr (MODE == 1) {
            const double s = block_sum(e, red);
            if (threadIdx.x == 0) epart_of(a, n + 1)[blk] = s;
        }
    }
}

// With a dense stiffness the step ends by applying Hinv_k to the right-hand side.  For
// a CP state the same kernel also forms the projections of the new level,
// s = Bf^T u^{n+1} and t = Cf^T u^{n+1}, and w = lam .* s .* t, from that right-hand side
// with the operator [Bf|Cf]^T Hinv_k built at context creation (the two products
// associate: Bf^T (Hinv_k rhs) = (Bf^T Hinv_k) rhs, with the same 2 N R flops as the
// projection of u^{n+1}).  The next step's scatter then starts at once, and a step is
// two kernels.  Blocks [0, nh) are Helmholtz row blocks, blocks [nh, nh + np)
// projection blocks (four row pairs each).
template <int DT, bool EVEN>
__device__ __forceinline__ void helm_proj_body(const HelmJob& jb, long long n, int blk) {
    if (blk < jb.nh) {
        helm_gemv_body<EVEN>(jb.a, n, blk);
        return;
    }
    typedef typename Store<DT>::T T;
    constexpr int V = 16 / (int)sizeof(T);
    const size_t rows = jb.layout ? (size_t)(jb.P + jb.R) : (size_t)2 * jb.Rp;
    const size_t mstride = (size_t)(bdf_order(n) - 1) * rows * jb.a.Np;
    Proj1Job pj{};
    pj.BCt = reinterpret_cast<const T*>(jb.Mst) + mstride;
    pj.BCt_lo = jb.Mst_lo ? jb.Mst_lo + mstride : nullptr;
    pj.lam = jb.lam;
    pj.N = jb.a.N;
    pj.Np = jb.a.Np;
    pj.Rp = jb.Rp;
    pj.layout = jb.layout;
    pj.P = jb.P;
    pj.R = jb.R;
    pj.u_base = jb.a.rhs;
    pj.w = jb.a.st;
    cp_proj_any_body<DT, V, 4>(pj, blk - jb.nh);
}


// ============================================================== SVD-ROM, one trajectory

// First product of the SVD-ROM (Sec. 4.4): w_r = sigma_r sum_j U[j][r] u_j over the rows
// of Ut [Rsp][Np] (rows past the rank are zero, so w is zero there).  One wavefront per
// row, four per block; the second product is the streaming kernel with R weighted slabs.

template <int DT, int V, int U>
__device__ __forceinline__ void svd_proj_body(const SvdProj& a, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int BYTES = V * (int)sizeof(T);
    constexpr bool X3 = (DT == DT_BF16X3);
    typedef typename RawT<BYTES>::T Raw;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int N = a.N, Np = a.Np;
    LdsU<DT> L;
    L.bind(smem, Np);
    const int lane = threadIdx.x % kWave;
    const int r = blk * 4 + (int)threadIdx.x / kWave;
    const bool live = r < a.Rsp;
    const T* row = reinterpret_cast<const T*>(a.Ut) + (size_t)(live ? r : 0) * Np;
    const unsigned short* rowlo = X3 ? a.Ut_lo + (size_t)(live ? r : 0) * Np : nullptr;
    Raw rv[U], rl[U];
    int k0 = lane * V;
    auto issue = [&](int kb) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = kb + q * kWave * V;
            if (live && k < Np) {
                rv[q] = ld_plain<BYTES>(row + k);
                if constexpr (X3) rl[q] = ld_plain<BYTES>(rowlo + k);
            }
        }
    };
    issue(k0);
    L.fill(a.u_base + (a.stepp ? (size_t)slot_of(*a.stepp) * a.slot_stride : 0), N, Np);
    __syncthreads();
    if (!live) return;
    Acc z = 0;
    while (k0 < Np) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int k = k0 + q * kWave * V;
            if (k < Np) z += dot_vec<DT, V>(rv[q], rl[q], L, k);
        }
        k0 += kWave * V * U;
        if (k0 < Np) issue(k0);
    }
    z = wave_sum(z);
    if (lane == 0) reinterpret_cast<Acc*>(a.w)[r] = reinterpret_cast<const Acc*>(a.sigma)[r] * z;
}


// ============================================================== BDF update from partials

// y^n from contraction partials part[c][b][i] (summed over c in order), then either
// the diagonal-stiffness update u^{n+1} = rhs / H_ii with its energy partials, or the
// right-hand side for the dense solve.  Block (bx, b) covers rows 256 bx .. 256 bx + 255
// of trajectory b (nbx blocks per trajectory).
template <class ACC, bool DIAG>
__device__ __forceinline__ void bdf_partials_body(const StepArgs& a, long long n, const ACC* __restrict__ part,
                                                  int nchunk, int pbstride, int bx, int b, int nbx) {
    __shared__ double red[4];
    const int k = bdf_order(n);
    const BdfCoef c = bdf_coef(k);
    const int i = bx * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < a.N) {
        // partial sums added in chunk order; loads issued 8 at a time
        double y = 0.0;
        const size_t cs = (size_t)pbstride * a.N;
        const ACC* pp = part + (size_t)b * a.N + i;
        int q = 0;
        for (; q + 8 <= nchunk; q += 8) {
            ACC v[8];
#pragma unroll
            for (int e2 = 0; e2 < 8; ++e2) v[e2] = pp[(size_t)(q + e2) * cs];
#pragma unroll
            for (int e2 = 0; e2 < 8; ++e2) y += (double)v[e2];
        }
        for (; q < nchunk; ++q) y += (double)pp[(size_t)q * cs];
        const double rhs = bdf_rhs_point(a, n, c, k, b, i, y);
        if (DIAG) {
            const double un = rhs * a.hdiag[(size_t)(k - 1) * a.N + i];
            write_level(a, n + 1, b, i, un);
            e = un * un;
        } else {
            a.rhs[(size_t)b * a.Np + i] = rhs;
        }
    }
    if (DIAG) {
        const double s = block_sum(e, red);
        if (threadIdx.x == 0) epart_of(a, n + 1)[(size_t)b * a.enmax + bx] = s;
    }
}


}  // namespace rom
