// rom_api.hip -- the C ABI of librom.so (include/rom.h): contexts (device operators,
// Helmholtz inverses, workspaces), states (trajectory histories, energy log), and the
// step sequencer that issues each BDF3/EXT3 step as a short chain of kernels and
// replays chunks of steps as captured HIP graphs.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "rom.h"
#include "als.h"
#include "rom_dev.h"
#include "kstep.h"

using namespace rom;

// ============================================================== errors

static thread_local std::string g_err;

static rom_status fail(rom_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static rom_status fail(rom_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE,          \
                        "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                        \
    } while (0)

// propagate a rom_status
#define TRYS(x)                        \
    do {                               \
        const rom_status s_ = (x);     \
        if (s_ != ROM_OK) return s_;   \
    } while (0)

extern "C" const char* rom_last_error(void) { return g_err.c_str(); }

// ============================================================== objects

namespace {

// Steps are replayed from captured graphs: a call of n steps is (n - 1) / 64 launches of a
// 64-step graph and one graph of the remaining 1..64 steps that ends with the closing
// kernel, so a call of up to 64 steps is a single graph launch.
constexpr int kGraphChunk = 64;

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

}  // namespace

struct rom_ctx_s {
    int N = 0, Np = 0, R = 0, Rp = 0, dtype = 0, max_batch = 1;
    int device = 0;                             // the GPU current at creation
    double nu = 0, dt = 0;
    bool dense = true, diagA = true;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // operators in the contraction format
    // (contracted indices padded with zeros: Np, Rp = N, R rounded up to multiples of 8)
    void *C = nullptr, *Clo = nullptr;         // dense [N][N][Np]
    void *Ct = nullptr, *Ct_lo = nullptr;      // dense, max_batch > 1: tiled copy for k_kr
    void *BCt = nullptr, *BCt_lo = nullptr;    // CP [2Rp][Np]: rows Bf^T then Cf^T
    void *Af = nullptr, *Af_lo = nullptr;      // CP [N][Rp]
    void* lam = nullptr;                        // CP [Rp] (FP64 or FP32)
    // CP with a dense stiffness: [Bf|Cf]^T Hinv_k for k = 1, 2, 3, [3][2Rp][Np]
    void *Mst = nullptr, *Mst_lo = nullptr;
    // CP factors with skew column pairs (skew_layout 1 or 2): the pair form of the
    // projection operator, [P + R][Np] (the P distinct columns of Bf, then the R columns of
    // Af, as rows), and with a dense stiffness its product with Hinv_k, [3][P + R][Np]
    int skew_layout = 0;
    void *SK = nullptr, *SK_lo = nullptr;
    void *Msk = nullptr, *Msk_lo = nullptr;
    // SVD form (svd): Ut [Rsp][Np] (columns of U as rows), sigma [Rsp] (accumulation
    // type), Vt [N][Rs][Np] (V[i][k][r] as slab r of row i)
    bool svd = false;
    int Rs = 0, Rsp = 0;
    void *Ut = nullptr, *Ut_lo = nullptr, *sig = nullptr, *Vt = nullptr, *Vt_lo = nullptr;
    double* hdiag = nullptr;                    // [3][N]
    double* hinv = nullptr;                     // [3][N][N]
    // full form of eq. nse_d1 (mass matrix, zeroth-mode terms): G = [L | M - I]
    // [N][2Np], fz = constant of the bracket, az = nu a0 (FP64)
    bool full = false;
    double *Gfull = nullptr, *fz = nullptr, *az = nullptr;
    // workspaces (shared by every state of the context; one stream serializes use)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int ws_gen = 0;
    // tiles (-1 = heuristic)
    // tile[4]: CP pair-form kernels (-1 default = on for one trajectory when the factors
    // have skew pairs, 0 off, 1 on for batches too); tile[5]: resident one-trajectory CP
    // steps (-1 default = on where the operator fits on chip, 0 off)
    int tile[6] = {-1, -1, -1, -1, -1, -1};
    // resident one-trajectory CP steps: geometry, valid while res_gen == ws_gen
    // (res_ok 0: not available for this context; res_refused: the runtime refused a run's
    // launch)
    int res_gen = -1, res_ok = 0, res_G = 0, res_nrg = 0, res_npg = 0, res_rg = 0, res_pg = 0;
    bool res_refused = false;
    size_t res_lds = 0;
    size_t lds_max = 65536;                     // dynamic LDS a batched kernel may take
    size_t bytes = 0;
    std::vector<void*> allocs;
};

struct rom_state_s {
    rom_ctx ctx = nullptr;
    int B = 0, Bpad = 0;
    StepArgs a{};
    long long h_step = 0;
    long long elog_base = 0;
    // single-trajectory states own their contraction scratch (partial sums or CP
    // projections), so several states of one context can be stepped in one grouped launch
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    double* xfull = nullptr;            // full form, batches: [Bpad][2Np] operand of X G^T
    double* slot_stage = nullptr;       // rom_state_set_slot: [5][N] staging of one history
    int sgen = 0;                       // bumped when scratch or the energy log moves
    long long* cnt = nullptr;           // the two slots of the device step counter
    // captured chunks of len = 1..64 steps, per parity of the first level (the kernels of
    // a step take the counter slots of its level's parity), without [0] and with [1] the
    // closing kernel at the end; valid while the workspace and scratch generations hold
    hipGraphExec_t graph[2][2][kGraphChunk + 1] = {};
    int graph_gen = -1, graph_sgen = -1;
    // resident one-trajectory CP steps: message words of x and w, the energy partials of a
    // run, the tag base (one allocation, res_buf)
    void* res_buf = nullptr;
    unsigned long long *res_x = nullptr, *res_w = nullptr;
    double* res_ep = nullptr;
    unsigned* res_seq = nullptr;
    bool pending = false;
    size_t bytes = 0;
    std::vector<void*> allocs;
};

static rom_status dmalloc(void** p, size_t bytes, size_t* acct, std::vector<void*>* list) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE,
                    "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    *acct += bytes;
    list->push_back(*p);
    return ROM_OK;
}

static size_t elem_bytes(int dt) { return dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2; }
static int acc_f64(int dt) { return dt == DT_F64 ? 1 : 0; }
static size_t acc_bytes(int dt) { return dt == DT_F64 ? 8 : 4; }

// ============================================================== workspace sizing

static SkewPairs skew_of(rom_ctx c);   // the skew column pairs in use (defined below)

namespace {

GemvTile gemv_tile(rom_ctx c) { return dense_gemv_variant(c->tile[0] < 0 ? 0 : c->tile[0]); }
// kinds 2 (CP projections) and 3 (CP scatter): k_gemm variants first, then the LDS-tile
// kernel's
SkinnyPlan skinny_plan(rom_ctx c, int kind, int Bpad) {
    SkinnyPlan sp{};
    const int v = c->tile[kind];
    const int M = kind == 2 ? 2 * c->Rp : c->N;
    if (v >= gemm_variants()) {
        sp.engine = 1;
        const MfmaTile t = mfma_variant(v - gemm_variants());
        sp.m = kind == 2 ? mfma_proj_plan(c->dtype, c->Np, c->Rp, Bpad, t) : mfma_scatter_plan(c->dtype, c->N, c->Rp, Bpad, t);
        sp.nsplit = sp.m.nsplit;
    } else {
        sp.engine = 0;
        sp.g = gemm_plan(M, Bpad, v);
        sp.nsplit = 1;
    }
    return sp;
}

void launch_proj(rom_ctx c, const SkinnyPlan& sp, int Bpad, const void* X, const void* Xlo, void* P, hipStream_t s) {
    if (sp.engine == 1) launch_mfma_proj(c->dtype, sp.m, c->BCt, c->BCt_lo, c->Np, c->Rp, Bpad, X, Xlo, P, s);
    else launch_gemm_proj(c->dtype, sp.g, c->BCt, c->BCt_lo, c->Np, c->Rp, Bpad, X, Xlo, P, s);
}

void launch_scatter(rom_ctx c, const SkinnyPlan& sp, int Bpad, const void* W, void* Y, hipStream_t s) {
    if (sp.engine == 1) launch_mfma_scatter(c->dtype, sp.m, c->Af, c->Af_lo, c->N, c->Rp, Bpad, W, Y, s);
    else launch_gemm_scatter(c->dtype, sp.g, c->Af, c->Af_lo, c->N, c->Rp, Bpad, W, Y, s);
}

// Batched CP term Y = Af (lam . Bf^T U . Cf^T U) (eq. tc_ap).  On the skinny GEMM the
// projection blocks pair the rows of Bf^T and Cf^T and write W themselves; the LDS-tile
// engine leaves partial projections that a separate pass turns into W.  With step
// arguments and the skinny GEMM for the scatter, the scatter also forms the step's
// right-hand side (and with a diagonal stiffness the update and step close); the
// return value says so.  Otherwise Y holds the scatter's partial sums.
bool launch_cp_batched(rom_ctx c, const SkinnyPlan& pp, const SkinnyPlan& ps, int Bpad, int B, const void* X,
                       const void* Xlo, void* P, void* W, void* Y, const StepArgs* sa, hipStream_t s) {
    // The pair-form GEMM covers half as many output tiles as the general form, each with
    // 1.5x the rows: at B <= 64 and R = 2000 it fills fewer CUs and runs 6-10% slower, so
    // batches take it only when knob 4 asks for it explicitly (value 1).
    const SkewPairs sk = c->tile[4] == 1 ? skew_of(c) : SkewPairs{};
    if (pp.engine == 0 && sk.layout) {
        launch_gemm_proj_skew(c->dtype, pp.g, c->SK, c->SK_lo, c->Np, sk.P, sk.layout, c->Rp, Bpad, X, Xlo, c->lam, W, s);
    } else if (pp.engine == 0) {
        launch_gemm_proj_pair(c->dtype, pp.g, c->BCt, c->BCt_lo, c->Np, c->Rp, Bpad, X, Xlo, c->lam, W, s);
    } else {
        launch_proj(c, pp, Bpad, X, Xlo, P, s);
        launch_hadamard(c->dtype, P, pp.nsplit, Bpad, B, c->Rp, c->lam, W, s);
    }
    if (sa && ps.engine == 0) {
        launch_gemm_scatter_step(c->dtype, ps.g, c->Af, c->Af_lo, c->N, c->Rp, Bpad, W, *sa, c->diagA ? 1 : 0, s);
        return true;
    }
    launch_scatter(c, ps, Bpad, W, Y, s);
    return false;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Zero `bytes` (a multiple of 16) of device memory with a kernel (unlike a memset node,
// safe inside a caller's graph capture).
__global__ void k_zero16(u32x4* p, size_t n) {
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        p[q] = z;
}
void launch_zero_fill(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4*)p, n);
}

// Contraction workspace of a batch of B (shared by the states of a context and by
// rom_nonlinear): layout and launch plans.
struct WsPlan {
    int B = 1, Bpad = 16;
    int nchunk = 0;                 // B = 1 dense: partial chunks per row
    DensePlan pd{};                 // B > 1: dense contraction
    SkinnyPlan pp{}, ps{};          // B > 1: CP projection, CP scatter
    size_t part_off = 0;            // dense / scatter partials, or CP s,t (B = 1)
    size_t part2_off = 0;           // CP projection partials (B > 1)
    size_t w_off = 0;               // CP Hadamard products W [Bpad][Rp] (B > 1)
    size_t ucv_off = 0, ucvlo_off = 0, usc_off = 0;   // rom_nonlinear operand copies (B > 1)
    size_t svdw_off = 0;            // SVD form (B = 1): slab weights w [Rsp]
    GemmPlan ph{};                  // B > 1, dense stiffness: FP64 Helmholtz apply
    size_t total = 0;
};

WsPlan plan_ws(rom_ctx c, int B) {
    WsPlan p;
    p.B = B;
    p.Bpad = (B + 15) / 16 * 16;
    const size_t ab = acc_bytes(c->dtype);
    size_t off = 0;
    if (B == 1) {
        if (c->dense || c->svd) {
            p.nchunk = dense_gemv_nchunk(c->N, gemv_tile(c));
            p.part_off = off;
            off = align256(off + (size_t)p.nchunk * c->N * ab);
            if (c->svd) {
                p.svdw_off = off;
                off = align256(off + (size_t)c->Rsp * ab);
            }
        } else {
            p.part_off = off;
            off = align256(off + 2 * (size_t)c->Rp * ab);
        }
    } else {
        const size_t eb = elem_bytes(c->dtype);
        if (c->dense) {
            p.pd = dense_batched_plan(c->dtype, c->N, c->Np, p.Bpad, c->tile[1], c->lds_max);
            p.part_off = off;
            off = align256(off + (size_t)p.pd.nsplit * p.Bpad * c->N * ab);
        } else {
            p.pp = skinny_plan(c, 2, p.Bpad);
            p.ps = skinny_plan(c, 3, p.Bpad);
            p.part2_off = off;
            off = align256(off + (size_t)p.pp.nsplit * p.Bpad * 2 * c->Rp * ab);
            p.w_off = off;
            off = align256(off + (size_t)p.Bpad * c->Rp * ab);
            p.part_off = off;
            off = align256(off + (size_t)p.ps.nsplit * p.Bpad * c->N * ab);
        }
        p.ucv_off = off;
        off = align256(off + (size_t)p.Bpad * c->Np * eb);
        p.ucvlo_off = off;
        off = align256(off + (c->dtype == DT_BF16X3 ? (size_t)p.Bpad * c->Np * 2 : 0));
        p.usc_off = off;
        off = align256(off + (size_t)p.Bpad * c->Np * ab);
        if (!c->diagA) p.ph = gemm_plan(c->N, p.Bpad, 0);
    }
    p.total = off + 256;
    return p;
}

rom_status ensure_ws(rom_ctx c, size_t bytes) {
    if (bytes <= c->ws_bytes) return ROM_OK;
    if (c->ws) {
        hipStreamSynchronize(c->stream);
        hipFree(c->ws);
        c->bytes -= c->ws_bytes;
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&c->ws, bytes);
    if (e != hipSuccess) {
        c->ws = nullptr;
        return fail(ROM_E_NOMEM, "workspace hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    hipMemsetAsync(c->ws, 0, bytes, c->stream);
    c->ws_bytes = bytes;
    c->bytes += bytes;
    c->ws_gen++;
    return ROM_OK;
}

}  // namespace

// ============================================================== create / destroy

// Upload `rows` rows of `cols` FP64 values and convert them into rows of pitch `dpitch`
// elements of the context's format (the destination padding was zeroed beforehand).
static rom_status upload_convert(rom_ctx c, const double* host, size_t rows, int cols, int dpitch, void* dst,
                                 void* dst_lo, double* stage, size_t stage_elems) {
    const size_t eb = elem_bytes(c->dtype);
    size_t rows_per = stage_elems / cols;
    if (rows_per < 1) rows_per = 1;
    for (size_t r0 = 0; r0 < rows; r0 += rows_per) {
        const size_t nr = (rows - r0 < rows_per) ? rows - r0 : rows_per;
        HIPCHK(hipMemcpyAsync(stage, host + r0 * cols, nr * cols * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
        launch_cvt_f64_to(c->dtype, stage, (char*)dst + r0 * dpitch * eb,
                          dst_lo ? (char*)dst_lo + r0 * dpitch * 2 : nullptr, (long long)nr, cols, dpitch,
                          c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return ROM_OK;
}

// Every operator allocation ends in kSlack zero bytes: the batched kernels' lane vectors
// may run up to one k-step past the last row (they meet zero weights).
static constexpr size_t kSlack = 256;

// Column pairs of CP factors that keep the partial skew-symmetry (Sec. 3.3, eq.
// skew_abc_struct): pair p = (c0, c1) with lam[c0] == lam[c1], Bf[:,c0] == Bf[:,c1],
// Cf[:,c0] == Af[:,c1] and Cf[:,c1] == -Af[:,c0], exactly.  1: c0 = 2p, c1 = 2p + 1
// (interleaved pairs); 2: c0 = p, c1 = R/2 + p (the paper's blocks); 0: neither.
static int skew_layout_of(int N, int R, const double* lam, const double* Af, const double* Bf, const double* Cf) {
    if (N < 1 || R < 2 || R % 2 != 0 || !lam || !Af || !Bf || !Cf) return 0;
    const int P = R / 2;
    for (int layout = 1; layout <= 2; ++layout) {
        bool ok = true;
        for (int p = 0; p < P && ok; ++p) {
            const int c0 = layout == 1 ? 2 * p : p, c1 = layout == 1 ? 2 * p + 1 : P + p;
            ok = lam[c0] == lam[c1];
            for (int n = 0; n < N && ok; ++n) {
                const size_t o = (size_t)n * R;
                ok = Bf[o + c0] == Bf[o + c1] && Cf[o + c0] == Af[o + c1] && Cf[o + c1] == -Af[o + c0];
            }
        }
        if (ok) return layout;
    }
    return 0;
}

// dst[k] = rows x Hinv_{k+1} for k = 0, 1, 2 ([3][rows][Np] in the contraction format):
// FP64 rows of length Np (zero padded) times the symmetric Hinv_k on the matrix cores,
// then one conversion.  Allocates dst (and dst_lo for BF16X3) in the context.
static rom_status hinv_products(rom_ctx c, const double* host_rows, size_t rows, void** dst, void** dst_lo) {
    const size_t N = c->N, Np = c->Np, eb = elem_bytes(c->dtype);
    const size_t rows16 = (rows + 15) / 16 * 16;        // the product's column tiles
    rom_status st = dmalloc(dst, 3 * rows * Np * eb + kSlack, &c->bytes, &c->allocs);
    if (st != ROM_OK) return st;
    HIPCHK(hipMemsetAsync(*dst, 0, 3 * rows * Np * eb + kSlack, c->stream));
    if (dst_lo) {
        st = dmalloc(dst_lo, 3 * rows * Np * 2 + kSlack, &c->bytes, &c->allocs);
        if (st != ROM_OK) return st;
        HIPCHK(hipMemsetAsync(*dst_lo, 0, 3 * rows * Np * 2 + kSlack, c->stream));
    }
    double *x_d = nullptr, *y_d = nullptr;
    hipError_t e = hipMalloc((void**)&x_d, sizeof(double) * rows16 * Np);
    if (e == hipSuccess) e = hipMalloc((void**)&y_d, sizeof(double) * rows16 * N);
    if (e == hipSuccess) e = hipMemsetAsync(x_d, 0, sizeof(double) * rows16 * Np, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(x_d, host_rows, sizeof(double) * rows * Np, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        const GemmPlan pl = gemm_plan((int)N, (int)rows16, 0);
        for (int k = 0; k < 3; ++k) {
            launch_gemm_f64(pl, c->hinv + (size_t)k * N * Np, (long long)Np, x_d, (long long)Np, y_d, (int)N,
                            (int)Np, (int)rows16, c->stream);
            launch_cvt_f64_to(c->dtype, y_d, (char*)*dst + (size_t)k * rows * Np * eb,
                              dst_lo ? (char*)*dst_lo + (size_t)k * rows * Np * 2 : nullptr, (long long)rows, (int)N,
                              (int)Np, c->stream);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (x_d) hipFree(x_d);
    if (y_d) hipFree(y_d);
    if (e != hipSuccess) return fail(ROM_E_DEVICE, "setup of the projection operators failed: %s", hipGetErrorString(e));
    return ROM_OK;
}

extern "C" int32_t rom_cp_skew_layout(int32_t N, int32_t R, const double* lambda, const double* Af, const double* Bf,
                                      const double* Cf) {
    return skew_layout_of(N, R, lambda, Af, Bf, Cf);
}

static void forget_plans_of(const void* obj);

// The order of resident runs across streams (one record per device).
constexpr int kResDevices = 16;
struct ResOrder {
    std::mutex mu;
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;     // stream of the latest run
};
static ResOrder& res_order(int device);
static void res_forget_stream(int device, hipStream_t s);

extern "C" void rom_destroy(rom_ctx c) {
    if (!c) return;
    forget_plans_of(c);
    res_forget_stream(c->device, c->stream);
    if (c->stream) hipStreamSynchronize(c->stream);
    for (void* p : c->allocs) hipFree(p);
    if (c->ws) hipFree(c->ws);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    delete c;
}

// The SVD form handed to rom_create_svd.
struct SvdDesc {
    int R;
    const double *U, *sigma, *V;
};

static rom_status create_ctx(const rom_desc* d, const SvdDesc* sv, const rom_full_terms* fd, rom_ctx* out) {
    if (!out) return fail(ROM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d) return fail(ROM_E_INVALID, "desc is NULL");
    if (d->N < 1) return fail(ROM_E_INVALID, "N must be >= 1 (got %d)", d->N);
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(ROM_E_INVALID, "dt must be > 0");
    if (!(d->nu >= 0.0) || !std::isfinite(d->nu)) return fail(ROM_E_INVALID, "nu must be >= 0");
    if (!d->A) return fail(ROM_E_INVALID, "stiffness A is NULL");
    if (d->dtype < ROM_FP64 || d->dtype > ROM_BF16X3) return fail(ROM_E_INVALID, "unknown dtype %d", d->dtype);
    if (d->max_batch < 1) return fail(ROM_E_INVALID, "max_batch must be >= 1");
    if (sv) {
        if (d->C || d->lambda || d->Af || d->Bf || d->Cf)
            return fail(ROM_E_INVALID, "the SVD form takes no dense tensor or CP factors");
        if (sv->R < 1) return fail(ROM_E_INVALID, "SVD rank must be >= 1");
        if (!sv->U || !sv->sigma || !sv->V) return fail(ROM_E_INVALID, "the SVD form needs U, sigma and V");
        if (d->N > 4096) return fail(ROM_E_UNSUPPORTED, "the SVD form is limited to N <= 4096");
        if (d->max_batch > 1) return fail(ROM_E_UNSUPPORTED, "the SVD form runs one trajectory per state");
    } else if (!d->C) {
        if (d->R < 1) return fail(ROM_E_INVALID, "CP rank R must be >= 1 when C is NULL");
        if (!d->lambda || !d->Af || !d->Bf || !d->Cf)
            return fail(ROM_E_INVALID, "CP mode needs lambda, Af, Bf and Cf");
    }
    const long long N = d->N;
    if (d->C && N > 4096) return fail(ROM_E_UNSUPPORTED, "dense tensors are limited to N <= 4096");
    if (fd && sv) return fail(ROM_E_UNSUPPORTED, "the full form takes the dense tensor or the CP factors");
    if (fd && (N + 7) / 8 * 8 > 4096)
        return fail(ROM_E_UNSUPPORTED, "the full form is limited to N <= 4096 (LDS staging of its GEMV)");
    if (fd && fd->M)
        for (long long i = 0; i < N; ++i)
            for (long long m = 0; m < i; ++m)
                if (fd->M[i * N + m] != fd->M[m * N + i])
                    return fail(ROM_E_INVALID, "mass matrix M is not symmetric (%lld, %lld)", i, m);
    if (N > 16384) return fail(ROM_E_UNSUPPORTED, "N > 16384 is not supported");
    // one-trajectory kernels stage u in LDS (64 KB per block): per padded mode 8 bytes
    // (FP64), 4 (FP32), 6 (BF16: words and weights) or 8 (BF16x3); the CP projections of
    // the BF16 formats hold a second image of -u, and the SVD slab stream adds R weights
    {
        const long long Npl = (N + 7) / 8 * 8;
        const long long per = d->dtype == ROM_FP64 ? 8 : d->dtype == ROM_FP32 ? 4 : d->dtype == ROM_BF16 ? 6 : 8;
        const long long acc = d->dtype == ROM_FP64 ? 8 : 4;
        long long need = per * Npl;
        if (!d->C && !sv && (d->dtype == ROM_BF16 || d->dtype == ROM_BF16X3)) need *= 2;
        if (sv) need += acc * (long long)sv->R;
        if (need > 65536)
            return fail(ROM_E_UNSUPPORTED, "N = %lld (with this format and rank) exceeds the 64 KB LDS staging of u",
                        N);
    }
    if (!d->C && !sv && (long long)d->R * (d->dtype == ROM_FP64 ? 8 : 4) > 65536)
        return fail(ROM_E_UNSUPPORTED, "CP rank %d exceeds the 64 KB LDS staging of the scatter kernel", d->R);
    // stiffness (and mass matrix): diagonal, or dense; a dense one is solved through an
    // explicit inverse whose setup and apply stage N doubles in LDS (and the CP projections
    // of a one-trajectory state stage the right-hand side), so N is limited
    bool diag = true;
    {
        const double* Mh = fd ? fd->M : nullptr;
        for (long long i = 0; i < N && diag; ++i)
            for (long long m = 0; m < N; ++m)
                if (i != m && (d->A[i * N + m] != 0.0 || (Mh && Mh[i * N + m] != 0.0))) {
                    diag = false;
                    break;
                }
    }
    if (!diag && N > 4096) return fail(ROM_E_UNSUPPORTED, "a non-diagonal stiffness is limited to N <= 4096");

    rom_ctx c = new rom_ctx_s();
    c->N = d->N;
    c->Np = (d->N + 7) / 8 * 8;
    c->R = (d->C || sv) ? 0 : d->R;
    c->Rp = (c->R + 7) / 8 * 8;
    c->dtype = d->dtype;
    c->nu = d->nu;
    c->dt = d->dt;
    c->max_batch = d->max_batch;
    c->dense = d->C != nullptr;
    c->svd = sv != nullptr;
    c->full = fd != nullptr;
    c->stream = (hipStream_t)d->stream;
    rom_status st = ROM_OK;
#define TRY(x)                          \
    do {                                \
        st = (x);                       \
        if (st != ROM_OK) {             \
            rom_destroy(c);             \
            return st;                  \
        }                               \
    } while (0)
#define HTRY(x)                                                                           \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            st = fail(e_ == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE, "%s: %s",  \
                      #x, hipGetErrorString(e_));                                         \
            rom_destroy(c);                                                               \
            return st;                                                                    \
        }                                                                                 \
    } while (0)

    // dynamic LDS the batched register kernel may request (the device limit, at most
    // 120 KB; 64 KB if raising the per-kernel limit is refused)
    {
        int dev = 0, lds = 0;
        HTRY(hipGetDevice(&dev));
        c->device = dev;
        HTRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        size_t want = lds > 122880 ? 122880 : (size_t)lds;
        if (want > 65536 && kr_set_lds_limit(want) != hipSuccess) {
            (void)hipGetLastError();
            want = 65536;
        }
        c->lds_max = want;
    }
    if (!c->stream) {
        HTRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }

    // ---- stiffness: Helmholtz data
    const double* Mh = fd ? fd->M : nullptr;   // mass matrix (NULL: the identity)
    c->diagA = diag;
    const size_t stage_elems = (size_t)1 << 25;   // 256 MB of FP64 per upload chunk
    double* stage = nullptr;
    const size_t nn = (size_t)N * N;
    HTRY(hipMalloc((void**)&stage, sizeof(double) * (nn > stage_elems ? nn : stage_elems)));
    struct StageGuard {
        double* p;
        ~StageGuard() { if (p) hipFree(p); }
    } guard{stage};
    HTRY(hipMemcpyAsync(stage, d->A, sizeof(double) * nn, hipMemcpyHostToDevice, c->stream));
    // full form: M, C1, C2, c0, a0 on the device for the Helmholtz matrices and G
    double* fdev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    struct FullGuard {
        double** p;
        ~FullGuard() {
            for (int q = 0; q < 5; ++q)
                if (p[q]) hipFree(p[q]);
        }
    } fguard{fdev};
    if (fd) {
        const double* src[5] = {fd->M, fd->C1, fd->C2, fd->c0, fd->a0};
        const size_t cnt[5] = {nn, (size_t)N * (N + 1), (size_t)N * (N + 1), (size_t)N, (size_t)N};
        for (int q = 0; q < 5; ++q) {
            if (!src[q]) continue;
            HTRY(hipMalloc((void**)&fdev[q], sizeof(double) * cnt[q]));
            HTRY(hipMemcpyAsync(fdev[q], src[q], sizeof(double) * cnt[q], hipMemcpyHostToDevice, c->stream));
        }
    }
    if (diag) {
        TRY(dmalloc((void**)&c->hdiag, sizeof(double) * 3 * N, &c->bytes, &c->allocs));
        helm_setup_diag((int)N, d->nu, d->dt, stage, fdev[0], c->hdiag, c->stream);
        HTRY(hipGetLastError());
        // SPD check of the three diagonal Helmholtz matrices
        for (long long i = 0; i < N; ++i) {
            const double h = (Mh ? Mh[i * N + i] : 1.0) / d->dt + d->nu * d->A[i * N + i];
            if (!(h > 0.0)) {
                st = fail(ROM_E_INVALID, "Helmholtz matrix not positive definite (row %lld)", i);
                rom_destroy(c);
                return st;
            }
        }
    } else {
        double* work = nullptr;
        int* info = nullptr;
        const size_t hbytes = sizeof(double) * 3 * (size_t)N * c->Np + 256;
        TRY(dmalloc((void**)&c->hinv, hbytes, &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->hinv, 0, hbytes, c->stream));
        HTRY(hipMalloc((void**)&work, sizeof(double) * 3 * nn));
        HTRY(hipMalloc((void**)&info, sizeof(int)));
        HTRY(hipMemsetAsync(info, 0, sizeof(int), c->stream));
        helm_setup_dense((int)N, c->Np, d->nu, d->dt, stage, fdev[0], c->hinv, work, info, c->stream);
        hipError_t le = hipGetLastError();
        int hinfo = 0;
        hipError_t se = hipStreamSynchronize(c->stream);
        if (le == hipSuccess && se == hipSuccess)
            se = hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost);
        hipFree(work);
        hipFree(info);
        if (le != hipSuccess || se != hipSuccess) {
            st = fail(ROM_E_DEVICE, "Helmholtz setup failed: %s", hipGetErrorString(le != hipSuccess ? le : se));
            rom_destroy(c);
            return st;
        }
        if (hinfo != 0) {
            st = fail(ROM_E_INVALID, "Helmholtz matrix (beta0/dt) M + nu A is not positive definite");
            rom_destroy(c);
            return st;
        }
    }
    if (fd) {
        TRY(dmalloc((void**)&c->Gfull, sizeof(double) * N * 2 * c->Np, &c->bytes, &c->allocs));
        TRY(dmalloc((void**)&c->fz, sizeof(double) * N, &c->bytes, &c->allocs));
        TRY(dmalloc((void**)&c->az, sizeof(double) * N, &c->bytes, &c->allocs));
        full_setup((int)N, c->Np, d->nu, fdev[0], fdev[1], fdev[2], fdev[3], fdev[4], c->Gfull, c->fz, c->az,
                   c->stream);
        HTRY(hipGetLastError());
    }
    HTRY(hipStreamSynchronize(c->stream));

    // ---- advection operator (zero-padded along the contracted index)
    const int dt = c->dtype;
    const size_t eb = elem_bytes(dt);
    const bool lo = dt == DT_BF16X3;
    const size_t Np = c->Np;
    if (sv) {
        // SVD form (Sec. 4.4): Ut rows are the columns of U, Vt[i][r][k] = V[i][k][r]
        const size_t Rs = (size_t)sv->R, Rsp = (Rs + 7) / 8 * 8;
        c->Rs = (int)Rs;
        c->Rsp = (int)Rsp;
        TRY(dmalloc(&c->Ut, Rsp * Np * eb + kSlack, &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->Ut, 0, Rsp * Np * eb + kSlack, c->stream));
        TRY(dmalloc(&c->Vt, (size_t)N * Rs * Np * eb + kSlack, &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->Vt, 0, (size_t)N * Rs * Np * eb + kSlack, c->stream));
        if (lo) {
            TRY(dmalloc(&c->Ut_lo, Rsp * Np * 2 + kSlack, &c->bytes, &c->allocs));
            HTRY(hipMemsetAsync(c->Ut_lo, 0, Rsp * Np * 2 + kSlack, c->stream));
            TRY(dmalloc(&c->Vt_lo, (size_t)N * Rs * Np * 2 + kSlack, &c->bytes, &c->allocs));
            HTRY(hipMemsetAsync(c->Vt_lo, 0, (size_t)N * Rs * Np * 2 + kSlack, c->stream));
        }
        TRY(dmalloc(&c->sig, Rsp * acc_bytes(dt), &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->sig, 0, Rsp * acc_bytes(dt), c->stream));
        std::vector<double> t(Rs * (size_t)N);
        for (size_t n = 0; n < (size_t)N; ++n)
            for (size_t r = 0; r < Rs; ++r) t[r * N + n] = sv->U[n * Rs + r];
        TRY(upload_convert(c, t.data(), Rs, (int)N, (int)Np, c->Ut, c->Ut_lo, stage, stage_elems));
        for (size_t i = 0; i < (size_t)N; ++i) {
            const double* Vi = sv->V + i * (size_t)N * Rs;           // [k][r] of row i
            for (size_t k = 0; k < (size_t)N; ++k)
                for (size_t r = 0; r < Rs; ++r) t[r * N + k] = Vi[k * Rs + r];
            TRY(upload_convert(c, t.data(), Rs, (int)N, (int)Np, (char*)c->Vt + i * Rs * Np * eb,
                               lo ? (char*)c->Vt_lo + i * Rs * Np * 2 : nullptr, stage, stage_elems));
        }
        HTRY(hipMemcpyAsync(stage, sv->sigma, sizeof(double) * Rs, hipMemcpyHostToDevice, c->stream));
        launch_cvt_lambda(dt, stage, c->sig, (long long)Rs, c->stream);
        HTRY(hipGetLastError());
    } else
    if (c->dense) {
        const size_t n3 = nn * Np;
        TRY(dmalloc(&c->C, n3 * eb + kSlack, &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->C, 0, n3 * eb + kSlack, c->stream));
        if (lo) {
            TRY(dmalloc(&c->Clo, n3 * 2 + kSlack, &c->bytes, &c->allocs));
            HTRY(hipMemsetAsync(c->Clo, 0, n3 * 2 + kSlack, c->stream));
        }
        TRY(upload_convert(c, d->C, nn, (int)N, (int)Np, c->C, c->Clo, stage, stage_elems));
        if (c->max_batch > 1) {
            // the batched kernel's tiled copy (a permutation of the converted words)
            const size_t tb = kr_tiled_bytes(dt, (int)N, (int)eb);
            TRY(dmalloc(&c->Ct, tb, &c->bytes, &c->allocs));
            launch_kr_tile(dt, (int)eb, c->C, c->Ct, (int)N, (int)Np, c->stream);
            if (lo) {
                TRY(dmalloc(&c->Ct_lo, kr_tiled_bytes(dt, (int)N, 2), &c->bytes, &c->allocs));
                launch_kr_tile(dt, 2, c->Clo, c->Ct_lo, (int)N, (int)Np, c->stream);
            }
            HTRY(hipGetLastError());
        }
    } else {
        const size_t R = c->R, Rp = c->Rp;
        TRY(dmalloc(&c->BCt, 2 * Rp * Np * eb + kSlack, &c->bytes, &c->allocs));
        TRY(dmalloc(&c->Af, N * Rp * eb + kSlack, &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->BCt, 0, 2 * Rp * Np * eb + kSlack, c->stream));
        HTRY(hipMemsetAsync(c->Af, 0, N * Rp * eb + kSlack, c->stream));
        if (lo) {
            TRY(dmalloc(&c->BCt_lo, 2 * Rp * Np * 2 + kSlack, &c->bytes, &c->allocs));
            TRY(dmalloc(&c->Af_lo, N * Rp * 2 + kSlack, &c->bytes, &c->allocs));
            HTRY(hipMemsetAsync(c->BCt_lo, 0, 2 * Rp * Np * 2 + kSlack, c->stream));
            HTRY(hipMemsetAsync(c->Af_lo, 0, N * Rp * 2 + kSlack, c->stream));
        }
        TRY(dmalloc(&c->lam, Rp * acc_bytes(dt), &c->bytes, &c->allocs));
        HTRY(hipMemsetAsync(c->lam, 0, Rp * acc_bytes(dt), c->stream));
        // Bf^T into rows [0, R) and Cf^T into rows [Rp, Rp + R) (host transposes of the
        // caller's [N][R] factors)
        std::vector<double> t(R * (size_t)N);
        for (size_t n = 0; n < (size_t)N; ++n)
            for (size_t r = 0; r < R; ++r) t[r * N + n] = d->Bf[n * R + r];
        TRY(upload_convert(c, t.data(), R, (int)N, (int)Np, c->BCt, c->BCt_lo, stage, stage_elems));
        for (size_t n = 0; n < (size_t)N; ++n)
            for (size_t r = 0; r < R; ++r) t[r * N + n] = d->Cf[n * R + r];
        TRY(upload_convert(c, t.data(), R, (int)N, (int)Np, (char*)c->BCt + Rp * Np * eb,
                           lo ? (char*)c->BCt_lo + Rp * Np * 2 : nullptr, stage, stage_elems));
        TRY(upload_convert(c, d->Af, N, (int)R, (int)Rp, c->Af, c->Af_lo, stage, stage_elems));
        HTRY(hipMemcpyAsync(stage, d->lambda, sizeof(double) * R, hipMemcpyHostToDevice, c->stream));
        launch_cvt_lambda(dt, stage, c->lam, (long long)R, c->stream);
        HTRY(hipGetLastError());
        if (!c->diagA) {
            // [Bf|Cf]^T Hinv_k for the one-trajectory step (the projections of u^{n+1}
            // straight from the right-hand side)
            const size_t rows2 = 2 * Rp;
            std::vector<double> bt(rows2 * Np, 0.0);
            for (size_t n = 0; n < (size_t)N; ++n)
                for (size_t r = 0; r < R; ++r) {
                    bt[r * Np + n] = d->Bf[n * R + r];
                    bt[(Rp + r) * Np + n] = d->Cf[n * R + r];
                }
            st = hinv_products(c, bt.data(), rows2, &c->Mst, lo ? &c->Mst_lo : nullptr);
            if (st != ROM_OK) {
                rom_destroy(c);
                return st;
            }
        }
        // Skew column pairs (Sec. 3.3, eq. skew_abc_struct): the pair form of the
        // projection operator, rows [Bf[:, c0(p)] for p < P; Af[:, r] for r < R]
        c->skew_layout = skew_layout_of((int)N, (int)R, d->lambda, d->Af, d->Bf, d->Cf);
        if (c->skew_layout) {
            const size_t P = R / 2, rows = P + R;
            std::vector<double> sk(rows * Np, 0.0);
            for (size_t p2 = 0; p2 < P; ++p2) {
                const size_t c0 = c->skew_layout == 1 ? 2 * p2 : p2;
                for (size_t n = 0; n < (size_t)N; ++n) sk[p2 * Np + n] = d->Bf[n * R + c0];
            }
            for (size_t r = 0; r < R; ++r)
                for (size_t n = 0; n < (size_t)N; ++n) sk[(P + r) * Np + n] = d->Af[n * R + r];
            TRY(dmalloc(&c->SK, rows * Np * eb + kSlack, &c->bytes, &c->allocs));
            HTRY(hipMemsetAsync(c->SK, 0, rows * Np * eb + kSlack, c->stream));
            if (lo) {
                TRY(dmalloc(&c->SK_lo, rows * Np * 2 + kSlack, &c->bytes, &c->allocs));
                HTRY(hipMemsetAsync(c->SK_lo, 0, rows * Np * 2 + kSlack, c->stream));
            }
            TRY(upload_convert(c, sk.data(), rows, (int)Np, (int)Np, c->SK, c->SK_lo, stage, stage_elems));
            if (!c->diagA) {
                st = hinv_products(c, sk.data(), rows, &c->Msk, lo ? &c->Msk_lo : nullptr);
                if (st != ROM_OK) {
                    rom_destroy(c);
                    return st;
                }
            }
        }
    }
    HTRY(hipStreamSynchronize(c->stream));
    *out = c;
#undef TRY
#undef HTRY
    return ROM_OK;
}

extern "C" rom_status rom_create(const rom_desc* d, rom_ctx* out) { return create_ctx(d, nullptr, nullptr, out); }
// The tensor-factor product of the ALS sweeps on its own FP64 MFMA kernel (k_als.hip)
// when 16 or 32 rows of the unfolding fit in 64 KB of LDS (N up to 496; the allowance is
// set here, before any capture), else on the skinny GEMM.  The transposed factor it reads
// gets kProductSlack zeroed elements past its end.
constexpr size_t kProductSlack = 16;
constexpr int kProductLds = 65536;

// Streams and graph of an ALS call: the capture stream cs (ordered after the caller's
// stream), a side stream for the SPD inverses, and one fork / join event pair per inverse
// of a sweep (kPairs - 1 for ALS-skew's subiterations, taken in turn, and the last for
// its tied system).  fork(q) makes the side stream wait for cs; join_mark(q) records the side
// stream's work; join(q) makes cs wait for it.  The side stream joins the capture through
// the fork and leaves it through the join, so the graph holds the inverse as a branch.
struct SweepStreams {
    static constexpr int kPairs = 9;
    hipStream_t cs = nullptr, side = nullptr;
    hipEvent_t start = nullptr, evf[kPairs] = {}, evj[kPairs] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool init(hipStream_t caller) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess)
            return false;
        for (int q = 0; q < kPairs; ++q)
            if (hipEventCreateWithFlags(&evf[q], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&evj[q], hipEventDisableTiming) != hipSuccess)
                return false;
        return hipEventRecord(start, caller) == hipSuccess && hipStreamWaitEvent(cs, start, 0) == hipSuccess;
    }
    bool fork(int q) {
        return q < kPairs && hipEventRecord(evf[q], cs) == hipSuccess && hipStreamWaitEvent(side, evf[q], 0) == hipSuccess;
    }
    bool join_mark(int q) { return q < kPairs && hipEventRecord(evj[q], side) == hipSuccess; }
    bool join(int q) { return q < kPairs && hipStreamWaitEvent(cs, evj[q], 0) == hipSuccess; }
    ~SweepStreams() {
        if (gexec) hipGraphExecDestroy(gexec);
        if (graph) hipGraphDestroy(graph);
        if (cs) {
            hipStreamSynchronize(cs);
            hipStreamDestroy(cs);
        }
        if (side) {
            hipStreamSynchronize(side);
            hipStreamDestroy(side);
        }
        if (start) hipEventDestroy(start);
        for (int q = 0; q < kPairs; ++q) {
            if (evf[q]) hipEventDestroy(evf[q]);
            if (evj[q]) hipEventDestroy(evj[q]);
        }
    }
};

extern "C" rom_status rom_cp_als(int32_t N, int32_t R, const double* C, double* A1, double* A2, double* A3,
                                  int32_t sweeps, void* stream) {
    if (N < 1 || N > 4096) return fail(ROM_E_INVALID, "N must be in [1, 4096] (got %d)", N);
    if (R < 1 || R > 4096) return fail(ROM_E_INVALID, "R must be in [1, 4096] (got %d)", R);
    if (sweeps < 0) return fail(ROM_E_INVALID, "sweeps must be >= 0");
    if (!C || !A1 || !A2 || !A3) return fail(ROM_E_INVALID, "a tensor or factor pointer is NULL");
    if (sweeps == 0) return ROM_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)N, r = (size_t)R, rp = (r + 7) / 8 * 8, npad = (n + 15) / 16 * 16;
    const size_t np = (n + 7) / 8 * 8, n2pad = (n * n + 15) / 16 * 16;
    // V and the two panel buffers of its inverse [R][R]; Vinv [R][Rp] and the right-hand
    // side Mb [Npad][Rp] with zero padding (the product's K = Rp; the product M V^-1 is
    // written straight into the factor's N rows); the two unfoldings of C [N^2 padded][Np],
    // a transposed factor [R][Np] and the tensor-factor product T [N^2 padded][R]
    constexpr int kBufs = 9;
    const size_t sizes[kBufs] = {r * r, r * r, r * r, r * rp, npad * rp, n2pad * np, n2pad * np,
                                 r * np + kProductSlack, n2pad * r};
    double* buf[kBufs] = {};
    int* info = nullptr;
    struct Guard {
        double** b;
        int** info;
        ~Guard() {
            for (int q = 0; q < kBufs; ++q)
                if (b[q]) hipFree(b[q]);
            if (*info) hipFree(*info);
        }
    } guard{buf, &info};
    for (int q = 0; q < kBufs; ++q) {
        const hipError_t e = hipMalloc((void**)&buf[q], sizeof(double) * sizes[q]);
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE, "CP-ALS workspace: %s",
                                         hipGetErrorString(e));
    }
    if (hipMalloc((void**)&info, sizeof(int)) != hipSuccess) return fail(ROM_E_NOMEM, "CP-ALS workspace");
    double *V = buf[0], *L = buf[1], *X = buf[2], *Vinv = buf[3], *Mb = buf[4];
    double *U0 = buf[5], *U1 = buf[6], *Ft = buf[7], *T = buf[8];
    if (hipMemsetAsync(Vinv, 0, sizeof(double) * sizes[3], s) != hipSuccess ||
        hipMemsetAsync(Mb, 0, sizeof(double) * sizes[4], s) != hipSuccess ||
        hipMemsetAsync(U0, 0, sizeof(double) * sizes[5], s) != hipSuccess ||
        hipMemsetAsync(U1, 0, sizeof(double) * sizes[6], s) != hipSuccess ||
        hipMemsetAsync(Ft, 0, sizeof(double) * sizes[7], s) != hipSuccess ||
        hipMemsetAsync(info, 0, sizeof(int), s) != hipSuccess)
        return fail(ROM_E_DEVICE, "CP-ALS workspace clear failed");
    launch_als_unfold(N, (int)np, 0, C, U0, s);     // rows (i, j), columns k
    launch_als_unfold(N, (int)np, 1, C, U1, s);     // rows (i, k), columns j
    // one sweep (about 3 R / 16 + 30 launches) is captured once into a graph on a stream of
    // this call, ordered after the caller's stream, and replayed `sweeps` times; each
    // inverse runs on a side stream beside the right-hand side of its update (a branch of
    // the graph)
    SweepStreams ss;
    if (!ss.init(s)) return fail(ROM_E_DEVICE, "CP-ALS stream setup failed");
    hipStream_t cs = ss.cs;
    hipGraph_t& graph = ss.graph;
    hipGraphExec_t& gexec = ss.gexec;
    double* F[3] = {A1, A2, A3};
    const GemmPlan pl = gemm_plan(R, (int)npad, 0), plt = gemm_plan(R, (int)n2pad, 0);
    const AlsProductPlan prod = als_product_plan((int)np, kProductLds);
    // T[row][m] = sum_c Ft[m][c] U[row][c]: the unfolding times one factor
    auto tensor_times = [&](const double* Uf, const double* Fk) {
        launch_als_transpose(N, R, (int)np, Fk, Ft, s);
        if (prod.ok) launch_als_product(prod, R, (int)np, (long long)n2pad, Uf, Ft, T, s);
        else launch_gemm_f64(plt, Ft, (long long)np, Uf, (long long)np, T, R, (int)np, (int)n2pad, s);
    };
    s = cs;   // every launch below (tensor_times included) goes to the capture stream
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(ROM_E_DEVICE, "CP-ALS graph capture failed to start");
    bool cap_ok = true;
    for (int mode = 0; mode < 3; ++mode) {
            const int a = mode == 0 ? 1 : 0, b = mode == 2 ? 1 : 2;
            launch_gram_hadamard(N, R, F[a], F[b], V, s);
            cap_ok = ss.fork(mode) && cap_ok;
            spd_inverse_gj(R, (int)rp, V, L, X, Vinv, info, ss.side);
            cap_ok = ss.join_mark(mode) && cap_ok;
            // right-hand side: modes 1 and 2 share T = C x_k A3 (A3 is fixed until mode 3);
            // mode 3 uses C x_j A2 over rows (i, k)
            if (mode == 0) tensor_times(U0, F[2]);
            if (mode == 2) tensor_times(U1, F[1]);
            if (mode == 0) launch_als_reduce(N, R, 1, T, F[1], Mb, (int)rp, s);       // sum_j T[(i,j)] A2[j]
            else launch_als_reduce(N, R, 0, T, F[0], Mb, (int)rp, s);                 // sum_i T[(i,.)] A1[i]
            cap_ok = ss.join(mode) && cap_ok;
            // F[mode][i][m] = sum_k Vinv[m][k] Mb[i][k]  (V symmetric)
            launch_gemm_f64_rows(pl, Vinv, (long long)rp, Mb, (long long)rp, F[mode], R, (int)rp, (int)npad, N, s);
    }
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess && !cap_ok) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    for (int sw = 0; sw < sweeps && e == hipSuccess; ++sw) e = hipGraphLaunch(gexec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    int hinfo = 0;
    if (e == hipSuccess) e = hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ROM_E_DEVICE, "CP-ALS failed: %s", hipGetErrorString(e));
    if (hinfo) return fail(ROM_E_INVALID, "CP-ALS normal equations not positive definite (rank-deficient factors)");
    return ROM_OK;
}

extern "C" rom_status rom_cp_als_skew(int32_t N, int32_t P, const double* C, double* A11, double* A12, double* B1,
                                       int32_t sweeps, int32_t subiters, double momentum, void* stream) {
    if (N < 1 || N > 4096) return fail(ROM_E_INVALID, "N must be in [1, 4096] (got %d)", N);
    if (P < 1 || P > 2048) return fail(ROM_E_INVALID, "P must be in [1, 2048] (got %d)", P);
    if (sweeps < 0 || subiters < 0) return fail(ROM_E_INVALID, "sweeps and subiters must be >= 0");
    if (!(momentum >= 0.0 && momentum < 1.0)) return fail(ROM_E_INVALID, "momentum must be in [0, 1)");
    if (!C || !A11 || !A12 || !B1) return fail(ROM_E_INVALID, "a tensor or factor pointer is NULL");
    if (sweeps == 0) return ROM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int R = 2 * P;
    const size_t n = (size_t)N, r = (size_t)R, rp = (r + 7) / 8 * 8, p = (size_t)P, pp = (p + 7) / 8 * 8;
    const size_t npad = (n + 15) / 16 * 16, np = (n + 7) / 8 * 8, n2pad = (n * n + 15) / 16 * 16;
    // factors A1, A2, A3 [N][R]; the untied normal system V, L, X [R][R], Vinv [R][Rp],
    // right-hand side Mb [Npad][Rp], solution Yb [Npad][R]; the tied system Vt, Lt, Xt
    // [P][P], Vtinv [P][Pp], Mt [Npad][Pp], Yt [Npad][P]; the unfolding U0 [N^2 padded][Np],
    // a transposed factor Ft [R][Np] and the product T [N^2 padded][R]
    constexpr int kBufs = 17;
    const size_t sizes[kBufs] = {n * r, n * r, n * r, r * r, r * r, r * r, r * rp, npad * rp, npad * r,
                                 p * p, p * p, p * p, p * pp, npad * pp, npad * p, n2pad * np, r * np + kProductSlack};
    const size_t tsize = n2pad * r;
    double* buf[kBufs + 1] = {};
    int* info = nullptr;
    struct Guard {
        double** b;
        int** info;
        ~Guard() {
            for (int q = 0; q <= kBufs; ++q)
                if (b[q]) hipFree(b[q]);
            if (*info) hipFree(*info);
        }
    } guard{buf, &info};
    for (int q = 0; q <= kBufs; ++q) {
        const hipError_t e = hipMalloc((void**)&buf[q], sizeof(double) * (q < kBufs ? sizes[q] : tsize));
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? ROM_E_NOMEM : ROM_E_DEVICE, "ALS-skew workspace: %s",
                                         hipGetErrorString(e));
    }
    if (hipMalloc((void**)&info, sizeof(int)) != hipSuccess) return fail(ROM_E_NOMEM, "ALS-skew workspace");
    double *A1 = buf[0], *A2 = buf[1], *A3 = buf[2], *V = buf[3], *L = buf[4], *X = buf[5], *Vinv = buf[6];
    double *Mb = buf[7], *Yb = buf[8], *Vt = buf[9], *Lt = buf[10], *Xt = buf[11], *Vtinv = buf[12], *Mt = buf[13];
    double *Yt = buf[14], *U0 = buf[15], *Ft = buf[16], *T = buf[17];
    if (hipMemsetAsync(Vinv, 0, sizeof(double) * sizes[6], s) != hipSuccess ||
        hipMemsetAsync(Mb, 0, sizeof(double) * sizes[7], s) != hipSuccess ||
        hipMemsetAsync(Vtinv, 0, sizeof(double) * sizes[12], s) != hipSuccess ||
        hipMemsetAsync(Mt, 0, sizeof(double) * sizes[13], s) != hipSuccess ||
        hipMemsetAsync(U0, 0, sizeof(double) * sizes[15], s) != hipSuccess ||
        hipMemsetAsync(Ft, 0, sizeof(double) * sizes[16], s) != hipSuccess ||
        hipMemsetAsync(info, 0, sizeof(int), s) != hipSuccess)
        return fail(ROM_E_DEVICE, "ALS-skew workspace clear failed");
    launch_als_unfold(N, (int)np, 0, C, U0, s);     // rows (i, j), columns k
    launch_skew_assemble(N, P, A11, A12, B1, A1, A2, A3, s);
    SweepStreams ss;
    if (!ss.init(s)) return fail(ROM_E_DEVICE, "ALS-skew stream setup failed");
    hipStream_t cs = ss.cs;
    hipGraph_t& graph = ss.graph;
    hipGraphExec_t& gexec = ss.gexec;
    const GemmPlan plt = gemm_plan(R, (int)n2pad, 0), plr = gemm_plan(R, (int)npad, 0),
                   plp = gemm_plan(P, (int)npad, 0);
    const AlsProductPlan prod = als_product_plan((int)np, kProductLds);
    s = cs;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(ROM_E_DEVICE, "ALS-skew graph capture failed to start");
    // T[(i, j)][m] = sum_k C[i][j][k] A3[k][m]: the unfolding times the third factor
    auto tensor_times_a3 = [&]() {
        launch_als_transpose(N, R, (int)np, A3, Ft, s);
        if (prod.ok) launch_als_product(prod, R, (int)np, (long long)n2pad, U0, Ft, T, s);
        else launch_gemm_f64(plt, Ft, (long long)np, U0, (long long)np, T, R, (int)np, (int)n2pad, s);
    };
    // one sweep: the tied second factor (least squares with A2 = B1 [I I]), then the
    // subiterations of the first factor with A3 fixed, each followed by the momentum
    // update and A3 = [A12 -A11]
    bool cap_ok = true;
    launch_gram_hadamard(N, R, A1, A3, V, s);
    // the tied system's inverse on the side stream, beside the product and the reduction
    const int qt = SweepStreams::kPairs - 1;
    launch_skew_tie(N, P, V, Vt, nullptr, (int)rp, Mt, (int)pp, s);   // Vt
    cap_ok = ss.fork(qt) && cap_ok;
    spd_inverse_gj(P, (int)pp, Vt, Lt, Xt, Vtinv, info, ss.side);
    cap_ok = ss.join_mark(qt) && cap_ok;
    tensor_times_a3();
    launch_als_reduce(N, R, 0, T, A1, Mb, (int)rp, s);                 // sum_i T[(i, j)] A1[i]
    launch_skew_tie(N, P, nullptr, Vt, Mb, (int)rp, Mt, (int)pp, s);  // Mt
    cap_ok = ss.join(qt) && cap_ok;
    launch_gemm_f64(plp, Vtinv, (long long)pp, Mt, (long long)pp, Yt, P, (int)pp, (int)npad, s);
    launch_skew_set_b(N, P, Yt, P, B1, A2, s);
    for (int it = 0; it < subiters; ++it) {
        launch_gram_hadamard(N, R, A2, A3, V, s);
        // the inverse on the side stream, beside the right-hand side
        const int q = it % (SweepStreams::kPairs - 1);
        cap_ok = ss.fork(q) && cap_ok;
        spd_inverse_gj(R, (int)rp, V, L, X, Vinv, info, ss.side);
        cap_ok = ss.join_mark(q) && cap_ok;
        if (it > 0) tensor_times_a3();                                 // A3 moved with A1
        launch_als_reduce(N, R, 1, T, A2, Mb, (int)rp, s);             // sum_j T[(i, j)] A2[j]
        cap_ok = ss.join(q) && cap_ok;
        launch_gemm_f64(plr, Vinv, (long long)rp, Mb, (long long)rp, Yb, R, (int)rp, (int)npad, s);
        launch_skew_momentum(N, P, momentum, Yb, R, A1, A3, A11, A12, s);
    }
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess && !cap_ok) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    for (int sw = 0; sw < sweeps && e == hipSuccess; ++sw) e = hipGraphLaunch(gexec, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    int hinfo = 0;
    if (e == hipSuccess) e = hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ROM_E_DEVICE, "ALS-skew failed: %s", hipGetErrorString(e));
    if (hinfo) return fail(ROM_E_INVALID, "ALS-skew normal equations not positive definite (rank-deficient factors)");
    return ROM_OK;
}

extern "C" rom_status rom_create_full(const rom_desc* d, const rom_full_terms* f, rom_ctx* out) {
    if (!f) {
        if (out) *out = nullptr;
        return fail(ROM_E_INVALID, "full terms are NULL");
    }
    return create_ctx(d, nullptr, f, out);
}

extern "C" rom_status rom_create_svd(const rom_desc* d, int32_t R, const double* U, const double* sigma,
                                     const double* V, rom_ctx* out) {
    const SvdDesc sv{R, U, sigma, V};
    return create_ctx(d, &sv, nullptr, out);
}

// ============================================================== contraction dispatch

// The state's kernel arguments for the step from level n: the counter slot of n's
// parity to read, the other one to advance.
static StepArgs step_args(rom_state s, long long n) {
    StepArgs a = s->a;
    a.step = s->cnt + (n & 1);
    a.step_next = s->cnt + ((n + 1) & 1);
    return a;
}

// The skew column pairs the one-trajectory CP kernels use (layout 0: the general form),
// and the matching projection operator.
static SkewPairs skew_of(rom_ctx c) {
    SkewPairs sk{};
    if (!c->dense && c->skew_layout && c->tile[4] != 0) {
        sk.layout = c->skew_layout;
        sk.P = c->R / 2;
        sk.R = c->R;
    }
    return sk;
}
static const void* proj_op(rom_ctx c) { return skew_of(c).layout ? c->SK : c->BCt; }
static const void* proj_op_lo(rom_ctx c) { return skew_of(c).layout ? c->SK_lo : c->BCt_lo; }

// The Helmholtz apply of a one-trajectory state (with the projections of the new level
// when the context is CP).
static HelmJob helm_job(rom_ctx c, const StepArgs& a) {
    HelmJob h{};
    h.a = a;
    h.nh = (c->N + 3) / 4;
    if (!c->dense) {
        const SkewPairs sk = skew_of(c);
        h.Mst = sk.layout ? c->Msk : c->Mst;
        h.Mst_lo = (const unsigned short*)(sk.layout ? c->Msk_lo : c->Mst_lo);
        h.lam = c->lam;
        h.Rp = c->Rp;
        h.layout = sk.layout;
        h.P = sk.P;
        h.R = sk.R;
        h.np = proj1_blocks(c->Rp, sk);
    }
    h.nblk = h.nh + h.np;
    return h;
}

// The Hadamard product of the projections of level n of a one-trajectory CP state with a
// dense stiffness (state creation and restart; every step then leaves that of the next
// level).
static void seed_projections(rom_ctx c, const StepArgs& a, hipStream_t stream) {
    if (c->dense || c->svd || c->diagA || a.B != 1) return;
    launch_cp_proj1(c->dtype, proj_op(c), proj_op_lo(c), c->lam, c->N, c->Np, c->Rp, skew_of(c), a.uring, a.step,
                    (long long)c->N, a.st, stream);
}

// Enqueue one BDF3/EXT3 step of state s from level n on `stream`: contraction (dense
// or CP, single-trajectory or batched kernels), FP64 update and energy; dense
// stiffness adds the Helmholtz apply.
static rom_status enqueue_step(rom_ctx c, rom_state s, hipStream_t stream, long long n) {
    const StepArgs a = step_args(s, n);
    const WsPlan p = plan_ws(c, s->B);
    const int accf = acc_f64(c->dtype);
    const int diag = c->diagA ? 1 : 0;
    // the full form's terms: the one-trajectory CP scatter forms them itself
    const bool fused_terms = c->full && s->B == 1 && !c->dense && !c->svd;
    if (c->full) {
        if (s->B == 1) {
            if (!fused_terms) launch_full_terms(a, c->Gfull, stream);
        } else {
            launch_full_x(a, s->xfull, stream);
            launch_gemm_f64(gemm_plan_splitk(c->N, 2 * c->Np, s->Bpad), c->Gfull, 2LL * c->Np, s->xfull, 2LL * c->Np, a.zfull,
                            c->N, 2 * c->Np, s->Bpad, stream);
        }
    }
    if (s->B == 1) {
        char* ws = (char*)s->scratch;
        if (c->dense) {
            launch_dense_gemv(c->dtype, c->C, c->Clo, c->N, c->Np, c->N, nullptr, a.uring, a.step, (long long)c->N,
                              ws + p.part_off, p.nchunk, gemv_tile(c), stream);
            launch_bdf_from_partials(a, accf, ws + p.part_off, p.nchunk, 1, diag, stream);
        } else if (c->svd) {
            launch_svd_proj(c->dtype, c->Ut, c->Ut_lo, c->sig, c->N, c->Np, c->Rs, a.uring, a.step, (long long)c->N,
                            ws + p.svdw_off, stream);
            launch_dense_gemv(c->dtype, c->Vt, c->Vt_lo, c->N, c->Np, c->Rs, ws + p.svdw_off, a.uring, a.step,
                              (long long)c->N, ws + p.part_off, p.nchunk, gemv_tile(c), stream);
            launch_bdf_from_partials(a, accf, ws + p.part_off, p.nchunk, 1, diag, stream);
        } else {
            // a.st holds w = lam .* s .* t of level n: computed here with a diagonal
            // stiffness, left by the previous step's Helmholtz kernel otherwise
            if (diag)
                launch_cp_proj1(c->dtype, proj_op(c), proj_op_lo(c), c->lam, c->N, c->Np, c->Rp, skew_of(c),
                                a.uring, a.step, (long long)c->N, a.st, stream);
            launch_cp_scatter1(c->dtype, c->Af, c->Af_lo, c->N, c->Rp, a.st, nullptr, &a, diag ? 1 : 2, stream,
                               fused_terms ? c->Gfull : nullptr);
        }
    } else {
        char* ws = (char*)c->ws;
        if (c->dense) {
            launch_dense_batched(c->dtype, p.pd, c->C, c->Clo, c->Ct, c->Ct_lo, c->N, c->Np, p.Bpad, a.ucv,
                                 a.ucv_lo, a.uj, ws + p.part_off, stream);
            launch_bdf_from_partials(a, accf, ws + p.part_off, p.pd.nsplit, p.Bpad, diag, stream);
        } else {
            if (!launch_cp_batched(c, p.pp, p.ps, p.Bpad, s->B, a.ucv, a.ucv_lo, ws + p.part2_off, ws + p.w_off,
                                   ws + p.part_off, &a, stream))
                launch_bdf_from_partials(a, accf, ws + p.part_off, p.ps.nsplit, p.Bpad, diag, stream);
        }
    }
    if (!c->diagA) {
        if (s->B == 1 && !c->dense && !c->svd) {
            launch_helm_proj(c->dtype, helm_job(c, a), stream);
        } else if (s->B == 1) {
            launch_helm_apply(a, stream);
        } else {
            launch_gemm_helm(p.ph, c->hinv, c->N, c->Np, p.Bpad, a.rhs, a.step, nullptr, &a, stream);
        }
    }
    HIPCHK(hipGetLastError());
    return ROM_OK;
}

// Shared body of rom_nonlinear and rom_nonlinear_timed: operand copies (batches), the
// contraction kernels, and the sum of the partial results into y.  With kernel_us the
// contraction is captured `reps` times into a HIP graph, launched once to warm up and
// once between two events; *kernel_us is the average per repetition.
static rom_status nonlinear_impl(rom_ctx c, int32_t batch, const double* u_dev, double* y_dev, int reps,
                                 double* kernel_us, char* ws_given = nullptr, size_t ws_given_bytes = 0) {
    if (!c) return fail(ROM_E_INVALID, "ctx is NULL");
    if (batch < 1 || batch > c->max_batch) return fail(ROM_E_INVALID, "batch %d outside [1, %d]", batch, c->max_batch);
    if (!u_dev || !y_dev) return fail(ROM_E_INVALID, "u_dev / y_dev is NULL");
    const WsPlan p = plan_ws(c, batch);
    char* ws = ws_given;
    if (ws) {
        // a caller-chosen workspace: it must hold the plan, and what the kernels may
        // read beyond the regions they write (lane vectors run up to one k-step past
        // the last row) must be zero, as a fresh workspace is
        if (p.total > ws_given_bytes)
            return fail(ROM_E_UNSUPPORTED, "the evaluation needs %zu bytes of workspace, more than the %zu available",
                        p.total, ws_given_bytes);
        launch_zero_fill(ws, p.total, c->stream);
    } else {
        rom_status st = ensure_ws(c, p.total);
        if (st != ROM_OK) return st;
        ws = (char*)c->ws;
    }
    const int accf = acc_f64(c->dtype);
    StepArgs a{};
    if (batch > 1) {
        // operand copies of the caller's u in the contraction format
        a.N = c->N;
        a.Np = c->Np;
        a.B = batch;
        a.Bpad = p.Bpad;
        a.dtype = c->dtype;
        a.batched = 1;
        a.ucv = ws + p.ucv_off;
        a.ucv_lo = ws + p.ucvlo_off;
        a.uj = ws + p.usc_off;
        launch_prep_ucv(a, u_dev, c->stream);
    }
    auto contract = [&]() {
        if (batch == 1) {
            if (c->dense) {
                launch_dense_gemv(c->dtype, c->C, c->Clo, c->N, c->Np, c->N, nullptr, u_dev, nullptr, 0,
                                  ws + p.part_off, p.nchunk, gemv_tile(c), c->stream);
            } else if (c->svd) {
                launch_svd_proj(c->dtype, c->Ut, c->Ut_lo, c->sig, c->N, c->Np, c->Rs, u_dev, nullptr, 0,
                                ws + p.svdw_off, c->stream);
                launch_dense_gemv(c->dtype, c->Vt, c->Vt_lo, c->N, c->Np, c->Rs, ws + p.svdw_off, u_dev, nullptr, 0,
                                  ws + p.part_off, p.nchunk, gemv_tile(c), c->stream);
            } else {
                launch_cp_proj1(c->dtype, proj_op(c), proj_op_lo(c), c->lam, c->N, c->Np, c->Rp, skew_of(c), u_dev,
                                nullptr, 0, ws + p.part_off, c->stream);
                launch_cp_scatter1(c->dtype, c->Af, c->Af_lo, c->N, c->Rp, ws + p.part_off, y_dev, nullptr, 0,
                                   c->stream);
            }
        } else if (c->dense) {
            launch_dense_batched(c->dtype, p.pd, c->C, c->Clo, c->Ct, c->Ct_lo, c->N, c->Np, p.Bpad, a.ucv, a.ucv_lo,
                                 a.uj, ws + p.part_off, c->stream);
        } else {
            launch_cp_batched(c, p.pp, p.ps, p.Bpad, batch, a.ucv, a.ucv_lo, ws + p.part2_off, ws + p.w_off,
                              ws + p.part_off, nullptr, c->stream);
        }
    };
    if (!kernel_us) {
        contract();
    } else {
        hipGraph_t gr = nullptr;
        hipGraphExec_t gx = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int r = 0; r < reps; ++r) contract();
            e = hipStreamEndCapture(c->stream, &gr);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = hipGraphLaunch(gx, c->stream);          // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess) e = hipGraphLaunch(gx, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        float ms = 0.f;
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (gx) hipGraphExecDestroy(gx);
        if (gr) hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(ROM_E_DEVICE, "timing the contraction failed: %s", hipGetErrorString(e));
        *kernel_us = 1e3 * (double)ms / reps;
    }
    if (batch == 1) {
        if (c->dense || c->svd) launch_sum_partials(accf, ws + p.part_off, p.nchunk, 1, 1, c->N, y_dev, c->stream);
    } else {
        launch_sum_partials(accf, ws + p.part_off, c->dense ? p.pd.nsplit : p.ps.nsplit, p.Bpad, batch, c->N, y_dev,
                            c->stream);
    }
    HIPCHK(hipGetLastError());
    return ROM_OK;
}

// ============================================================== scratch-free evaluation
//
// rom_nonlinear_noalloc runs rom_nonlinear's kernels with their workspace in `scratch`,
// one array per GPU that the code object brings along (held until the process ends),
// instead of the context's allocated workspace.  Host code never passes the array's
// name to a kernel: the device address of each GPU's copy is looked up once per GPU
// with hipGetSymbolAddress and kept in g_scratch_dev.

constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's `scratch` (looked up on the first call with `dev`
// current; the caller's current device is restored).
rom_status scratch_of(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return fail(ROM_E_UNSUPPORTED, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(ROM_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return ROM_OK;
}

}  // namespace

extern "C" rom_status rom_nonlinear_noalloc(rom_ctx c, int32_t batch, const double* u_dev, double* y_dev) {
    if (!c) return fail(ROM_E_INVALID, "ctx is NULL");
    void* ws = nullptr;
    TRYS(scratch_of(c->device, &ws));
    return nonlinear_impl(c, batch, u_dev, y_dev, 1, nullptr, (char*)ws, kStaticScratchBytes);
}

extern "C" rom_status rom_nonlinear(rom_ctx c, int32_t batch, const double* u_dev, double* y_dev) {
    return nonlinear_impl(c, batch, u_dev, y_dev, 1, nullptr);
}

extern "C" rom_status rom_nonlinear_timed(rom_ctx c, int32_t batch, const double* u_dev, double* y_dev, int32_t reps,
                                          double* kernel_us) {
    if (!kernel_us) return fail(ROM_E_INVALID, "kernel_us is NULL");
    if (reps < 1) return fail(ROM_E_INVALID, "reps must be >= 1");
    rom_status st = nonlinear_impl(c, batch, u_dev, y_dev, reps, kernel_us);
    if (st == ROM_OK && hipStreamSynchronize(c->stream) != hipSuccess)
        st = fail(ROM_E_DEVICE, "rom_nonlinear_timed: synchronize failed");
    return st;
}

// ============================================================== states

namespace {

__global__ void k_energy_level(StepArgs a, long long level) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const double* u = a.uring + ((size_t)(((level % 3) + 3) % 3) * a.B + b) * a.N;
    double s = 0.0;
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) s += u[i] * u[i];
    s += __shfl_xor(s, 32, 64);
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 8, 64);
    s += __shfl_xor(s, 4, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 1, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double e = 0.5 * (red[0] + red[1] + red[2] + red[3]);
        a.elog[(size_t)level * a.B + b] = e;
        if (!isfinite(e)) atomicMin(a.bad, level);
    }
}

__global__ void k_fill(double* p, size_t n, double v) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = v;
}

rom_status ensure_elog(rom_state s, long long levels_needed) {
    if (levels_needed <= s->a.elog_cap) return ROM_OK;
    long long cap = s->a.elog_cap > 0 ? s->a.elog_cap : 1024;
    while (cap < levels_needed) cap *= 2;
    double* nl = nullptr;
    hipError_t e = hipMalloc((void**)&nl, sizeof(double) * cap * s->B);
    if (e != hipSuccess) return fail(ROM_E_NOMEM, "energy log hipMalloc failed: %s", hipGetErrorString(e));
    rom_ctx c = s->ctx;
    const size_t total = (size_t)cap * s->B;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, nl, total,
                       std::nan(""));
    if (s->a.elog) {
        HIPCHK(hipMemcpyAsync(nl, s->a.elog, sizeof(double) * s->a.elog_cap * s->B, hipMemcpyDeviceToDevice,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        hipFree(s->a.elog);
        s->bytes -= sizeof(double) * s->a.elog_cap * s->B;
    }
    s->a.elog = nl;
    s->a.elog_cap = cap;
    s->bytes += sizeof(double) * cap * s->B;
    s->sgen++;
    return ROM_OK;
}

// Contraction scratch of a single-trajectory state (grows with the kernel tiles).
rom_status ensure_scratch(rom_state s) {
    if (s->B != 1) return ROM_OK;
    const size_t need = plan_ws(s->ctx, 1).total;
    if (need <= s->scratch_bytes) return ROM_OK;
    if (s->scratch) {
        hipStreamSynchronize(s->ctx->stream);
        hipFree(s->scratch);
        s->bytes -= s->scratch_bytes;
        s->scratch = nullptr;
        s->scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&s->scratch, need);
    if (e != hipSuccess) {
        s->scratch = nullptr;
        return fail(ROM_E_NOMEM, "state scratch hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
    }
    s->scratch_bytes = need;
    s->bytes += need;
    s->sgen++;
    return ROM_OK;
}

rom_status reset_counters(rom_state s, long long step) {
    rom_ctx c = s->ctx;
    const long long both[2] = {step, step};
    const long long health[2] = {LLONG_MAX, 0};
    const int none = 0;
    HIPCHK(hipMemcpyAsync(s->cnt, both, sizeof(both), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(s->a.bad, health, sizeof(health), hipMemcpyHostToDevice, c->stream));
    const int nocount[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(s->a.closep, &none, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(s->a.ecount, nocount, sizeof(nocount), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return ROM_OK;
}

// Room for energy partials per trajectory: the most blocks per trajectory of any kernel
// that can write level n+1 of a state (4 rows a block for one trajectory, 16 rows a
// block for batches).
int energy_slots(rom_ctx c, int B) { return B > 1 ? (c->N + 15) / 16 : (c->N + 3) / 4; }

}  // namespace

extern "C" void rom_state_destroy(rom_state s) {
    if (!s) return;
    forget_plans_of(s);
    if (s->ctx && s->ctx->stream) hipStreamSynchronize(s->ctx->stream);
    for (auto& par : s->graph)
        for (auto& row : par)
            for (auto g : row)
                if (g) hipGraphExecDestroy(g);
    for (void* p : s->allocs) hipFree(p);
    if (s->a.elog) hipFree(s->a.elog);
    if (s->scratch) hipFree(s->scratch);
    if (s->res_buf) hipFree(s->res_buf);
    if (s->slot_stage) hipFree(s->slot_stage);
    delete s;
}

extern "C" rom_status rom_state_create(rom_ctx c, int32_t batch, const double* u0_host, rom_state* out) {
    if (!out) return fail(ROM_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!c) return fail(ROM_E_INVALID, "ctx is NULL");
    if (batch < 1 || batch > c->max_batch) return fail(ROM_E_INVALID, "batch %d outside [1, %d]", batch, c->max_batch);
    if (!u0_host) return fail(ROM_E_INVALID, "u0_host is NULL");
    rom_state s = new rom_state_s();
    s->ctx = c;
    s->B = batch;
    s->Bpad = (batch + 15) / 16 * 16;
    const size_t N = c->N, B = batch, BN = B * N;
    rom_status st;
#define TRY(x)                      \
    do {                            \
        st = (x);                   \
        if (st != ROM_OK) {         \
            rom_state_destroy(s);   \
            return st;              \
        }                           \
    } while (0)
    StepArgs& a = s->a;
    a.N = c->N;
    a.Np = c->Np;
    a.B = batch;
    a.Bpad = s->Bpad;
    a.inv_dt = 1.0 / c->dt;
    a.dtype = c->dtype;
    a.batched = batch > 1 ? 1 : 0;
    a.hdiag = c->hdiag;
    a.hinv = c->hinv;
    TRY(dmalloc((void**)&a.uring, sizeof(double) * 3 * BN, &s->bytes, &s->allocs));
    TRY(dmalloc((void**)&a.yring, sizeof(double) * 3 * BN, &s->bytes, &s->allocs));
    TRY(dmalloc((void**)&a.rhs, sizeof(double) * s->Bpad * c->Np, &s->bytes, &s->allocs));
    a.enmax = energy_slots(c, batch);
    TRY(dmalloc((void**)&a.epart, sizeof(double) * 2 * B * a.enmax, &s->bytes, &s->allocs));
    TRY(dmalloc((void**)&a.ecount, 2 * sizeof(int), &s->bytes, &s->allocs));
    TRY(dmalloc((void**)&s->cnt, 2 * sizeof(long long), &s->bytes, &s->allocs));
    a.step = s->cnt;
    a.step_next = s->cnt + 1;
    // bad[0]: first non-finite level; bad[1]: nonzero when a resident run's wait gave up
    TRY(dmalloc((void**)&a.bad, 2 * sizeof(long long), &s->bytes, &s->allocs));
    TRY(dmalloc((void**)&a.closep, sizeof(int), &s->bytes, &s->allocs));
    if (!c->dense && !c->svd && batch == 1)
        TRY(dmalloc(&a.st, c->Rp * acc_bytes(c->dtype), &s->bytes, &s->allocs));
    if (c->full) {
        // zfull takes Bpad rows (the batched product writes its padding rows); X of the
        // batched product starts zero and only its live entries are ever written
        // batches: one partial product of X G^T per K range of the split product
        a.zsplit = batch > 1 ? gemm_plan_splitk(c->N, 2 * c->Np, s->Bpad).ksplit : 1;
        a.zstride = (long long)s->Bpad * N;
        TRY(dmalloc((void**)&a.zfull, sizeof(double) * a.zsplit * s->Bpad * N, &s->bytes, &s->allocs));
        a.fz = c->fz;
        a.az = c->az;
        if (batch > 1) {
            const size_t xb = sizeof(double) * s->Bpad * 2 * c->Np;
            TRY(dmalloc((void**)&s->xfull, xb, &s->bytes, &s->allocs));
            if (hipMemsetAsync(s->xfull, 0, xb, c->stream) != hipSuccess) {
                rom_state_destroy(s);
                return fail(ROM_E_DEVICE, "clearing the full-form operand failed");
            }
        }
    }
    if (a.batched) {
        const size_t cells = (size_t)s->Bpad * c->Np;
        TRY(dmalloc(&a.ucv, cells * elem_bytes(c->dtype), &s->bytes, &s->allocs));
        TRY(dmalloc(&a.uj, cells * acc_bytes(c->dtype), &s->bytes, &s->allocs));
        if (c->dtype == DT_BF16X3) TRY(dmalloc(&a.ucv_lo, cells * 2, &s->bytes, &s->allocs));
        if (hipMemsetAsync(a.ucv, 0, cells * elem_bytes(c->dtype), c->stream) != hipSuccess ||
            hipMemsetAsync(a.uj, 0, cells * acc_bytes(c->dtype), c->stream) != hipSuccess ||
            (a.ucv_lo && hipMemsetAsync(a.ucv_lo, 0, cells * 2, c->stream) != hipSuccess)) {
            rom_state_destroy(s);
            return fail(ROM_E_DEVICE, "state clear failed");
        }
    }
    if (hipMemsetAsync(a.rhs, 0, sizeof(double) * s->Bpad * c->Np, c->stream) != hipSuccess ||
        hipMemsetAsync(a.uring, 0, sizeof(double) * 3 * BN, c->stream) != hipSuccess ||
        hipMemsetAsync(a.yring, 0, sizeof(double) * 3 * BN, c->stream) != hipSuccess) {
        rom_state_destroy(s);
        return fail(ROM_E_DEVICE, "state clear failed");
    }
    if (hipMemcpyAsync(a.uring, u0_host, sizeof(double) * BN, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        rom_state_destroy(s);
        return fail(ROM_E_DEVICE, "upload of u0 failed");
    }
    TRY(reset_counters(s, 0));
    TRY(ensure_elog(s, 1024));
    hipLaunchKernelGGL(k_energy_level, dim3(batch), dim3(256), 0, c->stream, a, 0LL);
    seed_projections(c, step_args(s, 0), c->stream);
    if (a.batched) launch_prep_ucv(a, a.uring, c->stream);
    TRY(ensure_ws(c, plan_ws(c, batch).total));
    TRY(ensure_scratch(s));
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        rom_state_destroy(s);
        return fail(ROM_E_DEVICE, "state setup failed");
    }
#undef TRY
    *out = s;
    return ROM_OK;
}

// ============================================================== stepping

static bool res_usable(rom_ctx c, rom_state s);
static rom_status ensure_res(rom_ctx c, rom_state s);

static rom_status prepare(rom_ctx c, rom_state s, int64_t nsteps) {
    rom_status st = ensure_ws(c, plan_ws(c, s->B).total);
    if (st != ROM_OK) return st;
    st = ensure_scratch(s);
    if (st != ROM_OK) return st;
    if (res_usable(c, s)) {
        st = ensure_res(c, s);
        if (st != ROM_OK) return st;
    }
    return ensure_elog(s, s->h_step + nsteps + 1);
}

// Capture `len` steps of state s starting at a level of parity `par` into *gx, with the
// closing kernel of the newest level at the end when `close` is set.
static rom_status capture_chunk(rom_ctx c, rom_state s, int par, int len, int close, hipGraphExec_t* gx) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    rom_status cst = ROM_OK;
    for (int q = 0; q < len && cst == ROM_OK; ++q) cst = enqueue_step(c, s, c->stream, par + q);
    if (cst == ROM_OK && close) launch_close(step_args(s, par + len), c->stream);
    hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (cst != ROM_OK) {
        if (g) hipGraphDestroy(g);
        return cst;
    }
    if (ee != hipSuccess) return fail(ROM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ee));
    hipError_t ie = hipGraphInstantiate(gx, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) {
        *gx = nullptr;
        return fail(ROM_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
    }
    // move the executable graph to the device now rather than at its first launch
    ie = hipGraphUpload(*gx, c->stream);
    if (ie != hipSuccess) return fail(ROM_E_DEVICE, "graph upload failed: %s", hipGetErrorString(ie));
    return ROM_OK;
}

// The graph of `len` steps from a level of parity `par` (captured on first use; every
// cached graph is dropped when the workspace or the state's scratch has moved).
static rom_status chunk_graph(rom_ctx c, rom_state s, int par, int len, int close, hipGraphExec_t* out) {
    if (s->graph_gen != c->ws_gen || s->graph_sgen != s->sgen) {
        for (auto& pr : s->graph)
            for (auto& row : pr)
                for (auto& g : row)
                    if (g) {
                        hipGraphExecDestroy(g);
                        g = nullptr;
                    }
        s->graph_gen = c->ws_gen;
        s->graph_sgen = s->sgen;
    }
    hipGraphExec_t& gx = s->graph[par][close][len];
    if (!gx) TRYS(capture_chunk(c, s, par, len, close, &gx));
    *out = gx;
    return ROM_OK;
}

// Walk the graphs of a call of nsteps from level n0: launch them, or (launch = false)
// only make sure they are captured.
static rom_status walk_graphs(rom_ctx c, rom_state s, long long n0, int64_t nsteps, bool launch) {
    long long n = n0;
    int64_t left = nsteps;
    while (left > 0) {
        const int len = left > kGraphChunk ? kGraphChunk : (int)left;
        const int close = left <= kGraphChunk ? 1 : 0;
        hipGraphExec_t gx = nullptr;
        TRYS(chunk_graph(c, s, (int)(n & 1), len, close, &gx));
        if (launch) HIPCHK(hipGraphLaunch(gx, c->stream));
        else if (len == kGraphChunk && !close) {
            // the 64-step graph repeats from the same parity: one capture serves them all
            const int64_t reps = (left - 1) / kGraphChunk;
            n += reps * kGraphChunk;
            left -= reps * kGraphChunk;
            continue;
        }
        n += len;
        left -= len;
    }
    return ROM_OK;
}

// ---- resident one-trajectory CP runs (k_res.hip)

constexpr int kResMin = 16;        // shortest run worth a launch (shorter tails use graphs)
constexpr int kResMax = 512;       // levels per run (the energy partials of a run)
constexpr unsigned kResSpin = 1u << 21;   // polling rounds before a wait gives up (seconds)

// Whether the one-trajectory CP steps of context c run resident, and their geometry:
// every block of the run co-resident (one per compute unit at most), the block's rows and
// vectors in its LDS, the vectors a block waits for within kResWaitWords message words.
static bool res_plan(rom_ctx c) {
    if (c->res_refused) return false;
    if (c->res_gen == c->ws_gen) return c->res_ok != 0;
    c->res_gen = c->ws_gen;
    c->res_ok = 0;
    if (c->dense || c->svd || c->full || c->tile[5] == 0) return false;
    const int wpe = c->dtype == DT_F64 ? 2 : 1;
    if (2 * c->N > kResWaitWords || c->Rp * wpe > kResWaitWords) return false;
    int ncu = 0, lds_dev = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_dev, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const SkewPairs sk = skew_of(c);
    const int nrg = (c->N + 3) / 4, npg = proj1_blocks(c->Rp, sk);
    const int G = std::min(ncu, std::max(nrg, npg));
    const int rg = (nrg + G - 1) / G, pg = (npg + G - 1) / G;
    if (rg > 4 || pg > 8) return false;       // the kernel's per-block tables
    const size_t lds = res_layout(c->dtype, c->N, c->Np, c->Rp, sk.layout, c->diagA ? 0 : 1, rg, pg).total;
    const size_t cap = (size_t)lds_dev - 2048;   // room for the kernel's static LDS
    if (lds > cap) return false;
    int per_cu = 0;
    if (res_attr(c->dtype, c->N, cap, lds, &per_cu) != hipSuccess || per_cu < 1 || (long long)per_cu * ncu < G) {
        (void)hipGetLastError();
        return false;
    }
    c->res_ok = 1;
    c->res_G = G;
    c->res_nrg = nrg;
    c->res_npg = npg;
    c->res_rg = rg;
    c->res_pg = pg;
    c->res_lds = lds;
    return true;
}

static bool res_usable(rom_ctx c, rom_state s) { return s->B == 1 && res_plan(c); }

// Message words, energy partials and tag base of a state's resident runs (zeroed once;
// the tag base only grows, so old words never match a later run's tags).
static rom_status ensure_res(rom_ctx c, rom_state s) {
    if (s->res_buf) return ROM_OK;
    const int wpe = c->dtype == DT_F64 ? 2 : 1;
    const size_t xb = align256(sizeof(unsigned long long) * 2 * c->N);
    const size_t wb = align256(sizeof(unsigned long long) * (size_t)c->Rp * wpe);
    const size_t eb = align256(sizeof(double) * (size_t)kResMax * ((c->N + 3) / 4));
    const size_t total = xb + wb + eb + 256;
    hipError_t e = hipMalloc(&s->res_buf, total);
    if (e != hipSuccess) {
        s->res_buf = nullptr;
        return fail(ROM_E_NOMEM, "resident step buffers hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
    }
    s->bytes += total;
    char* p = (char*)s->res_buf;
    s->res_x = (unsigned long long*)p;
    s->res_w = (unsigned long long*)(p + xb);
    s->res_ep = (double*)(p + xb + wb);
    s->res_seq = (unsigned*)(p + xb + wb + eb);
    launch_zero_fill(s->res_buf, total, c->stream);
    HIPCHK(hipGetLastError());
    return ROM_OK;
}

// A resident run needs every one of its blocks on the device at once (they wait for each
// other's messages).  It is an ordinary launch of at most one block per compute unit, which
// an otherwise idle device places at once; two runs overlapping on two streams could each
// hold part of the device, so the runs of this process are ordered across streams: a run on
// another stream than the previous run's first waits for all work enqueued on that stream
// (an event recorded there when the stream changes; none while runs stay on one stream).
// Any other wait that does not end within the kernel's polling bound raises its error flag.
static ResOrder& res_order(int device) {
    static ResOrder ord[kResDevices];
    return ord[(unsigned)device % kResDevices];
}

static void res_forget_stream(int device, hipStream_t s) {
    ResOrder& ord = res_order(device);
    std::lock_guard<std::mutex> lk(ord.mu);
    if (ord.last == s) ord.last = nullptr;
}

// One resident run of L steps from level n0 >= 2, then its closing block.  Returns
// *refused = true (and ROM_OK) when the runtime refuses the launch: nothing was enqueued,
// and the context takes the per-step kernels from then on.
static rom_status launch_resident(rom_ctx c, rom_state s, long long n0, int L, bool close_last, bool* refused) {
    *refused = false;
    const SkewPairs sk = skew_of(c);
    ResJob jb{};
    jb.a = step_args(s, n0);
    jb.n0 = n0;
    jb.nsteps = L;
    jb.dense_h = c->diagA ? 0 : 1;
    jb.Af = c->Af;
    jb.Af_lo = (const unsigned short*)c->Af_lo;
    if (jb.dense_h) {
        // order 3 of [3][rows][Np]
        const size_t rows = sk.layout ? (size_t)(sk.P + sk.R) : (size_t)2 * c->Rp;
        const size_t off = 2 * rows * c->Np;
        jb.Pop = (const char*)(sk.layout ? c->Msk : c->Mst) + off * elem_bytes(c->dtype);
        const void* lo = sk.layout ? c->Msk_lo : c->Mst_lo;
        jb.Pop_lo = lo ? (const unsigned short*)lo + off : nullptr;
    } else {
        jb.Pop = proj_op(c);
        jb.Pop_lo = (const unsigned short*)proj_op_lo(c);
    }
    jb.lam = c->lam;
    jb.Rp = c->Rp;
    jb.layout = sk.layout;
    jb.P = sk.P;
    jb.R = sk.R;
    jb.nrg = c->res_nrg;
    jb.npg = c->res_npg;
    jb.rg_per = c->res_rg;
    jb.pg_per = c->res_pg;
    jb.xmsg = s->res_x;
    jb.wmsg = s->res_w;
    jb.epall = s->res_ep;
    jb.seq = s->res_seq;
    jb.err = (int*)(s->a.bad + 1);
    jb.spin_max = kResSpin;
    ResOrder& ord = res_order(c->device);
    std::lock_guard<std::mutex> lk(ord.mu);
    if (ord.last && ord.last != c->stream) {
        if (!ord.ev) HIPCHK(hipEventCreateWithFlags(&ord.ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ord.ev, ord.last));
        HIPCHK(hipStreamWaitEvent(c->stream, ord.ev, 0));
    }
    hipError_t e = res_launch(c->dtype, jb, c->res_G, c->res_lds, c->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->res_refused = true;
        *refused = true;
        return ROM_OK;
    }
    ord.last = c->stream;
    res_close_launch(step_args(s, n0), step_args(s, n0 + L), n0, L, s->res_ep, c->res_nrg, s->res_seq, close_last,
                     c->stream);
    HIPCHK(hipGetLastError());
    return ROM_OK;
}

// The launches of nsteps steps from level n0: resident runs from level 2 on when the
// context allows them (the first two levels and a tail shorter than kResMin through the
// captured graphs), else the graphs alone.  launch = false only captures the graphs.
static rom_status walk_steps(rom_ctx c, rom_state s, long long n0, int64_t nsteps, bool launch) {
    const int64_t head = n0 < 2 ? std::min<int64_t>(2 - n0, nsteps) : 0;
    bool res = nsteps - head >= kResMin && res_usable(c, s);
    if (res && launch) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) res = false;
    }
    if (!res) return walk_graphs(c, s, n0, nsteps, launch);
    long long n = n0;
    int64_t left = nsteps;
    if (head > 0) {
        TRYS(walk_graphs(c, s, n, head, launch));
        n += head;
        left -= head;
    }
    while (left >= kResMin) {
        const int L = (int)std::min<int64_t>(left, kResMax);
        if (launch) {
            bool refused = false;
            TRYS(launch_resident(c, s, n, L, left == L, &refused));   // the last run closes its last level
            if (refused) break;                      // the rest through the graphs
        }
        n += L;
        left -= L;
    }
    if (left > 0) TRYS(walk_graphs(c, s, n, left, launch));
    return ROM_OK;
}

static rom_status step_enqueue(rom_ctx c, rom_state s, int64_t nsteps) {
    rom_status st = prepare(c, s, nsteps);
    if (st != ROM_OK) return st;
    if (nsteps == 0) return ROM_OK;
    // every update kernel closes the level before its own; the graph of the last chunk
    // (or the closing kernel after a resident run) closes the newest one
    TRYS(walk_steps(c, s, s->h_step, nsteps, true));
    HIPCHK(hipGetLastError());
    s->h_step += nsteps;
    s->pending = true;
    return ROM_OK;
}

extern "C" rom_status rom_step_prepare(rom_ctx c, rom_state s, int64_t nsteps) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    if (nsteps < 0) return fail(ROM_E_INVALID, "nsteps < 0");
    TRYS(prepare(c, s, nsteps));
    // the graphs depend on the parity of the first level only: both parities are
    // captured, so steps of any count may come between this call and the prepared one
    TRYS(walk_steps(c, s, s->h_step, nsteps, false));
    TRYS(walk_steps(c, s, s->h_step + 1, nsteps, false));
    HIPCHK(hipStreamSynchronize(c->stream));
    return ROM_OK;
}

extern "C" rom_status rom_step_sync(rom_ctx c, rom_state s, int64_t* first_bad_step) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    if (first_bad_step) *first_bad_step = -1;
    HIPCHK(hipStreamSynchronize(c->stream));
    s->pending = false;
    long long health[2] = {LLONG_MAX, 0};
    HIPCHK(hipMemcpy(health, s->a.bad, sizeof(health), hipMemcpyDeviceToHost));
    if (health[1] != 0)
        return fail(ROM_E_DEVICE, "a resident step run gave up waiting for another block's data");
    const long long bad = health[0];
    if (bad != LLONG_MAX) {
        if (first_bad_step) *first_bad_step = bad;
        return fail(ROM_E_NONFINITE, "trajectory became non-finite at step %lld", bad);
    }
    return ROM_OK;
}

extern "C" rom_status rom_step_async(rom_ctx c, rom_state s, int64_t nsteps) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    if (nsteps < 0) return fail(ROM_E_INVALID, "nsteps < 0");
    return step_enqueue(c, s, nsteps);
}

extern "C" rom_status rom_step(rom_ctx c, rom_state s, int64_t nsteps, int64_t* first_bad_step) {
    if (first_bad_step) *first_bad_step = -1;
    rom_status st = rom_step_async(c, s, nsteps);
    if (st != ROM_OK) return st;
    return rom_step_sync(c, s, first_bad_step);
}

extern "C" rom_status rom_energy(rom_ctx c, rom_state s, double* E_host, double* Elog_host) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    HIPCHK(hipStreamSynchronize(c->stream));
    if (E_host)
        HIPCHK(hipMemcpy(E_host, s->a.elog + (size_t)s->h_step * s->B, sizeof(double) * s->B,
                         hipMemcpyDeviceToHost));
    if (Elog_host)
        HIPCHK(hipMemcpy(Elog_host, s->a.elog, sizeof(double) * (size_t)(s->h_step + 1) * s->B,
                         hipMemcpyDeviceToHost));
    return ROM_OK;
}

extern "C" rom_status rom_state_get(rom_ctx c, rom_state s, double* u_hist, double* y_hist, int64_t* step) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t BN = (size_t)s->B * c->N;
    const long long n = s->h_step;
    for (int q = 0; q < 3 && u_hist; ++q) {
        const long long lev = n - q;
        if (lev < 0) memset(u_hist + q * BN, 0, sizeof(double) * BN);
        else HIPCHK(hipMemcpy(u_hist + q * BN, s->a.uring + (size_t)(lev % 3) * BN, sizeof(double) * BN,
                              hipMemcpyDeviceToHost));
    }
    for (int q = 0; q < 2 && y_hist; ++q) {
        const long long lev = n - 1 - q;
        if (lev < 0) memset(y_hist + q * BN, 0, sizeof(double) * BN);
        else HIPCHK(hipMemcpy(y_hist + q * BN, s->a.yring + (size_t)(lev % 3) * BN, sizeof(double) * BN,
                              hipMemcpyDeviceToHost));
    }
    if (step) *step = n;
    return ROM_OK;
}

extern "C" rom_status rom_state_set(rom_ctx c, rom_state s, const double* u_hist, const double* y_hist,
                                    int64_t step) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    if (!u_hist || !y_hist) return fail(ROM_E_INVALID, "u_hist / y_hist is NULL");
    if (step < 0) return fail(ROM_E_INVALID, "step < 0");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t BN = (size_t)s->B * c->N;
    for (int q = 0; q < 3; ++q) {
        const long long lev = step - q;
        if (lev < 0) continue;
        HIPCHK(hipMemcpy(s->a.uring + (size_t)(lev % 3) * BN, u_hist + q * BN, sizeof(double) * BN,
                         hipMemcpyHostToDevice));
    }
    for (int q = 0; q < 2; ++q) {
        const long long lev = step - 1 - q;
        if (lev < 0) continue;
        HIPCHK(hipMemcpy(s->a.yring + (size_t)(lev % 3) * BN, y_hist + q * BN, sizeof(double) * BN,
                         hipMemcpyHostToDevice));
    }
    rom_status st = ensure_elog(s, step + 1024);
    if (st != ROM_OK) return st;
    const size_t total = (size_t)s->a.elog_cap * s->B;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, s->a.elog, total,
                       std::nan(""));
    st = reset_counters(s, step);
    if (st != ROM_OK) return st;
    s->h_step = step;
    hipLaunchKernelGGL(k_energy_level, dim3(s->B), dim3(256), 0, c->stream, s->a, (long long)step);
    seed_projections(c, step_args(s, step), c->stream);
    if (s->a.batched) launch_prep_ucv(s->a, s->a.uring + (size_t)(step % 3) * BN, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return ROM_OK;
}

namespace {

// Trajectory b of a state at level n from h [5][N] (u^n, u^{n-1}, u^{n-2}, y^{n-1},
// y^{n-2}; levels below 0 skipped): the rings, the batched operand copies of level n, and
// E^n in the energy log.  One block.
__global__ __launch_bounds__(256) void k_set_slot(StepArgs a, long long n, int b, const double* __restrict__ h) {
    __shared__ double red[4];
    const size_t BN = (size_t)a.B * a.N, off = (size_t)b * a.N;
    double e = 0.0;
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) {
        for (int q = 0; q < 3; ++q)
            if (n - q >= 0) a.uring[(size_t)slot_of(n - q) * BN + off + i] = h[(size_t)q * a.N + i];
        for (int q = 0; q < 2; ++q)
            if (n - 1 - q >= 0) a.yring[(size_t)slot_of(n - 1 - q) * BN + off + i] = h[(size_t)(3 + q) * a.N + i];
        const double u = h[i];
        if (a.batched) write_ucv(a, b, i, u);
        e += u * u;
    }
    const double sum = block_sum(e, red);
    if (threadIdx.x == 0 && n < a.elog_cap) a.elog[(size_t)n * a.B + b] = 0.5 * sum;
}

}  // namespace

extern "C" rom_status rom_state_set_slot(rom_ctx c, rom_state s, int32_t b, const double* u_hist,
                                         const double* y_hist, int32_t clear_health) {
    if (!c || !s || s->ctx != c) return fail(ROM_E_INVALID, "bad ctx/state");
    if (b < 0 || b >= s->B) return fail(ROM_E_INVALID, "slot %d outside [0, %d)", b, s->B);
    if (!u_hist || !y_hist) return fail(ROM_E_INVALID, "u_hist / y_hist is NULL");
    HIPCHK(hipStreamSynchronize(c->stream));
    const size_t N = c->N;
    if (!s->slot_stage) {
        const hipError_t e = hipMalloc((void**)&s->slot_stage, sizeof(double) * 5 * N);
        if (e != hipSuccess) {
            s->slot_stage = nullptr;
            return fail(ROM_E_NOMEM, "slot staging hipMalloc failed: %s", hipGetErrorString(e));
        }
        s->bytes += sizeof(double) * 5 * N;
    }
    HIPCHK(hipMemcpy(s->slot_stage, u_hist, sizeof(double) * 3 * N, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->slot_stage + 3 * N, y_hist, sizeof(double) * 2 * N, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(256), 0, c->stream, s->a, (long long)s->h_step, (int)b,
                       (const double*)s->slot_stage);
    // a one-trajectory CP state with a dense stiffness carries the projections of its
    // level from step to step: form them from the new u^n
    seed_projections(c, step_args(s, s->h_step), c->stream);
    HIPCHK(hipGetLastError());
    if (clear_health) {
        const long long none = LLONG_MAX;
        HIPCHK(hipMemcpyAsync(s->a.bad, &none, sizeof(long long), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return ROM_OK;
}

extern "C" rom_status rom_state_u(rom_ctx c, rom_state s, double* u_dev) {
    if (!c || !s || s->ctx != c || !u_dev) return fail(ROM_E_INVALID, "bad arguments");
    const size_t BN = (size_t)s->B * c->N;
    HIPCHK(hipMemcpyAsync(u_dev, s->a.uring + (size_t)(s->h_step % 3) * BN, sizeof(double) * BN,
                          hipMemcpyDeviceToDevice, c->stream));
    return ROM_OK;
}

// ============================================================== uneven-N batching
//
// rom_step_multi advances many (context, state) pairs together.  Every one-trajectory
// state contributes jobs to four mixed launches per step (k_multi.hip): phase 0 full-form
// terms and SVD first products, phase 1 dense / SVD slab streams and CP projections,
// phase 2 BDF updates and CP scatters, phase 3 Helmholtz applies (with the next CP
// projections), whatever the mix of N, R, formats, stiffness kinds and operator forms.
// Batches (B > 1) run their own kernels (enqueue_step) inside the same captured steps.
// The job tables of a set of pairs (one per parity of the step index: a state's kernels
// take the counter slots of its level's parity) are built and uploaded once and cached
// with their captured graphs; a plan is dropped when one of its states or contexts is
// destroyed, or rebuilt when a workspace, scratch or energy log has moved.

namespace {

constexpr int kMixPhases = 4;

struct MultiPlan {
    std::vector<rom_ctx> ctxs;
    std::vector<rom_state> states;
    std::vector<int> wsgen, sgen;
    std::vector<char> par;                  // level parity of each state at the plan's start
    std::vector<int> batched;               // pairs stepped by their own kernels
    char* dev = nullptr;                    // the job tables
    size_t off[2][kMixPhases] = {};
    int njobs[2][kMixPhases] = {}, blocks[2][kMixPhases] = {};
    size_t lds[2][kMixPhases] = {};
    size_t fin_off[2] = {};                 // closing jobs after an even / odd number of steps
    int nfin = 0;
    // graphs of len steps (index len) from the plan's start parities, without [0] and with
    // [1] the closing kernels at the end
    hipGraphExec_t graph[2][kGraphChunk + 1] = {};
    hipStream_t stream = nullptr;

    ~MultiPlan() {
        for (auto& row : graph)
            for (auto g : row)
                if (g) hipGraphExecDestroy(g);
        if (dev) {
            if (stream) hipStreamSynchronize(stream);
            hipFree(dev);
        }
    }
};

constexpr size_t kMaxPlans = 8;
std::mutex g_plan_mu;
std::vector<MultiPlan*> g_plans;            // most recently used last

// Drop every plan that refers to `obj` (a context or a state about to be destroyed).
void forget_plans(const void* obj) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (size_t q = 0; q < g_plans.size();) {
        MultiPlan* pl = g_plans[q];
        bool hit = false;
        for (size_t r = 0; r < pl->states.size() && !hit; ++r)
            hit = (const void*)pl->states[r] == obj || (const void*)pl->ctxs[r] == obj;
        if (hit) {
            delete pl;
            g_plans.erase(g_plans.begin() + (long)q);
        } else {
            ++q;
        }
    }
}

bool plan_matches(const MultiPlan* pl, int n, const rom_ctx* ctxs, const rom_state* states) {
    if ((int)pl->states.size() != n || pl->stream != ctxs[0]->stream) return false;
    for (int q = 0; q < n; ++q)
        if (pl->ctxs[q] != ctxs[q] || pl->states[q] != states[q] || pl->wsgen[q] != ctxs[q]->ws_gen ||
            pl->sgen[q] != states[q]->sgen || pl->par[q] != (char)(states[q]->h_step & 1))
            return false;
    return true;
}

// The mixed jobs of one-trajectory pair (c, st) for the step from level `lev`, by phase.
void pair_jobs(rom_ctx c, rom_state st, long long lev, std::vector<MixJob> (&ph)[kMixPhases]) {
    const StepArgs sa = step_args(st, lev);
    const WsPlan p = plan_ws(c, 1);
    char* scr = (char*)st->scratch;
    const int diag = c->diagA ? 1 : 0;
    auto add = [&](int phase, MixJob jb) {
        jb.dtype = c->dtype;
        jb.nblk = mix_job_blocks(jb);
        ph[phase].push_back(jb);
    };
    if (c->full) {
        MixJob jb{};
        jb.kind = MIX_FULL;
        jb.f.a = sa;
        jb.f.G = c->Gfull;
        add(0, jb);
    }
    if (c->dense || c->svd) {
        const void* wj = nullptr;
        if (c->svd) {
            MixJob jv{};
            jv.kind = MIX_SVDP;
            jv.v.Ut = c->Ut;
            jv.v.Ut_lo = (const unsigned short*)c->Ut_lo;
            jv.v.sigma = c->sig;
            jv.v.N = c->N;
            jv.v.Np = c->Np;
            jv.v.Rsp = c->Rsp;
            jv.v.u_base = sa.uring;
            jv.v.stepp = sa.step;
            jv.v.slot_stride = c->N;
            jv.v.w = scr + p.svdw_off;
            wj = jv.v.w;
            add(0, jv);
        }
        MixJob jg{};
        jg.kind = MIX_GEMV;
        jg.g = c->svd ? make_gemv_job(c->dtype, c->Vt, c->Vt_lo, c->N, c->Np, c->Rs, wj, sa.uring, sa.step, c->N,
                                      scr + p.part_off, p.nchunk, gemv_tile(c))
                      : make_gemv_job(c->dtype, c->C, c->Clo, c->N, c->Np, c->N, nullptr, sa.uring, sa.step, c->N,
                                      scr + p.part_off, p.nchunk, gemv_tile(c));
        add(1, jg);
        MixJob jb{};
        jb.kind = MIX_BDF;
        jb.mode = diag;
        jb.b.a = sa;
        jb.b.part = scr + p.part_off;
        jb.b.nchunk = p.nchunk;
        jb.b.pb = 1;
        jb.b.nblk = (c->N + 255) / 256;
        add(2, jb);
    } else {
        // with a dense stiffness the projections come from the previous step's Helmholtz
        // kernel (phase 3)
        if (diag) {
            MixJob jp{};
            jp.kind = MIX_PROJ;
            const SkewPairs sk = skew_of(c);
            jp.p.BCt = proj_op(c);
            jp.p.BCt_lo = (const unsigned short*)proj_op_lo(c);
            jp.p.lam = c->lam;
            jp.p.N = c->N;
            jp.p.Np = c->Np;
            jp.p.Rp = c->Rp;
            jp.p.layout = sk.layout;
            jp.p.P = sk.P;
            jp.p.R = sk.R;
            jp.p.u_base = sa.uring;
            jp.p.stepp = sa.step;
            jp.p.slot_stride = c->N;
            jp.p.w = sa.st;
            jp.p.nblk = proj1_blocks(c->Rp, sk);
            add(1, jp);
        }
        MixJob js{};
        js.kind = MIX_SCAT;
        js.mode = diag ? 1 : 2;
        js.s.Af = c->Af;
        js.s.Af_lo = (const unsigned short*)c->Af_lo;
        js.s.N = c->N;
        js.s.Rp = c->Rp;
        js.s.w = sa.st;
        js.s.a = sa;
        js.s.nblk = (c->N + 3) / 4;
        add(2, js);
    }
    if (!diag) {
        MixJob jh{};
        jh.kind = MIX_HELM;
        jh.h = helm_job(c, sa);
        if (c->dense || c->svd) {
            jh.h.np = 0;
            jh.h.Mst = nullptr;
        }
        add(3, jh);
    }
}

// Build and upload the job tables of a set of pairs from their current levels.
rom_status build_plan(MultiPlan* pl, int n, const rom_ctx* ctxs, const rom_state* states) {
    pl->stream = ctxs[0]->stream;
    std::vector<MixJob> ph[2][kMixPhases];
    std::vector<FinJob> fin[2];
    for (int q = 0; q < n; ++q) {
        rom_ctx c = ctxs[q];
        rom_state st = states[q];
        pl->ctxs.push_back(c);
        pl->states.push_back(st);
        pl->wsgen.push_back(c->ws_gen);
        pl->sgen.push_back(st->sgen);
        pl->par.push_back((char)(st->h_step & 1));
        if (st->B != 1) {
            pl->batched.push_back(q);
            continue;
        }
        for (int k = 0; k < 2; ++k) {
            pair_jobs(c, st, st->h_step + k, ph[k]);
            FinJob fj{};
            fj.a = step_args(st, st->h_step + k);      // counter slots of the last level's parity
            fin[k].push_back(fj);
        }
    }
    // blob: tables per parity and phase (block ranges assigned in order), then the
    // closing jobs
    std::vector<char> blob;
    auto put_bytes = [&](const void* src, size_t bytes) {
        const size_t o = (blob.size() + 255) & ~(size_t)255;
        blob.resize(o + bytes);
        if (bytes) memcpy(blob.data() + o, src, bytes);
        return o;
    };
    for (int k = 0; k < 2; ++k)
        for (int f = 0; f < kMixPhases; ++f) {
            int b = 0;
            size_t lds = 0;
            for (auto& jb : ph[k][f]) {
                jb.blk0 = b;
                b += jb.nblk;
                const size_t l = mix_job_lds(jb);
                if (l > lds) lds = l;
            }
            pl->off[k][f] = put_bytes(ph[k][f].data(), sizeof(MixJob) * ph[k][f].size());
            pl->njobs[k][f] = (int)ph[k][f].size();
            pl->blocks[k][f] = b;
            pl->lds[k][f] = lds;
        }
    for (int k = 0; k < 2; ++k) pl->fin_off[k] = put_bytes(fin[k].data(), sizeof(FinJob) * fin[k].size());
    pl->nfin = (int)fin[0].size();
    if (!blob.empty()) {
        HIPCHK(hipMalloc((void**)&pl->dev, blob.size()));
        HIPCHK(hipMemcpy(pl->dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
    }
    return ROM_OK;
}

// Step k of a call (levels h_step + k of every pair).
rom_status multi_enqueue_step(MultiPlan* pl, int64_t k) {
    hipStream_t stream = pl->stream;
    const int par = (int)(k & 1);
    for (int f = 0; f < kMixPhases; ++f)
        launch_mix((const MixJob*)(pl->dev + pl->off[par][f]), pl->njobs[par][f], pl->blocks[par][f], pl->lds[par][f],
                   stream);
    for (int q : pl->batched) TRYS(enqueue_step(pl->ctxs[q], pl->states[q], stream, pl->states[q]->h_step + k));
    HIPCHK(hipGetLastError());
    return ROM_OK;
}

void multi_enqueue_close(MultiPlan* pl, int64_t nsteps) {
    launch_close_group((const FinJob*)(pl->dev + pl->fin_off[nsteps & 1]), pl->nfin, pl->stream);
    for (int q : pl->batched) launch_close(step_args(pl->states[q], pl->states[q]->h_step + nsteps), pl->stream);
}

rom_status multi_graph(MultiPlan* pl, int len, int close, hipGraphExec_t* out) {
    hipGraphExec_t& gx = pl->graph[close][len];
    if (!gx) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
        rom_status cst = ROM_OK;
        for (int k = 0; k < len && cst == ROM_OK; ++k) cst = multi_enqueue_step(pl, k);
        if (cst == ROM_OK && close) multi_enqueue_close(pl, len);
        hipError_t ee = hipStreamEndCapture(pl->stream, &g);
        if (cst != ROM_OK) {
            if (g) hipGraphDestroy(g);
            return cst;
        }
        if (ee != hipSuccess) return fail(ROM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ee));
        hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ie != hipSuccess) {
            gx = nullptr;
            return fail(ROM_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
        }
        ie = hipGraphUpload(gx, pl->stream);
        if (ie != hipSuccess) return fail(ROM_E_DEVICE, "graph upload failed: %s", hipGetErrorString(ie));
    }
    *out = gx;
    return ROM_OK;
}

}  // namespace

extern "C" rom_status rom_step_multi(int32_t n, const rom_ctx* ctxs, const rom_state* states, int64_t nsteps,
                                     int64_t* first_bad_step) {
    if (first_bad_step) *first_bad_step = -1;
    if (n < 1 || !ctxs || !states) return fail(ROM_E_INVALID, "rom_step_multi needs n >= 1 pairs");
    if (nsteps < 0) return fail(ROM_E_INVALID, "nsteps < 0");
    for (int q = 0; q < n; ++q) {
        if (!ctxs[q] || !states[q] || states[q]->ctx != ctxs[q])
            return fail(ROM_E_INVALID, "pair %d: state does not belong to its context", q);
        for (int r = 0; r < q; ++r)
            if (states[r] == states[q]) return fail(ROM_E_INVALID, "state listed twice (pairs %d and %d)", r, q);
    }
    hipStream_t stream = ctxs[0]->stream;
    for (int q = 0; q < n; ++q) HIPCHK(hipStreamSynchronize(ctxs[q]->stream));
    for (int q = 0; q < n; ++q) {
        rom_status st = prepare(ctxs[q], states[q], nsteps);
        if (st != ROM_OK) return st;
    }
    if (nsteps == 0) return ROM_OK;

    // the cached plan of this set of pairs (most recently used last), or a new one
    std::unique_lock<std::mutex> lk(g_plan_mu);
    MultiPlan* pl = nullptr;
    for (size_t q = 0; q < g_plans.size(); ++q)
        if (plan_matches(g_plans[q], n, ctxs, states)) {
            pl = g_plans[q];
            g_plans.erase(g_plans.begin() + (long)q);
            break;
        }
    if (!pl) {
        pl = new MultiPlan();
        rom_status bs = build_plan(pl, n, ctxs, states);
        if (bs != ROM_OK) {
            delete pl;
            return bs;
        }
        if (g_plans.size() >= kMaxPlans) {
            delete g_plans.front();
            g_plans.erase(g_plans.begin());
        }
    }
    g_plans.push_back(pl);

    // (nsteps - 1) / 64 replays of the 64-step graph, then one graph of the rest with the
    // closing kernels
    rom_status status = ROM_OK;
    int64_t left = nsteps;
    while (status == ROM_OK && left > 0) {
        const int len = left > kGraphChunk ? kGraphChunk : (int)left;
        const int close = left <= kGraphChunk ? 1 : 0;
        hipGraphExec_t gx = nullptr;
        status = multi_graph(pl, len, close, &gx);
        if (status == ROM_OK && hipGraphLaunch(gx, stream) != hipSuccess)
            status = fail(ROM_E_DEVICE, "graph launch failed");
        left -= len;
    }
    lk.unlock();
    hipError_t se = hipStreamSynchronize(stream);
    if (status != ROM_OK) return status;
    if (se != hipSuccess) return fail(ROM_E_DEVICE, "rom_step_multi: %s", hipGetErrorString(se));
    long long worst = LLONG_MAX;
    for (int q = 0; q < n; ++q) {
        states[q]->h_step += nsteps;
        states[q]->pending = false;
        long long bad = LLONG_MAX;
        HIPCHK(hipMemcpy(&bad, states[q]->a.bad, sizeof(long long), hipMemcpyDeviceToHost));
        if (bad < worst) worst = bad;
    }
    if (worst != LLONG_MAX) {
        if (first_bad_step) *first_bad_step = worst;
        return fail(ROM_E_NONFINITE, "a trajectory became non-finite at step %lld", worst);
    }
    return ROM_OK;
}

static void forget_plans_of(const void* obj) { forget_plans(obj); }

extern "C" rom_status rom_query(rom_ctx c, rom_state s, int32_t what, int64_t* value) {
    if (!value) return fail(ROM_E_INVALID, "value is NULL");
    switch (what) {
        case 0: if (!c) break; *value = (int64_t)c->bytes; return ROM_OK;
        case 1: if (!s) break; *value = (int64_t)s->bytes; return ROM_OK;
        case 2: if (!c) break; *value = c->N; return ROM_OK;
        case 3: if (!c) break; *value = c->R; return ROM_OK;
        case 4: if (!c) break; *value = c->dtype; return ROM_OK;
        case 5: if (!s) break; *value = s->B; return ROM_OK;
        case 6: if (!s) break; *value = s->h_step; return ROM_OK;
        case 7: if (!c) break; *value = skew_of(c).layout; return ROM_OK;
        case 8: if (!c) break; *value = c->dense ? 0 : c->svd ? 2 : 1; return ROM_OK;
        case 9: if (!c) break; *value = c->Rs; return ROM_OK;
        case 10: {
            if (!s) break;
            long long bad = LLONG_MAX;
            HIPCHK(hipStreamSynchronize(s->ctx->stream));
            HIPCHK(hipMemcpy(&bad, s->a.bad, sizeof(long long), hipMemcpyDeviceToHost));
            *value = bad == LLONG_MAX ? -1 : (int64_t)bad;
            return ROM_OK;
        }
        case 11: if (!s) break; *value = res_usable(s->ctx, s) ? s->ctx->res_G : 0; return ROM_OK;
        default: return fail(ROM_E_INVALID, "unknown query %d", what);
    }
    return fail(ROM_E_INVALID, "query %d needs a %s", what,
                what == 1 || (what >= 5 && what <= 6) || what >= 10 ? "state" : "context");
}

extern "C" int32_t rom_tile_count(int32_t kind) {
    switch (kind) {
        case 0: return dense_gemv_variants();
        case 1: return dense_batched_variants();
        case 2: case 3: return gemm_variants() + mfma_variants();
        case 4: return 2;
        case 5: return 2;
        default: return 0;
    }
}

extern "C" rom_status rom_set_tile(rom_ctx c, int32_t kind, int32_t value) {
    if (!c) return fail(ROM_E_INVALID, "ctx is NULL");
    if (kind < 0 || kind > 5) return fail(ROM_E_INVALID, "unknown kernel kind %d", kind);
    if (value < -1 || value >= rom_tile_count(kind)) return fail(ROM_E_INVALID, "tile index %d out of range", value);
    if (kind == 4 && value == 1 && !c->skew_layout)
        return fail(ROM_E_UNSUPPORTED, "the CP factors have no skew column pairs");
    c->tile[kind] = value;
    c->ws_gen++;   // captured graphs bake tile shapes: force a recapture
    return ROM_OK;
}
