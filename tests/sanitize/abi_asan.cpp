// abi_asan.cpp -- drives the C ABI (include/rom.h) in a build whose host code (the
// runtime in rom_api.hip and this driver) carries AddressSanitizer and
// UndefinedBehaviorSanitizer; the GPU kernels are the library's own (test
// infrastructure).
//
// Without a GPU it exercises the host-side argument checks of every entry point that
// has them.  With a GPU it also runs each operator form through creation, stepping
// (graphs, resident runs, grouped steps), checkpoint/restart, slot replacement,
// evaluation and destruction, checking relations the library documents:
//   - a call of n steps equals calls of a and n - a steps, to the bit;
//   - rom_step_multi equals rom_step on each state alone, to the bit;
//   - rom_nonlinear_noalloc equals rom_nonlinear, to the bit;
//   - rom_state_get after rom_state_set returns what was set;
//   - CP-ALS and ALS-skew run, and rank-deficient factors are reported.
// Prints "mode=gpu" or "mode=host" and exits 0 when every check holds.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rom.h"

namespace {

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (%s)\n", what, rom_last_error() ? rom_last_error() : "");
        ++failures;
    }
}

uint64_t rng = 0x243f6a8885a308d3ull;
double uniform() {   // splitmix64 -> [-1, 1)
    uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
std::vector<double> vec(size_t n, double scale = 1.0) {
    std::vector<double> v(n);
    for (auto& x : v) x = scale * uniform();
    return v;
}

struct Problem {
    int N, R;
    std::vector<double> A, C, lam, Af, Bf, Cf, u0;
};

// Stiffness diag(k^2) (or that plus a small symmetric part), a rough dense tensor or CP
// factors small enough that the trajectory stays bounded.
Problem problem(int N, int R, bool dense_stiffness) {
    Problem p{N, R, {}, {}, {}, {}, {}, {}, {}};
    p.A.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) p.A[(size_t)i * N + i] = (double)(i + 1) * (i + 1);
    if (dense_stiffness)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < i; ++j) p.A[(size_t)i * N + j] = p.A[(size_t)j * N + i] = 0.05 * uniform();
    const double s = 0.3 / N;
    if (R == 0) {
        p.C = vec((size_t)N * N * N, s);
    } else {
        p.lam = vec(R, 1.0);
        p.Af = vec((size_t)N * R, std::sqrt(s));
        p.Bf = vec((size_t)N * R, std::sqrt(s));
        p.Cf = vec((size_t)N * R, std::sqrt(s));
    }
    p.u0 = vec(N, 0.1);
    return p;
}

rom_desc desc(const Problem& p, int dtype, int max_batch) {
    rom_desc d{};
    d.N = p.N;
    d.R = p.R;
    d.nu = 1e-2;
    d.dt = 1e-3;
    d.A = p.A.data();
    d.C = p.C.empty() ? nullptr : p.C.data();
    d.lambda = p.lam.empty() ? nullptr : p.lam.data();
    d.Af = p.Af.empty() ? nullptr : p.Af.data();
    d.Bf = p.Bf.empty() ? nullptr : p.Bf.data();
    d.Cf = p.Cf.empty() ? nullptr : p.Cf.data();
    d.dtype = dtype;
    d.max_batch = max_batch;
    d.stream = nullptr;
    return d;
}

void host_checks() {
    Problem p = problem(12, 8, false);
    rom_ctx ctx = nullptr;
    check(rom_create(nullptr, &ctx) == ROM_E_INVALID, "create(NULL)");
    rom_desc d = desc(p, ROM_FP32, 1);
    d.N = 0;
    check(rom_create(&d, &ctx) == ROM_E_INVALID, "create N = 0");
    d = desc(p, ROM_FP32, 1);
    d.dt = 0.0;
    check(rom_create(&d, &ctx) == ROM_E_INVALID, "create dt = 0");
    d = desc(p, ROM_FP32, 1);
    d.nu = -1.0;
    check(rom_create(&d, &ctx) == ROM_E_INVALID, "create nu < 0");
    d = desc(p, ROM_FP32, 1);
    d.lambda = nullptr;
    check(rom_create(&d, &ctx) == ROM_E_INVALID, "create CP without lambda");
    d = desc(p, ROM_FP32, 1);
    d.dtype = 9;
    check(rom_create(&d, &ctx) != ROM_OK, "create unknown dtype");
    d = desc(p, ROM_FP32, 2);
    d.lambda = d.Af = d.Bf = d.Cf = nullptr;
    std::vector<double> U = vec(12 * 3), sg = vec(3), V = vec(12 * 12 * 3);
    check(rom_create_svd(&d, 3, U.data(), sg.data(), V.data(), &ctx) == ROM_E_UNSUPPORTED, "svd max_batch 2");
    d.max_batch = 1;
    check(rom_create_svd(&d, 0, U.data(), sg.data(), V.data(), &ctx) == ROM_E_INVALID, "svd rank 0");
    check(rom_create_full(&d, nullptr, &ctx) == ROM_E_INVALID, "full without terms");
    std::vector<double> M((size_t)12 * 12, 0.0);
    for (int i = 0; i < 12; ++i) M[(size_t)i * 12 + i] = 1.0;
    M[1] = 0.5;   // not symmetric
    rom_full_terms ft{M.data(), nullptr, nullptr, nullptr, nullptr};
    d = desc(p, ROM_FP32, 1);
    check(rom_create_full(&d, &ft, &ctx) == ROM_E_INVALID, "full with a non-symmetric mass matrix");
    check(rom_cp_als(0, 3, nullptr, nullptr, nullptr, nullptr, 1, nullptr) == ROM_E_INVALID, "als N = 0");
    check(rom_cp_als(4, 3, nullptr, nullptr, nullptr, nullptr, 1, nullptr) == ROM_E_INVALID, "als NULL");
    check(rom_cp_als_skew(4, 0, nullptr, nullptr, nullptr, nullptr, 1, 1, 0.5, nullptr) == ROM_E_INVALID,
          "als-skew P = 0");
    check(rom_cp_als_skew(4, 2, nullptr, nullptr, nullptr, nullptr, 1, 1, 1.0, nullptr) == ROM_E_INVALID,
          "als-skew momentum 1");
    int64_t v = 0;
    check(rom_query(nullptr, nullptr, 2, &v) == ROM_E_INVALID, "query NULL");
    check(rom_step(nullptr, nullptr, 1, nullptr) == ROM_E_INVALID, "step NULL");
    check(rom_nonlinear(nullptr, 1, nullptr, nullptr) == ROM_E_INVALID, "nonlinear NULL");
    check(rom_set_tile(nullptr, 0, 0) == ROM_E_INVALID, "set_tile NULL");
    check(rom_tile_count(0) >= 1 && rom_tile_count(99) == 0, "tile counts");
    rom_destroy(nullptr);
    rom_state_destroy(nullptr);

    // skew column pairs: interleaved (1), blocked (2), broken (0), odd rank and NULL (0)
    const int N = 9, P = 5, R = 2 * P;
    std::vector<double> a = vec(N * P), c = vec(N * P), b = vec(N * P), lp = vec(P);
    std::vector<double> lam(R), Af(N * R), Bf(N * R), Cf(N * R), lamb(R), Afb(N * R), Bfb(N * R), Cfb(N * R);
    for (int q = 0; q < P; ++q) {
        lam[2 * q] = lam[2 * q + 1] = lamb[q] = lamb[P + q] = lp[q];
        for (int i = 0; i < N; ++i) {
            const double ai = a[i * P + q], ci = c[i * P + q], bi = b[i * P + q];
            Af[i * R + 2 * q] = ai, Af[i * R + 2 * q + 1] = ci;
            Bf[i * R + 2 * q] = Bf[i * R + 2 * q + 1] = bi;
            Cf[i * R + 2 * q] = ci, Cf[i * R + 2 * q + 1] = -ai;
            Afb[i * R + q] = ai, Afb[i * R + P + q] = ci;
            Bfb[i * R + q] = Bfb[i * R + P + q] = bi;
            Cfb[i * R + q] = ci, Cfb[i * R + P + q] = -ai;
        }
    }
    check(rom_cp_skew_layout(N, R, lam.data(), Af.data(), Bf.data(), Cf.data()) == 1, "interleaved pairs");
    check(rom_cp_skew_layout(N, R, lamb.data(), Afb.data(), Bfb.data(), Cfb.data()) == 2, "blocked pairs");
    Cf[5] += 1e-3;
    check(rom_cp_skew_layout(N, R, lam.data(), Af.data(), Bf.data(), Cf.data()) == 0, "broken pair");
    check(rom_cp_skew_layout(N, R - 1, lam.data(), Af.data(), Bf.data(), Cf.data()) == 0, "odd rank");
    check(rom_cp_skew_layout(N, R, nullptr, Af.data(), Bf.data(), Cf.data()) == 0, "NULL lambda");
}

// Energies of `steps` levels of a fresh state, stepped in the given chunks.
std::vector<double> stepped(rom_ctx ctx, const std::vector<double>& u0, int batch, const std::vector<int>& chunks) {
    rom_state st = nullptr;
    std::vector<double> E;
    if (rom_state_create(ctx, batch, u0.data(), &st) != ROM_OK) {
        check(false, "state_create");
        return E;
    }
    int64_t total = 0;
    for (int c : chunks) {
        int64_t bad = 0;
        check(rom_step(ctx, st, c, &bad) == ROM_OK && bad == -1, "step");
        total += c;
    }
    E.assign((size_t)(total + 1) * batch, 0.0);
    check(rom_energy(ctx, st, nullptr, E.data()) == ROM_OK, "energy");
    rom_state_destroy(st);
    return E;
}

void gpu_checks() {
    struct Case {
        int N, R, dtype, batch;
        bool dense_stiffness;
    };
    const Case cases[] = {{40, 30, ROM_FP32, 1, false}, {40, 30, ROM_BF16X3, 1, true}, {24, 0, ROM_FP64, 3, true},
                          {33, 20, ROM_BF16, 5, false}, {18, 0, ROM_FP32, 1, false}};
    std::vector<rom_ctx> ctxs;
    std::vector<Problem> probs;
    for (const Case& cs : cases) {
        probs.push_back(problem(cs.N, cs.R, cs.dense_stiffness));
        Problem& p = probs.back();
        rom_desc d = desc(p, cs.dtype, cs.batch);
        rom_ctx ctx = nullptr;
        check(rom_create(&d, &ctx) == ROM_OK, "create");
        ctxs.push_back(ctx);
        std::vector<double> u0;
        for (int b = 0; b < cs.batch; ++b) u0.insert(u0.end(), p.u0.begin(), p.u0.end());
        const auto e1 = stepped(ctx, u0, cs.batch, {70});
        const auto e2 = stepped(ctx, u0, cs.batch, {9, 61});
        check(!e1.empty() && e1.size() == e2.size() &&
                  std::memcmp(e1.data(), e2.data(), e1.size() * sizeof(double)) == 0,
              "step splits agree");
        // evaluation through both entry points
        double *ud = nullptr, *y1 = nullptr, *y2 = nullptr;
        const size_t bytes = sizeof(double) * (size_t)cs.batch * cs.N;
        check(hipMalloc((void**)&ud, bytes) == hipSuccess && hipMalloc((void**)&y1, bytes) == hipSuccess &&
                  hipMalloc((void**)&y2, bytes) == hipSuccess,
              "hipMalloc");
        check(hipMemcpy(ud, u0.data(), bytes, hipMemcpyHostToDevice) == hipSuccess, "upload");
        check(rom_nonlinear(ctx, cs.batch, ud, y1) == ROM_OK, "nonlinear");
        check(rom_nonlinear_noalloc(ctx, cs.batch, ud, y2) == ROM_OK, "nonlinear_noalloc");
        check(hipDeviceSynchronize() == hipSuccess, "sync");
        std::vector<double> h1((size_t)cs.batch * cs.N), h2(h1.size());
        check(hipMemcpy(h1.data(), y1, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
                  hipMemcpy(h2.data(), y2, bytes, hipMemcpyDeviceToHost) == hipSuccess,
              "download");
        check(std::memcmp(h1.data(), h2.data(), bytes) == 0, "noalloc equals nonlinear");
        (void)hipFree(ud);
        (void)hipFree(y1);
        (void)hipFree(y2);
        // checkpoint / restart / slot replacement
        rom_state st = nullptr;
        check(rom_state_create(ctx, cs.batch, u0.data(), &st) == ROM_OK, "state_create");
        check(rom_step(ctx, st, 5, nullptr) == ROM_OK, "step 5");
        std::vector<double> uh((size_t)3 * cs.batch * cs.N), yh((size_t)2 * cs.batch * cs.N);
        int64_t lvl = -1;
        check(rom_state_get(ctx, st, uh.data(), yh.data(), &lvl) == ROM_OK && lvl == 5, "state_get");
        check(rom_state_set(ctx, st, uh.data(), yh.data(), lvl) == ROM_OK, "state_set");
        std::vector<double> uh2(uh.size()), yh2(yh.size());
        check(rom_state_get(ctx, st, uh2.data(), yh2.data(), &lvl) == ROM_OK && uh2 == uh && yh2 == yh,
              "get after set");
        std::vector<double> us((size_t)3 * cs.N, 0.0), ys((size_t)2 * cs.N, 0.0);
        check(rom_state_set_slot(ctx, st, cs.batch - 1, us.data(), ys.data(), 0) == ROM_OK, "set_slot");
        check(rom_step(ctx, st, 20, nullptr) == ROM_OK, "step after set_slot");
        for (int w = 0; w <= 11; ++w) check(rom_query(ctx, st, w, &lvl) == ROM_OK, "query");
        rom_state_destroy(st);
    }

    // grouped steps of the one-trajectory states against stepping each alone
    std::vector<rom_ctx> mc;
    std::vector<rom_state> ms;
    std::vector<std::vector<double>> alone;
    for (size_t q = 0; q < ctxs.size(); ++q) {
        if (cases[q].batch != 1) continue;
        alone.push_back(stepped(ctxs[q], probs[q].u0, 1, {40}));
        rom_state st = nullptr;
        check(rom_state_create(ctxs[q], 1, probs[q].u0.data(), &st) == ROM_OK, "state_create");
        mc.push_back(ctxs[q]);
        ms.push_back(st);
    }
    for (int rep = 0; rep < 2; ++rep) {   // the second call reuses the cached tables
        int64_t bad = 0;
        check(rom_step_multi((int)mc.size(), mc.data(), ms.data(), 20, &bad) == ROM_OK && bad == -1, "step_multi");
    }
    for (size_t q = 0; q < ms.size(); ++q) {
        std::vector<double> E(41);
        check(rom_energy(mc[q], ms[q], nullptr, E.data()) == ROM_OK, "energy");
        check(alone[q].size() == 41 && std::memcmp(E.data(), alone[q].data(), sizeof(double) * 41) == 0,
              "multi equals alone");
    }
    rom_state_destroy(ms.back());   // drops the set's tables; the rest steps on
    ms.pop_back();
    mc.pop_back();
    check(rom_step_multi((int)mc.size(), mc.data(), ms.data(), 3, nullptr) == ROM_OK, "step_multi after destroy");
    for (rom_state s : ms) rom_state_destroy(s);
    for (rom_ctx c : ctxs) rom_destroy(c);

    // ALS: a short fit, and a rank-deficient start reported
    const int N = 10, R = 4;
    std::vector<double> X = vec((size_t)N * N * N), F[3] = {vec(N * R), vec(N * R), vec(N * R)};
    double *Xd = nullptr, *Fd[3] = {nullptr, nullptr, nullptr};
    check(hipMalloc((void**)&Xd, X.size() * sizeof(double)) == hipSuccess, "hipMalloc");
    check(hipMemcpy(Xd, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess, "upload");
    for (int m = 0; m < 3; ++m) {
        check(hipMalloc((void**)&Fd[m], F[m].size() * sizeof(double)) == hipSuccess, "hipMalloc");
        check(hipMemcpy(Fd[m], F[m].data(), F[m].size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess,
              "upload");
    }
    check(rom_cp_als(N, R, Xd, Fd[0], Fd[1], Fd[2], 3, nullptr) == ROM_OK, "cp_als");
    check(rom_cp_als_skew(N, R / 2, Xd, Fd[0], Fd[1], Fd[2], 2, 2, 0.5, nullptr) == ROM_OK, "cp_als_skew");
    std::vector<double> z((size_t)N * R, 0.0);
    check(hipMemcpy(Fd[1], z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess, "upload");
    check(rom_cp_als(N, R, Xd, Fd[0], Fd[1], Fd[2], 1, nullptr) == ROM_E_INVALID, "rank-deficient reported");
    (void)hipFree(Xd);
    for (double* f : Fd) (void)hipFree(f);
}

}  // namespace

int main() {
    host_checks();
    int ndev = 0;
    const bool gpu = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
    std::printf("mode=%s\n", gpu ? "gpu" : "host");
    std::fflush(stdout);
    if (gpu) gpu_checks();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("abi sanitizer run: all checks hold\n");
    std::fflush(stdout);     // before the runtimes' own teardown at exit
    return 0;
}
