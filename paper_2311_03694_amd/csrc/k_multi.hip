// k_multi.hip -- one launch per step phase over a heterogeneous work table: the
// one-trajectory states of rom_step_multi, whatever their N, CP rank, number format,
// stiffness kind (diagonal or dense) and operator form (dense tensor, CP factors, SVD
// form, full form with mass matrix and zeroth-mode terms), advance together.  Block q of a
// launch runs block q - blk0 of the job whose block range holds it; the job's kind and
// format select the body (kbody.h) that the kernels of a single state run, so a state
// gives the same results to the bit alone and in a mix.
#include "kbody.h"

namespace rom {

namespace {

template <int DT>
__device__ __forceinline__ void mix_body(const MixJob& jb, int blk) {
    typedef typename Store<DT>::T T;
    typedef typename Store<DT>::Acc Acc;
    constexpr int V = 16 / (int)sizeof(T);
    switch (jb.kind) {
        case MIX_GEMV:
            dense_gemv_body<DT, V, 4, 256>(jb.g, blk);
            break;
        case MIX_PROJ:
            cp_proj_any_body<DT, V, 4>(jb.p, blk);
            break;
        case MIX_BDF: {
            const long long n = *jb.b.a.step;
            if (jb.mode == 1) {
                if (blk == 0) close_and_advance(jb.b.a, n, jb.nblk);
                bdf_partials_body<Acc, true>(jb.b.a, n, reinterpret_cast<const Acc*>(jb.b.part), jb.b.nchunk, jb.b.pb,
                                             blk, 0, jb.nblk);
            } else {
                bdf_partials_body<Acc, false>(jb.b.a, n, reinterpret_cast<const Acc*>(jb.b.part), jb.b.nchunk, jb.b.pb,
                                              blk, 0, jb.nblk);
            }
            break;
        }
        case MIX_SCAT: {
            const long long n = *jb.s.a.step;
            if (jb.mode == 1) {
                if (blk == 0) close_and_advance(jb.s.a, n, jb.nblk);
                cp_scatter1_body<DT, V, 8, 1>(jb.s, nullptr, blk, n);
            } else {
                cp_scatter1_body<DT, V, 8, 2>(jb.s, nullptr, blk, n);
            }
            break;
        }
        case MIX_HELM: {
            const long long n = *jb.h.a.step;
            if (blk == 0) close_and_advance(jb.h.a, n, jb.h.nh);
            if (jb.h.a.N % 2 == 0) helm_proj_body<DT, true>(jb.h, n, blk);
            else helm_proj_body<DT, false>(jb.h, n, blk);
            break;
        }
        case MIX_SVDP:
            svd_proj_body<DT, V, 4>(jb.v, blk);
            break;
        default:
            full_terms_body(jb.f.a, jb.f.G, blk, 0);
            break;
    }
}

__global__ __launch_bounds__(256) void k_mix(const MixJob* __restrict__ jobs, int njobs) {
    const int p = find_job(jobs, njobs, (int)blockIdx.x);
    const MixJob& jb = jobs[p];
    const int blk = (int)blockIdx.x - jb.blk0;
    switch (jb.dtype) {
        case DT_F64: mix_body<DT_F64>(jb, blk); break;
        case DT_F32: mix_body<DT_F32>(jb, blk); break;
        case DT_BF16: mix_body<DT_BF16>(jb, blk); break;
        default: mix_body<DT_BF16X3>(jb, blk); break;
    }
}

// The staged coefficient image of a format (kdot.h), and the projections' second image of
// -u for the BF16 formats.
size_t lds_u(int dt, int Np) {
    switch (dt) {
        case DT_F64: return LdsU<DT_F64>::bytes(Np);
        case DT_F32: return LdsU<DT_F32>::bytes(Np);
        case DT_BF16: return LdsU<DT_BF16>::bytes(Np);
        default: return LdsU<DT_BF16X3>::bytes(Np);
    }
}
size_t acc_size(int dt) { return dt == DT_F64 ? 8 : 4; }
size_t proj_lds_of(int dt, int Np) { return (dt == DT_BF16 || dt == DT_BF16X3 ? 2 : 1) * lds_u(dt, Np); }

}  // namespace

int mix_job_blocks(const MixJob& jb) {
    switch (jb.kind) {
        case MIX_GEMV: return jb.g.nblk;
        case MIX_PROJ: return jb.p.nblk;
        case MIX_BDF: return jb.b.nblk;
        case MIX_SCAT: return jb.s.nblk;
        case MIX_HELM: return jb.h.nh + jb.h.np;
        case MIX_SVDP: return (jb.v.Rsp + 3) / 4;
        default: return (jb.f.a.N + 3) / 4;              // four rows per 256-thread block
    }
}

size_t mix_job_lds(const MixJob& jb) {
    switch (jb.kind) {
        case MIX_GEMV: return lds_u(jb.dtype, jb.g.Np) + (jb.g.wj ? acc_size(jb.dtype) * (size_t)jb.g.J : 0);
        case MIX_PROJ: return proj_lds_of(jb.dtype, jb.p.Np);
        case MIX_BDF: return 0;
        case MIX_SCAT: return acc_size(jb.dtype) * (size_t)jb.s.Rp;
        case MIX_HELM: {
            const size_t h = sizeof(double) * (size_t)jb.h.a.N, q = jb.h.np ? proj_lds_of(jb.dtype, jb.h.a.Np) : 0;
            return h > q ? h : q;
        }
        case MIX_SVDP: return lds_u(jb.dtype, jb.v.Np);
        default: return sizeof(double) * 2 * (size_t)jb.f.a.Np;
    }
}

void launch_mix(const MixJob* jobs_dev, int njobs, int blocks, size_t lds, hipStream_t s) {
    if (njobs > 0 && blocks > 0) hipLaunchKernelGGL(k_mix, dim3((unsigned)blocks), dim3(256), lds, s, jobs_dev, njobs);
}

}  // namespace rom
