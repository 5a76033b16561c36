// reg_kernels.hip -- register-resident variant of the fused step kernel.
//
// Same scheme and phases as step_kernel (kernels.hip), but each thread keeps
// the step-invariant coefficients of its branches (alpha, beta, F, 1/d') and
// the eliminated right-hand side in VGPRs for the whole epoch.  A thread owns
// up to S branches of at most L CVs; every round of the level sweep uses one
// register slot j on all of its threads (the host assigns them), so the
// per-slot register arrays are indexed with compile-time constants.  Per CV
// and step the LDS traffic is one load of V, one of the point/nonlinear
// current, and one store of the new V; branches exchange only their end
// values: a child leaves F * rhs' of its proximal CV in R at that CV's slot
// for the parent's elimination, and the parent's new V is read from LDS by
// the children's substitution.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"
#include "kernels.hpp"

namespace arbmi {

namespace {

using namespace dev;

template <int S, int L>
struct Regs {
    double A[S][L], B[S][L], F[S][L], D[S][L], R[S][L];
};

// Elimination of one branch held in register slot J, distal to proximal.
template <int J, int S, int L>
__device__ inline void elim(Regs<S, L>& g, const double* sV, double* sR, int base, int w, int len, double csum) {
    double v[L], rn[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int sl = base + min(k, len - 1) * w;
        v[k] = sV[sl];
        rn[k] = sR[sl];
    }
    double acc = 0.0;
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
        if (k < len) {
            const double t = g.A[J][k] * v[k] + g.B[J][k] + rn[k];
            const double fnext = (k + 1 < L) ? g.F[J][(k + 1 < L) ? k + 1 : k] : 0.0;
            acc = (k == len - 1) ? t - csum : t - fnext * acc;
            g.R[J][k] = acc;
        }
    }
    sR[base] = g.F[J][0] * g.R[J][0];  // contribution to the parent's elimination
}

// Substitution of one branch held in register slot J, proximal to distal.
template <int J, int S, int L>
__device__ inline void subst(Regs<S, L>& g, double* sV, double* sR, int base, int w, int len, double x) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
        if (k < len) {
            x = g.R[J][k] * g.D[J][k] - g.F[J][k] * x;
            sV[base + k * w] = x;
        }
    }
    sR[base] = 0.0;  // clear the contribution left for the parent
}

template <int J, int S, int L>
__device__ inline void load_slot(Regs<S, L>& g, const StepArgs& a, const PackDesc& pk, const RoundDesc* s_rd,
                                 const TaskDesc* s_tk, int r, int tid) {
    if (r < 0) {
#pragma unroll
        for (int k = 0; k < L; ++k) g.A[J][k] = g.B[J][k] = g.F[J][k] = g.D[J][k] = g.R[J][k] = 0.0;
        return;
    }
    const RoundDesc R = s_rd[r];
    const int i = round_index(R, tid);
    const TaskDesc t = s_tk[R.task0 + i];
    const int64_t base = pk.slot0 + R.slot0 + i;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int64_t sl = base + int64_t(min(k, t.len - 1)) * R.w;
        g.A[J][k] = a.alpha[sl];
        g.B[J][k] = a.beta[sl];
        g.F[J][k] = a.F[sl];
        g.D[J][k] = a.invd[sl];
        g.R[J][k] = 0.0;
    }
}

template <int T, int S, int L>
__global__ void __launch_bounds__(T) reg_step_kernel(StepArgs a) {
    extern __shared__ double lds[];
    const int p = blockIdx.x;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    // ---- LDS layout (coefficient mode 2 layout of pack_lds_bytes) ----
    double* sV = lds;
    double* sR = sV + ns;
    double* sg = sR + ns;
    double* sm = sg + pk.nsyn;
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    RoundDesc* s_rd = reinterpret_cast<RoundDesc*>(sn + pk.nhh);
    TaskDesc* s_tk = reinterpret_cast<TaskDesc*>(s_rd + pk.nrd);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(s_tk + pk.ntk);
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);

    const double* g_gna = a.hh_gna + pk.hh0;
    const double* g_gk = a.hh_gk + pk.hh0;
    const double* g_se = a.syn_e + pk.syn0;
    const double* g_sdec = a.syn_decay + pk.syn0;

    for (int i = tid; i < ns; i += T) {
        sV[i] = a.V[pk.slot0 + i];
        sR[i] = 0.0;
    }
    for (int i = tid; i < pk.nsyn; i += T) sg[i] = a.syn_g[pk.syn0 + i];
    for (int i = tid; i < pk.nhh; i += T) {
        sm[i] = a.hh_m[pk.hh0 + i];
        sh[i] = a.hh_h[pk.hh0 + i];
        sn[i] = a.hh_n[pk.hh0 + i];
    }
    for (int i = tid; i < pk.nrd; i += T) s_rd[i] = a.rd[pk.rd0 + i];
    for (int i = tid; i < pk.ntk; i += T) s_tk[i] = a.tk[pk.tk0 + i];
    for (int i = tid; i < pk.nnl; i += T) s_nl[i] = a.nl[pk.nl0 + i];
    for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_slot[pk.ch0 + i];

    int64_t step0 = a.step0;
    int32_t bucket = a.bucket;
    if (a.epoch_ptr) {
        const int64_t e = *a.epoch_ptr;
        step0 = e * a.nsteps;
        bucket = int32_t(e % a.n_buckets);
    }
    const int64_t bk_base = (int64_t(bucket) * a.n_packs + p);
    const uint64_t* ev = a.bk_ev + bk_base * a.bk_cap;
    int32_t ncur = 0, nend = 0;
    int64_t xcur = 0;
    uint64_t nkey = ~uint64_t(0);
    int64_t xstep = INT64_MAX;
    if (tid == 0) {
        xcur = a.pk_xcur[p];
        ncur = a.pk_ncur[p];
        const uint32_t c = a.bk_cnt[bk_base];
        nend = int32_t(c < uint32_t(a.bk_cap) ? c : uint32_t(a.bk_cap));
        if (ncur < nend) nkey = ev[ncur];
        if (xcur < pk.xe1) xstep = a.xe_step[xcur];
    }
    const int soma = (tid < pk.ncell) ? a.pc_soma[pk.cell0 + tid] : -1;
    double vold = 0.0;
    __syncthreads();

    // this thread's round in each register slot, then its coefficients
    int myr[S];
#pragma unroll
    for (int j = 0; j < S; ++j) myr[j] = -1;
    for (int r = 0; r < pk.nrd; ++r) {
        const RoundDesc R = s_rd[r];
        if (round_index(R, tid) >= 0) {
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (R.j == j) myr[j] = r;
        }
    }
    Regs<S, L> g;
    load_slot<0, S, L>(g, a, pk, s_rd, s_tk, myr[0], tid);
    if constexpr (S > 1) load_slot<1, S, L>(g, a, pk, s_rd, s_tk, myr[1], tid);
    if constexpr (S > 2) load_slot<2, S, L>(g, a, pk, s_rd, s_tk, myr[2], tid);

    for (int s = 0; s < a.nsteps; ++s) {
        const int64_t n = step0 + s;

        // A: events due at the start of step n (network, then external)
        if (tid == 0) {
            while (int64_t(nkey >> 32) == n) {
                const uint32_t r = uint32_t(nkey);
                sg[a.cr_syn[r]] += a.cr_w[r];
                ++ncur;
                nkey = (ncur < nend) ? ev[ncur] : ~uint64_t(0);
            }
            while (xstep == n) {
                sg[a.xe_syn[xcur]] += a.xe_w[xcur];
                ++xcur;
                xstep = (xcur < pk.xe1) ? a.xe_step[xcur] : INT64_MAX;
            }
        }
        __syncthreads();

        if (a.rec_V) {  // state entering the step, for the adjoint
            double* rv = a.rec_V + int64_t(s) * a.n_slots_total + pk.slot0;
            for (int i = tid; i < ns; i += T) rv[i] = sV[i];
            double* rm = a.rec_m + int64_t(s) * a.n_hh_total + pk.hh0;
            double* rh = a.rec_h + int64_t(s) * a.n_hh_total + pk.hh0;
            double* rn = a.rec_n + int64_t(s) * a.n_hh_total + pk.hh0;
            for (int i = tid; i < pk.nhh; i += T) {
                rm[i] = sm[i];
                rh[i] = sh[i];
                rn[i] = sn[i];
            }
            double* rg = a.rec_g + int64_t(s) * a.n_syn_total + pk.syn0;
            for (int i = tid; i < pk.nsyn; i += T) rg[i] = sg[i];
        }

        // B: nonlinear and point currents at V^n, stored as -I in R
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double v = sV[d.slot];
            double I = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = sm[q], h = sh[q], x = sn[q];
                I += g_gna[q] * (m * m * m * h) * (v - kENa);
                I += g_gk[q] * (x * x * x * x) * (v - kEK);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                I += sg[q] * (v - g_se[q]);
            }
            sR[d.slot] = -I;
        }
        if (soma >= 0) vold = sV[soma];
        if (pk.nic > 0) {
            __syncthreads();
            if (tid == 0)
                for (int q = pk.ic0; q < pk.ic0 + pk.nic; ++q)
                    if (a.ic_on[q] <= n && n < a.ic_off[q]) sR[a.ic_slot[q]] += a.ic_amp[q];
        }
        __syncthreads();

        // C: elimination, deepest rounds first
        for (int r = 0; r < pk.nrd; ++r) {
            const RoundDesc R = s_rd[r];
            const int i = round_index(R, tid);
            if (i >= 0) {
                const TaskDesc t = s_tk[R.task0 + i];
                double csum = 0.0;
                for (int c = 0; c < t.nch; ++c) csum += sR[s_ch[t.ch0 + c]];
                const int base = R.slot0 + i;
                const int j = __builtin_amdgcn_readfirstlane(R.j);
                if (j == 0) elim<0, S, L>(g, sV, sR, base, R.w, t.len, csum);
                if constexpr (S > 1) if (j == 1) elim<(S > 1 ? 1 : 0), S, L>(g, sV, sR, base, R.w, t.len, csum);
                if constexpr (S > 2) if (j == 2) elim<(S > 2 ? 2 : 0), S, L>(g, sV, sR, base, R.w, t.len, csum);
            }
            __syncthreads();
        }

        // D: substitution, shallowest rounds first
        for (int r = pk.nrd - 1; r >= 0; --r) {
            const RoundDesc R = s_rd[r];
            const int i = round_index(R, tid);
            if (i >= 0) {
                const TaskDesc t = s_tk[R.task0 + i];
                const double x = (t.par >= 0) ? sV[t.par] : 0.0;
                const int base = R.slot0 + i;
                const int j = __builtin_amdgcn_readfirstlane(R.j);
                if (j == 0) subst<0, S, L>(g, sV, sR, base, R.w, t.len, x);
                if constexpr (S > 1) if (j == 1) subst<(S > 1 ? 1 : 0), S, L>(g, sV, sR, base, R.w, t.len, x);
                if constexpr (S > 2) if (j == 2) subst<(S > 2 ? 2 : 0), S, L>(g, sV, sR, base, R.w, t.len, x);
            }
            __syncthreads();
        }

        // E: states with V^{n+1}, threshold, probes
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            if (d.hh >= 0) {
                const int q = d.hh;
                const Rates rt = hh_rates(sV[d.slot]);
                sm[q] = gate_step(sm[q], rt.am, rt.bm, a.dt);
                sh[q] = gate_step(sh[q], rt.ah, rt.bh, a.dt);
                sn[q] = gate_step(sn[q], rt.an, rt.bn, a.dt);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                sg[q] *= g_sdec[q];
            }
        }
        if (soma >= 0) {
            const double vnew = sV[soma];
            if (vold < a.threshold && vnew >= a.threshold) {
                const uint32_t pos = atomicAdd(&a.ctr->sp_count, 1u);
                if (pos < a.sp_cap) {
                    a.sp_gid[pos] = uint32_t(a.pc_gid[pk.cell0 + tid]);
                    a.sp_step[pos] = n + 1;
                    a.sp_t[pos] = (double(n) + (a.threshold - vold) / (vnew - vold)) * a.dt;
                } else {
                    atomicOr(&a.ctr->flags, kFlagSpikeOverflow);
                }
            }
        }
        if (a.trace) {
            const int64_t col = n - a.trace_step0;
            if (col >= 0 && col < a.trace_cap)
                for (int j = tid; j < pk.npr; j += T)
                    a.trace[int64_t(a.pr_id[pk.pr0 + j]) * a.trace_cap + col] = sV[a.pr_slot[pk.pr0 + j]];
        }
        __syncthreads();
    }

    if (a.rec_V) {
        double* rv = a.rec_V + int64_t(a.nsteps) * a.n_slots_total + pk.slot0;
        for (int i = tid; i < ns; i += T) rv[i] = sV[i];
    }
    for (int i = tid; i < ns; i += T) a.V[pk.slot0 + i] = sV[i];
    for (int i = tid; i < pk.nsyn; i += T) a.syn_g[pk.syn0 + i] = sg[i];
    for (int i = tid; i < pk.nhh; i += T) {
        a.hh_m[pk.hh0 + i] = sm[i];
        a.hh_h[pk.hh0 + i] = sh[i];
        a.hh_n[pk.hh0 + i] = sn[i];
    }
    if (tid == 0) {
        a.pk_xcur[p] = xcur;
        a.pk_ncur[p] = ncur;
        if (a.epoch_end) a.bk_cnt[bk_base] = 0u;
    }
}

template <int T, int S, int L>
hipError_t launch_reg(const StepArgs& a, int lds, int n_packs, hipStream_t st) {
    hipLaunchKernelGGL((reg_step_kernel<T, S, L>), dim3(n_packs), dim3(T), lds, st, a);
    return hipGetLastError();
}

template <int T, int S, int L>
void allow_lds(int lds_max) {
    const void* f = reinterpret_cast<const void*>(&reg_step_kernel<T, S, L>);
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
}

template <int T>
hipError_t launch_reg_T(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.reg_len == 8) {
        switch (cfg.reg_slots) {
            case 1: return launch_reg<T, 1, 8>(a, cfg.lds_bytes, n_packs, st);
            case 2: return launch_reg<T, 2, 8>(a, cfg.lds_bytes, n_packs, st);
            case 3: return launch_reg<T, 3, 8>(a, cfg.lds_bytes, n_packs, st);
            default: break;
        }
    } else if (cfg.reg_len == 16 && cfg.reg_slots == 1) {
        return launch_reg<T, 1, 16>(a, cfg.lds_bytes, n_packs, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t prepare_reg_kernels(int lds_max) {
    allow_lds<64, 1, 8>(lds_max);
    allow_lds<64, 2, 8>(lds_max);
    allow_lds<64, 3, 8>(lds_max);
    allow_lds<64, 1, 16>(lds_max);
    allow_lds<128, 1, 8>(lds_max);
    allow_lds<128, 2, 8>(lds_max);
    allow_lds<128, 3, 8>(lds_max);
    allow_lds<128, 1, 16>(lds_max);
    allow_lds<256, 1, 8>(lds_max);
    allow_lds<256, 2, 8>(lds_max);
    allow_lds<256, 3, 8>(lds_max);
    allow_lds<256, 1, 16>(lds_max);
    return hipSuccess;
}

hipError_t launch_reg_step(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    switch (cfg.block_threads) {
        case 64: return launch_reg_T<64>(a, cfg, n_packs, st);
        case 128: return launch_reg_T<128>(a, cfg, n_packs, st);
        case 256: return launch_reg_T<256>(a, cfg, n_packs, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace arbmi
