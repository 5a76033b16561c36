// reg_kernels.hip -- register-resident variant of the fused step kernel.
//
// Same scheme and phases as step_kernel (kernels.hip): events, point
// currents, elimination by rounds (deepest first), substitution, states and
// threshold.  Here each thread holds, for the whole launch, everything about
// its branches that does not change between steps: the step coefficients
// (alpha, F = u/d', 1/d'), the LDS offsets of the branch's CVs, of its
// parent's CV and of its children's proximal CVs.  A thread owns up to S
// branches of at most L CVs; the host gives every round one register slot j
// on all of its threads, so the per-slot arrays are indexed with
// compile-time constants.  The rounds themselves need no descriptor loads.
// The kernel does not record states for the adjoint (the host refuses that).
//
// LDS keeps V and R (the right-hand side) as interleaved pairs, so one
// 128-bit load brings both operands of a CV; between a branch's elimination
// and its substitution its V entries hold rhs'/d'.  R starts every step as beta
// (the step-invariant part of the right-hand side); the point-current pass
// writes beta - I at the CVs with currents, a branch's elimination leaves
// F * rhs' of its proximal CV in that CV's R for the parent and its
// substitution puts beta back.  A branch shorter than L is padded: the pad
// CVs read a pair of zeros and carry the children's sum through unchanged
// (F = -1, and +1 at the first pad), their results go to a discard pair.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"
#include "kernels.hpp"

namespace arbmi {

namespace {

using namespace dev;

__device__ __forceinline__ double2 ld_pair(const char* vr, int off) {
    return *reinterpret_cast<const double2*>(vr + off);
}
__device__ __forceinline__ double ld_V(const char* vr, int off) { return *reinterpret_cast<const double*>(vr + off); }
__device__ __forceinline__ double ld_R(const char* vr, int off) {
    return *reinterpret_cast<const double*>(vr + off + 8);
}
__device__ __forceinline__ void st_V(char* vr, int off, double x) { *reinterpret_cast<double*>(vr + off) = x; }
__device__ __forceinline__ void st_R(char* vr, int off, double x) { *reinterpret_cast<double*>(vr + off + 8) = x; }

// The registers of one branch slot.  Offsets are bytes into the pair array.
template <int L>
struct Slot {
    double A[L], F[L], D[L];        // alpha, F (pads: +1 then -1), 1/d' (pads: 0)
    double B0;                      // beta of the proximal CV
    int ea[L];                      // pairs of the CVs (pads: the zero pair)
    int r;                          // round of the branch, -1 if the slot is empty
    int len;
    int par;                        // pair of the parent's CV (zero pair at a soma)
    int c0, c1;                     // pairs of the first two children (zero pair if fewer)
    int cx0, ncx;                   // further children: s_ch[cx0 .. cx0 + ncx)
};

// Elimination of one branch, distal to proximal:
// rhs'_k = alpha_k V_k + R_k - F_{k+1} rhs'_{k+1}, the distal CV taking the
// children's contributions instead of the last term.  V_k is not read again
// before the substitution writes its new value, so rhs'_k / d'_k waits there.
template <int L>
__device__ __forceinline__ void elim(const Slot<L>& g, char* vr, const int32_t* s_ch, int discard) {
    double2 p[L];
#pragma unroll
    for (int k = 0; k < L; ++k) p[k] = ld_pair(vr, g.ea[k]);
    double csum = ld_R(vr, g.c0) + ld_R(vr, g.c1);
    for (int q = 0; q < g.ncx; ++q) csum += ld_R(vr, 16 * s_ch[g.cx0 + q]);
    double acc = (g.len == L) ? csum : -csum;
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
        const double t = g.A[k] * p[k].x + p[k].y;
        const double r = (k == L - 1) ? t - acc : t - g.F[(k + 1 < L) ? k + 1 : k] * acc;
        st_V(vr, (k == 0 || k < g.len) ? g.ea[k] : discard, r * g.D[k]);
        acc = r;
    }
    st_R(vr, g.ea[0], g.F[0] * acc);  // contribution to the parent's elimination
}

// Substitution of one branch, proximal to distal: V_k = rhs'_k/d'_k - F_k V_{k-1}
// (V_{-1} the parent's CV); then beta back into R.
template <int L>
__device__ __forceinline__ void subst(const Slot<L>& g, char* vr, int discard) {
    double y[L];
#pragma unroll
    for (int k = 0; k < L; ++k) y[k] = ld_V(vr, g.ea[k]);
    double x = ld_V(vr, g.par);
#pragma unroll
    for (int k = 0; k < L; ++k) {
        x = y[k] - g.F[k] * x;
        st_V(vr, (k == 0 || k < g.len) ? g.ea[k] : discard, x);
    }
    st_R(vr, g.ea[0], g.B0);
}

// Fill slot g with the branch this thread takes in round r of the pack (an
// empty slot if r < 0).  Branch-free: an empty slot reads valid entries of
// the pack and keeps neutral values.
template <int L>
__device__ __forceinline__ void load_slot(Slot<L>& g, const StepArgs& a, const PackDesc& pk, int r, int tid,
                                          int zero) {
    const bool has = r >= 0;
    const RoundDesc R = a.rd[pk.rd0 + (has ? r : 0)];
    const int i = has ? round_index(R, tid) : 0;
    const TaskDesc t = a.tk[pk.tk0 + (has ? R.task0 + i : 0)];
    const int len = has ? t.len : 1;
    const int base = has ? R.slot0 + i : 0;
    const int w = has ? R.w : 0;
    g.r = has ? r : -1;
    g.len = len;
    g.par = (has && t.par >= 0) ? 16 * t.par : zero;
    g.c0 = zero;
    g.c1 = zero;
    if (has && t.nch > 0) g.c0 = 16 * a.ch_slot[pk.ch0 + t.ch0];
    if (has && t.nch > 1) g.c1 = 16 * a.ch_slot[pk.ch0 + t.ch0 + 1];
    g.cx0 = t.ch0 + 2;
    g.ncx = has ? max(0, t.nch - 2) : 0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const bool real = has && k < len;
        const int loc = base + min(k, len - 1) * w;
        const int64_t sl = pk.slot0 + loc;
        const double al = a.alpha[sl], f = a.F[sl], dv = a.invd[sl];
        g.ea[k] = real ? 16 * loc : zero;
        g.A[k] = real ? al : 0.0;
        g.D[k] = real ? dv : 0.0;
        g.F[k] = real ? f : (k == len ? 1.0 : -1.0);
    }
    const double b0 = a.beta[pk.slot0 + base];
    g.B0 = has ? b0 : 0.0;
}

// Waves per SIMD the registers allow without spilling: three for one slot
// of 8 CVs, two for two such slots, one otherwise.
template <int T, int S, int L>
__global__ void __launch_bounds__(T, (S * L <= 8) ? 3 : (S == 2 && L == 8 ? 2 : 1)) reg_step_kernel(StepArgs a) {
    extern __shared__ __align__(16) char lds_raw[];
    const int p = blockIdx.x + a.pack0;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    // ---- LDS layout (the mode-3 layout of pack_lds_bytes) ----
    char* vr = lds_raw;                                        // (V, R) pairs [ns + 2]
    const int zero = 16 * ns, discard = 16 * (ns + 1);
    double* sg = reinterpret_cast<double*>(vr + 16 * (ns + 2));
    double* s_se = sg + pk.nsyn;
    double* s_sdec = s_se + pk.nsyn;
    double* sm = s_sdec + pk.nsyn;
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    double* s_gna = sn + pk.nhh;
    double* s_gk = s_gna + pk.nhh;
    double* s_nlb = s_gk + pk.nhh;                             // beta of each nonlinear CV
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(s_nlb + pk.nnl);
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);

    for (int i = tid; i < ns; i += T) {
        st_V(vr, 16 * i, a.V[pk.slot0 + i]);
        st_R(vr, 16 * i, a.beta[pk.slot0 + i]);
    }
    if (tid < 2) {
        st_V(vr, zero + 16 * tid, 0.0);
        st_R(vr, zero + 16 * tid, 0.0);
    }
    for (int i = tid; i < pk.nsyn; i += T) {
        sg[i] = a.syn_g[pk.syn0 + i];
        s_se[i] = a.syn_e[pk.syn0 + i];
        s_sdec[i] = a.syn_decay[pk.syn0 + i];
    }
    for (int i = tid; i < pk.nhh; i += T) {
        sm[i] = a.hh_m[pk.hh0 + i];
        sh[i] = a.hh_h[pk.hh0 + i];
        sn[i] = a.hh_n[pk.hh0 + i];
        s_gna[i] = a.hh_gna[pk.hh0 + i];
        s_gk[i] = a.hh_gk[pk.hh0 + i];
    }
    for (int i = tid; i < pk.nnl; i += T) {
        const NlDesc d = a.nl[pk.nl0 + i];
        s_nl[i] = d;
        s_nlb[i] = a.beta[pk.slot0 + d.slot];
    }
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
    const int soma = (tid < pk.ncell) ? 16 * a.pc_soma[pk.cell0 + tid] : -1;
    double vold = 0.0;

    // this thread's round in each register slot, then its branches
    int myr[S];
#pragma unroll
    for (int j = 0; j < S; ++j) myr[j] = -1;
    for (int r = 0; r < pk.nrd; ++r) {
        const RoundDesc R = a.rd[pk.rd0 + r];
        if (round_index(R, tid) >= 0) {
#pragma unroll
            for (int j = 0; j < S; ++j)
                if (R.j == j) myr[j] = r;
        }
    }
    Slot<L> g0, g1, g2;
    load_slot<L>(g0, a, pk, myr[0], tid, zero);
    if constexpr (S > 1) load_slot<L>(g1, a, pk, myr[1], tid, zero);
    if constexpr (S > 2) load_slot<L>(g2, a, pk, myr[2], tid, zero);
    __syncthreads();

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

        // B: R = beta - I at the CVs with nonlinear and point currents (V^n)
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double v = ld_V(vr, 16 * d.slot);
            double I = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = sm[q], h = sh[q], x = sn[q];
                I += s_gna[q] * (m * m * m * h) * (v - kENa);
                I += s_gk[q] * (x * x * x * x) * (v - kEK);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                I += sg[q] * (v - s_se[q]);
            }
            st_R(vr, 16 * d.slot, s_nlb[j] - I);
        }
        if (soma >= 0) vold = ld_V(vr, soma);
        if (pk.nic > 0) {
            __syncthreads();
            if (tid == 0)
                for (int q = pk.ic0; q < pk.ic0 + pk.nic; ++q)
                    if (a.ic_on[q] <= n && n < a.ic_off[q]) {
                        const int o = 16 * a.ic_slot[q];
                        st_R(vr, o, ld_R(vr, o) + a.ic_amp[q]);
                    }
        }
        __syncthreads();

        // C: elimination, deepest rounds first
        for (int r = 0; r < pk.nrd; ++r) {
            if (g0.r == r) elim<L>(g0, vr, s_ch, discard);
            if constexpr (S > 1) {
                if (g1.r == r) elim<L>(g1, vr, s_ch, discard);
            }
            if constexpr (S > 2) {
                if (g2.r == r) elim<L>(g2, vr, s_ch, discard);
            }
            __syncthreads();
        }

        // D: substitution, shallowest rounds first
        for (int r = pk.nrd - 1; r >= 0; --r) {
            if (g0.r == r) subst<L>(g0, vr, discard);
            if constexpr (S > 1) {
                if (g1.r == r) subst<L>(g1, vr, discard);
            }
            if constexpr (S > 2) {
                if (g2.r == r) subst<L>(g2, vr, discard);
            }
            __syncthreads();
        }

        // E: states with V^{n+1}, threshold, probes
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            if (d.hh >= 0) {
                const int q = d.hh;
                const Rates rt = hh_rates(ld_V(vr, 16 * d.slot));
                sm[q] = gate_step(sm[q], rt.am, rt.bm, a.dt);
                sh[q] = gate_step(sh[q], rt.ah, rt.bh, a.dt);
                sn[q] = gate_step(sn[q], rt.an, rt.bn, a.dt);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                sg[q] *= s_sdec[q];
            }
        }
        if (soma >= 0) {
            const double vnew = ld_V(vr, soma);
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
                    a.trace[int64_t(a.pr_id[pk.pr0 + j]) * a.trace_cap + col] = ld_V(vr, 16 * a.pr_slot[pk.pr0 + j]);
        }
        __syncthreads();
    }

    for (int i = tid; i < ns; i += T) a.V[pk.slot0 + i] = ld_V(vr, 16 * i);
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
