// reg_adjoint_kernels.hip -- the discrete adjoint of the step on the
// register-resident layout.
//
// The paper computes no gradients; this differentiates exactly the forward
// scheme of reg_kernels.hip (Sec. II's operator split: currents at V^n, the
// implicit-Euler solve with A = C/dt + L, states with V^{n+1}).  Going
// backwards through step n with lambda_V = dL/dV^{n+1} (everything after the
// step, except the gate update of this step) and lambda_x = dL/dx^{n+1}:
//   u = lambda_V + sum_x (dPhi_x/dV^{n+1}) lambda_x,   lambda_x <- E_x lambda_x
//   A w = u                                   (the same split Hines solve: A = A^T)
//   lambda_V <- (C/dt - G_lin) w - (dI_nl/dV) w    (+ dL/dtrace of the step before)
//   lambda_x <- lambda_x - (dI/dx) w
//   dL/dtheta -= (dI/dtheta)^T w
// with E_x = dPhi_x/dx = exp(-dt (a + b)).  The forward's recompute records,
// per step, V after the step, the gates before their update and the synapse
// conductances after the step's events (reg_step_kernel with recording).
//
// One workgroup runs one pack backwards through a segment of recorded steps.
// A thread keeps its branches' factorisation in registers exactly as the
// forward does (reg_solve.hpp).  LDS holds, per slot, w (V entry) and
// lambda_V (R entry), the per-CV gradient sums sum w and sum w V, and the
// records of the running step and of the one before it: every thread issues
// the loads of step s-1's records at the top of step s and stores them to LDS
// at its end, so the records' latency hides behind a whole step.
#include <hip/hip_runtime.h>

#include "adjoint_kernels.hpp"
#include "kernel_common.hpp"
#include "reg_solve.hpp"

namespace arbmi {

namespace {

using namespace dev;
using namespace reg;

// Records a thread prefetches per step; a pack with more (ns + 3 nhh + nsyn
// > kPrefetch * T) loads the rest when it stores them.
constexpr int kPrefetch = 8;

struct GateSens {
    double E;     // dPhi/dx = exp(-dt (a + b))
    double dPhi;  // dPhi/dV
};

// Sensitivities of the exact gate update Phi = x_inf + (x - x_inf) e^{-dt s},
// s = a + b, x_inf = a/s, at the gate's value before the update.
__device__ __forceinline__ GateSens gate_sens(double x, double a, double b, double da, double db, double dt) {
    const double s = a + b;
    const double E = exp_pair(-dt * s).e;
    const double rs = 1.0 / s;
    const double xinf = a * rs;
    const double dxinf = (da * b - a * db) * rs * rs;
    GateSens g;
    g.E = E;
    g.dPhi = dxinf * (1.0 - E) - (x - xinf) * E * dt * (da + db);
    return g;
}

// x/(e^x - 1) and its derivative from one exp_pair (a short series for the
// derivative near the removable singularity)
__device__ __forceinline__ void exprelr_d(double x, double& f, double& df) {
    const ExpPair p = exp_pair(x);
    f = (1.0 + x == 1.0) ? 1.0 : x / p.em1;
    df = (fabs(x) < 1e-4) ? -0.5 + x * (1.0 / 6.0) - x * x * x * (1.0 / 180.0)
                          : (p.em1 - x * p.e) / (p.em1 * p.em1);
}

// lambda_V of a branch's rows into R, w into V (for the nonlinear CVs'
// terms), and the per-CV gradient sums; an empty register slot only stores
// into its spare slot.
template <int L>
__device__ __forceinline__ void adj_store(const Slot<L>& g, double* sV, const double* y, double* sA0, double* sA1,
                                          const double* vrow) {
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int sl = g.base + k * g.w;
        const int c = vix(sl);
        sV[c] = y[k];
        sV[c + kRoff] = g.A[k] * y[k];
    }
    if (g.r < 0) return;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int sl = g.base + k * g.w;
        sA0[sl] += y[k];
        sA1[sl] += y[k] * vrow[sl];
    }
}

// The right-hand side u (R entries) of the branch's rows; the soma's row
// also takes the loss term of its voltage.
template <int L>
__device__ __forceinline__ void rhs_load(const Slot<L>& g, const double* sV, double* t, double loss) {
#pragma unroll
    for (int k = 0; k < L; ++k) t[k] = sV[cv_slot(g, k) + kRoff];
    t[0] += loss;
}

// The gid of the cell whose soma is the branch in slot g, or -1.
template <int L>
__device__ __forceinline__ int soma_gid(const Slot<L>& g, const StepArgs& a, const PackDesc& pk) {
    int gid = -1;
    if (g.r >= 0 && g.lev == 0)
        for (int c = 0; c < pk.ncell; ++c)
            if (a.pc_soma[pk.cell0 + c] == g.base) gid = a.pc_gid[pk.cell0 + c];
    return gid;
}

template <int T, int S, int L>
__global__ void __launch_bounds__(T, 1) reg_adjoint_kernel(StepArgs a, AdjArgs b) {
    extern __shared__ __align__(16) char lds_raw[];
    const int p = blockIdx.x;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;
    const int nsp = (ns > pk.spare + 1) ? ns : pk.spare + 1;
    const int nhh = pk.nhh, nsyn = pk.nsyn;

    // ---- LDS layout (reg_adjoint_lds_bytes) ----
    double* sV = reinterpret_cast<double*>(lds_raw);  // w (V entries) and lambda_V (R entries)
    double* sA0 = sV + vr_block_doubles(ns, pk.spare);  // per slot: sum w
    double* sA1 = sA0 + nsp;                            // per slot: sum w V
    double* sVst = sA1 + nsp;                           // V records, three rows (row r at r % 3)
    double* sXst = sVst + 3 * nsp;                      // gate records m, h, n, two rows (r % 2)
    double* sGst = sXst + 6 * nhh;                      // synapse records, two rows
    double* sLm = sGst + 2 * nsyn;                      // lambda_m, lambda_h, lambda_n
    double* sLh = sLm + nhh;
    double* sLn = sLh + nhh;
    double* sGna = sLn + nhh;                           // gradient sums of gNa, gK terms
    double* sGk = sGna + nhh;
    double* s_gna = sGk + nhh;                          // nS
    double* s_gk = s_gna + nhh;
    double* sC = s_gk + nhh;                            // per task (+2), as in the forward
    double* sX = sC;
    double* sF = sC + (pk.ntk + 2);
    double* sY = sF;
    double* sQ = sF + (pk.ntk + 2);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(sQ + (pk.binary ? pk.ntk + 2 : 0));
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);
    int32_t* s_hhs = s_ch + (pk.binary ? 0 : pk.nch);   // per hh instance: its CV's pack-local slot

    const int64_t NS = b.n_slots_total, NH = b.n_hh_total, NY = b.n_syn_total;
    const int ntot = ns + 3 * nhh + nsyn;  // records of one step of the pack
    // source of record element e of step r, and its place in LDS
    auto rec_src = [&](int e, int r) -> const double* {
        if (e < ns) return b.rec_V + int64_t(r) * NS + pk.slot0 + e;
        e -= ns;
        if (e < 3 * nhh) {
            const int w = e / nhh, q = e - w * nhh;
            const double* base = (w == 0) ? b.rec_m : (w == 1) ? b.rec_h : b.rec_n;
            return base + int64_t(r) * NH + pk.hh0 + q;
        }
        return b.rec_g + int64_t(r) * NY + pk.syn0 + (e - 3 * nhh);
    };
    auto rec_dst = [&](int e, int r) -> double* {
        if (e < ns) return sVst + (r % 3) * nsp + e;
        e -= ns;
        if (e < 3 * nhh) return sXst + (r & 1) * 3 * nhh + e;
        return sGst + (r & 1) * nsyn + (e - 3 * nhh);
    };

    for (int i = tid; i < nsp; i += T) {
        const bool real = i < ns;
        sV[vix(i)] = 0.0;
        sV[vix(i) + kRoff] = real ? b.lamV[pk.slot0 + i] : 0.0;
        sA0[i] = 0.0;
        sA1[i] = 0.0;
        sVst[i] = 0.0;
        sVst[nsp + i] = 0.0;
        sVst[2 * nsp + i] = 0.0;
    }
    if (tid < 2) {
        sC[pk.ntk + tid] = 0.0;
        sF[pk.ntk + tid] = 0.0;
        if (pk.binary) sQ[pk.ntk + tid] = 0.0;
    }
    for (int i = tid; i < nhh; i += T) {
        sLm[i] = b.lamM[pk.hh0 + i];
        sLh[i] = b.lamH[pk.hh0 + i];
        sLn[i] = b.lamN[pk.hh0 + i];
        sGna[i] = 0.0;
        sGk[i] = 0.0;
        s_gna[i] = a.hh_gna[pk.hh0 + i];
        s_gk[i] = a.hh_gk[pk.hh0 + i];
    }
    for (int i = tid; i < pk.nnl; i += T) {
        const NlDesc d = a.nl[pk.nl0 + i];
        s_nl[i] = d;
        if (d.hh >= 0) s_hhs[d.hh] = d.slot;
    }
    if (!pk.binary)
        for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_task[pk.ch0 + i];
    __syncthreads();
    // the records of the last step: V after it and before it, gates and g
    const int last = b.nsteps - 1;
    for (int i = tid; i < ns; i += T) sVst[((last + 1) % 3) * nsp + i] = b.rec_V[int64_t(last + 1) * NS + pk.slot0 + i];
    for (int e = tid; e < ntot; e += T) *rec_dst(e, last) = *rec_src(e, last);

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
    load_slot<L>(g0, a, pk, myr[0], tid);
    if constexpr (S > 1) load_slot<L>(g1, a, pk, myr[1], tid);
    if constexpr (S > 2) load_slot<L>(g2, a, pk, myr[2], tid);
    // the soma tasks' cells (loss terms): gid, or -1
    int gid[S];
    gid[0] = soma_gid<L>(g0, a, pk);
    if constexpr (S > 1) gid[1] = soma_gid<L>(g1, a, pk);
    if constexpr (S > 2) gid[2] = soma_gid<L>(g2, a, pk);
    if (pk.binary) {
        if (g0.r >= 0) sQ[g0.task] = g0.FQ;
        if constexpr (S > 1) {
            if (g1.r >= 0) sQ[g1.task] = g1.FQ;
        }
        if constexpr (S > 2) {
            if (g2.r >= 0) sQ[g2.task] = g2.FQ;
        }
    }
    // loss terms of the last step (trace column n - trace_step0)
    double loss[S];
#pragma unroll
    for (int j = 0; j < S; ++j)
        loss[j] = (gid[j] >= 0) ? b.dLdtrace[int64_t(gid[j]) * b.trace_len + (b.step0 + last - b.trace_step0)] : 0.0;
    __syncthreads();

    for (int s = last; s >= 0; --s) {
        // prefetch: step s-1's records into registers, and its loss terms
        double pf[kPrefetch];
        double lnext[S];
        if (s > 0) {
#pragma unroll
            for (int k = 0; k < kPrefetch; ++k) {
                const int e = tid + k * T;
                pf[k] = (e < ntot) ? *rec_src(e, s - 1) : 0.0;
            }
#pragma unroll
            for (int j = 0; j < S; ++j)
                lnext[j] = (gid[j] >= 0)
                               ? b.dLdtrace[int64_t(gid[j]) * b.trace_len + (b.step0 + s - 1 - b.trace_step0)]
                               : 0.0;
        }
        const double* vrow1 = sVst + ((s + 1) % 3) * nsp;  // V^{n+1}
        const double* vrow0 = sVst + (s % 3) * nsp;        // V^n
        const double* xrow = sXst + (s & 1) * 3 * nhh;     // gates before the step
        const double* grow = sGst + (s & 1) * nsyn;        // g after the step's events

        // G: the gate update's terms at V^{n+1}: u += dPhi/dV lambda_x, lambda_x *= E
        for (int q = tid; q < nhh; q += T) {
            const int sl = s_hhs[q];
            const double v = vrow1[sl];
            double am, dam, an, dan;
            exprelr_d(-(v + 40.0) * 0.1, am, dam);
            dam *= -0.1;
            exprelr_d(-(v + 55.0) * 0.1, an, dan);
            an *= 0.1;
            dan *= -0.01;
            const double ebm = exp_pair(-(v + 65.0) * (1.0 / 18.0)).e;
            const double bm = 4.0 * ebm, dbm = -(4.0 / 18.0) * ebm;
            const double eah = exp_pair(-(v + 65.0) * 0.05).e;
            const double ah = 0.07 * eah, dah = -(0.07 * 0.05) * eah;
            const double u = exp_pair(-(v + 35.0) * 0.1).e;
            const double bh = 1.0 / (u + 1.0), dbh = 0.1 * u * bh * bh;
            const double ebn = exp_pair(-(v + 65.0) * (1.0 / 80.0)).e;
            const double bn = 0.125 * ebn, dbn = -(0.125 / 80.0) * ebn;
            const GateSens gm = gate_sens(xrow[q], am, bm, dam, dbm, b.dt);
            const GateSens gh = gate_sens(xrow[nhh + q], ah, bh, dah, dbh, b.dt);
            const GateSens gn = gate_sens(xrow[2 * nhh + q], an, bn, dan, dbn, b.dt);
            const double lm = sLm[q], lh = sLh[q], ln = sLn[q];
            sV[vix(sl) + kRoff] += gm.dPhi * lm + gh.dPhi * lh + gn.dPhi * ln;
            sLm[q] = gm.E * lm;
            sLh[q] = gh.E * lh;
            sLn[q] = gn.E * ln;
        }
        round_sync<T>();

        // the solve A w = u, exactly the forward's
        double y0[L], y1[L], y2[L];
        rhs_load<L>(g0, sV, y0, loss[0]);
        if constexpr (S > 1) rhs_load<L>(g1, sV, y1, loss[1]);
        if constexpr (S > 2) rhs_load<L>(g2, sV, y2, loss[2]);
        local_chain<L>(g0, y0);
        if constexpr (S > 1) local_chain<L>(g1, y1);
        if constexpr (S > 2) local_chain<L>(g2, y2);
        local_store<L>(g0, sC, sF);
        if constexpr (S > 1) local_store<L>(g1, sC, sF);
        if constexpr (S > 2) local_store<L>(g2, sC, sF);
        round_sync<T>();
        up_pass<T, S, L>(pk, g0, g1, g2, sF, sQ, sC, s_ch);
        full_chain<L>(g0, y0);
        if constexpr (S > 1) full_chain<L>(g1, y1);
        if constexpr (S > 2) full_chain<L>(g2, y2);
        grounded_store<L>(g0, sY, sX);
        if constexpr (S > 1) grounded_store<L>(g1, sY, sX);
        if constexpr (S > 2) grounded_store<L>(g2, sY, sX);
        round_sync<T>();
        down_pass<T, S, L>(pk, g0, g1, g2, sY, sX);
        subst_chain<L>(g0, y0);
        if constexpr (S > 1) subst_chain<L>(g1, y1);
        if constexpr (S > 2) subst_chain<L>(g2, y2);
        // lambda_V <- alpha w (the linear terms), w for the nonlinear CVs, sums
        adj_store<L>(g0, sV, y0, sA0, sA1, vrow0);
        if constexpr (S > 1) adj_store<L>(g1, sV, y1, sA0, sA1, vrow0);
        if constexpr (S > 2) adj_store<L>(g2, sV, y2, sA0, sA1, vrow0);
        round_sync<T>();

        // N: the nonlinear currents' terms at V^n
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const int c = vix(d.slot);
            const double w = sV[c];
            const double v = vrow0[d.slot];
            double gnl = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = xrow[q], h = xrow[nhh + q], x = xrow[2 * nhh + q];
                const double gna = s_gna[q], gk = s_gk[q];
                const double m2 = m * m, x3 = x * x * x;
                const double m3h = m2 * m * h, n4 = x3 * x;
                const double ena = (v - kENa) * w, ek = (v - kEK) * w;
                gnl += gna * m3h + gk * n4;
                sLm[q] -= gna * 3.0 * m2 * h * ena;
                sLh[q] -= gna * m2 * m * ena;
                sLn[q] -= gk * 4.0 * x3 * ek;
                sGna[q] -= m3h * ena;
                sGk[q] -= n4 * ek;
            }
            for (int k = 0; k < d.nsyn; ++k) gnl += grow[d.syn0 + k];
            sV[c + kRoff] -= gnl * w;
        }
        // the prefetched records of step s-1 into the rows this step no
        // longer reads (V row s + 2, gate and synapse rows s + 1)
        if (s > 0) {
#pragma unroll
            for (int k = 0; k < kPrefetch; ++k) {
                const int e = tid + k * T;
                if (e < ntot) *rec_dst(e, s - 1) = pf[k];
            }
            for (int e = tid + kPrefetch * T; e < ntot; e += T) *rec_dst(e, s - 1) = *rec_src(e, s - 1);
#pragma unroll
            for (int j = 0; j < S; ++j) loss[j] = lnext[j];
        }
        round_sync<T>();
    }

    for (int i = tid; i < ns; i += T) {
        b.lamV[pk.slot0 + i] = sV[vix(i) + kRoff];
        b.accP0[pk.slot0 + i] += sA0[i];
        b.accP1[pk.slot0 + i] += sA1[i];
    }
    for (int i = tid; i < nhh; i += T) {
        b.lamM[pk.hh0 + i] = sLm[i];
        b.lamH[pk.hh0 + i] = sLh[i];
        b.lamN[pk.hh0 + i] = sLn[i];
        b.accNa[pk.hh0 + i] += sGna[i];
        b.accK[pk.hh0 + i] += sGk[i];
    }
}

template <int T, int S, int L>
hipError_t launch_one(const StepArgs& a, const AdjArgs& b, int lds, int n_packs, hipStream_t st) {
    hipLaunchKernelGGL((reg_adjoint_kernel<T, S, L>), dim3(n_packs), dim3(T), lds, st, a, b);
    return hipGetLastError();
}

template <int T, int S, int L>
void allow_one(int lds_max) {
    const void* f = reinterpret_cast<const void*>(&reg_adjoint_kernel<T, S, L>);
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
}

template <int T>
hipError_t launch_T(const StepArgs& a, const AdjArgs& b, int slots, int len, int lds, int n_packs, hipStream_t st) {
    if (len == 8) {
        switch (slots) {
            case 1: return launch_one<T, 1, 8>(a, b, lds, n_packs, st);
            case 2: return launch_one<T, 2, 8>(a, b, lds, n_packs, st);
            case 3: return launch_one<T, 3, 8>(a, b, lds, n_packs, st);
            default: break;
        }
    } else if (len == 16 && slots == 1) {
        return launch_one<T, 1, 16>(a, b, lds, n_packs, st);
    }
    return hipErrorInvalidValue;
}

template <int T>
void allow_T(int lds_max) {
    allow_one<T, 1, 8>(lds_max);
    allow_one<T, 2, 8>(lds_max);
    allow_one<T, 3, 8>(lds_max);
    allow_one<T, 1, 16>(lds_max);
}

}  // namespace

hipError_t prepare_reg_adjoint_kernels(int lds_max) {
    allow_T<64>(lds_max);
    allow_T<128>(lds_max);
    allow_T<256>(lds_max);
    return hipSuccess;
}

hipError_t launch_reg_adjoint(const StepArgs& a, const AdjArgs& b, const LaunchCfg& cfg, int lds_bytes, int n_packs,
                              hipStream_t st) {
    switch (cfg.block_threads) {
        case 64: return launch_T<64>(a, b, cfg.reg_slots, cfg.reg_len, lds_bytes, n_packs, st);
        case 128: return launch_T<128>(a, b, cfg.reg_slots, cfg.reg_len, lds_bytes, n_packs, st);
        case 256: return launch_T<256>(a, b, cfg.reg_slots, cfg.reg_len, lds_bytes, n_packs, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace arbmi
