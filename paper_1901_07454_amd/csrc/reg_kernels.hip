// reg_kernels.hip -- register-resident variant of the fused step kernel.
//
// Same phases as step_kernel (kernels.hip): events, point currents, the
// Hines solve, states and threshold.  Each thread holds, for the whole
// launch, everything about its branches that does not change between
// steps: the step coefficients (alpha, F = u/d', 1/d') and where the
// branch's CVs, its parent and its children live.  A thread owns up to S
// branches of at most L CVs; the host gives every round one register slot
// j on all of its threads, so the per-slot arrays are indexed with
// compile-time constants.
//
// The solve is the split Hines solve of reg_solve.hpp: all branches'
// local elimination; rounds deepest first passing the contributions up (one
// multiply-add per branch); all branches' full elimination with their
// children's sum and the local substitution; rounds shallowest first passing
// the distal V down, two tree levels a round (a branch forms its parent's V
// from its grandparent's: x_p = Y_p + Z_p x_gp); all branches' substitution
// with the parent's V.  In packs with at most binary branch points every
// register slot takes part in every round (up_pass, down_pass).
//
// LDS keeps V and R (the right-hand side) per slot, in blocks of 64 slots
// (64 V then 64 R): V-only accesses of consecutive slots are 8 bytes apart
// and R is a fixed offset from V.  R holds beta (the step-invariant part of
// the right-hand side) minus the point currents.
// Through the solve a row's values stay in its thread's registers; only
// the per-branch scalars passed between branches go through LDS (the task
// arrays sC, sF, sQ, with sX and sY reusing sC and sF for the downward
// pass).  Every branch has L rows in the layout; a shorter
// branch's spare rows hold pad CVs (alpha = beta = 1/d' = 0) that carry the
// recurrences through unchanged (F = +1 at the first pad, -1 after it).
// An empty register slot works on a slot no CV uses (a pad row, or one past
// the pack's slots).
// With recording on (REC, for the adjoint's recompute) every step also
// writes the state the adjoint needs to HBM: V after the step, the gates
// before their update and the synapse conductances after the step's events.
#include <hip/hip_runtime.h>

#include "gen/mechanisms.hpp"
#include "kernel_common.hpp"
#include "kernels.hpp"
#include "reg_solve.hpp"

namespace arbmi {

namespace {

using namespace dev;
using namespace reg;

// Waves per SIMD the registers allow without spilling (built without
// machine loop-invariant code motion): three for one slot of 8 CVs, two for
// 16 CVs in all, one otherwise.  G: some pack of the launch keeps state in
// HBM, its synapses' or its hh conductances' (without it, those paths are
// compiled out).  REC: the
// sim is built for gradients; the steps record their states when a.rec_V
// is set (the adjoint's recompute), and the gradient forward runs the same
// code with it unset, so both produce the same trajectory bit for bit (one
// wave per SIMD fewer than the plain variant: the recording's addresses take
// the registers).  M: the model has generated density mechanisms (their
// currents join the nonlinear CVs' right-hand sides, their states advance
// with the gates; parameters and states stay in HBM).
template <int T, int S, int L, bool G, bool REC, bool M = false>
__global__ void __launch_bounds__(T, REC ? ((S * L <= 8) ? 2 : 1) : ((S * L <= 8) ? 3 : (S * L <= 16 ? 2 : 1)))
    reg_step_kernel(StepArgs a) {
    extern __shared__ __align__(16) char lds_raw[];
    const int p = blockIdx.x + a.pack0;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    // ---- LDS layout (the mode-3 layout of pack_lds_bytes) ----
    double* sV = reinterpret_cast<double*>(lds_raw);           // V and R blocks (pack_lds_bytes)
    // synapse state in LDS, or in HBM (pack_lds_bytes) for synapse-heavy packs
    const bool syn_hbm = G && pk.syn_global;
    const int nsyn_lds = syn_hbm ? 0 : pk.nsyn;
    double* sg = sV + vr_block_doubles(ns, pk.spare);
    double* s_se = sg + nsyn_lds;
    double* s_sdec = s_se + nsyn_lds;
    double* sm = s_sdec + nsyn_lds;
    double* g_g = a.syn_g + pk.syn0;                           // HBM synapse state of the pack
    const double* g_se = a.syn_e + pk.syn0;
    const double* g_sdec = a.syn_decay + pk.syn0;
    double* sgv = syn_hbm ? g_g : sg;                    // where events add to g
    // hh conductances and the nonlinear CVs' beta in LDS, or in HBM for a
    // pack too large for LDS otherwise
    const bool hh_hbm = G && pk.hh_global;
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    double* s_gna = sn + pk.nhh;
    double* s_gk = s_gna + (hh_hbm ? 0 : pk.nhh);
    double* s_nlb = s_gk + (hh_hbm ? 0 : pk.nhh);              // beta of each nonlinear CV
    // per task, two spare entries (zero, discard) each: contribution, then
    // distal V; contribution with no children, then distal V for a grounded
    // parent; F_0 Q_0 (binary packs)
    double* sC = s_nlb + (hh_hbm ? 0 : pk.nnl);
    double* sX = sC;
    double* sF = sC + (pk.ntk + 2);
    double* sY = sF;
    double* sQ = sF + (pk.ntk + 2);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(sQ + (pk.binary ? pk.ntk + 2 : 0));
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);  // children's tasks (other packs)
    int32_t* s_hhs = s_ch + (pk.binary ? 0 : pk.nch);          // per hh instance: its CV's slot

    const bool rec = REC && a.rec_V != nullptr;
    for (int i = tid; i < ns; i += T) {
        const double v = a.V[pk.slot0 + i];
        sV[vix(i)] = v;
        sV[vix(i) + kRoff] = a.beta[pk.slot0 + i];
        if (rec) a.rec_V[pk.slot0 + i] = v;  // row 0: the state before the launch's first step
    }
    if (tid == 0 && pk.spare == ns) {
        sV[vix(ns)] = 0.0;
        sV[vix(ns) + kRoff] = 0.0;
    }
    if (tid < 2) {
        sC[pk.ntk + tid] = 0.0;
        sF[pk.ntk + tid] = 0.0;
        if (pk.binary) sQ[pk.ntk + tid] = 0.0;
    }
    for (int i = tid; i < nsyn_lds; i += T) {
        sg[i] = g_g[i];
        s_se[i] = g_se[i];
        s_sdec[i] = g_sdec[i];
    }
    for (int i = tid; i < pk.nhh; i += T) {
        sm[i] = a.hh_m[pk.hh0 + i];
        sh[i] = a.hh_h[pk.hh0 + i];
        sn[i] = a.hh_n[pk.hh0 + i];
        if (!hh_hbm) {
            s_gna[i] = a.hh_gna[pk.hh0 + i];
            s_gk[i] = a.hh_gk[pk.hh0 + i];
        }
    }
    for (int i = tid; i < pk.nnl; i += T) {
        const NlDesc d = a.nl[pk.nl0 + i];
        s_nl[i] = d;
        if (!hh_hbm) s_nlb[i] = a.beta[pk.slot0 + d.slot];
        if (d.hh >= 0) s_hhs[d.hh] = vix(d.slot);
    }
    if (!pk.binary)
        for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_task[pk.ch0 + i];

    int64_t step0 = a.step0;
    if (a.epoch_ptr) step0 = *a.epoch_ptr * a.nsteps;
    // network events: where each step of the epoch starts in the pack's
    // bucket; external-event cursor, the same in every thread
    const int64_t estart = step0 - step0 % a.epoch_steps;
    const uint32_t* eoff = a.bk_off ? a.bk_off + int64_t(p) * (a.epoch_steps + 1) : nullptr;
    const int32_t* eq = a.bk_q + int64_t(p) * a.bk_cap;
    const double* ew = a.bk_w + int64_t(p) * a.bk_cap;
    // the next step of the epoch with network events: steps without any
    // load nothing
    const uint32_t* enxt = eoff ? a.bk_nxt + int64_t(p) * (a.epoch_steps + 1) : nullptr;
    // a pack with at most kSpreadHH hh instances gives each gate a thread:
    // this thread's instance and gate, and the gate's constants
    static_assert(3 * kSpreadHH <= T, "one gate per thread");
    const int hq = tid / 3, hw = tid - 3 * hq;
    const HHGate hc = hh_gate_consts(hw);
    int32_t eb = eoff ? int32_t(enxt[step0 - estart]) : INT32_MAX;
    int64_t xcur = a.pk_xcur[p];
    int64_t xstep = (xcur < pk.xe1) ? a.xe_step[xcur] : INT64_MAX;
    const int soma = (tid < pk.ncell) ? vix(a.pc_soma[pk.cell0 + tid]) : -1;
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
    load_slot<L>(g0, a, pk, myr[0], tid);
    if constexpr (S > 1) load_slot<L>(g1, a, pk, myr[1], tid);
    if constexpr (S > 2) load_slot<L>(g2, a, pk, myr[2], tid);
    if (pk.binary) {
        if (g0.r >= 0) sQ[g0.task] = g0.FQ;
        if constexpr (S > 1) {
            if (g1.r >= 0) sQ[g1.task] = g1.FQ;
        }
        if constexpr (S > 2) {
            if (g2.r >= 0) sQ[g2.task] = g2.FQ;
        }
    }
    __syncthreads();
    // the V entry of this thread's gate in the spread update, fixed for the launch
    const int hv = (pk.nhh <= kSpreadHH && tid < 3 * pk.nhh) ? s_hhs[hq] : 0;

    for (int s = 0; s < a.nsteps; ++s) {
        const int64_t n = step0 + s;

        // A: events due at the start of step n, network ones (in connection
        // rank order, so a synapse's events are adjacent) before external ones
        // (sorted by step, then synapse).  The thread holding the first event
        // of a run of same-synapse events adds the whole run in order, so
        // every synapse's sum is the serial one.  A thread takes up to four
        // network events at once: their synapses and weights are loaded
        // together, then their conductances (distinct synapses), then the
        // sums are stored.
        if (int32_t(n - estart) == eb) {
            const uint32_t i0 = eoff[eb], i1 = eoff[eb + 1];
            eb = int32_t(enxt[eb + 1]);
            for (uint32_t c = i0; c < i1; c += 4 * T) {
                int q[4];
                double w[4], gq[4];
                bool head[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t i = c + uint32_t(u * T + tid);
                    head[u] = false;
                    q[u] = 0;
                    w[u] = 0.0;
                    if (i < i1) {
                        q[u] = eq[i];
                        w[u] = ew[i];
                        head[u] = i == i0 || eq[i - 1] != q[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) gq[u] = head[u] ? sgv[q[u]] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (head[u]) {
                        double x = gq[u] + w[u];
                        for (uint32_t j = c + uint32_t(u * T + tid) + 1; j < i1 && eq[j] == q[u]; ++j) x += ew[j];
                        sgv[q[u]] = x;
                    }
            }
            if (syn_hbm) __threadfence_block();
            round_sync<T>();
        }
        if (xstep == n) {
            const int64_t first = xcur;
            for (;;) {
                const int64_t i = xcur + tid;
                const bool due = i < pk.xe1 && a.xe_step[i] == n;
                if (due) {
                    const int q = a.xe_syn[i];
                    if (i == first || a.xe_syn[i - 1] != q) {
                        double gq = sgv[q] + a.xe_w[i];
                        for (int64_t j = i + 1; j < pk.xe1 && a.xe_step[j] == n && a.xe_syn[j] == q; ++j)
                            gq += a.xe_w[j];
                        sgv[q] = gq;
                    }
                }
                const int cnt = block_count<T>(due);
                xcur += cnt;
                if (cnt < T) break;
            }
            xstep = (xcur < pk.xe1) ? a.xe_step[xcur] : INT64_MAX;
            if (syn_hbm) __threadfence_block();  // the adds reach the other threads' loads
        }
        round_sync<T>();

        // B: R = beta - I at the CVs with nonlinear and point currents (V^n)
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double v = sV[vix(d.slot)];
            double I = 0.0, bnl;
            if (hh_hbm) {
                bnl = a.beta[pk.slot0 + d.slot];
                if (d.hh >= 0) {
                    const int q = d.hh;
                    const double m = sm[q], h = sh[q], x = sn[q];
                    I += a.hh_gna[pk.hh0 + q] * (m * m * m * h) * (v - kENa);
                    I += a.hh_gk[pk.hh0 + q] * (x * x * x * x) * (v - kEK);
                }
            } else {
                bnl = s_nlb[j];
                if (d.hh >= 0) {
                    const int q = d.hh;
                    const double m = sm[q], h = sh[q], x = sn[q];
                    I += s_gna[q] * (m * m * m * h) * (v - kENa);
                    I += s_gk[q] * (x * x * x * x) * (v - kEK);
                }
            }
            if constexpr (M) {
                for (int q = a.gen_off[pk.nl0 + j]; q < a.gen_off[pk.nl0 + j + 1]; ++q) {
                    // shared parameter rows stay in cache; the mechanism
                    // comes with the row index (one dependent load less)
                    const int rr = a.gen_row[q], r = rr & 0xffffff;
                    I += a.gen_w[q] * gen::current(rr >> 24, v, a.gen_prm + int64_t(r) * gen::kMaxParams,
                                                   a.gen_st + q, a.gen_n);
                }
            }
            if (!syn_hbm) {
                // the decay of phase E is applied here too: g is not read
                // again before the next step's events
                for (int k = 0; k < d.nsyn; ++k) {
                    const int q = d.syn0 + k;
                    const double gq = sg[q], eq = s_se[q], dq = s_sdec[q];  // loads issued together
                    if (rec) a.rec_g[int64_t(s) * a.n_syn_total + pk.syn0 + q] = gq;
                    I += gq * (v - eq);
                    sg[q] = gq * dq;
                }
            } else {
                // HBM synapses, interleaved over the threads of this group
                // of entries (stride w), four at a time so their loads
                // overlap; the decay of phase E is applied here (g is not
                // read again before the next step's events)
                const int w = min(T, pk.nnl - (j / T) * T);
                if (pk.syn_uniform) {  // shared e_syn and decay: only g moves
                    const double e = pk.syn_e, dec = pk.syn_decay;
                    for (int k0 = 0; k0 < d.nsyn; k0 += 4) {
                        double gg[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) gg[i] = g_g[d.syn0 + min(k0 + i, d.nsyn - 1) * w];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (k0 + i < d.nsyn) {
                                I += gg[i] * (v - e);
                                g_g[d.syn0 + (k0 + i) * w] = gg[i] * dec;
                            }
                    }
                } else {
                    for (int k0 = 0; k0 < d.nsyn; k0 += 4) {
                        double gg[4], ee[4], dd[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int q = d.syn0 + min(k0 + i, d.nsyn - 1) * w;
                            gg[i] = g_g[q];
                            ee[i] = g_se[q];
                            dd[i] = g_sdec[q];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (k0 + i < d.nsyn) {
                                I += gg[i] * (v - ee[i]);
                                g_g[d.syn0 + (k0 + i) * w] = gg[i] * dd[i];
                            }
                    }
                }
            }
            sV[vix(d.slot) + kRoff] = bnl - I;
        }
        if (soma >= 0) vold = sV[soma];
        if (pk.nic > 0) {
            round_sync<T>();
            if (tid == 0)
                for (int q = pk.ic0; q < pk.ic0 + pk.nic; ++q)
                    if (a.ic_on[q] <= n && n < a.ic_off[q]) {
                        sV[vix(a.ic_slot[q]) + kRoff] += a.ic_amp[q];
                    }
        }
        round_sync<T>();

        // C: the solve.  Each row's t, then rhs'/d', stays in the owning
        // thread's registers from the local elimination to the substitution
        // (no other thread reads them); the V entries keep V^n until then.
        double y0[L], y1[L], y2[L];
        local_load<L>(g0, sV, y0);
        if constexpr (S > 1) local_load<L>(g1, sV, y1);
        if constexpr (S > 2) local_load<L>(g2, sV, y2);
        local_chain<L>(g0, y0);
        if constexpr (S > 1) local_chain<L>(g1, y1);
        if constexpr (S > 2) local_chain<L>(g2, y2);
        local_store<L>(g0, sC, sF);
        if constexpr (S > 1) local_store<L>(g1, sC, sF);
        if constexpr (S > 2) local_store<L>(g2, sC, sF);
        round_sync<T>();
        up_pass<T, S, L>(pk, g0, g1, g2, sF, sQ, sC, s_ch);
        {
            full_chain<L>(g0, y0);
            if constexpr (S > 1) full_chain<L>(g1, y1);
            if constexpr (S > 2) full_chain<L>(g2, y2);
            grounded_store<L>(g0, sY, sX);
            if constexpr (S > 1) grounded_store<L>(g1, sY, sX);
            if constexpr (S > 2) grounded_store<L>(g2, sY, sX);
        }
        round_sync<T>();
        down_pass<T, S, L>(pk, g0, g1, g2, sY, sX);
        {
            subst_chain<L>(g0, y0);
            if constexpr (S > 1) subst_chain<L>(g1, y1);
            if constexpr (S > 2) subst_chain<L>(g2, y2);
            store_v<L>(g0, sV, y0);
            if constexpr (S > 1) store_v<L>(g1, sV, y1);
            if constexpr (S > 2) store_v<L>(g2, sV, y2);
            if (rec) {  // V^{n+1} into row s + 1, from the owners' registers
                double* row = a.rec_V + int64_t(s + 1) * a.n_slots_total + pk.slot0;
                record_v<L>(g0, row, y0);
                if constexpr (S > 1) record_v<L>(g1, row, y1);
                if constexpr (S > 2) record_v<L>(g2, row, y2);
            }
        }
        round_sync<T>();

        // E: states with V^{n+1} (synapses decayed in phase B); threshold.  A
        // pack with few hh instances gives each gate of an instance its own
        // thread (which computes that gate's two rates and the update);
        // otherwise a thread takes a whole instance.
        if (pk.nhh <= kSpreadHH) {
            if (tid < 3 * pk.nhh) {
                double* x = (hw == 0) ? sm : (hw == 1) ? sh : sn;
                if (rec) {  // the gate before its update
                    double* r = (hw == 0) ? a.rec_m : (hw == 1) ? a.rec_h : a.rec_n;
                    r[int64_t(s) * a.n_hh_total + pk.hh0 + hq] = x[hq];
                }
                x[hq] = hh_gate_step(hc, sV[hv], x[hq], a.dt);
            }
        } else {
            for (int q = tid; q < pk.nhh; q += T) {
                const Rates rt = hh_rates(sV[s_hhs[q]]);
                if (rec) {  // the gates before their update
                    const int64_t at = int64_t(s) * a.n_hh_total + pk.hh0 + q;
                    a.rec_m[at] = sm[q];
                    a.rec_h[at] = sh[q];
                    a.rec_n[at] = sn[q];
                }
                sm[q] = gate_step(sm[q], rt.am, rt.bm, a.dt);
                sh[q] = gate_step(sh[q], rt.ah, rt.bh, a.dt);
                sn[q] = gate_step(sn[q], rt.an, rt.bn, a.dt);
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
                    a.trace[int64_t(a.pr_id[pk.pr0 + j]) * a.trace_cap + col] = sV[vix(a.pr_slot[pk.pr0 + j])];
        }
        if constexpr (M) {  // generated mechanisms' states with V^{n+1}
            for (int q = a.gen_pk[p] + tid; q < a.gen_pk[p + 1]; q += T) {
                const int rr = a.gen_row[q], r = rr & 0xffffff;
                gen::advance(rr >> 24, sV[vix(a.gen_slot[q])], a.dt, a.gen_prm + int64_t(r) * gen::kMaxParams,
                             a.gen_st + q, a.gen_n);
            }
            __threadfence_block();  // before the next step's currents read them
        }
        if (syn_hbm) __threadfence_block();  // phase B's g stores before the next step's events
        round_sync<T>();
    }

    for (int i = tid; i < ns; i += T) a.V[pk.slot0 + i] = sV[vix(i)];
    for (int i = tid; i < nsyn_lds; i += T) g_g[i] = sg[i];
    for (int i = tid; i < pk.nhh; i += T) {
        a.hh_m[pk.hh0 + i] = sm[i];
        a.hh_h[pk.hh0 + i] = sh[i];
        a.hh_n[pk.hh0 + i] = sn[i];
    }
    if (tid == 0) a.pk_xcur[p] = xcur;
}

template <int T, int S, int L>
hipError_t launch_reg(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.gen) {  // generated mechanisms: state in LDS, no recording
        if (cfg.rec || cfg.syn_hbm) return hipErrorInvalidValue;
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, false, false, true>), dim3(n_packs), dim3(T), cfg.lds_bytes, st,
                           a);
    } else if (cfg.rec) {  // gradient sims never keep synapse state in HBM
        if (cfg.syn_hbm) return hipErrorInvalidValue;
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, false, true>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a);
    } else if (cfg.syn_hbm) {
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, true, false>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a);
    } else {
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, false, false>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a);
    }
    return hipGetLastError();
}

template <int T, int S, int L, bool G, bool REC, bool M = false>
void allow_lds_one(int lds_max) {
    const void* f = reinterpret_cast<const void*>(&reg_step_kernel<T, S, L, G, REC, M>);
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
}

template <int T, int S, int L>
void allow_lds(int lds_max) {
    allow_lds_one<T, S, L, false, false>(lds_max);
    allow_lds_one<T, S, L, true, false>(lds_max);
    allow_lds_one<T, S, L, false, true>(lds_max);
    allow_lds_one<T, S, L, false, false, true>(lds_max);
}

template <int T>
hipError_t launch_reg_T(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.reg_len == 8) {
        switch (cfg.reg_slots) {
            case 1: return launch_reg<T, 1, 8>(a, cfg, n_packs, st);
            case 2: return launch_reg<T, 2, 8>(a, cfg, n_packs, st);
            case 3: return launch_reg<T, 3, 8>(a, cfg, n_packs, st);
            default: break;
        }
    } else if (cfg.reg_len == 16 && cfg.reg_slots == 1) {
        return launch_reg<T, 1, 16>(a, cfg, n_packs, st);
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
