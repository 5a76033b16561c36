// var_kernels.hip -- the variable time step (Sec. II: a step is shortened
// so that every event arrives at the beginning of a step).
//
// Each workgroup advances one cell in the register-resident layout (the
// layout of reg_kernels.hip), with its own time t.  From t in the grid
// interval [k dt, (k+1) dt) the cell first takes every event due at or
// before t (network events, then external ones), then steps to
// min((k+1) dt, its next event's time); a step from k dt to (k+1) dt has
// length dt exactly.  Events, spikes and epochs keep continuous times: a
// spike carries its threshold crossing interpolated within its step, and its
// events arrive at that time plus the connection's delay.  An epoch is K
// steps of the grid (K dt at most the minimum delay), so every launch starts
// and ends on the grid.
//
// A step of length dt runs exactly as the fixed step does, with the
// factorisation computed once on the host and held in registers.  A
// shortened step of length h changes the matrix (C/h + the axial
// conductances): the branches refactor their registers for h, level by
// level of the branch tree from the deepest (the continued fraction
// d'_k = C_k/h + sum sigma - u_{k+1} F_{k+1} does not split across branches
// the way the right-hand side does), the same split solve runs, and the
// step-dt coefficients are reloaded afterwards.  Gates and synapses decay
// over h.
//
// The pull (one wave per cell) bins the epoch's network events by grid
// interval, comparing arrival times with the grid points k dt as the step
// kernel computes them, and sorts each interval's events by (time, synapse,
// weight), so that each cell reads its events in time order and equal
// times always add in one order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kernel_common.hpp"
#include "kernels.hpp"
#include "reg_solve.hpp"
#include "var_kernels.hpp"

namespace arbmi {

namespace {

using namespace dev;
using namespace reg;

// Refactor a branch in its registers for a step of length h.  The step-dt
// factorisation held there gives what the new one needs, with the branch's
// capacitances C (read from HBM, every row's load issued at once, at clamped
// rows for the pads): u_k = F_k / D_k (F = u/d', D = 1/d'; the quotients
// from refined reciprocals, recip), and with dh =
// 1/h - 1/dt and the distal neighbour's parts c = u F of the eliminated
// diagonal at dt (c_dt) and at h (c_h),
//   d'_h = 1/D + c_dt - c_h + C dh,   alpha_h = alpha + C dh,
// so that d'_h = C/h + sum sigma - c_h, the elimination of the matrix for h
// (Sec. II, the step's own dt).  cdt and ch are the children's sums at the
// distal CV; returns the branch's own parts (u_0 F_0 at dt and at h) for its
// parent.  Pads keep their neutral values.
template <int L>
__device__ __forceinline__ void var_refactor(Slot<L>& g, const VarArgs& v, const PackDesc& pk, double ih, double dh,
                                             double cdt, double ch, double& out_dt, double& out_h) {
    // the rows' addresses are formed here, at each use: hoisted out of the
    // time loop they would hold 2 L registers for the whole launch
    int base = g.base, w = g.w, len = g.len;
    asm volatile("" : "+v"(base), "+v"(w), "+v"(len));
    double cap[L];
#pragma unroll
    for (int k = 0; k < L; ++k) cap[k] = v.cap[pk.slot0 + base + int64_t(min(k, len - 1)) * w];
    (void)ih;
    // branch-free over the rows: a pad row (k >= len; D = 0) computes
    // values that the selects discard
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
        const bool real = k < len;
        const double id = recip(g.D[k]);  // d' at dt
        const double u = g.F[k] * id;
        const double d = id + cdt - ch + cap[k] * dh;
        const double rd = recip(d);
        const double f = u * rd;
        cdt = real ? g.F[k] * u : cdt;
        ch = real ? f * u : ch;
        g.A[k] = real ? g.A[k] + cap[k] * dh : g.A[k];
        g.F[k] = real ? f : g.F[k];
        g.D[k] = real ? rd : g.D[k];
    }
    double q = 1.0, z = 1.0;
#pragma unroll
    for (int k = 0; k < L; ++k)
        if (k < len) {
            z *= -g.F[k];
            if (k >= 1) q *= -g.F[k];
        }
    g.FQ = g.F[0] * q;
    g.Z = z;
    out_dt = cdt;
    out_h = ch;
}

// The children's sums of a branch's parts in the refactoring pass (binary
// packs hold grandchildren in x0/x1, so only c0 and c1 are children there).
template <int L>
__device__ __forceinline__ void child_sums(const Slot<L>& g, const double* sC, const double* sF, const int32_t* s_ch,
                                           bool binary, double& cdt, double& ch) {
    cdt = sF[g.c0] + sF[g.c1];
    ch = sC[g.c0] + sC[g.c1];
    if (!binary)
        for (int q = 0; q < g.x1; ++q) {
            const int c = s_ch[g.x0 + q];
            cdt += sF[c];
            ch += sC[c];
        }
}

template <int L>
__device__ __forceinline__ void refactor_level(Slot<L>& g, int lv, const VarArgs& v, const PackDesc& pk, double ih,
                                               double dh, double* sC, double* sF, const int32_t* s_ch) {
    if (g.lev != lv) return;
    double cdt, ch, odt, oh;
    child_sums<L>(g, sC, sF, s_ch, pk.binary, cdt, ch);
    var_refactor<L>(g, v, pk, ih, dh, cdt, ch, odt, oh);
    sF[g.task] = odt;
    sC[g.task] = oh;
}

// The step-dt coefficients of a branch back from HBM after a shortened
// step (the branch's position fields are unchanged): every row's loads issued
// at once, at clamped rows for the pads, as load_slot does.
template <int L>
__device__ __forceinline__ void restore_coefficients(Slot<L>& g, const StepArgs& a, const PackDesc& pk) {
    if (g.r < 0) return;
    int base = g.base, w = g.w, len = g.len;
    asm volatile("" : "+v"(base), "+v"(w), "+v"(len));
    double q = 1.0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int64_t sl = pk.slot0 + base + int64_t(min(k, len - 1)) * w;
        const double al = a.alpha[sl], f = a.F[sl], dv = a.invd[sl];
        if (k < len) {
            g.A[k] = al;
            g.F[k] = f;
            g.D[k] = dv;
            if (k >= 1) q *= -f;
        }
    }
    g.FQ = g.F[0] * q;
    g.Z = a.tk_Z[pk.tk0 + g.task];
    g.Zp = (g.ptask != pk.ntk) ? a.tk_Z[pk.tk0 + g.ptask] : 0.0;
}

// The cell's time, its event cursors and their next times are the same in
// every thread: kept in scalar registers, so that the vector registers stay
// with the branches' coefficients.
__device__ __forceinline__ double uniform(double x) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int64_t uniform(int64_t x) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint64_t(x) & 0xffffffffu)));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint64_t(x) >> 32)));
    return int64_t((uint64_t(hi) << 32) | lo);
}

template <int T, int S, int L>
__global__ void __launch_bounds__(T, (S * L <= 8) ? 3 : (S * L <= 16 ? 2 : 1))
    var_step_kernel(StepArgs a, VarArgs v) {
    extern __shared__ __align__(16) char lds_raw[];
    const int p = blockIdx.x + a.pack0;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    // ---- LDS: the register layout's (pack_lds_bytes, mode 3, state in LDS) ----
    double* sV = reinterpret_cast<double*>(lds_raw);
    double* sg = sV + vr_block_doubles(ns, pk.spare);
    double* s_se = sg + pk.nsyn;
    double* s_sdec = s_se + pk.nsyn;
    double* sm = s_sdec + pk.nsyn;
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    double* s_gna = sn + pk.nhh;
    double* s_gk = s_gna + pk.nhh;
    double* s_nlb = s_gk + pk.nhh;
    double* sC = s_nlb + pk.nnl;
    double* sX = sC;
    double* sF = sC + (pk.ntk + 2);
    double* sY = sF;
    double* sQ = sF + (pk.ntk + 2);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(sQ + (pk.binary ? pk.ntk + 2 : 0));
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);
    int32_t* s_hhs = s_ch + (pk.binary ? 0 : pk.nch);

    for (int i = tid; i < ns; i += T) {
        sV[vix(i)] = a.V[pk.slot0 + i];
        sV[vix(i) + kRoff] = a.beta[pk.slot0 + i];
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
        if (d.hh >= 0) s_hhs[d.hh] = vix(d.slot);
    }
    if (!pk.binary)
        for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_task[pk.ch0 + i];

    int64_t step0 = a.step0;
    if (a.epoch_ptr) step0 = *a.epoch_ptr * a.nsteps;
    const int64_t estart = step0 - step0 % a.epoch_steps;
    // The cell's event cursors, its time and the next decision live in LDS
    // and are read and written by thread 0, which delivers the events: the
    // other threads carry only the grid step and the end of the current run
    // of steps of dt from one decision to the next.  Network events of the
    // epoch are in time order; the launch starts at the first one of its
    // grid interval (earlier ones were taken before).
    __shared__ double cb_t, cb_t0, cb_tn, cb_tx, cb_h;
    __shared__ int64_t cb_ncur, cb_xcur, cb_nend, cb_kf, cb_nsub;
    __shared__ int32_t cb_full, cb_on_grid;
    const double kInf = __builtin_inf();
    if (tid == 0) {
        const uint32_t* eoff = a.bk_off ? a.bk_off + int64_t(p) * (a.epoch_steps + 1) : nullptr;
        const double* et = v.bk_t + int64_t(p) * a.bk_cap;
        const int64_t ncur = eoff ? int64_t(eoff[step0 - estart]) : 0;
        const int64_t nend = eoff ? int64_t(eoff[a.epoch_steps]) : 0;
        const int64_t xcur = a.pk_xcur[p];
        cb_ncur = ncur;
        cb_nend = nend;
        cb_xcur = xcur;
        cb_tn = (ncur < nend) ? et[ncur] : kInf;         // next network event
        cb_tx = (xcur < pk.xe1) ? v.xe_t[xcur] : kInf;   // next external event
        cb_t = double(step0) * a.dt;
        cb_nsub = 0;
    }
    const int soma = (tid < pk.ncell) ? vix(a.pc_soma[pk.cell0 + tid]) : -1;
    // a pack with at most kSpreadHH hh instances gives each gate a thread:
    // this thread's instance and gate, and the gate's constants
    static_assert(3 * kSpreadHH <= T, "one gate per thread");
    const int hq = tid / 3, hw = tid - 3 * hq;
    const HHGate hc = hh_gate_consts(hw);
    double vold = 0.0;

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

    const int64_t kend = step0 + a.nsteps;
    int64_t k = step0;
    int64_t kf = k;  // steps of dt run while k < kf, with no event due
    while (k < kend) {
        bool full = k < kf;
        double t = double(k) * a.dt, h = a.dt;
        bool on_grid = true;
        if (!full) {
            if (tid == 0) {
                // A: every event due at or before t, network ones first
                const double tc = cb_t;
                double tn = cb_tn, tx = cb_tx;
                if (tn <= tc || tx <= tc) {
                    const int32_t* eq = a.bk_q + int64_t(p) * a.bk_cap;
                    const double* ew = a.bk_w + int64_t(p) * a.bk_cap;
                    const double* et = v.bk_t + int64_t(p) * a.bk_cap;
                    int64_t ncur = cb_ncur, xcur = cb_xcur;
                    const int64_t nend = cb_nend;
                    while (tn <= tc) {
                        sg[eq[ncur]] += ew[ncur];
                        ++ncur;
                        tn = (ncur < nend) ? et[ncur] : kInf;
                    }
                    while (tx <= tc) {
                        sg[a.xe_syn[xcur]] += a.xe_w[xcur];
                        ++xcur;
                        tx = (xcur < pk.xe1) ? v.xe_t[xcur] : kInf;
                    }
                    cb_ncur = ncur;
                    cb_xcur = xcur;
                    cb_tn = tn;
                    cb_tx = tx;
                }
                const double next = fmin(tn, tx);  // > tc
                const double grid1 = double(k + 1) * a.dt;
                if (tc == double(k) * a.dt && !(next < grid1)) {
                    // on the grid, no event inside the coming interval:
                    // steps of dt up to the grid point at or before the
                    // next event
                    int64_t e = kend;
                    if (next < double(kend) * a.dt) {
                        e = int64_t(next / a.dt);
                        while (e > k + 1 && double(e) * a.dt > next) --e;
                        while (e + 1 < kend && double(e + 1) * a.dt <= next) ++e;
                        e = e < k + 1 ? k + 1 : e;
                    }
                    cb_full = 1;
                    cb_kf = e;
                    cb_t = double(e) * a.dt;
                    cb_nsub += e - k;
                } else {
                    // a step cut at the next event, or ending on the grid
                    // from an off-grid time
                    const double target = (next < grid1) ? next : grid1;
                    cb_full = 0;
                    cb_t0 = tc;
                    cb_h = target - tc;
                    cb_on_grid = !(next < grid1);
                    cb_t = target;
                    cb_nsub += 1;
                }
            }
            round_sync<T>();
            full = __builtin_amdgcn_readfirstlane(cb_full) != 0;
            if (full) {
                kf = uniform(cb_kf);
            } else {
                h = uniform(cb_h);
                t = uniform(cb_t0);
                on_grid = __builtin_amdgcn_readfirstlane(cb_on_grid) != 0;
            }
            round_sync<T>();  // every thread has read the decision before it changes
        }
        if (!full) {  // the branches' coefficients for h, deepest level first
            const double ih = 1.0 / h, dh = ih - 1.0 / a.dt;
            for (int lv = pk.nlev - 1; lv >= 0; --lv) {
                refactor_level<L>(g0, lv, v, pk, ih, dh, sC, sF, s_ch);
                if constexpr (S > 1) refactor_level<L>(g1, lv, v, pk, ih, dh, sC, sF, s_ch);
                if constexpr (S > 2) refactor_level<L>(g2, lv, v, pk, ih, dh, sC, sF, s_ch);
                round_sync<T>();
            }
            // each branch's Z for its children, F_0 Q_0 for the up passes
            if (g0.r >= 0) sF[g0.task] = g0.Z;
            if constexpr (S > 1) {
                if (g1.r >= 0) sF[g1.task] = g1.Z;
            }
            if constexpr (S > 2) {
                if (g2.r >= 0) sF[g2.task] = g2.Z;
            }
            if (pk.binary) {
                if (g0.r >= 0) sQ[g0.task] = g0.FQ;
                if constexpr (S > 1) {
                    if (g1.r >= 0) sQ[g1.task] = g1.FQ;
                }
                if constexpr (S > 2) {
                    if (g2.r >= 0) sQ[g2.task] = g2.FQ;
                }
            }
            round_sync<T>();
            if (g0.r >= 0) g0.Zp = sF[g0.ptask];
            if constexpr (S > 1) {
                if (g1.r >= 0) g1.Zp = sF[g1.ptask];
            }
            if constexpr (S > 2) {
                if (g2.r >= 0) g2.Zp = sF[g2.ptask];
            }
            round_sync<T>();
        }

        // B: R = beta - I at the nonlinear CVs (V at t); synapses decay over
        // the step here (g is not read again before the next events)
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double vv = sV[vix(d.slot)];
            double I = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = sm[q], hg = sh[q], x = sn[q];
                I += s_gna[q] * (m * m * m * hg) * (vv - kENa);
                I += s_gk[q] * (x * x * x * x) * (vv - kEK);
            }
            if (full) {
                for (int c = 0; c < d.nsyn; ++c) {
                    const int q = d.syn0 + c;
                    const double gq = sg[q];
                    I += gq * (vv - s_se[q]);
                    sg[q] = gq * s_sdec[q];
                }
            } else {
                for (int c = 0; c < d.nsyn; ++c) {
                    const int q = d.syn0 + c;
                    const double gq = sg[q];
                    I += gq * (vv - s_se[q]);
                    sg[q] = gq * exp(-h / v.syn_tau[pk.syn0 + q]);
                }
            }
            sV[vix(d.slot) + kRoff] = s_nlb[j] - I;
        }
        if (soma >= 0) vold = sV[soma];
        round_sync<T>();

        // C/D: the split Hines solve with the registers' coefficients
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
        store_v<L>(g0, sV, y0);
        if constexpr (S > 1) store_v<L>(g1, sV, y1);
        if constexpr (S > 2) store_v<L>(g2, sV, y2);
        round_sync<T>();

        // E: gates over h with the new V; threshold, the crossing time
        // interpolated within the step
        if (pk.nhh <= kSpreadHH) {
            if (tid < 3 * pk.nhh) {
                double* x = (hw == 0) ? sm : (hw == 1) ? sh : sn;
                x[hq] = hh_gate_step(hc, sV[hv], x[hq], h);
            }
        } else {
            for (int q = tid; q < pk.nhh; q += T) {
                const Rates rt = hh_rates(sV[s_hhs[q]]);
                sm[q] = gate_step(sm[q], rt.am, rt.bm, h);
                sh[q] = gate_step(sh[q], rt.ah, rt.bh, h);
                sn[q] = gate_step(sn[q], rt.an, rt.bn, h);
            }
        }
        if (soma >= 0) {
            const double vnew = sV[soma];
            if (vold < a.threshold && vnew >= a.threshold) {
                const double ts = t + h * (a.threshold - vold) / (vnew - vold);
                const uint32_t pos = atomicAdd(&a.ctr->sp_count, 1u);
                if (pos < a.sp_cap) {
                    a.sp_gid[pos] = uint32_t(a.pc_gid[pk.cell0 + tid]);
                    a.sp_step[pos] = __double_as_longlong(ts);  // the exchange carries the time
                    a.sp_t[pos] = ts;
                } else {
                    atomicOr(&a.ctr->flags, kFlagSpikeOverflow);
                }
            }
        }
        if (on_grid && a.trace) {
            const int64_t col = k - a.trace_step0;
            if (col >= 0 && col < a.trace_cap)
                for (int j = tid; j < pk.npr; j += T)
                    a.trace[int64_t(a.pr_id[pk.pr0 + j]) * a.trace_cap + col] = sV[vix(a.pr_slot[pk.pr0 + j])];
        }
        if (!full) {  // the step-dt coefficients back
            restore_coefficients<L>(g0, a, pk);
            if constexpr (S > 1) restore_coefficients<L>(g1, a, pk);
            if constexpr (S > 2) restore_coefficients<L>(g2, a, pk);
            if (pk.binary) {
                if (g0.r >= 0) sQ[g0.task] = g0.FQ;
                if constexpr (S > 1) {
                    if (g1.r >= 0) sQ[g1.task] = g1.FQ;
                }
                if constexpr (S > 2) {
                    if (g2.r >= 0) sQ[g2.task] = g2.FQ;
                }
            }
        }
        round_sync<T>();
        if (full || on_grid) ++k;
    }

    for (int i = tid; i < ns; i += T) a.V[pk.slot0 + i] = sV[vix(i)];
    for (int i = tid; i < pk.nsyn; i += T) a.syn_g[pk.syn0 + i] = sg[i];
    for (int i = tid; i < pk.nhh; i += T) {
        a.hh_m[pk.hh0 + i] = sm[i];
        a.hh_h[pk.hh0 + i] = sh[i];
        a.hh_n[pk.hh0 + i] = sn[i];
    }
    if (tid == 0) {
        a.pk_xcur[p] = cb_xcur;
        v.pk_steps[p] += cb_nsub;
    }
}

// The grid interval j (relative to the epoch's first, lo) holding arrival
// time ta: (lo + j) dt <= ta < (lo + j + 1) dt with the grid points as the
// step kernel computes them; -1 outside the epoch.  An arrival before the
// epoch from a spike of the epoch just ended is due at once: interval 0.
__device__ __forceinline__ int arrival_bin(double ts, double ta, int64_t lo, int K, double dt) {
    if (ta < double(lo) * dt) return (ts >= double(lo - K) * dt) ? 0 : -1;
    if (!(ta < double(lo + K) * dt)) return -1;
    int64_t j = int64_t(ta / dt) - lo;
    j = j < 0 ? 0 : (j > K - 1 ? K - 1 : j);
    while (j > 0 && double(lo + j) * dt > ta) --j;
    while (j + 1 < K && double(lo + j + 1) * dt <= ta) ++j;
    return int(j);
}

__device__ __forceinline__ bool event_less(double ta, int32_t qa, double wa, double tb, int32_t qb, double wb) {
    if (ta != tb) return ta < tb;
    if (qa != qb) return qa < qb;
    return wa < wb;
}

// One wave per pack: count the epoch's events per grid interval, scan the
// counts into the intervals' first positions, place the events (any order
// within an interval), then sort each interval by (time, synapse, weight).
__global__ void __launch_bounds__(64) pull_timed_kernel(TimedPullArgs a) {
    extern __shared__ uint32_t bins[];  // [K] counts, then cursors; [K + 1] starts
    const int K = a.epoch_steps;
    uint32_t* start = bins + K;
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t e = a.epoch_ptr ? *a.epoch_ptr : a.epoch;
    const int64_t lo = e * K;
    const int64_t r0 = a.in_off[p], r1 = a.in_off[p + 1];
    uint32_t* off = a.bk_off + int64_t(p) * (K + 1);
    if (a.sx_off[a.n_src] == 0) {  // no spikes in the history: no events this epoch
        for (int b = lane; b <= K; b += 64) off[b] = 0u;
        return;
    }
    for (int b = lane; b < K; b += 64) bins[b] = 0u;
    __syncthreads();
    for (int64_t r = r0 + lane; r < r1; r += 64) {
        const uint32_t src = a.cr_src[r];
        const double d = a.cr_delay_ms[r];
        for (int64_t k = a.sx_off[src]; k < a.sx_off[src + 1]; ++k) {
            const double ts = __longlong_as_double(a.sx_step[k]);
            const int b = arrival_bin(ts, ts + d, lo, K, a.dt);
            if (b >= 0) atomicAdd(&bins[b], 1u);
        }
    }
    __syncthreads();
    uint32_t run = 0;
    for (int b0 = 0; b0 < K; b0 += 64) {
        const int b = b0 + lane;
        const uint32_t c = b < K ? bins[b] : 0u;
        uint32_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (b < K) {
            bins[b] = run + x - c;
            start[b] = run + x - c;
        }
        run += __shfl(x, 63);
    }
    const uint32_t total = run;
    const uint32_t cap = uint32_t(a.bk_cap);
    if (lane == 0) start[K] = total;
    __syncthreads();
    for (int b = lane; b <= K; b += 64) off[b] = start[b] < cap ? start[b] : cap;
    int32_t* oq = a.bk_q + int64_t(p) * a.bk_cap;
    double* ow = a.bk_w + int64_t(p) * a.bk_cap;
    double* ot = a.bk_t + int64_t(p) * a.bk_cap;
    for (int64_t r = r0 + lane; r < r1; r += 64) {
        const uint32_t src = a.cr_src[r];
        const double d = a.cr_delay_ms[r];
        const int64_t k0 = a.sx_off[src], k1 = a.sx_off[src + 1];
        if (k1 == k0) continue;
        const int32_t q = a.cr_syn[r];
        const double w = a.cr_w[r];
        for (int64_t k = k0; k < k1; ++k) {
            const double ts = __longlong_as_double(a.sx_step[k]);
            const double ta = ts + d;
            const int b = arrival_bin(ts, ta, lo, K, a.dt);
            if (b < 0) continue;
            const uint32_t pos = atomicAdd(&bins[b], 1u);
            if (pos < cap) {
                oq[pos] = q;
                ow[pos] = w;
                ot[pos] = ta;
            }
        }
    }
    __threadfence_block();
    __syncthreads();
    // insertion sort of each interval (intervals hold few events)
    for (int b = lane; b < K; b += 64) {
        const uint32_t s0 = start[b] < cap ? start[b] : cap;
        const uint32_t s1 = start[b + 1] < cap ? start[b + 1] : cap;
        for (uint32_t i = s0 + 1; i < s1; ++i) {
            const double ti = ot[i], wi = ow[i];
            const int32_t qi = oq[i];
            uint32_t j = i;
            while (j > s0 && event_less(ti, qi, wi, ot[j - 1], oq[j - 1], ow[j - 1])) {
                ot[j] = ot[j - 1];
                oq[j] = oq[j - 1];
                ow[j] = ow[j - 1];
                --j;
            }
            ot[j] = ti;
            oq[j] = qi;
            ow[j] = wi;
        }
    }
    if (lane == 0 && total > cap) atomicOr(&a.ctr->flags, kFlagEventOverflow);
}

template <int T, int S, int L>
hipError_t launch_var(const StepArgs& a, const VarArgs& v, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    hipLaunchKernelGGL((var_step_kernel<T, S, L>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a, v);
    return hipGetLastError();
}

template <int T>
hipError_t launch_var_T(const StepArgs& a, const VarArgs& v, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.reg_len == 8) {
        switch (cfg.reg_slots) {
            case 1: return launch_var<T, 1, 8>(a, v, cfg, n_packs, st);
            case 2: return launch_var<T, 2, 8>(a, v, cfg, n_packs, st);
            case 3: return launch_var<T, 3, 8>(a, v, cfg, n_packs, st);
            default: break;
        }
    } else if (cfg.reg_len == 16 && cfg.reg_slots == 1) {
        return launch_var<T, 1, 16>(a, v, cfg, n_packs, st);
    }
    return hipErrorInvalidValue;
}

void allow_lds_fn(const void* f, int lds_max) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
}

template <int T>
void allow_lds_T(int lds_max) {
    allow_lds_fn(reinterpret_cast<const void*>(&var_step_kernel<T, 1, 8>), lds_max);
    allow_lds_fn(reinterpret_cast<const void*>(&var_step_kernel<T, 2, 8>), lds_max);
    allow_lds_fn(reinterpret_cast<const void*>(&var_step_kernel<T, 3, 8>), lds_max);
    allow_lds_fn(reinterpret_cast<const void*>(&var_step_kernel<T, 1, 16>), lds_max);
}

}  // namespace

hipError_t prepare_var_kernels(int lds_max) {
    allow_lds_T<64>(lds_max);
    allow_lds_T<128>(lds_max);
    allow_lds_T<256>(lds_max);
    allow_lds_fn(reinterpret_cast<const void*>(&pull_timed_kernel), lds_max);
    return hipSuccess;
}

hipError_t launch_var_step(const StepArgs& a, const VarArgs& v, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.coef_mode != 3 || cfg.syn_hbm || cfg.rec) return hipErrorInvalidValue;
    switch (cfg.block_threads) {
        case 64: return launch_var_T<64>(a, v, cfg, n_packs, st);
        case 128: return launch_var_T<128>(a, v, cfg, n_packs, st);
        case 256: return launch_var_T<256>(a, v, cfg, n_packs, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pull_timed(const TimedPullArgs& a, int32_t n_packs, hipStream_t st) {
    hipLaunchKernelGGL(pull_timed_kernel, dim3(n_packs), dim3(64), size_t(2 * a.epoch_steps + 1) * 4, st, a);
    return hipGetLastError();
}

}  // namespace arbmi
