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
// The solve of a branch is split so that only one multiply-add per branch
// waits on the tree.  With the children's sum s and the parent's new V xp
// as unknowns, the branch's recurrences are linear in them:
//   rhs'_k = P_k - Q_k s,  F_0 rhs'_0 = F_0 P_0 - (F_0 Q_0) s,
//   V_last = Y_last + Z xp,
// where P and Y come from the branch's own CVs (all branches at once) and
// F_0 Q_0 = F_0 prod_{k>=1}(-F_k), Z = prod_k(-F_k) are step-invariant.  So a
// step runs: all branches' local elimination; rounds deepest first passing
// the contributions up (one multiply-add per branch); all branches' full
// elimination with their s and the local substitution; rounds shallowest
// first passing the distal V down, two tree levels a round (a branch forms
// its parent's V from its grandparent's: x_p = Y_p + Z_p x_gp); all
// branches' substitution with xp.
// The elimination and substitution themselves are the Hines recurrences of
// the serial solve; only the values passed between branches are formed
// through the split.
//
// LDS keeps V and R (the right-hand side) per slot, in blocks of 64 slots
// (64 V then 64 R): V-only accesses of consecutive slots are 8 bytes apart
// and R is a fixed offset from V.  R holds beta (the step-invariant part of
// the right-hand side) minus the point currents.
// Between the phases of the solve, a branch keeps its intermediate values
// in its own V entries.  Every branch has L rows in the layout; a shorter
// branch's spare rows hold pad CVs (alpha = beta = 1/d' = 0) that carry the
// recurrences through unchanged (F = +1 at the first pad, -1 after it).
// An empty register slot works on a slot no CV uses (a pad row, or one past
// the pack's slots).
// The kernel does not record states for the adjoint (the host refuses that).
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"
#include "kernels.hpp"

namespace arbmi {

namespace {

using namespace dev;

// The registers of one branch slot.
template <int L>
struct Slot {
    double A[L], F[L], D[L];  // alpha, F (pads: +1 then -1), 1/d' (pads: 0)
    double FQ;                // F_0 Q_0
    double Z, Zp;             // prod_k (-F_k) of this branch and of its parent
    double fp, cs, yl, xp;    // per step: F_0 P_0, children's sum, V_last with xp = 0, parent's V
    int base, w, len;         // CV k of the branch is slot base + k w
    int r;                    // round of the branch, -1 if the slot is empty
    int lev;                  // depth level (the soma is 0)
    int task, ptask, gptask;  // own, parent's and grandparent's task (none: a zero entry)
    int c0, c1;               // first two children's tasks (a zero entry if fewer)
    int x0, x1;               // binary packs: grandchildren's tasks, two 16-bit fields each
                              // (children of c0, of c1); other packs: further children
                              // s_ch[x0 .. x0 + x1)
};

// V and R sit in blocks of 64 slots: 64 V, then the same slots' 64 R.  So
// consecutive slots are 8 bytes apart (no bank conflicts for V alone) and R
// is a fixed 512 bytes past V.
__device__ __forceinline__ int vix(int slot) { return slot + (slot & ~63); }
constexpr int kRoff = 64;

// V index of the branch's CV k
template <int L>
__device__ __forceinline__ int cv_slot(const Slot<L>& g, int k) {
    return vix(g.base + k * g.w);
}

// The three all-branch parts of the solve, each split into loads, arithmetic
// and stores so that the kernel can issue every slot's loads before any
// slot's stores (LDS stores may alias later loads, so the compiler keeps
// them in source order) and overlap the slots' recurrences.

// Local elimination (children's sum taken as 0): t_k = alpha_k V_k + R_k,
// P_k = t_k - F_{k+1} P_{k+1}.  t stays in the thread's registers; F_0 P_0
// is the branch's contribution if it has no children.
template <int L>
__device__ __forceinline__ void local_load(const Slot<L>& g, const double* sV, double* t) {
#pragma unroll
    for (int k = 0; k < L; ++k) t[k] = g.A[k] * sV[cv_slot(g, k)] + sV[cv_slot(g, k) + kRoff];
}
template <int L>
__device__ __forceinline__ void local_chain(Slot<L>& g, const double* t) {
    double acc = 0.0;
#pragma unroll
    for (int k = L - 1; k >= 0; --k) acc = (k == L - 1) ? t[k] : t[k] - g.F[(k + 1 < L) ? k + 1 : k] * acc;
    g.fp = g.F[0] * acc;
}
template <int L>
__device__ __forceinline__ void local_store(const Slot<L>& g, double* sC, double* sF) {
    sC[g.task] = g.fp;
    sF[g.task] = g.fp;
}

// Full elimination with the children's sum (t becomes rhs'/d', kept in
// registers for the substitution), and the distal V for a grounded parent.
template <int L>
__device__ __forceinline__ void full_chain(Slot<L>& g, double* t) {
    double acc = (g.len == L) ? g.cs : -g.cs;
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
        const double r = (k == L - 1) ? t[k] - acc : t[k] - g.F[(k + 1 < L) ? k + 1 : k] * acc;
        t[k] = r * g.D[k];
        acc = r;
    }
    double x = 0.0;
#pragma unroll
    for (int k = 0; k < L; ++k) x = t[k] - g.F[k] * x;
    g.yl = (g.len == L) ? x : -x;
}
template <int L>
__device__ __forceinline__ void store_v(const Slot<L>& g, double* sV, const double* t) {
#pragma unroll
    for (int k = 0; k < L; ++k) sV[cv_slot(g, k)] = t[k];
}

// Substitution with the parent's V: V_k = rhs'_k/d'_k - F_k V_{k-1}.
template <int L>
__device__ __forceinline__ void subst_chain(const Slot<L>& g, double* y) {
    double x = g.xp;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        x = y[k] - g.F[k] * x;
        y[k] = x;
    }
}

// Fill slot g with the branch this thread takes in round r of the pack (an
// empty slot, len 0, if r < 0).  Branch-free: an empty slot reads valid
// entries of the pack and keeps neutral values.
template <int L>
__device__ __forceinline__ void load_slot(Slot<L>& g, const StepArgs& a, const PackDesc& pk, int r, int tid) {
    const bool has = r >= 0;
    const int none = pk.ntk, dump = pk.ntk + 1;
    const RoundDesc R = a.rd[pk.rd0 + (has ? r : 0)];
    const int i = has ? round_index(R, tid) : 0;
    const int task = has ? R.task0 + i : 0;
    const TaskDesc t = a.tk[pk.tk0 + task];
    const int len = has ? t.len : 0;
    g.r = has ? r : -1;
    g.len = len;
    g.base = has ? R.slot0 + i : pk.spare;
    g.w = has ? R.w : 0;
    g.task = has ? task : dump;
    const int pt = a.tk_ptask[pk.tk0 + task];
    g.ptask = (has && pt >= 0) ? pt : none;
    const int gpt = (g.ptask != none) ? a.tk_ptask[pk.tk0 + g.ptask] : -1;
    g.gptask = (gpt >= 0) ? gpt : none;
    g.lev = has ? a.tk_lev[pk.tk0 + task] : -1000;  // empty: no round matches
    g.Zp = (g.ptask != none) ? a.tk_Z[pk.tk0 + g.ptask] : 0.0;
    g.c0 = none;
    g.c1 = none;
    if (has && t.nch > 0) g.c0 = a.ch_task[pk.ch0 + t.ch0];
    if (has && t.nch > 1) g.c1 = a.ch_task[pk.ch0 + t.ch0 + 1];
    if (pk.binary) {
        int gc[4] = {none, none, none, none};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = h ? g.c1 : g.c0;
            if (c != none) {
                const TaskDesc tc = a.tk[pk.tk0 + c];
                if (tc.nch > 0) gc[2 * h] = a.ch_task[pk.ch0 + tc.ch0];
                if (tc.nch > 1) gc[2 * h + 1] = a.ch_task[pk.ch0 + tc.ch0 + 1];
            }
        }
        g.x0 = gc[0] | (gc[1] << 16);
        g.x1 = gc[2] | (gc[3] << 16);
    } else {
        g.x0 = t.ch0 + 2;
        g.x1 = has ? max(0, t.nch - 2) : 0;
    }
    double q = 1.0, z = 1.0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const bool real = k < len;
        const int64_t sl = pk.slot0 + (has ? g.base + int64_t(min(k, len - 1)) * g.w : 0);
        const double al = a.alpha[sl], f = a.F[sl], dv = a.invd[sl];
        g.A[k] = real ? al : 0.0;
        g.D[k] = real ? dv : 0.0;
        g.F[k] = real ? f : (k == len ? 1.0 : -1.0);
        if (real) z *= -g.F[k];
        if (real && k >= 1) q *= -g.F[k];
    }
    g.FQ = g.F[0] * q;
    g.Z = has ? a.tk_Z[pk.tk0 + task] : z;
    g.fp = 0.0;
    g.cs = 0.0;
    g.yl = 0.0;
    g.xp = 0.0;
}

// Up round, one level at a time: the children's sum and this branch's
// contribution to its parent.
template <int L>
__device__ __forceinline__ void pass_up(Slot<L>& g, double* sC, const int32_t* s_ch) {
    double cs = sC[g.c0] + sC[g.c1];
    for (int q = 0; q < g.x1; ++q) cs += sC[s_ch[g.x0 + q]];
    g.cs = cs;
    sC[g.task] = g.fp - g.FQ * cs;
}

// Up round, two levels at a time (packs of at most binary branch points):
// each child's contribution formed from its local value and its own
// children's final contributions, C_c = F_0 P_0(c) - F_0 Q_0(c) sum C_g, so a
// branch and its children share a round.
template <int L>
__device__ __forceinline__ void pass_up2(Slot<L>& g, const double* sF, const double* sQ, double* sC) {
    const int g00 = g.x0 & 0xffff, g01 = int(unsigned(g.x0) >> 16);
    const int g10 = g.x1 & 0xffff, g11 = int(unsigned(g.x1) >> 16);
    const double s0 = sF[g.c0] - sQ[g.c0] * (sC[g00] + sC[g01]);
    const double s1 = sF[g.c1] - sQ[g.c1] * (sC[g10] + sC[g11]);
    g.cs = s0 + s1;
    sC[g.task] = g.fp - g.FQ * g.cs;
}

// Down round, two levels at a time: the parent's V from the grandparent's
// (x_p = Y_p + Z_p x_gp, so a branch and its parent can take the same round),
// then this branch's distal V.
template <int L>
__device__ __forceinline__ void pass_down(Slot<L>& g, const double* sY, double* sX) {
    g.xp = sY[g.ptask] + g.Zp * sX[g.gptask];
    sX[g.task] = g.yl + g.Z * g.xp;
}

// End of a round of the tree passes.  A one-wave workgroup needs no
// barrier and no wait: a wave's LDS operations take effect in issue order,
// so the next round's loads see this round's stores.
template <int T>
__device__ __forceinline__ int block_count(bool pred) {
    if constexpr (T == 64)
        return __popcll(__ballot(pred));
    else
        return __syncthreads_count(pred);
}

template <int T>
__device__ __forceinline__ void round_sync() {
    if constexpr (T == 64)
        __builtin_amdgcn_wave_barrier();
    else
        __syncthreads();
}

// Waves per SIMD the registers allow without spilling (built without
// machine loop-invariant code motion): three for one slot of 8 CVs, two for
// 16 CVs in all, one otherwise.  G: some pack of the launch keeps its
// synapse state in HBM (without it, that path is compiled out).
template <int T, int S, int L, bool G>
__global__ void __launch_bounds__(T, (S * L <= 8) ? 3 : (S * L <= 16 ? 2 : 1)) reg_step_kernel(StepArgs a) {
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
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    double* s_gna = sn + pk.nhh;
    double* s_gk = s_gna + pk.nhh;
    double* s_nlb = s_gk + pk.nhh;                             // beta of each nonlinear CV
    // per task, two spare entries (zero, discard) each: contribution, then
    // distal V; contribution with no children, then distal V for a grounded
    // parent; F_0 Q_0 (binary packs)
    double* sC = s_nlb + pk.nnl;
    double* sX = sC;
    double* sF = sC + (pk.ntk + 2);
    double* sY = sF;
    double* sQ = sF + (pk.ntk + 2);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(sQ + (pk.binary ? pk.ntk + 2 : 0));
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);  // children's tasks (other packs)
    int32_t* s_hhs = s_ch + (pk.binary ? 0 : pk.nch);          // per hh instance: its CV's slot

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
    for (int i = tid; i < nsyn_lds; i += T) {
        sg[i] = g_g[i];
        s_se[i] = g_se[i];
        s_sdec[i] = g_sdec[i];
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
    // network events: where each step of the epoch starts in the pack's
    // bucket; external-event cursor, the same in every thread
    const int64_t estart = step0 - step0 % a.epoch_steps;
    const uint32_t* eoff = a.bk_off ? a.bk_off + int64_t(p) * (a.epoch_steps + 1) : nullptr;
    const int32_t* eq = a.bk_q + int64_t(p) * a.bk_cap;
    const double* ew = a.bk_w + int64_t(p) * a.bk_cap;
    // the next step of the epoch with network events: steps without any
    // load nothing
    const uint32_t* enxt = eoff ? a.bk_nxt + int64_t(p) * (a.epoch_steps + 1) : nullptr;
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
            double I = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = sm[q], h = sh[q], x = sn[q];
                I += s_gna[q] * (m * m * m * h) * (v - kENa);
                I += s_gk[q] * (x * x * x * x) * (v - kEK);
            }
            if (!syn_hbm) {
                // the decay of phase E is applied here too: g is not read
                // again before the next step's events
                for (int k = 0; k < d.nsyn; ++k) {
                    const int q = d.syn0 + k;
                    const double gq = sg[q];
                    I += gq * (v - s_se[q]);
                    sg[q] = gq * s_sdec[q];
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
            sV[vix(d.slot) + kRoff] = s_nlb[j] - I;
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
        if (pk.binary) {  // contributions up, two levels a round, deepest first
            for (int sr = 0; 2 * sr < pk.nlev; ++sr) {
                if (((pk.nlev - 1 - g0.lev) >> 1) == sr && g0.c0 != pk.ntk) pass_up2<L>(g0, sF, sQ, sC);
                if constexpr (S > 1) {
                    if (((pk.nlev - 1 - g1.lev) >> 1) == sr && g1.c0 != pk.ntk) pass_up2<L>(g1, sF, sQ, sC);
                }
                if constexpr (S > 2) {
                    if (((pk.nlev - 1 - g2.lev) >> 1) == sr && g2.c0 != pk.ntk) pass_up2<L>(g2, sF, sQ, sC);
                }
                round_sync<T>();
            }
        } else {
            for (int r = 0; r < pk.nrd; ++r) {  // contributions up, deepest rounds first
                if (g0.r == r && g0.c0 != pk.ntk) pass_up<L>(g0, sC, s_ch);
                if constexpr (S > 1) {
                    if (g1.r == r && g1.c0 != pk.ntk) pass_up<L>(g1, sC, s_ch);
                }
                if constexpr (S > 2) {
                    if (g2.r == r && g2.c0 != pk.ntk) pass_up<L>(g2, sC, s_ch);
                }
                round_sync<T>();
            }
        }
        {
            full_chain<L>(g0, y0);
            if constexpr (S > 1) full_chain<L>(g1, y1);
            if constexpr (S > 2) full_chain<L>(g2, y2);
            sY[g0.task] = g0.yl;
            if constexpr (S > 1) sY[g1.task] = g1.yl;
            if constexpr (S > 2) sY[g2.task] = g2.yl;
        }
        round_sync<T>();
        for (int sr = 0; 2 * sr < pk.nlev; ++sr) {  // distal V down, two levels a round, shallowest first
            if ((g0.lev >> 1) == sr) pass_down<L>(g0, sY, sX);
            if constexpr (S > 1) {
                if ((g1.lev >> 1) == sr) pass_down<L>(g1, sY, sX);
            }
            if constexpr (S > 2) {
                if ((g2.lev >> 1) == sr) pass_down<L>(g2, sY, sX);
            }
            round_sync<T>();
        }
        {
            subst_chain<L>(g0, y0);
            if constexpr (S > 1) subst_chain<L>(g1, y1);
            if constexpr (S > 2) subst_chain<L>(g2, y2);
            store_v<L>(g0, sV, y0);
            if constexpr (S > 1) store_v<L>(g1, sV, y1);
            if constexpr (S > 2) store_v<L>(g2, sV, y2);
        }
        round_sync<T>();

        // E: states with V^{n+1} (synapses decayed in phase B); threshold.  A
        // pack with few hh instances gives each gate of an instance its own
        // thread (which computes that gate's two rates and the update);
        // otherwise a thread takes a whole instance.
        if (pk.nhh <= kSpreadHH) {
            for (int j = tid; j < 3 * pk.nhh; j += T) {
                const int q = j / 3, w = j - 3 * q;
                double al, be;
                hh_gate_rates(w, sV[s_hhs[q]], al, be);
                double* x = (w == 0) ? sm : (w == 1) ? sh : sn;
                x[q] = gate_step_pair(x[q], al, be, a.dt);
            }
        } else {
            for (int q = tid; q < pk.nhh; q += T) {
                const Rates rt = hh_rates(sV[s_hhs[q]]);
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
    if (cfg.syn_hbm)
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, true>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a);
    else
        hipLaunchKernelGGL((reg_step_kernel<T, S, L, false>), dim3(n_packs), dim3(T), cfg.lds_bytes, st, a);
    return hipGetLastError();
}

template <int T, int S, int L, bool G>
void allow_lds_one(int lds_max) {
    const void* f = reinterpret_cast<const void*>(&reg_step_kernel<T, S, L, G>);
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, f) != hipSuccess) return;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
}

template <int T, int S, int L>
void allow_lds(int lds_max) {
    allow_lds_one<T, S, L, false>(lds_max);
    allow_lds_one<T, S, L, true>(lds_max);
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
