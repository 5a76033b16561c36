// reg_solve.hpp -- the register-resident layout's per-thread branch state
// and the split Hines solve on it, shared by the step kernel
// (reg_kernels.hip) and its adjoint (reg_adjoint_kernels.hip).
//
// A thread owns up to S branches ("register slots") of at most L CVs; the
// host gives every round one register slot j on all of its threads.  The
// solve of a branch is split so that only one multiply-add per branch waits
// on the tree.  With the children's sum s and the parent's new value xp as
// unknowns, the branch's recurrences are linear in them:
//   rhs'_k = P_k - Q_k s,  F_0 rhs'_0 = F_0 P_0 - (F_0 Q_0) s,
//   x_last = Y_last + Z xp,
// where P and Y come from the branch's own CVs (all branches at once) and
// F_0 Q_0 = F_0 prod_{k>=1}(-F_k), Z = prod_k(-F_k) are step-invariant.  The
// elimination and substitution themselves are the Hines recurrences of the
// serial solve (Sec. II); only the values passed between branches are formed
// through the split.
#pragma once
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"
#include "kernels.hpp"

namespace arbmi {
namespace reg {

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
    double x = t[0];
#pragma unroll
    for (int k = 1; k < L; ++k) x = t[k] - g.F[k] * x;
    g.yl = (g.len == L) ? x : -x;
}
template <int L>
__device__ __forceinline__ void store_v(const Slot<L>& g, double* sV, const double* t) {
#pragma unroll
    for (int k = 0; k < L; ++k) sV[cv_slot(g, k)] = t[k];
}

// The branch's rows (pads included) into a row of HBM indexed by pack-local
// slot; an empty register slot writes nothing.
template <int L>
__device__ __forceinline__ void record_v(const Slot<L>& g, double* row, const double* t) {
    if (g.r < 0) return;
#pragma unroll
    for (int k = 0; k < L; ++k) row[g.base + k * g.w] = t[k];
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

// The same two passes with every slot taking part in every round, so that a
// round has no branches and issues all of its slots' loads before any
// arithmetic (one LDS round trip a round instead of one per slot and
// child).  A branch's inputs are final from the round before its own (its
// children's or grandchildren's round going up, its grandparent's going
// down) and nothing
// reads its entry before the round after its own; so the rounds before its
// own compute values that are never read, and the rounds after it recompute
// the same values from the same inputs and store identical bits.  An empty
// slot reads zero entries and writes the discard entry.  Results equal
// pass_up2 and pass_down bit for bit.
struct Up2In {
    double f0, q0, a0, b0;  // first child: F_0 P_0, F_0 Q_0, its children's contributions
    double f1, q1, a1, b1;  // second child
};
template <int L>
__device__ __forceinline__ Up2In up2_load(const Slot<L>& g, const double* sF, const double* sQ, const double* sC) {
    Up2In u;
    u.f0 = sF[g.c0];
    u.q0 = sQ[g.c0];
    u.a0 = sC[g.x0 & 0xffff];
    u.b0 = sC[int(unsigned(g.x0) >> 16)];
    u.f1 = sF[g.c1];
    u.q1 = sQ[g.c1];
    u.a1 = sC[g.x1 & 0xffff];
    u.b1 = sC[int(unsigned(g.x1) >> 16)];
    return u;
}
template <int L>
__device__ __forceinline__ void up2_store(Slot<L>& g, const Up2In& u, double* sC) {
    const double s0 = u.f0 - u.q0 * (u.a0 + u.b0);
    const double s1 = u.f1 - u.q1 * (u.a1 + u.b1);
    g.cs = s0 + s1;
    sC[g.task] = g.fp - g.FQ * g.cs;
}
struct DownIn {
    double y, x;  // parent's V with a grounded grandparent, grandparent's distal V
};
template <int L>
__device__ __forceinline__ DownIn down_load(const Slot<L>& g, const double* sY, const double* sX) {
    return DownIn{sY[g.ptask], sX[g.gptask]};
}
template <int L>
__device__ __forceinline__ void down_store(Slot<L>& g, const DownIn& d, double* sX) {
    g.xp = d.y + g.Zp * d.x;
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

// The upward pass of the split solve over the thread's S slots.  Packs with
// at most binary branch points run every slot in every round: in workgroups
// of up to two waves one tree level a round (a branch adds its children's
// contributions: two loads per slot and round), in larger workgroups, where
// each round costs a barrier across more waves, two levels a round
// (up2_load, up2_store: eight loads per slot and round, half the rounds).
// Both store the same contributions bit for bit.  Other packs take one round
// of the host's schedule at a time, each slot in its own round.
template <int T, int S, int L>
__device__ __forceinline__ void up_pass(const PackDesc& pk, Slot<L>& g0, Slot<L>& g1, Slot<L>& g2, const double* sF,
                                        const double* sQ, double* sC, const int32_t* s_ch) {
    if (T <= 128 && pk.binary) {
        // the deepest level's branches are leaves, final from the local
        // elimination on: the root is final after nlev - 1 rounds
        for (int r = 0; r + 1 < pk.nlev; ++r) {
            double a0 = sC[g0.c0], b0 = sC[g0.c1], a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0;
            if constexpr (S > 1) {
                a1 = sC[g1.c0];
                b1 = sC[g1.c1];
            }
            if constexpr (S > 2) {
                a2 = sC[g2.c0];
                b2 = sC[g2.c1];
            }
            g0.cs = a0 + b0;
            sC[g0.task] = g0.fp - g0.FQ * g0.cs;
            if constexpr (S > 1) {
                g1.cs = a1 + b1;
                sC[g1.task] = g1.fp - g1.FQ * g1.cs;
            }
            if constexpr (S > 2) {
                g2.cs = a2 + b2;
                sC[g2.task] = g2.fp - g2.FQ * g2.cs;
            }
            round_sync<T>();
        }
    } else if (pk.binary) {
        // after round r every level from nlev - 3 - 2 r down is final
        for (int sr = 0; 2 * sr + 1 < pk.nlev; ++sr) {
            Up2In u0, u1, u2;
            u0 = up2_load<L>(g0, sF, sQ, sC);
            if constexpr (S > 1) u1 = up2_load<L>(g1, sF, sQ, sC);
            if constexpr (S > 2) u2 = up2_load<L>(g2, sF, sQ, sC);
            up2_store<L>(g0, u0, sC);
            if constexpr (S > 1) up2_store<L>(g1, u1, sC);
            if constexpr (S > 2) up2_store<L>(g2, u2, sC);
            round_sync<T>();
        }
    } else {
        for (int r = 0; r < pk.nrd; ++r) {  // deepest rounds first
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
}

// The values the downward pass starts from, stored after the full
// elimination: every branch's distal value with a grounded parent (Y) and
// the same as its distal voltage (X), which is final for the root (its
// parent's voltage is zero) and rewritten by the rounds for the others.
template <int L>
__device__ __forceinline__ void grounded_store(const Slot<L>& g, double* sY, double* sX) {
    sY[g.task] = g.yl;
    sX[g.task] = g.yl + g.Z * 0.0;
}

// The downward pass: two tree levels a round, shallowest first, every slot
// in every round (down_load, down_store).  With the root final beforehand
// (grounded_store), after round r every level up to 2 r + 2 is final.
template <int T, int S, int L>
__device__ __forceinline__ void down_pass(const PackDesc& pk, Slot<L>& g0, Slot<L>& g1, Slot<L>& g2, const double* sY,
                                          double* sX) {
    for (int sr = 0; 2 * sr + 1 < pk.nlev; ++sr) {
        DownIn d0, d1, d2;
        d0 = down_load<L>(g0, sY, sX);
        if constexpr (S > 1) d1 = down_load<L>(g1, sY, sX);
        if constexpr (S > 2) d2 = down_load<L>(g2, sY, sX);
        down_store<L>(g0, d0, sX);
        if constexpr (S > 1) down_store<L>(g1, d1, sX);
        if constexpr (S > 2) down_store<L>(g2, d2, sX);
        round_sync<T>();
    }
}


}  // namespace reg
}  // namespace arbmi
