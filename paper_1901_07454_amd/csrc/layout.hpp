// layout.hpp -- device-side data layout shared by the host lowering and the
// HIP kernels of the cell stepper.
//
// A *pack* is the set of cells one workgroup advances.  Its control volumes
// (CVs) occupy a contiguous run of *slots*.  Cells' branches are grouped by
// depth in the branch tree (the soma is depth 0, a branch hanging off the
// soma depth 1, ...); the branches of one depth in a pack form one or more
// *rounds* of at most `block_threads` branches.  In a round of width w and
// length L (its longest branch), CV k (0 = proximal) of the branch handled by
// thread t sits at slot  round.slot0 + k*w + t, so that the threads of a
// round touch consecutive slots (coalesced in HBM, conflict-free in LDS).
// Rounds are stored deepest first: the elimination sweep runs them in order
// and the substitution sweep in reverse.
#pragma once
#include <algorithm>
#include <stdint.h>

namespace arbmi {

// hh reversal potentials (mV): textbook squid-axon values
constexpr double kENa = 50.0;
constexpr double kEK = -77.0;
constexpr double kEL = -54.3;

struct PackDesc {
    int64_t slot0;   // first global slot of the pack
    int32_t nslot;   // slots (incl. padding)
    int32_t rd0;     // first round
    int32_t nrd;     // rounds
    int32_t cell0;   // first entry in the pack-cell arrays
    int32_t ncell;
    int32_t nl0;     // first nonlinear CV entry (CVs with hh, synapses or clamps)
    int32_t nnl;
    int32_t hh0;     // first hh instance
    int32_t nhh;
    int32_t syn0;    // first synapse (pack-local synapse q is global q - syn0 + syn0)
    int32_t nsyn;
    int32_t pr0;     // probes
    int32_t npr;
    int32_t tk0;     // first task (tasks of a pack are contiguous)
    int32_t ntk;
    int32_t ch0;     // first child-slot entry
    int32_t nch;
    int32_t ic0;     // first clamp entry
    int32_t nic;
    int32_t spare;   // register-resident layout: a slot no CV uses (a pad row, or nslot)
    int32_t nlev;    // depth levels of the pack's cells (the soma is level 0)
    int32_t binary;  // 1 if no task of the pack has more than two children
    int32_t syn_global;  // register-resident layout: synapse state stays in HBM
    int32_t syn_uniform; // all synapses of the pack share e_syn and decay (below)
    int32_t hh_global;   // register-resident layout: hh conductances and the nonlinear CVs'
                         // beta stay in HBM (a cell too large for LDS otherwise)
    int64_t xe0, xe1; // external events [xe0, xe1), sorted by (step, syn, input order)
    double syn_e, syn_decay;  // the shared values when syn_uniform
};

// Bytes of dynamic LDS the step kernel uses for a pack.  Layout in the
// streamed and LDS-resident kernels: doubles V, R, [alpha, beta, F, 1/d'], g,
// m, h, n, [gNa, gK, e_syn, decay]; then rounds, tasks, nonlinear entries,
// child slots.  Bracketed parts are staged only in coefficient mode 1 (mode 2
// streams them).  The register-resident kernel (mode 3) keeps its branches'
// descriptors in registers and stages: V and R for every slot (and the
// spare slot, when it lies past them), in blocks of 64 slots (64 V, 64 R),
// g, e_syn, decay, m, h, n, gNa, gK, beta of each nonlinear CV, per-task
// scalars with two spare entries each (a branch's contribution to its parent,
// then its distal V; its contribution with no children, then its distal V
// for a grounded parent; in packs of at most binary branch points, F_0 Q_0),
// the nonlinear entries, the children's tasks (other packs) and the slot of
// each hh instance.

// Packs with at most this many hh instances give each gate its own thread
// in the register-resident kernel.
constexpr int kSpreadHH = 20;

// A register-resident pack whose synapses would take more LDS than this
// keeps their state in HBM and streams it every step.  A pack of one cell
// too large for LDS otherwise reads its hh conductances and the step-invariant
// right-hand side of its nonlinear CVs from HBM each step (hh_global).
constexpr int64_t kSynLdsMax = 16384;

// Incoming connections a pack of several cells may have: one workgroup
// pulls and delivers all of its pack's network events.
constexpr int64_t kPackInMax = 4096;

// Longest epoch of a network (steps): events are placed per step with one
// LDS counter per step of the epoch.
constexpr int32_t kMaxEpochSteps = 16384;

// Doubles of the register-resident kernel's V and R blocks (64 V then 64 R per
// 64 slots) for a pack: every slot and the spare slot.  The kernel and the
// LDS accounting below both use this.
constexpr int vr_block_doubles(int nslot, int spare) {
    return 128 * (((nslot > spare + 1 ? nslot : spare + 1) + 63) / 64);
}

inline int64_t pack_lds_bytes(const PackDesc& D, int coef_mode) {
    if (coef_mode == 3) {
        const int64_t dbl = vr_block_doubles(D.nslot, D.spare) + (D.syn_global ? 0 : 3 * int64_t(D.nsyn)) +
                            (D.hh_global ? 3 : 5) * int64_t(D.nhh) +
                            (D.hh_global ? 0 : int64_t(D.nnl)) + (D.binary ? 3 : 2) * (int64_t(D.ntk) + 2);
        return 8 * dbl + 16 * int64_t(D.nnl) + (D.binary ? 0 : 4 * int64_t(D.nch)) + 4 * int64_t(D.nhh);
    }
    const bool cl = coef_mode == 1;
    const int64_t dbl = (cl ? 6 : 2) * int64_t(D.nslot) + int64_t(D.nsyn) + 3 * int64_t(D.nhh) +
                        (cl ? 2 * (int64_t(D.nhh) + int64_t(D.nsyn)) : 0);
    return 8 * dbl + 24 * int64_t(D.nrd) + 16 * int64_t(D.ntk) + 16 * int64_t(D.nnl) + 4 * int64_t(D.nch);
}

// Bytes of dynamic LDS the register-resident adjoint kernel uses for a pack
// (reg_adjoint_kernels.hip): the V and R blocks (w and lambda_V), two
// gradient sums per slot, three rows of voltage records, two rows of gate
// and synapse records, seven doubles per hh instance (three adjoint gates,
// two gradient sums, the two conductances), the per-task scalars of the
// solve, the nonlinear entries, the children's tasks (other packs) and each
// hh instance's slot.
inline int64_t reg_adjoint_lds_bytes(const PackDesc& D) {
    const int64_t nsp = std::max<int64_t>(D.nslot, int64_t(D.spare) + 1);
    const int64_t dbl = vr_block_doubles(D.nslot, D.spare) + 5 * nsp + 13 * int64_t(D.nhh) +
                        2 * int64_t(D.nsyn) + (D.binary ? 3 : 2) * (int64_t(D.ntk) + 2);
    return 8 * dbl + 16 * int64_t(D.nnl) + (D.binary ? 0 : 4 * int64_t(D.nch)) + 4 * int64_t(D.nhh);
}

struct RoundDesc {
    int32_t slot0;  // pack-local slot of (k = 0, first thread)
    int32_t w;      // branches in the round
    int32_t len;    // longest branch
    int32_t task0;  // first task (one per branch)
    int32_t t0;     // threads t0 .. t0 + w - 1 take the round's branches in order
    int32_t j;      // register slot the round's threads use (register-resident kernel)
};

struct TaskDesc {
    int32_t len;    // CVs of the branch (1 for a soma)
    int32_t par;    // pack-local slot of the parent CV of the proximal CV, -1 at a soma
    int32_t ch0;    // children: ch_slot[ch0 .. ch0+nch), pack-local slots of the
    int32_t nch;    //   proximal CVs of the child branches, in branch order
};

struct NlDesc {     // one CV carrying an hh instance, synapses or current clamps
    int32_t slot;   // pack-local slot
    int32_t hh;     // pack-local hh instance, -1 if none
    int32_t syn0;   // pack-local synapses syn0 + k s, k < nsyn, with s = 1, or in a pack
    int32_t nsyn;   //   keeping synapses in HBM s = the entries of its group of T
};

// Device counters and flags of a sim.
struct Counters {
    uint32_t sp_count;      // spikes in the buffer
    uint32_t sp_exch;       // spikes [0, sp_exch) already exchanged
    uint32_t flags;         // kFlag*
    uint32_t pad;
};
constexpr uint32_t kFlagSpikeOverflow = 1u;
constexpr uint32_t kFlagEventOverflow = 2u;

}  // namespace arbmi
