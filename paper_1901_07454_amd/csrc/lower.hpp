// lower.hpp -- host-side lowering of a model into the packed device layout.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/arbmi.h"
#include "layout.hpp"

namespace arbmi {

struct Region {
    uint32_t mech;
    double gna, gk, gl, gpas, epas;  // S/cm^2, mV
};

// Everything the device needs, in packed order, plus what the host keeps to
// recompute coefficients when parameters change.
struct Lowered {
    // sizes
    int32_t n_cells = 0;
    int64_t n_cv = 0, n_slots = 0;
    int32_t block_threads = 64;
    int32_t coef_mode = 1;
    int32_t reg_slots = 0, reg_len = 0;
    double dt = 0.025, threshold = -10.0, v_init = -65.0;

    std::vector<PackDesc> packs;
    std::vector<RoundDesc> rounds;
    std::vector<TaskDesc> tasks;
    std::vector<int32_t> ch_slot;
    std::vector<int32_t> ch_task;     // per child entry: the child's pack-local task
    std::vector<int32_t> tk_ptask;    // per task: the parent's pack-local task, -1 at a soma
    std::vector<int32_t> tk_lev;      // per task: depth level (the soma is 0)
    std::vector<double> tk_Z;         // per task: prod over its CVs of (-F), the distal V's weight on the parent's
    std::vector<NlDesc> nl;
    std::vector<int32_t> pc_gid, pc_soma;  // per pack cell: gid, pack-local soma slot

    // per global slot
    std::vector<double> cap;                  // pF (0 in padding)
    std::vector<double> alpha, beta, F, invd; // step coefficients
    std::vector<double> d_elim;               // eliminated diagonal (kept for checks)
    std::vector<double> sigsum;               // sum of the axial conductances at the CV (nS)
    std::vector<double> uoff;                 // -sigma to the parent CV (0 at a soma and in padding)
    std::vector<double> gmem;                 // linear membrane conductance (pas, hh leak; nS)
    std::vector<int64_t> perm;                // user CV -> global slot
    std::vector<int32_t> slot_cell;           // global slot -> gid (-1 padding)

    // membrane pieces of each user CV (for parameter updates and gradients)
    std::vector<int64_t> piece_off;           // [n_cv + 1]
    std::vector<int32_t> piece_reg;           // global region
    std::vector<double> piece_area;           // um^2
    std::vector<Region> regions;              // [n_cells + n_branches], soma first per cell
    std::vector<int64_t> cell_reg0;           // [n_cells + 1]
    std::vector<int64_t> cell_cv0;            // [n_cells + 1] user CV offsets
    std::vector<double> glin_extra;           // per user CV: hh leak part of the linear conductance

    // hh instances, pack order
    std::vector<int64_t> hh_cv;               // user CV
    std::vector<double> hh_gna, hh_gk;        // nS
    // synapses, pack order
    std::vector<int64_t> syn_global;          // pack-order index -> global synapse
    std::vector<int64_t> syn_pack_index;      // global synapse -> pack-order index
    std::vector<double> syn_e, syn_decay;
    std::vector<double> syn_tau;              // ms (variable step: decay over any step length)
    // clamps, per pack, ordered by (slot, input order)
    std::vector<int32_t> ic_slot;             // pack-local slot
    std::vector<int64_t> ic_on, ic_off;
    std::vector<double> ic_amp;               // pA
    // external events, pack order
    std::vector<int64_t> xe_step;
    std::vector<double> xe_t;                 // variable step: event times (ms)
    std::vector<int32_t> xe_syn;              // pack-local synapse
    std::vector<double> xe_w;                 // nS
    // connections: ranks sorted by (dst pack, dst pack-local synapse, src, index)
    int64_t n_src = 0;                        // source gids: n_cells, or R n_cells in dry-run mode
    std::vector<int32_t> cr_pack, cr_syn, cr_delay;
    std::vector<double> cr_delay_ms;          // variable step: delays (ms)
    std::vector<uint32_t> cr_src;             // source gid of each rank
    std::vector<double> cr_w;                 // nS
    // generated density mechanisms: one instance per (CV, density entry on a
    // region the CV covers); instances are grouped by nonlinear entry
    std::vector<int32_t> gen_off;             // [n_nl + 1] first instance of each nonlinear entry
    std::vector<int32_t> gen_pk;              // [n_packs + 1] first instance of each pack
    std::vector<int32_t> gen_mech;            // per instance: catalogue index (host side only)
    std::vector<int32_t> gen_row;             // per instance: its parameter row (low 24 bits) and
                                              // catalogue index (high bits)
    std::vector<int32_t> gen_slot;            // per instance: pack-local slot of its CV
    std::vector<double> gen_w;                // per instance: 10 x its membrane area (um^2): S/cm^2 -> nS
    std::vector<int32_t> gen_rmech;           // per parameter row: catalogue index (host side only)
    std::vector<double> gen_prm;              // [n_rows][gen::kMaxParams], one row per distinct
                                              // (mechanism, parameters) pair
    std::vector<double> gen_st0;              // [gen::kMaxStates][n_inst] states at rest at v_init,
                                              // state-major (a state of consecutive instances is contiguous)
    std::vector<int64_t> in_off;              // [n_packs + 1] first rank of each pack
    int32_t dry_run_ranks = 1;                // R: ranks the exchange emulates (1 = none)
    bool timed = false;                       // variable time step (continuous event times)
    double min_delay_ms = 0, max_delay_ms = 0;
    int32_t min_delay = 0, max_delay = 0;
    int64_t max_in_per_pack = 0;              // incoming connections of the busiest pack
    int64_t n_hh_total = 0;
};

struct LowerOptions {
    int32_t block_threads = 64;
    int32_t coef_mode = 1;            // 1 LDS, 2 streamed
    int64_t lds_budget = 160 * 1024;  // target bytes per workgroup when packing several cells
    int64_t lds_hard_max = 160 * 1024; // a single cell may use up to this
    int64_t max_cells_per_pack = int64_t(1) << 30;
    int32_t reg_slots = 0;            // register-resident layout: branches per thread (0 = LDS layout)
    int32_t reg_len = 8;              // and the longest branch it takes
    bool grads = false;               // packs must also fit the adjoint kernel (register layout:
                                      // its LDS, and synapse state in LDS)
    // variable time step: continuous connection delays (ms, input order) and
    // external event times (ms, input order); both null for the fixed step
    const double* conn_delay_ms = nullptr;
    const double* ev_t_ms = nullptr;
};

// Validates and lowers.  Returns ARB_OK or ARB_EINVAL (message in err).
int lower_model(const arb_cell* cells, int32_t n_cells, const arb_branch* br, int64_t n_br,
                const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, int64_t n_conn,
                const arb_event* ev, int64_t n_ev, const arb_iclamp* ic, int32_t n_ic,
                const arb_params& p, const LowerOptions& opt, Lowered& out, std::string& err);

// Check the packed layout's invariants; empty string if all hold.
std::string verify_layout(const Lowered& lw);

// The dynamic state of a sim as a host blob (arb_get_state / arb_set_state):
// a header, then kStateParts parts in this order: V, hh m, h, n, synapse g,
// external-event cursors, the running epoch's network events (offsets,
// next-step table, synapses, weights), counters, spike buffer (gid, step,
// time), spike history (counts, gids, steps), generated mechanisms' states.
struct StateShape {
    int32_t K = 1;            // epoch steps
    int32_t bk_cap = 0;       // network events per pack and epoch
    uint32_t sp_cap = 0;      // spike buffer
    int32_t n_hist = 1;       // history epochs
    uint32_t hist_cap = 0;    // spikes per history epoch
    bool net = false;         // the event tables exist
};
struct StateHeader {
    uint64_t magic;
    int64_t step, n_slots, n_hh, n_syn, n_packs, n_bk, bk_cap, sp_cap, sp_user;
};
constexpr uint64_t kStateMagic = 0x41524233535441ull;
constexpr int kStateParts = 18;
// Bytes of each part.
void state_part_bytes(const Lowered& L, const StateShape& sh, int64_t bytes[kStateParts]);
// Every check arb_set_state makes before any byte reaches the device: the
// header names this model, and every value a kernel indexes with (step and
// spike counters, event cursors, spike gids, bucket offsets and synapses,
// history counts and gids) lies in range.  "" if the blob is acceptable.
std::string check_state_blob(const Lowered& L, const StateShape& sh, const void* blob, int64_t n);

// Recompute alpha, beta, hh_gna, hh_gk from lw.regions (after a parameter change).
void recompute_coefficients(Lowered& lw);

}  // namespace arbmi
