// kernels.hpp -- launch interface of the HIP kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace arbmi {

// Everything the fused step kernel reads or writes.  All pointers are device
// pointers into the sim's arena.
struct StepArgs {
    const PackDesc* pk;
    const RoundDesc* rd;
    const TaskDesc* tk;
    const int32_t* ch_slot;
    const int32_t* ch_task;    // per child entry: the child's pack-local task
    const int32_t* tk_ptask;   // per task: the parent's pack-local task, -1 at a soma
    const int32_t* tk_lev;     // per task: depth level (the soma is 0)
    const double* tk_Z;        // per task: prod over its CVs of (-F)
    const NlDesc* nl;
    const int32_t* pc_gid;
    const int32_t* pc_soma;
    double* V;                 // [n_slots]
    const double* alpha;
    const double* beta;
    const double* F;
    const double* invd;
    double* hh_m;              // [n_hh] gates
    double* hh_h;
    double* hh_n;
    const double* hh_gna;      // nS
    const double* hh_gk;
    double* syn_g;             // [n_syn] nS
    const double* syn_e;
    const double* syn_decay;   // exp(-dt/tau)
    const int32_t* ic_slot;    // pack-local slot of each clamp
    const int64_t* ic_on;
    const int64_t* ic_off;
    const double* ic_amp;      // pA
    const int64_t* xe_step;    // external events
    const int32_t* xe_syn;
    const double* xe_w;        // nS
    int64_t* pk_xcur;          // [n_packs] cursor into the external events
    // network events of the current epoch (null without a network): per
    // pack the events in (step, connection rank) order, and where each step
    // of the epoch starts among them
    const uint32_t* bk_off;    // [n_packs][epoch_steps + 1]
    const uint32_t* bk_nxt;    // [n_packs][epoch_steps + 1] first step >= b with events (epoch_steps if none)
    const int32_t* bk_q;       // [n_packs][bk_cap] pack-local synapse
    const double* bk_w;        // [n_packs][bk_cap] weight nS
    int32_t bk_cap;
    int32_t epoch_steps;       // K: epochs start at multiples of K
    // spikes
    uint32_t* sp_gid;
    int64_t* sp_step;
    double* sp_t;
    uint32_t sp_cap;
    uint32_t pad1;
    Counters* ctr;
    // probes
    const int32_t* pr_slot;    // per pack probe entries (pack-local slot)
    const int32_t* pr_id;
    double* trace;             // [n_probe][trace_cap]
    int64_t trace_cap;
    int64_t trace_step0;       // step whose end value goes to column 0
    // gradient checkpoint recording (null when not recording): per step of
    // the launch, the state before the step
    double* rec_V;             // [nsteps][n_slots]
    double* rec_m;             // [nsteps][n_hh] ...
    double* rec_h;
    double* rec_n;
    double* rec_g;             // [nsteps][n_syn] g after the step's events
    int64_t n_slots_total;
    int64_t n_hh_total;
    int64_t n_syn_total;
    double dt;
    double threshold;
    int64_t step0;             // first step of this launch
    int32_t nsteps;            // steps in this launch
    int32_t epoch_end;         // 1 if the launch completes an epoch
    // graph replay: when set, the launch is the full epoch *epoch_ptr
    // (step0 = epoch * nsteps)
    const int64_t* epoch_ptr;
    int32_t pad0;
    int32_t pack0;             // first pack of this launch (block b runs pack pack0 + b)
    // generated density mechanisms (null when the model has none): the
    // instances of each nonlinear entry and of each pack, their mechanism,
    // CV, weight (10 x area, S/cm^2 -> nS), parameters and states
    const int32_t* gen_off;    // [n_nl + 1]
    const int32_t* gen_pk;     // [n_packs + 1]
    const int32_t* gen_row;    // per instance: parameter row | catalogue index << 24
    const int32_t* gen_slot;   // pack-local slot
    const double* gen_w;
    const double* gen_prm;     // [n_rows][kMaxParams]
    double* gen_st;            // [kMaxStates][n_inst], state-major
    int64_t gen_n;             // instances (the state-major stride)
};

// Per-launch configuration chosen by the host.
struct LaunchCfg {
    int block_threads;  // 64, 128, 256
    int coef_mode;      // 1 LDS, 2 streamed, 3 register-resident
    int lds_bytes;      // dynamic LDS per workgroup
    int reg_slots;      // mode 3: branches per thread
    int reg_len;        // mode 3: CVs per branch held in registers (8 or 16)
    int syn_hbm;        // mode 3: some pack keeps its synapse state in HBM
    int rec;            // mode 3: the sim is built for gradients (kernels that can record states)
    int gen;            // mode 3: the model has generated density mechanisms
};

hipError_t launch_step(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st);
hipError_t prepare_step_kernels(int max_lds_bytes);
hipError_t launch_reg_step(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st);
hipError_t prepare_reg_kernels(int max_lds_bytes);

// ++*epoch (end of a replayed epoch)
hipError_t launch_advance_epoch(int64_t* epoch, hipStream_t st);

// Spike exchange between epochs (Sec. II min-delay epochs, Sec. IV-A).
// Epoch end: copy the spikes [ctr.sp_exch, ctr.sp_count) into history slot
// epoch % n_hist (h_cap entries each; overflow is flagged) and mark them
// exchanged.  `epoch_ptr`, when set, holds the epoch instead of `epoch`.
hipError_t launch_collect_spikes(Counters* ctr, const uint32_t* sp_gid, const int64_t* sp_step, uint32_t sp_cap,
                                 uint32_t* h_gid, int64_t* h_step, uint32_t* h_cnt, uint32_t h_cap, int32_t n_hist,
                                 int64_t epoch, const int64_t* epoch_ptr, hipStream_t st);
// Epoch start: index the history's spikes by source gid: off[n_src + 1]
// (exclusive offsets, n_src = ranks x n_cells) and sx_step (their steps).
// With ranks R > 1 (dry run) each local spike of gid g also stands for the
// spikes of gids g + k n_cells, k < R; at most sx_cap are indexed (more
// flag an event overflow).  cnt[n_src] is scratch that must be zero on entry
// and is zero again on return; tile_sum holds index_tiles(n_src) values.
struct IndexLaunch {
    const uint32_t* h_gid;
    const int64_t* h_step;
    const uint32_t* h_cnt;
    uint32_t h_cap;
    int32_t n_hist;
    int32_t ranks;
    int32_t n_cells;
    int64_t sx_cap;
    int32_t* cnt;
    int64_t* off;
    int64_t* tile_sum;
    int64_t* sx_step;
    Counters* ctr;
};
int64_t index_tiles(int64_t n_src);
hipError_t launch_index_spikes(const IndexLaunch& x, hipStream_t st);
// Epoch start, after the index: each pack's network events of the epoch in
// (step, rank) order, with each step's start, into its bucket.
struct PullArgs {
    const int64_t* in_off;     // [n_packs + 1] first connection rank of each pack
    const uint32_t* cr_src;    // per rank: source gid
    const int32_t* cr_delay;   // per rank: delay in steps
    const int32_t* cr_syn;     // per rank: pack-local synapse
    const double* cr_w;        // per rank: weight nS
    const int64_t* sx_off;     // [n_src + 1]
    const int64_t* sx_step;
    int64_t n_src;             // source gids (ranks x cells)
    uint32_t* bk_off;          // [n_packs][epoch_steps + 1]
    uint32_t* bk_nxt;          // [n_packs][epoch_steps + 1]
    int32_t* bk_q;             // [n_packs][bk_cap]
    double* bk_w;              // [n_packs][bk_cap]
    Counters* ctr;
    const int64_t* epoch_ptr;  // or null: `epoch`
    int64_t epoch;
    int32_t bk_cap;
    int32_t epoch_steps;       // K: LDS holds one counter per step
};
hipError_t launch_pull_events(const PullArgs& a, int32_t n_packs, hipStream_t st);

// dst[i] = V[perm[i]] for i < n
hipError_t launch_gather(const double* V, const int64_t* perm, double* dst, int64_t n, hipStream_t st);
// V[perm[i]] = src[i]
hipError_t launch_scatter(double* V, const int64_t* perm, const double* src, int64_t n, hipStream_t st);

}  // namespace arbmi
