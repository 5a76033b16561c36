// sim.hpp -- the simulation object behind the opaque arb_sim handle.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/arbmi.h"
#include "kernels.hpp"
#include "lower.hpp"
#include "var_kernels.hpp"

struct arb_sim_ {};

namespace arbmi {

struct RecordArgs {
    double *V, *m, *h, *n, *g;
};

// Launch shape and packing chosen before lowering.
struct Plan {
    int block_threads = 64;
    int coef_mode = 1;
    int64_t lds_budget = 160 * 1024;
    int64_t lds_hard_max = 160 * 1024;
    int64_t max_cells_per_pack = 64;
    int reg_slots = 0, reg_len = 8;
    int64_t fallback_cells_per_pack = 1;  // streamed mode, if the chosen layout fails
    int64_t fallback_lds_budget = 0;
    int64_t fallback_lds_hard_max = 0;
};
Plan choose_plan(const arb_cell* cells, int32_t n_cells, const arb_branch* br, int64_t n_br, const arb_params& p,
                 int64_t lds_max, int n_cu);

struct GradState;

struct Sim : arb_sim_ {
    arb_params p{};
    hipStream_t st = nullptr;
    int device = 0, n_cu = 256;
    int64_t lds_max = 0;
    Lowered L;
    int32_t K = 1;          // epoch length in steps
    LaunchCfg cfg{};
    // launch classes: contiguous pack ranges run as separate concurrent
    // kernels, each with the LDS its largest pack needs
    // streams the launch classes run on at most (the sim's and auxiliary ones)
    static constexpr int kClassStreams = 4;
    struct Class {
        int32_t pack0, npack, lds;
        int hbm;     // some pack of the class keeps state in HBM (the kernel variant that can)
        int slots;   // register slots its packs use (register layout), else 0
        int stream;  // 0: the sim's stream, k > 0: aux[k - 1]
    };
    std::vector<Class> classes;
    std::vector<hipStream_t> aux;       // the streams besides the sim's that classes run on
    std::vector<hipEvent_t> fork_ev, join_ev;
    int32_t bk_cap = 0;
    int32_t n_hist = 1;     // epochs of spike history the longest delay needs
    uint32_t hist_cap = 0;  // spikes per history epoch
    uint32_t sp_cap = 0, sp_user = 0;
    int64_t step = 0;
    double m0 = 0, h0 = 0, n0 = 0;
    std::vector<int64_t> xcur0;

    std::vector<void*> allocs;
    std::vector<int64_t> alloc_bytes;
    int64_t device_bytes = 0;
    std::vector<hipEvent_t> timer_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timer_pending;

    PackDesc* d_pk = nullptr;
    RoundDesc* d_rd = nullptr;
    TaskDesc* d_tk = nullptr;
    int32_t* d_ch = nullptr;
    int32_t* d_ch_task = nullptr;
    int32_t* d_tk_ptask = nullptr;
    int32_t* d_tk_lev = nullptr;
    double* d_tk_Z = nullptr;
    NlDesc* d_nl = nullptr;
    int32_t *d_pc_gid = nullptr, *d_pc_soma = nullptr;
    double *d_V = nullptr, *d_alpha = nullptr, *d_beta = nullptr, *d_F = nullptr, *d_invd = nullptr;
    double *d_hh_m = nullptr, *d_hh_h = nullptr, *d_hh_n = nullptr, *d_hh_gna = nullptr, *d_hh_gk = nullptr;
    double *d_syn_g = nullptr, *d_syn_e = nullptr, *d_syn_decay = nullptr;
    int32_t* d_ic_slot = nullptr;
    int64_t *d_ic_on = nullptr, *d_ic_off = nullptr;
    double* d_ic_amp = nullptr;
    int64_t* d_xe_step = nullptr;
    int32_t* d_xe_syn = nullptr;
    double* d_xe_w = nullptr;
    int64_t* d_pk_xcur = nullptr;
    uint32_t* d_bk_off = nullptr;  // network events of the running epoch (StepArgs)
    uint32_t* d_bk_nxt = nullptr;
    int32_t* d_bk_q = nullptr;
    double* d_bk_w = nullptr;
    int32_t *d_cr_syn = nullptr, *d_cr_delay = nullptr;
    uint32_t* d_cr_src = nullptr;
    double* d_cr_w = nullptr;
    int64_t* d_in_off = nullptr;
    // spike history ring and its per-source index
    uint32_t* d_hist_gid = nullptr;
    int64_t* d_hist_step = nullptr;
    uint32_t* d_hist_cnt = nullptr;
    int32_t* d_sx_cnt = nullptr;
    int64_t *d_sx_off = nullptr, *d_sx_step = nullptr, *d_tile_sum = nullptr;
    int64_t sx_cap = 0;  // indexed spikes (proxies included) per epoch
    uint32_t* d_sp_gid = nullptr;
    int64_t* d_sp_step = nullptr;
    double* d_sp_t = nullptr;
    Counters* d_ctr = nullptr;
    int64_t* d_perm = nullptr;
    double* d_tmp = nullptr;
    int64_t tmp_n = 0;
    // probes
    int32_t *d_pr_slot = nullptr, *d_pr_id = nullptr;
    double* d_trace = nullptr;
    // the buffers arb_set_probes allocated (released when probes are replaced)
    int32_t *own_pr_slot = nullptr, *own_pr_id = nullptr;
    double* own_trace = nullptr;
    int64_t n_probe = 0, trace_cap = 0, trace_step0 = 0;
    // graph replay of whole epochs (ARB_FLAG_GRAPH)
    int64_t* d_epoch = nullptr;
    hipGraphExec_t graph = nullptr;
    hipStream_t st_capture = nullptr;  // capture happens here; replays go on st
    bool graph_dirty = true;
    int capture_epoch_graph();
    // variable time step (continuous event times; arb_build_cells_timed)
    bool timed = false;
    double *d_xe_t = nullptr, *d_bk_t = nullptr, *d_cr_delay_ms = nullptr;
    double *d_cap = nullptr, *d_gmem = nullptr, *d_sigsum = nullptr, *d_uoff = nullptr, *d_syn_tau = nullptr;
    int64_t* d_pk_steps = nullptr;
    // generated density mechanisms (StepArgs.gen_*)
    int32_t *d_gen_off = nullptr, *d_gen_pk = nullptr, *d_gen_row = nullptr, *d_gen_slot = nullptr;
    double *d_gen_w = nullptr, *d_gen_prm = nullptr, *d_gen_st = nullptr;
    VarArgs var_args() const;
    // gradients
    GradState* grad = nullptr;
    bool grad_valid = false;

    void* raw_alloc(size_t bytes);
    void release(void* ptr);  // frees one allocation of raw_alloc (no-op for others)
    void release_all();
    int upload(void* dst, const void* src, size_t bytes);
    int fill_zero(void* dst, size_t bytes);
    StepArgs step_args() const;
    int advance(int64_t n, const RecordArgs* rec);
    int launch_epoch_sequence(const StepArgs& a, bool net, bool graph_mode);
    int launch_pull(int64_t epoch, const int64_t* epoch_ptr);     // the epoch's network events
    int launch_collect(int64_t epoch, const int64_t* epoch_ptr);  // the epoch's spikes into the history
    int launch_classes(const StepArgs& a);
    int check_flags(bool& spikes_lost, bool& events_lost);
    // the dynamic state's parts (state_part_bytes order) and their device addresses
    StateShape state_shape() const;
    void state_part_ptrs(void* ptr[kStateParts]) const;
};

struct ModelView {
    const arb_cell* cells;
    int32_t n_cells;
    const arb_branch* br;
    int64_t n_br;
    const arb_synapse* syn;
    int64_t n_syn;
    const arb_connection* conn;
    int64_t n_conn;
    const arb_event* ev;
    int64_t n_ev;
    const arb_iclamp* ic;
    int32_t n_ic;
    // variable time step: connection delays and event times (ms), or null
    const double* conn_delay_ms = nullptr;
    const double* ev_t_ms = nullptr;
};

struct DeviceLimits {
    bool have_dev = false;
    int dev = 0;
    int64_t lds_max = 160 * 1024;
    int n_cu = 256;
};

// Lower and upload a model with the launch parameters in p (0 = planned).
int build_sim(const ModelView& m, const arb_params& p, const DeviceLimits& d, Sim** out, std::string& err);
void destroy_sim(Sim* s);
// Time candidate launch shapes on a sample of the model's cells; returns p
// with block_threads, coef_mode and cells_per_pack set to the fastest.
arb_params autotune(const ModelView& m, const arb_params& p, const DeviceLimits& d);

int set_error(int code, const std::string& msg);
// Look up, once per device (the device current), the static staging buffer of
// arb_get_voltages_noalloc.
hipError_t noalloc_setup(int device);
int set_hip_error(hipError_t e, const char* where);

}  // namespace arbmi
