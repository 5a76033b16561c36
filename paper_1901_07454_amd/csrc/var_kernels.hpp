// var_kernels.hpp -- host interface of the variable-step kernels
// (var_kernels.hip): the step kernel that shortens steps at event times
// (Sec. II) and the pull of the epoch's network events at continuous times.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace arbmi {

// What the variable step reads beyond the fixed step's arguments.
struct VarArgs {
    const double* xe_t;     // external event times (ms), pack order, sorted by time within a pack
    const double* bk_t;     // [n_packs][bk_cap] arrival times (ms) of the epoch's network events
    const double* cap;      // per slot: membrane capacitance (pF; 0 in padding)
    const double* gmem;     // per slot: linear membrane conductance, pas and hh leak (nS)
    const double* sigsum;   // per slot: sum of the axial conductances at the CV (nS)
    const double* uoff;     // per slot: -sigma to the parent CV (0 at a soma)
    const double* syn_tau;  // per synapse, pack order (ms)
    int64_t* pk_steps;      // [n_packs] steps taken, accumulated over launches
};

// The timed pull: the epoch's network events of every pack, binned by grid
// interval and sorted by arrival time within each interval.
struct TimedPullArgs {
    const int64_t* in_off;       // [n_packs + 1] first connection rank of each pack
    const uint32_t* cr_src;      // per rank: source gid
    const double* cr_delay_ms;   // per rank: delay (ms)
    const int32_t* cr_syn;       // per rank: pack-local synapse
    const double* cr_w;          // per rank: weight nS
    const int64_t* sx_off;       // [n_src + 1] the index by source gid
    const int64_t* sx_step;      // indexed spikes: the bits of their times (ms)
    int64_t n_src;
    uint32_t* bk_off;            // [n_packs][epoch_steps + 1] first event of each grid interval
    int32_t* bk_q;               // [n_packs][bk_cap]
    double* bk_w;                // [n_packs][bk_cap]
    double* bk_t;                // [n_packs][bk_cap]
    Counters* ctr;
    const int64_t* epoch_ptr;    // or null: `epoch`
    int64_t epoch;
    double dt;
    int32_t bk_cap;
    int32_t epoch_steps;         // K grid steps per epoch
};

hipError_t prepare_var_kernels(int max_lds_bytes);
hipError_t launch_var_step(const StepArgs& a, const VarArgs& v, const LaunchCfg& cfg, int n_packs, hipStream_t st);
hipError_t launch_pull_timed(const TimedPullArgs& a, int32_t n_packs, hipStream_t st);

}  // namespace arbmi
