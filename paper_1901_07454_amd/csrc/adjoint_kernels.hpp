// adjoint_kernels.hpp -- launch interface of the adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "layout.hpp"

namespace arbmi {

struct AdjArgs {
    const PackDesc* pk;
    const RoundDesc* rd;
    const TaskDesc* tk;
    const int32_t* ch_slot;
    const NlDesc* nl;
    const int32_t* pc_gid;
    const int32_t* pc_soma;
    const double* alpha;
    const double* F;
    const double* invd;
    const double* hh_gna;
    const double* hh_gk;
    // forward states of the segment: V rows 0..nsteps, gates and g rows 0..nsteps-1
    const double* rec_V;
    const double* rec_m;
    const double* rec_h;
    const double* rec_n;
    const double* rec_g;
    int64_t n_slots_total, n_hh_total, n_syn_total;
    // adjoint state carried between segments
    double *lamV, *lamM, *lamH, *lamN;
    // gradient sums: per slot sum(w V), sum(w); per hh instance the gNa, gK terms
    double *accP1, *accP0, *accNa, *accK;
    const double* dLdtrace;  // [cell][trace_len]
    int64_t trace_len;
    int64_t trace_step0;
    double dt;
    int64_t step0;           // first step of the segment
    int32_t nsteps;
    int32_t pad;
};

// Dynamic LDS of the adjoint kernel for a pack: doubles lambda_V, w, sum wV,
// sum w per slot; lambda_m/h/n and two gradient sums per hh instance; then
// rounds, tasks, nonlinear entries, child slots.
inline int64_t adjoint_lds_bytes(const PackDesc& D) {
    return 8 * (4 * int64_t(D.nslot) + 5 * int64_t(D.nhh)) + 24 * int64_t(D.nrd) + 16 * int64_t(D.ntk) +
           16 * int64_t(D.nnl) + 4 * int64_t(D.nch);
}

struct GradReduceArgs {
    int64_t n_reg;
    const int64_t* rp_off;   // [n_reg + 1] membrane pieces of each region
    const int64_t* rp_slot;  // global slot of the piece's CV
    const int64_t* rp_hh;    // global hh instance of that CV, -1 if none
    const double* rp_area;   // um^2
    const uint32_t* reg_mech;
    const double* reg_epas;
    const double *accP1, *accP0, *accNa, *accK;
    double* out;             // [n_reg][3]
};

// Up to kCopyParts device-to-device copies of whole 32-bit words in one
// launch (the dynamic state into and out of a checkpoint).
constexpr int kCopyParts = 24;
struct CopyList {
    int32_t n;
    int32_t pad;
    const uint32_t* src[kCopyParts];
    uint32_t* dst[kCopyParts];
    int64_t words[kCopyParts];
};
hipError_t launch_copy_parts(const CopyList& c, hipStream_t st);

hipError_t prepare_adjoint_kernels(int lds_max);
hipError_t launch_adjoint(const AdjArgs& a, int block_threads, int lds_bytes, int n_packs, hipStream_t st);
hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t st);

// The register-resident adjoint (reg_adjoint_kernels.hip): one workgroup per
// pack of the sim's register layout (a: the sim's step arguments, for the
// layout and coefficients; cfg: its launch shape), LDS reg_adjoint_lds_bytes.
hipError_t prepare_reg_adjoint_kernels(int lds_max);
hipError_t launch_reg_adjoint(const StepArgs& a, const AdjArgs& b, const LaunchCfg& cfg, int lds_bytes, int n_packs,
                              hipStream_t st);

}  // namespace arbmi
