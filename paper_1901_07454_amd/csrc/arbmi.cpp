// arbmi.cpp -- the C ABI: sim lifetime, device memory, the epoch loop.
#include "../../include/arbmi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "lower.hpp"
#include "gen/mechanisms_desc.hpp"
#include "sim.hpp"

using namespace arbmi;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ARB_EHIP;
}

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
    } while (0)

}  // namespace

namespace arbmi {

void* Sim::raw_alloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = nullptr;
    if (p.alloc) {
        ptr = p.alloc(bytes, p.alloc_ctx);
    } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
        ptr = nullptr;
    }
    if (ptr) {
        allocs.push_back(ptr);
        alloc_bytes.push_back(int64_t(bytes));
        device_bytes += int64_t(bytes);
    }
    return ptr;
}

void Sim::release(void* ptr) {
    if (!ptr) return;
    for (size_t k = 0; k < allocs.size(); ++k)
        if (allocs[k] == ptr) {
            if (p.free)
                p.free(ptr, p.alloc_ctx);
            else
                (void)hipFree(ptr);
            device_bytes -= alloc_bytes[k];
            allocs.erase(allocs.begin() + int64_t(k));
            alloc_bytes.erase(alloc_bytes.begin() + int64_t(k));
            return;
        }
}

void Sim::release_all() {
    for (void* q : allocs) {
        if (p.free)
            p.free(q, p.alloc_ctx);
        else
            (void)hipFree(q);
    }
    allocs.clear();
    alloc_bytes.clear();
    device_bytes = 0;
}

int Sim::upload(void* dst, const void* src, size_t bytes) {
    if (!bytes) return ARB_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return ARB_OK;
}

int Sim::fill_zero(void* dst, size_t bytes) {
    if (!bytes) return ARB_OK;
    HIP_TRY(hipMemsetAsync(dst, 0, bytes, st));
    return ARB_OK;
}

StepArgs Sim::step_args() const {
    StepArgs a{};
    a.pk = d_pk;
    a.rd = d_rd;
    a.tk = d_tk;
    a.ch_slot = d_ch;
    a.ch_task = d_ch_task;
    a.tk_ptask = d_tk_ptask;
    a.tk_lev = d_tk_lev;
    a.tk_Z = d_tk_Z;
    a.nl = d_nl;
    a.pc_gid = d_pc_gid;
    a.pc_soma = d_pc_soma;
    a.V = d_V;
    a.alpha = d_alpha;
    a.beta = d_beta;
    a.F = d_F;
    a.invd = d_invd;
    a.hh_m = d_hh_m;
    a.hh_h = d_hh_h;
    a.hh_n = d_hh_n;
    a.hh_gna = d_hh_gna;
    a.hh_gk = d_hh_gk;
    a.syn_g = d_syn_g;
    a.syn_e = d_syn_e;
    a.syn_decay = d_syn_decay;
    a.ic_slot = d_ic_slot;
    a.ic_on = d_ic_on;
    a.ic_off = d_ic_off;
    a.ic_amp = d_ic_amp;
    a.xe_step = d_xe_step;
    a.xe_syn = d_xe_syn;
    a.xe_w = d_xe_w;
    a.pk_xcur = d_pk_xcur;
    a.bk_off = d_bk_off;
    a.bk_nxt = d_bk_nxt;
    a.bk_q = d_bk_q;
    a.bk_w = d_bk_w;
    a.bk_cap = bk_cap;
    a.epoch_steps = K;
    a.sp_gid = d_sp_gid;
    a.sp_step = d_sp_step;
    a.sp_t = d_sp_t;
    a.sp_cap = sp_cap;
    a.ctr = d_ctr;
    a.pr_slot = d_pr_slot;
    a.pr_id = d_pr_id;
    a.trace = d_trace;
    a.trace_cap = trace_cap;
    a.trace_step0 = trace_step0;
    a.n_slots_total = L.n_slots;
    a.n_hh_total = int64_t(L.hh_cv.size());
    a.n_syn_total = int64_t(L.syn_global.size());
    a.dt = L.dt;
    a.threshold = L.threshold;
    a.gen_off = d_gen_off;
    a.gen_pk = d_gen_pk;
    a.gen_row = d_gen_row;
    a.gen_slot = d_gen_slot;
    a.gen_w = d_gen_w;
    a.gen_prm = d_gen_prm;
    a.gen_st = d_gen_st;
    a.gen_n = int64_t(L.gen_mech.size());
    return a;
}

VarArgs Sim::var_args() const {
    VarArgs v{};
    v.xe_t = d_xe_t;
    v.bk_t = d_bk_t;
    v.cap = d_cap;
    v.gmem = d_gmem;
    v.sigsum = d_sigsum;
    v.uoff = d_uoff;
    v.syn_tau = d_syn_tau;
    v.pk_steps = d_pk_steps;
    return v;
}

// The step kernel over every pack: one launch per class, each on the stream
// the class was given (the sim's stream or an auxiliary one forked from and
// joined back into it; classes sharing a stream run one after the other).
int Sim::launch_classes(const StepArgs& a0) {
    if (classes.size() <= 1) {
        StepArgs a = a0;
        a.pack0 = 0;
        if (timed)
            HIP_TRY(launch_var_step(a, var_args(), cfg, int32_t(L.packs.size()), st));
        else
            HIP_TRY(launch_step(a, cfg, int32_t(L.packs.size()), st));
        return ARB_OK;
    }
    HIP_TRY(hipEventRecord(fork_ev[0], st));
    for (hipStream_t x : aux) HIP_TRY(hipStreamWaitEvent(x, fork_ev[0], 0));
    for (size_t c = 0; c < classes.size(); ++c) {
        StepArgs a = a0;
        a.pack0 = classes[c].pack0;
        LaunchCfg lc = cfg;
        lc.lds_bytes = classes[c].lds;
        lc.syn_hbm = classes[c].hbm;
        if (cfg.coef_mode == 3) lc.reg_slots = classes[c].slots;
        hipStream_t s_c = (classes[c].stream == 0) ? st : aux[classes[c].stream - 1];
        if (timed)
            HIP_TRY(launch_var_step(a, var_args(), lc, classes[c].npack, s_c));
        else
            HIP_TRY(launch_step(a, lc, classes[c].npack, s_c));
    }
    for (size_t k = 0; k < aux.size(); ++k) {
        HIP_TRY(hipEventRecord(join_ev[k], aux[k]));
        HIP_TRY(hipStreamWaitEvent(st, join_ev[k], 0));
    }
    return ARB_OK;
}

// The epoch's network events: index the spike history by source, then every
// pack pulls its events of the epoch into its bucket.
int Sim::launch_pull(int64_t epoch, const int64_t* epoch_ptr) {
    IndexLaunch ix{};
    ix.h_gid = d_hist_gid;
    ix.h_step = d_hist_step;
    ix.h_cnt = d_hist_cnt;
    ix.h_cap = hist_cap;
    ix.n_hist = n_hist;
    ix.ranks = L.dry_run_ranks;
    ix.n_cells = L.n_cells;
    ix.sx_cap = sx_cap;
    ix.cnt = d_sx_cnt;
    ix.off = d_sx_off;
    ix.tile_sum = d_tile_sum;
    ix.sx_step = d_sx_step;
    ix.ctr = d_ctr;
    HIP_TRY(launch_index_spikes(ix, st));
    if (timed) {
        TimedPullArgs x{};
        x.in_off = d_in_off;
        x.cr_src = d_cr_src;
        x.cr_delay_ms = d_cr_delay_ms;
        x.cr_syn = d_cr_syn;
        x.cr_w = d_cr_w;
        x.sx_off = d_sx_off;
        x.sx_step = d_sx_step;
        x.n_src = L.n_src;
        x.bk_off = d_bk_off;
        x.bk_q = d_bk_q;
        x.bk_w = d_bk_w;
        x.bk_t = d_bk_t;
        x.ctr = d_ctr;
        x.epoch_ptr = epoch_ptr;
        x.epoch = epoch;
        x.dt = L.dt;
        x.bk_cap = bk_cap;
        x.epoch_steps = K;
        HIP_TRY(launch_pull_timed(x, int32_t(L.packs.size()), st));
        return ARB_OK;
    }
    PullArgs x{};
    x.in_off = d_in_off;
    x.cr_src = d_cr_src;
    x.cr_delay = d_cr_delay;
    x.cr_syn = d_cr_syn;
    x.cr_w = d_cr_w;
    x.sx_off = d_sx_off;
    x.sx_step = d_sx_step;
    x.n_src = L.n_src;
    x.bk_off = d_bk_off;
    x.bk_nxt = d_bk_nxt;
    x.bk_q = d_bk_q;
    x.bk_w = d_bk_w;
    x.ctr = d_ctr;
    x.epoch_ptr = epoch_ptr;
    x.epoch = epoch;
    x.bk_cap = bk_cap;
    x.epoch_steps = K;
    HIP_TRY(launch_pull_events(x, int32_t(L.packs.size()), st));
    return ARB_OK;
}

// The finished epoch's spikes into its history slot.
int Sim::launch_collect(int64_t epoch, const int64_t* epoch_ptr) {
    HIP_TRY(launch_collect_spikes(d_ctr, d_sp_gid, d_sp_step, sp_cap, d_hist_gid, d_hist_step, d_hist_cnt, hist_cap,
                                  n_hist, epoch, epoch_ptr, st));
    return ARB_OK;
}

// One epoch's kernels after the step arguments are set: (network) the
// epoch's events, the step kernel, (network) the spikes into the history;
// in graph mode the device epoch counter's advance after them.
int Sim::launch_epoch_sequence(const StepArgs& a, bool net, bool graph_mode) {
    if (graph_mode && net) {
        const int rc = launch_pull(0, d_epoch);
        if (rc != ARB_OK) return rc;
    }
    {
        const int rc = launch_classes(a);
        if (rc != ARB_OK) return rc;
    }
    if (net && a.epoch_end) {
        const int rc = launch_collect(a.step0 / K, graph_mode ? d_epoch : nullptr);
        if (rc != ARB_OK) return rc;
    }
    if (graph_mode) HIP_TRY(launch_advance_epoch(d_epoch, st));
    return ARB_OK;
}

// Capture one full epoch, with its step read from d_epoch.
int Sim::capture_epoch_graph() {
    if (graph) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    const bool net = !L.cr_src.empty();
    StepArgs a = step_args();
    a.epoch_ptr = d_epoch;
    a.nsteps = K;
    a.epoch_end = 1;
    hipGraph_t g = nullptr;
    if (!st_capture) HIP_TRY(hipStreamCreateWithFlags(&st_capture, hipStreamNonBlocking));
    hipStream_t keep = st;
    st = st_capture;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = launch_epoch_sequence(a, net, true);
    hipGraph_t captured = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &captured);
    st = keep;
    if (rc != ARB_OK) return rc;
    HIP_TRY(e);
    g = captured;
    hipError_t ie = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ie);
    graph_dirty = false;
    return ARB_OK;
}

// Enqueue steps [step, step + n): epochs of K steps aligned at multiples of
// K; network events are sorted at each epoch start and spikes exchanged at
// each epoch end.  `rec` (optional) records the pre-step state of every step
// for the adjoint.  With ARB_FLAG_GRAPH, whole epochs replay a captured graph.
int Sim::advance(int64_t n, const RecordArgs* rec) {
    const bool net = !L.cr_src.empty();
    int64_t done = 0;
    while (n > 0) {
        const int64_t e = step / K, pos = step % K;
        if ((p.flags & ARB_FLAG_GRAPH) && !rec && pos == 0 && n >= K) {
            const int64_t ne = n / K;
            if (graph_dirty || !graph) {
                const int rc = capture_epoch_graph();
                if (rc != ARB_OK) return rc;
            }
            HIP_TRY(hipMemcpyAsync(d_epoch, &e, sizeof e, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));  // e lives on this stack frame
            for (int64_t q = 0; q < ne; ++q) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (p.flags & ARB_FLAG_TIME_KERNELS) {
                    if (timer_free.size() < 2) {
                        hipEvent_t x;
                        HIP_TRY(hipEventCreate(&x));
                        timer_free.push_back(x);
                        HIP_TRY(hipEventCreate(&x));
                        timer_free.push_back(x);
                    }
                    e0 = timer_free.back();
                    timer_free.pop_back();
                    e1 = timer_free.back();
                    timer_free.pop_back();
                    HIP_TRY(hipEventRecord(e0, st));
                }
                HIP_TRY(hipGraphLaunch(graph, st));
                if (e0) {
                    HIP_TRY(hipEventRecord(e1, st));
                    timer_pending.push_back({e0, e1});
                }
            }
            step += ne * K;
            n -= ne * K;
            done += ne * K;
            continue;
        }
        const int64_t nthis = std::min<int64_t>(n, K - pos);
        if (net && pos == 0) {
            const int rc = launch_pull(e, nullptr);
            if (rc != ARB_OK) return rc;
        }
        StepArgs a = step_args();
        a.step0 = step;
        a.nsteps = int32_t(nthis);
        a.epoch_end = (pos + nthis == K) ? 1 : 0;
        if (rec) {  // rows offset by the steps already done in this call
            if (cfg.coef_mode == 3 && !cfg.rec)
                return set_error(ARB_ESTATE, "recording needs a sim built with ARB_FLAG_GRADIENTS");
            a.rec_V = rec->V + done * L.n_slots;
            a.rec_m = rec->m + done * int64_t(L.hh_cv.size());
            a.rec_h = rec->h + done * int64_t(L.hh_cv.size());
            a.rec_n = rec->n + done * int64_t(L.hh_cv.size());
            a.rec_g = rec->g + done * int64_t(L.syn_global.size());
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (p.flags & ARB_FLAG_TIME_KERNELS) {
            if (timer_free.size() < 2) {
                hipEvent_t x;
                HIP_TRY(hipEventCreate(&x));
                timer_free.push_back(x);
                HIP_TRY(hipEventCreate(&x));
                timer_free.push_back(x);
            }
            e0 = timer_free.back();
            timer_free.pop_back();
            e1 = timer_free.back();
            timer_free.pop_back();
            HIP_TRY(hipEventRecord(e0, st));
        }
        {
            const int rc = launch_classes(a);
            if (rc != ARB_OK) return rc;
        }
        if (e0) {
            HIP_TRY(hipEventRecord(e1, st));
            timer_pending.push_back({e0, e1});
        }
        step += nthis;
        n -= nthis;
        done += nthis;
        if (net && a.epoch_end) {
            const int rc = launch_collect(e, nullptr);
            if (rc != ARB_OK) return rc;
        }
    }
    return ARB_OK;
}

StateShape Sim::state_shape() const {
    StateShape sh;
    sh.K = K;
    sh.bk_cap = bk_cap;
    sh.sp_cap = sp_cap;
    sh.n_hist = n_hist;
    sh.hist_cap = hist_cap;
    sh.net = d_bk_off != nullptr;
    return sh;
}

void Sim::state_part_ptrs(void* ptr[kStateParts]) const {
    void* const v[kStateParts] = {d_V,      d_hh_m,   d_hh_h,    d_hh_n,    d_syn_g,    d_pk_xcur,
                                  d_bk_off, d_bk_nxt, d_bk_q,    d_bk_w,    d_ctr,      d_sp_gid,
                                  d_sp_step, d_sp_t,  d_hist_cnt, d_hist_gid, d_hist_step, d_gen_st};
    for (int k = 0; k < kStateParts; ++k) ptr[k] = v[k];
}

int Sim::check_flags(bool& spikes_lost, bool& events_lost) {
    Counters c{};
    HIP_TRY(hipMemcpyAsync(&c, d_ctr, sizeof c, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    spikes_lost = (c.flags & kFlagSpikeOverflow) != 0;
    events_lost = (c.flags & kFlagEventOverflow) != 0;
    return ARB_OK;
}

}  // namespace arbmi

namespace {

template <class T>
T* dalloc(Sim* s, size_t n, int& rc) {
    if (rc != ARB_OK) return nullptr;
    T* ptr = static_cast<T*>(s->raw_alloc(n * sizeof(T)));
    if (!ptr) rc = fail(ARB_ENOMEM, "device allocation failed");
    return ptr;
}

template <class T>
T* dupload(Sim* s, const std::vector<T>& v, int& rc) {
    T* ptr = dalloc<T>(s, std::max<size_t>(v.size(), 1), rc);
    if (rc == ARB_OK && !v.empty()) rc = s->upload(ptr, v.data(), v.size() * sizeof(T));
    return ptr;
}

int build_device(Sim* s) {
    Lowered& L = s->L;
    int rc = ARB_OK;
    const int np = int(L.packs.size());
    s->d_pk = dupload(s, L.packs, rc);
    s->d_rd = dupload(s, L.rounds, rc);
    s->d_tk = dupload(s, L.tasks, rc);
    s->d_ch = dupload(s, L.ch_slot, rc);
    s->d_ch_task = dupload(s, L.ch_task, rc);
    s->d_tk_ptask = dupload(s, L.tk_ptask, rc);
    s->d_tk_lev = dupload(s, L.tk_lev, rc);
    s->d_tk_Z = dupload(s, L.tk_Z, rc);
    s->d_nl = dupload(s, L.nl, rc);
    s->d_pc_gid = dupload(s, L.pc_gid, rc);
    s->d_pc_soma = dupload(s, L.pc_soma, rc);
    std::vector<double> v0(L.n_slots, 0.0);
    for (int64_t i = 0; i < L.n_cv; ++i) v0[L.perm[i]] = L.v_init;
    s->d_V = dupload(s, v0, rc);
    s->d_alpha = dupload(s, L.alpha, rc);
    s->d_beta = dupload(s, L.beta, rc);
    s->d_F = dupload(s, L.F, rc);
    s->d_invd = dupload(s, L.invd, rc);
    // gates at steady state for v_init (host evaluation of the same rates)
    const size_t nhh = L.hh_cv.size();
    {
        const double v = L.v_init;
        auto ex = [](double x) { return (1.0 + x == 1.0) ? 1.0 : x / std::expm1(x); };
        const double am = ex(-(v + 40.0) * 0.1), bm = 4.0 * std::exp(-(v + 65.0) * (1.0 / 18.0));
        const double ah = 0.07 * std::exp(-(v + 65.0) * 0.05), bh = 1.0 / (std::exp(-(v + 35.0) * 0.1) + 1.0);
        const double an = 0.1 * ex(-(v + 55.0) * 0.1), bn = 0.125 * std::exp(-(v + 65.0) * (1.0 / 80.0));
        s->m0 = am / (am + bm);
        s->h0 = ah / (ah + bh);
        s->n0 = an / (an + bn);
    }
    s->d_hh_m = dupload(s, std::vector<double>(nhh, s->m0), rc);
    s->d_hh_h = dupload(s, std::vector<double>(nhh, s->h0), rc);
    s->d_hh_n = dupload(s, std::vector<double>(nhh, s->n0), rc);
    s->d_hh_gna = dupload(s, L.hh_gna, rc);
    s->d_hh_gk = dupload(s, L.hh_gk, rc);
    const size_t nsyn = L.syn_global.size();
    s->d_syn_g = dupload(s, std::vector<double>(nsyn, 0.0), rc);
    s->d_syn_e = dupload(s, L.syn_e, rc);
    s->d_syn_decay = dupload(s, L.syn_decay, rc);
    s->d_ic_slot = dupload(s, L.ic_slot, rc);
    s->d_ic_on = dupload(s, L.ic_on, rc);
    s->d_ic_off = dupload(s, L.ic_off, rc);
    s->d_ic_amp = dupload(s, L.ic_amp, rc);
    s->d_xe_step = dupload(s, L.xe_step, rc);
    s->d_xe_syn = dupload(s, L.xe_syn, rc);
    s->d_xe_w = dupload(s, L.xe_w, rc);
    if (!L.gen_mech.empty()) {
        s->d_gen_off = dupload(s, L.gen_off, rc);
        s->d_gen_pk = dupload(s, L.gen_pk, rc);
        s->d_gen_row = dupload(s, L.gen_row, rc);
        s->d_gen_slot = dupload(s, L.gen_slot, rc);
        s->d_gen_w = dupload(s, L.gen_w, rc);
        s->d_gen_prm = dupload(s, L.gen_prm, rc);
        s->d_gen_st = dupload(s, L.gen_st0, rc);
    }
    if (s->timed) {
        s->d_xe_t = dupload(s, L.xe_t, rc);
        s->d_cr_delay_ms = dupload(s, L.cr_delay_ms, rc);
        s->d_cap = dupload(s, L.cap, rc);
        s->d_gmem = dupload(s, L.gmem, rc);
        s->d_sigsum = dupload(s, L.sigsum, rc);
        s->d_uoff = dupload(s, L.uoff, rc);
        s->d_syn_tau = dupload(s, L.syn_tau, rc);
        s->d_pk_steps = dupload(s, std::vector<int64_t>(np, 0), rc);
    }
    std::vector<int64_t> xcur(np);
    for (int k = 0; k < np; ++k) xcur[k] = L.packs[k].xe0;
    s->xcur0 = xcur;
    s->d_pk_xcur = dupload(s, xcur, rc);
    s->d_cr_syn = dupload(s, L.cr_syn, rc);
    s->d_cr_delay = dupload(s, L.cr_delay, rc);
    s->d_cr_src = dupload(s, L.cr_src, rc);
    s->d_cr_w = dupload(s, L.cr_w, rc);
    s->d_in_off = dupload(s, L.in_off, rc);
    s->d_perm = dupload(s, L.perm, rc);
    // spikes
    int64_t spc = s->p.spike_capacity;
    if (spc <= 0) spc = std::max<int64_t>(1 << 16, int64_t(L.n_cells) * 64);
    spc = std::min<int64_t>(spc, int64_t(1) << 31);
    s->sp_cap = uint32_t(spc);
    s->d_sp_gid = dalloc<uint32_t>(s, s->sp_cap, rc);
    s->d_sp_step = dalloc<int64_t>(s, s->sp_cap, rc);
    s->d_sp_t = dalloc<double>(s, s->sp_cap, rc);
    // network: one event bucket per pack for the running epoch, and the spike
    // history of the epochs whose spikes can still arrive (a spike of epoch
    // e - n_hist + 1 .. e - 1 can deliver into epoch e, none of epoch e)
    const bool net = !L.cr_src.empty();
    if (net) {
        int64_t cap = s->p.event_capacity;
        if (cap <= 0) cap = std::max<int64_t>(64, 4 * L.max_in_per_pack);
        s->bk_cap = int32_t(std::min<int64_t>(cap, INT32_MAX));
        s->n_hist = int32_t(1 + (L.max_delay + s->K - 1) / s->K);
        s->hist_cap = s->sp_cap;
    } else {
        s->bk_cap = 0;
        s->n_hist = 1;
        s->hist_cap = 0;
    }
    if (net) {
        const size_t noff = size_t(np) * (size_t(s->K) + 1);
        s->d_bk_off = dalloc<uint32_t>(s, noff, rc);
        if (rc == ARB_OK) rc = s->fill_zero(s->d_bk_off, noff * sizeof(uint32_t));
        s->d_bk_nxt = dalloc<uint32_t>(s, noff, rc);
        if (rc == ARB_OK) rc = s->fill_zero(s->d_bk_nxt, noff * sizeof(uint32_t));
        s->d_bk_q = dalloc<int32_t>(s, size_t(np) * size_t(s->bk_cap), rc);
        s->d_bk_w = dalloc<double>(s, size_t(np) * size_t(s->bk_cap), rc);
        if (s->timed) s->d_bk_t = dalloc<double>(s, size_t(np) * size_t(s->bk_cap), rc);
    }
    const size_t nh = std::max<size_t>(1, size_t(s->n_hist) * s->hist_cap);
    s->d_hist_gid = dalloc<uint32_t>(s, nh, rc);
    s->d_hist_step = dalloc<int64_t>(s, nh, rc);
    s->d_hist_cnt = dalloc<uint32_t>(s, size_t(s->n_hist), rc);
    if (rc == ARB_OK) rc = s->fill_zero(s->d_hist_cnt, size_t(s->n_hist) * sizeof(uint32_t));
    // the source index: one count and offset per source gid (ranks x cells
    // in a dry run), and the indexed spikes, proxies included (a dry run
    // holds at most 4 per local cell, history epoch and rank)
    const size_t nsrc = size_t(std::max<int64_t>(L.n_src, L.n_cells));
    s->sx_cap = (L.dry_run_ranks > 1) ? int64_t(L.dry_run_ranks) * s->n_hist *
                                            std::min<int64_t>(s->hist_cap, 4 * int64_t(L.n_cells))
                                      : int64_t(nh);
    s->d_sx_cnt = dalloc<int32_t>(s, nsrc + 1, rc);
    if (rc == ARB_OK) rc = s->fill_zero(s->d_sx_cnt, (nsrc + 1) * sizeof(int32_t));
    s->d_sx_off = dalloc<int64_t>(s, nsrc + 1, rc);
    s->d_sx_step = dalloc<int64_t>(s, size_t(std::max<int64_t>(1, s->sx_cap)), rc);
    s->d_tile_sum = dalloc<int64_t>(s, size_t(std::max<int64_t>(1, index_tiles(int64_t(nsrc)))), rc);
    s->d_epoch = dalloc<int64_t>(s, 1, rc);
    s->d_ctr = dalloc<Counters>(s, 1, rc);
    if (rc == ARB_OK) rc = s->fill_zero(s->d_ctr, sizeof(Counters));
    if (rc != ARB_OK) return rc;
    return ARB_OK;
}

}  // namespace

namespace arbmi {

int build_sim(const ModelView& m, const arb_params& pp, const DeviceLimits& d, Sim** out, std::string& err) {
    const arb_params* p = &pp;
    *out = nullptr;
    Sim* s = new Sim();
    s->p = *p;
    s->st = static_cast<hipStream_t>(p->hip_stream);
    s->device = d.dev;
    s->n_cu = d.n_cu;
    s->lds_max = d.lds_max;
    const Plan plan = choose_plan(m.cells, m.n_cells, m.br, m.n_br, *p, d.lds_max, d.n_cu);
    LowerOptions opt;
    opt.block_threads = plan.block_threads;
    opt.coef_mode = plan.coef_mode;
    opt.lds_budget = plan.lds_budget;
    opt.lds_hard_max = plan.lds_hard_max;
    opt.max_cells_per_pack = plan.max_cells_per_pack;
    opt.reg_slots = plan.coef_mode == 3 ? plan.reg_slots : 0;
    opt.reg_len = plan.reg_len;
    opt.grads = (p->flags & ARB_FLAG_GRADIENTS) != 0;
    opt.conn_delay_ms = m.conn_delay_ms;
    opt.ev_t_ms = m.ev_t_ms;
    const bool timed = m.conn_delay_ms != nullptr || m.ev_t_ms != nullptr;
    int rc = ARB_OK;
    if (timed) {
        // one cell per workgroup in the register layout; unless the caller
        // fixed the workgroup size, the smallest one whose register slots
        // hold every cell
        opt.coef_mode = 3;
        opt.max_cells_per_pack = 1;
        opt.lds_budget = opt.lds_hard_max;
        for (int T : {64, 128, 256}) {
            if (p->block_threads && T != p->block_threads) continue;
            arb_params pt = *p;
            pt.block_threads = T;
            pt.coef_mode = 3;
            pt.cells_per_pack = 1;
            const Plan pl = choose_plan(m.cells, m.n_cells, m.br, m.n_br, pt, d.lds_max, d.n_cu);
            opt.block_threads = T;
            opt.reg_slots = pl.reg_slots;
            opt.reg_len = pl.reg_len;
            s->L = Lowered();
            err.clear();
            rc = lower_model(m.cells, m.n_cells, m.br, m.n_br, m.syn, m.n_syn, m.conn, m.n_conn, m.ev, m.n_ev, m.ic,
                             m.n_ic, *p, opt, s->L, err);
            if (rc == ARB_OK || (err.find("LDS") == std::string::npos && err.find("register") == std::string::npos))
                break;
        }
    } else {
        rc = lower_model(m.cells, m.n_cells, m.br, m.n_br, m.syn, m.n_syn, m.conn, m.n_conn, m.ev, m.n_ev, m.ic,
                         m.n_ic, *p, opt, s->L, err);
    }
    const bool auto_mode = p->coef_mode == 0 || (p->flags & ARB_FLAG_AUTOTUNE);
    if (rc == ARB_EINVAL && auto_mode && !timed && opt.coef_mode != 2 &&
        (err.find("LDS") != std::string::npos || err.find("register") != std::string::npos)) {
        // a cell too large for LDS- or register-resident coefficients: stream them
        opt.coef_mode = 2;
        opt.reg_slots = 0;
        opt.block_threads = p->block_threads ? p->block_threads : 256;
        opt.max_cells_per_pack = std::max<int64_t>(1, plan.fallback_cells_per_pack);
        opt.lds_budget = plan.fallback_lds_budget;
        opt.lds_hard_max = plan.fallback_lds_hard_max;
        s->L = Lowered();
        rc = lower_model(m.cells, m.n_cells, m.br, m.n_br, m.syn, m.n_syn, m.conn, m.n_conn, m.ev, m.n_ev, m.ic,
                         m.n_ic, *p, opt, s->L, err);
    }
    if (rc != ARB_OK) {
        delete s;
        return rc;
    }
    if (!d.have_dev) {
        delete s;
        err = "no HIP device available";
        return ARB_EHIP;
    }
    s->timed = s->L.timed;
    const bool net = !s->L.cr_src.empty();
    s->K = p->epoch_steps > 0 ? p->epoch_steps : (net ? std::min(s->L.min_delay, kMaxEpochSteps) : 1000);
    if (net && s->K > kMaxEpochSteps) {
        delete s;
        err = "epoch_steps exceeds 16384 in a network";
        return ARB_EINVAL;
    }
    s->cfg.block_threads = s->L.block_threads;
    s->cfg.coef_mode = s->L.coef_mode;
    s->cfg.reg_slots = s->L.reg_slots;
    s->cfg.reg_len = s->L.reg_len;
    s->cfg.syn_hbm = 0;
    s->cfg.rec = (s->L.coef_mode == 3 && (p->flags & ARB_FLAG_GRADIENTS)) ? 1 : 0;
    s->cfg.gen = s->L.gen_mech.empty() ? 0 : 1;
    int64_t lds = 0;
    for (const PackDesc& D : s->L.packs) {
        lds = std::max(lds, pack_lds_bytes(D, s->L.coef_mode));
        if (s->L.coef_mode == 3 && (D.syn_global || D.hh_global)) s->cfg.syn_hbm = 1;
    }
    if (s->cfg.rec && s->cfg.syn_hbm) {  // the lowering keeps gradient sims' synapses in LDS
        delete s;
        err = "internal: a gradient sim keeps synapse state in HBM";
        return ARB_EINVAL;
    }
    if (lds > d.lds_max - 256) {
        delete s;
        err = "a pack needs more LDS than the device has";
        return ARB_EINVAL;
    }
    s->cfg.lds_bytes = int(std::max<int64_t>(lds, 8));
    // Classes: runs of packs that need the same kernel variant (register
    // slots in use, state in HBM) and allow the same number of workgroups
    // per CU by LDS (1, 2, 3, 4 or more).  The lowering orders the packs so
    // that each class is a contiguous range; a class's LDS is its largest
    // pack's, and it runs as its own launch.
    {
        const Lowered& L = s->L;
        const int64_t lim = d.lds_max - 256;
        auto cat = [&](int64_t b) { return b > lim / 2 ? 1 : b > lim / 3 ? 2 : b > lim / 4 ? 3 : 4; };
        const int32_t np = int32_t(L.packs.size());
        auto slots_of = [&](int32_t k) {
            int used = 1;
            for (int32_t r = 0; r < L.packs[k].nrd; ++r) used = std::max(used, L.rounds[L.packs[k].rd0 + r].j + 1);
            return L.coef_mode == 3 ? used : 0;
        };
        auto hbm_of = [&](int32_t k) {
            return (L.coef_mode == 3 && (L.packs[k].syn_global || L.packs[k].hh_global)) ? 1 : 0;
        };
        struct Key {
            int slots, hbm, cat;
            bool operator==(const Key& o) const { return slots == o.slots && hbm == o.hbm && cat == o.cat; }
        };
        auto key_of = [&](int32_t k) {
            return Key{slots_of(k), hbm_of(k), cat(pack_lds_bytes(L.packs[k], L.coef_mode))};
        };
        int32_t start = 0;
        Key cur = np ? key_of(0) : Key{0, 0, 0};
        int64_t mx = 0;
        for (int32_t k = 0; k <= np; ++k) {
            const bool end_run = (k == np) || !(key_of(k) == cur);
            if (end_run && k > start) {
                s->classes.push_back({start, k - start, int(std::max<int64_t>(mx, 8)), cur.hbm, cur.slots, 0});
                start = k;
                mx = 0;
                if (k < np) cur = key_of(k);
            }
            if (k < np) mx = std::max(mx, pack_lds_bytes(L.packs[k], L.coef_mode));
        }
        // a class of a few packs is not worth a stream of its own: merge it
        // into the previous class if that uses as many register slots (the
        // variant that can keep state in HBM also runs packs that keep none)
        std::vector<Sim::Class> merged;
        for (const Sim::Class& c : s->classes) {
            if (!merged.empty() && c.npack < 2 * d.n_cu && merged.back().slots == c.slots) {
                merged.back().npack += c.npack;
                merged.back().lds = std::max(merged.back().lds, c.lds);
                merged.back().hbm |= c.hbm;
                continue;
            }
            merged.push_back(c);
        }
        s->classes = merged;
        if (s->classes.size() == 1 && s->L.coef_mode == 3 && !s->cfg.rec) s->cfg.reg_slots = s->classes[0].slots;
        // Classes onto at most kClassStreams streams (the device runs a
        // process's streams on four hardware queues; two busy streams on one
        // queue run one after the other): longest first, each onto the
        // stream with the least work so far, a class's work taken as its
        // packs' CV rows.
        int n_streams = 1;
        if (s->classes.size() > 1) {
            n_streams = int(std::min<size_t>(s->classes.size(), Sim::kClassStreams));
            std::vector<int64_t> work(s->classes.size(), 0), load(n_streams, 0);
            for (size_t c = 0; c < s->classes.size(); ++c)
                for (int32_t k = s->classes[c].pack0; k < s->classes[c].pack0 + s->classes[c].npack; ++k)
                    work[c] += L.packs[k].nslot;
            std::vector<size_t> order(s->classes.size());
            std::iota(order.begin(), order.end(), size_t(0));
            std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return work[x] > work[y]; });
            for (size_t c : order) {
                const int at = int(std::min_element(load.begin(), load.end()) - load.begin());
                s->classes[c].stream = at;
                load[at] += work[c];
            }
        }
        if (n_streams > 1) {
            for (int c = 1; c < n_streams; ++c) {
                hipStream_t x;
                hipEvent_t e;
                if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
                    destroy_sim(s);  // the streams and events made so far
                    err = "stream creation failed";
                    return ARB_EHIP;
                }
                s->aux.push_back(x);
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                    destroy_sim(s);  // the streams and events made so far
                    err = "event creation failed";
                    return ARB_EHIP;
                }
                s->join_ev.push_back(e);
            }
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                destroy_sim(s);  // the streams and events made so far
                err = "event creation failed";
                return ARB_EHIP;
            }
            s->fork_ev.push_back(e);
        }
    }
    hipError_t he = prepare_step_kernels(int(d.lds_max));
    if (he == hipSuccess && s->timed) he = prepare_var_kernels(int(d.lds_max));
    if (he != hipSuccess) {
        destroy_sim(s);
        err = std::string("prepare_step_kernels: ") + hipGetErrorString(he);
        return ARB_EHIP;
    }
    rc = build_device(s);
    if (rc == ARB_OK) {
        hipError_t e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) rc = hip_fail(e, "upload");
    }
    // the no-allocation voltage read's staging buffer on this device (a
    // failed lookup only disables that call)
    if (rc == ARB_OK) (void)noalloc_setup(s->device);
    if (rc != ARB_OK) {
        err = g_err;
        destroy_sim(s);  // buffers, streams and events
        return rc;
    }
    *out = s;
    return ARB_OK;
}

void destroy_sim(Sim* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->st);
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (s->st_capture) (void)hipStreamDestroy(s->st_capture);
    for (hipStream_t x : s->aux) (void)hipStreamDestroy(x);
    for (hipEvent_t e : s->fork_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->join_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->timer_free) (void)hipEventDestroy(e);
    for (auto& pr : s->timer_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    grad_release(s);
    s->release_all();
    delete s;
}

}  // namespace arbmi

namespace {

int build_cells(const arb_cell* cells, int32_t n_cells, const arb_branch* branches, int64_t n_branches,
                const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, int64_t n_conn,
                const arb_event* ev, int64_t n_ev, const arb_iclamp* stim, int32_t n_stim,
                const double* conn_delay_ms, const double* ev_t_ms, const arb_params* p, arb_sim* out) {
    g_err.clear();
    if (!out) return fail(ARB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(ARB_EINVAL, "params is NULL");
    if (p->block_threads != 0 && p->block_threads != 64 && p->block_threads != 128 && p->block_threads != 256)
        return fail(ARB_EINVAL, "block_threads must be 0, 64, 128 or 256");
    if (p->coef_mode < 0 || p->coef_mode > 3) return fail(ARB_EINVAL, "coef_mode must be 0, 1, 2 or 3");
    if (p->cells_per_pack < 0) return fail(ARB_EINVAL, "cells_per_pack must be >= 0");
    if ((p->alloc == nullptr) != (p->free == nullptr)) return fail(ARB_EINVAL, "alloc and free must be given together");

    // device limits (validation runs even without a device)
    DeviceLimits d;
    int ndev = 0;
    d.have_dev = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
    if (d.have_dev) {
        if (hipGetDevice(&d.dev) != hipSuccess) d.dev = 0;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d.dev) == hipSuccess && v > 0)
            d.lds_max = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d.dev) == hipSuccess && v > 0) d.n_cu = v;
    }
    ModelView m{cells, n_cells, branches, n_branches, syn, n_syn, conn, n_conn, ev, n_ev, stim, n_stim};
    m.conn_delay_ms = conn_delay_ms;
    m.ev_t_ms = ev_t_ms;
    const bool timed = conn_delay_ms != nullptr || ev_t_ms != nullptr;
    const bool dens = p->n_densities != 0;
    arb_params q = *p;
    if (dens && q.coef_mode == 0) q.coef_mode = 3;  // generated mechanisms run in the register layout
    if ((p->flags & ARB_FLAG_AUTOTUNE) && d.have_dev && !timed && !dens && p->block_threads == 0 &&
        p->coef_mode == 0 && p->cells_per_pack == 0)
        q = autotune(m, *p, d);
    Sim* s = nullptr;
    std::string err;
    const int rc = build_sim(m, q, d, &s, err);
    if (rc != ARB_OK) return fail(rc, err);
    *out = s;
    return ARB_OK;
}

}  // namespace

extern "C" {

int arb_build_cells(const arb_cell* cells, int32_t n_cells, const arb_branch* branches, int64_t n_branches,
                    const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, int64_t n_conn,
                    const arb_event* ev, int64_t n_ev, const arb_iclamp* stim, int32_t n_stim,
                    const arb_params* p, arb_sim* out) {
    return build_cells(cells, n_cells, branches, n_branches, syn, n_syn, conn, n_conn, ev, n_ev, stim, n_stim,
                       nullptr, nullptr, p, out);
}

int arb_build_cells_timed(const arb_cell* cells, int32_t n_cells, const arb_branch* branches, int64_t n_branches,
                          const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, const double* delay_ms,
                          int64_t n_conn, const arb_event* ev, const double* t_ms, int64_t n_ev,
                          const arb_params* p, arb_sim* out) {
    static const double kNone = 0.0;  // a non-null marker for empty arrays
    if ((n_conn > 0 && !delay_ms) || (n_ev > 0 && !t_ms)) {
        g_err.clear();
        if (out) *out = nullptr;
        return fail(ARB_EINVAL, "delay_ms and t_ms must be given for every connection and event");
    }
    return build_cells(cells, n_cells, branches, n_branches, syn, n_syn, conn, n_conn, ev, n_ev, nullptr, 0,
                       delay_ms ? delay_ms : &kNone, t_ms ? t_ms : &kNone, p, out);
}

int arb_mechanism_count(void) { return gen::kNumMechs; }

int arb_mechanism_info(int32_t id, arb_mech_info* out) {
    if (!out) return fail(ARB_EINVAL, "null argument");
    if (id < 0 || id >= gen::kNumMechs) return fail(ARB_EINVAL, "mechanism id out of range");
    const gen::MechDesc& M = gen::kMechs[id];
    arb_mech_info I{};
    std::snprintf(I.name, sizeof I.name, "%s", M.name);
    I.n_params = M.n_params;
    I.n_states = M.n_states;
    for (int k = 0; k < M.n_params && k < 8; ++k) {
        std::snprintf(I.param_names[k], sizeof I.param_names[k], "%s", M.param_names[k]);
        I.defaults[k] = M.defaults[k];
    }
    *out = I;
    return ARB_OK;
}

int arb_get_mechanism_instances(arb_sim s_, int64_t* counts, int32_t n) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !counts) return fail(ARB_EINVAL, "null argument");
    if (n < gen::kNumMechs) return fail(ARB_EINVAL, "counts smaller than the catalogue");
    for (int32_t k = 0; k < n; ++k) counts[k] = 0;
    for (int32_t id : s->L.gen_mech) counts[id]++;
    return ARB_OK;
}

int arb_get_step_count(arb_sim s_, int64_t* n_out) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !n_out) return fail(ARB_EINVAL, "null argument");
    *n_out = 0;
    const int64_t np = int64_t(s->L.packs.size());
    if (!s->timed) {  // every cell takes every step of the grid
        *n_out = s->step * int64_t(s->L.n_cells);
        return ARB_OK;
    }
    std::vector<int64_t> c(size_t(std::max<int64_t>(np, 1)), 0);
    HIP_TRY(hipStreamSynchronize(s->st));
    if (np) HIP_TRY(hipMemcpy(c.data(), s->d_pk_steps, size_t(np) * 8, hipMemcpyDeviceToHost));
    int64_t tot = 0;
    for (int64_t k = 0; k < np; ++k) tot += c[size_t(k)];
    *n_out = tot;
    return ARB_OK;
}

int arb_plan_layout(const arb_cell* cells, int32_t n_cells, const arb_branch* branches, int64_t n_branches,
                    const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, int64_t n_conn,
                    const arb_event* ev, int64_t n_ev, const arb_iclamp* stim, int32_t n_stim,
                    const arb_params* p, arb_info* info) {
    g_err.clear();
    if (!p || !info) return fail(ARB_EINVAL, "null argument");
    if (p->block_threads != 0 && p->block_threads != 64 && p->block_threads != 128 && p->block_threads != 256)
        return fail(ARB_EINVAL, "block_threads must be 0, 64, 128 or 256");
    if (p->coef_mode < 0 || p->coef_mode > 3) return fail(ARB_EINVAL, "coef_mode must be 0, 1, 2 or 3");
    if (p->cells_per_pack < 0) return fail(ARB_EINVAL, "cells_per_pack must be >= 0");
    DeviceLimits d;  // MI355X: 256 CUs, 160 KiB LDS
    const Plan plan = choose_plan(cells, n_cells, branches, n_branches, *p, d.lds_max, d.n_cu);
    LowerOptions opt;
    opt.block_threads = plan.block_threads;
    opt.coef_mode = plan.coef_mode;
    opt.lds_budget = plan.lds_budget;
    opt.lds_hard_max = plan.lds_hard_max;
    opt.max_cells_per_pack = plan.max_cells_per_pack;
    opt.reg_slots = plan.coef_mode == 3 ? plan.reg_slots : 0;
    opt.reg_len = plan.reg_len;
    opt.grads = (p->flags & ARB_FLAG_GRADIENTS) != 0;
    Lowered L;
    std::string err;
    int rc = lower_model(cells, n_cells, branches, n_branches, syn, n_syn, conn, n_conn, ev, n_ev, stim, n_stim, *p,
                         opt, L, err);
    const bool auto_mode = p->coef_mode == 0 || (p->flags & ARB_FLAG_AUTOTUNE);
    if (rc == ARB_EINVAL && auto_mode && opt.coef_mode != 2 &&
        (err.find("LDS") != std::string::npos || err.find("register") != std::string::npos)) {
        opt.coef_mode = 2;
        opt.reg_slots = 0;
        opt.block_threads = p->block_threads ? p->block_threads : 256;
        opt.max_cells_per_pack = std::max<int64_t>(1, plan.fallback_cells_per_pack);
        opt.lds_budget = plan.fallback_lds_budget;
        opt.lds_hard_max = plan.fallback_lds_hard_max;
        L = Lowered();
        rc = lower_model(cells, n_cells, branches, n_branches, syn, n_syn, conn, n_conn, ev, n_ev, stim, n_stim, *p,
                         opt, L, err);
    }
    if (rc != ARB_OK) return fail(rc, err);
    const std::string bad = verify_layout(L);
    if (!bad.empty()) return fail(ARB_EINVAL, "layout invariant violated: " + bad);
    arb_info I{};
    I.n_cells = L.n_cells;
    I.n_packs = int32_t(L.packs.size());
    I.n_cv = L.n_cv;
    I.n_slots = L.n_slots;
    I.n_hh = int64_t(L.hh_cv.size());
    I.n_syn = int64_t(L.syn_pack_index.size());  // the model's synapses (pack order may pad)
    I.n_conn = int64_t(L.cr_src.size());
    I.epoch_steps = p->epoch_steps > 0 ? p->epoch_steps
                                       : (L.cr_src.empty() ? 1000 : std::min(L.min_delay, kMaxEpochSteps));
    I.block_threads = L.block_threads;
    I.coef_mode = L.coef_mode;
    int64_t lds = 0;
    for (const PackDesc& D : L.packs) lds = std::max(lds, pack_lds_bytes(D, L.coef_mode));
    I.lds_bytes = int32_t(lds);
    I.bytes_per_step = 44 * L.n_cv + 56 * I.n_hh + 20 * I.n_syn;
    I.reg_slots = L.coef_mode == 3 ? L.reg_slots : 0;
    I.reg_len = L.coef_mode == 3 ? L.reg_len : 0;
    I.syn_hbm = 0;
    for (const PackDesc& D : L.packs)
        if (L.coef_mode == 3 && (D.syn_global || D.hh_global)) I.syn_hbm = 1;
    *info = I;
    return ARB_OK;
}

int arb_step(arb_sim s_, int64_t n_steps) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s) return fail(ARB_EINVAL, "sim is NULL");
    if (n_steps < 0) return fail(ARB_EINVAL, "n_steps < 0");
    if (s->step + n_steps >= (int64_t(1) << 31)) return fail(ARB_EINVAL, "step count beyond 2^31");
    s->grad_valid = false;
    return s->advance(n_steps, nullptr);
}

int arb_get_voltages(arb_sim s_, double* dst, int64_t n, int dst_on_device) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !dst) return fail(ARB_EINVAL, "null argument");
    if (n < s->L.n_cv) return fail(ARB_EINVAL, "destination smaller than the CV count");
    const int64_t ncv = s->L.n_cv;
    if (dst_on_device) {
        HIP_TRY(launch_gather(s->d_V, s->d_perm, dst, ncv, s->st));
        HIP_TRY(hipStreamSynchronize(s->st));
        return ARB_OK;
    }
    int rc = ARB_OK;
    if (!s->d_tmp || s->tmp_n < ncv) {
        s->d_tmp = dalloc<double>(s, size_t(ncv), rc);
        if (rc != ARB_OK) return rc;
        s->tmp_n = ncv;
    }
    HIP_TRY(launch_gather(s->d_V, s->d_perm, s->d_tmp, ncv, s->st));
    HIP_TRY(hipMemcpyAsync(dst, s->d_tmp, size_t(ncv) * 8, hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    return ARB_OK;
}

int arb_get_spikes(arb_sim s_, arb_spike* dst, int64_t cap, int64_t* n_out) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !n_out) return fail(ARB_EINVAL, "null argument");
    *n_out = 0;
    Counters c{};
    HIP_TRY(hipMemcpyAsync(&c, s->d_ctr, sizeof c, hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    const uint32_t have = std::min(c.sp_count, s->sp_cap);
    const int64_t n = int64_t(have) - int64_t(s->sp_user);
    if (n > cap || (n > 0 && !dst)) return fail(ARB_EOVERFLOW, "destination too small for the pending spikes");
    if (n > 0) {
        std::vector<uint32_t> gid(n);
        std::vector<int64_t> stp(n);
        std::vector<double> t(n);
        HIP_TRY(hipMemcpyAsync(gid.data(), s->d_sp_gid + s->sp_user, n * 4, hipMemcpyDeviceToHost, s->st));
        HIP_TRY(hipMemcpyAsync(stp.data(), s->d_sp_step + s->sp_user, n * 8, hipMemcpyDeviceToHost, s->st));
        HIP_TRY(hipMemcpyAsync(t.data(), s->d_sp_t + s->sp_user, n * 8, hipMemcpyDeviceToHost, s->st));
        HIP_TRY(hipStreamSynchronize(s->st));
        std::vector<int64_t> idx(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = i;
        if (s->timed)  // the step field carries the time's bits: order by time
            std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
                if (t[a] != t[b]) return t[a] < t[b];
                return gid[a] < gid[b];
            });
        else
            std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
                if (stp[a] != stp[b]) return stp[a] < stp[b];
                return gid[a] < gid[b];
            });
        for (int64_t i = 0; i < n; ++i) {
            dst[i].gid = gid[idx[i]];
            dst[i].reserved = 0;
            dst[i].step = s->timed ? -1 : stp[idx[i]];
            dst[i].t_ms = t[idx[i]];
        }
    }
    *n_out = n;
    s->sp_user = have;
    // everything returned and (in a network) exchanged: start the buffer over
    const bool exchanged = s->L.cr_src.empty() || c.sp_exch == have;
    if (exchanged && have == c.sp_count && (c.flags & kFlagSpikeOverflow) == 0) {
        Counters z = c;
        z.sp_count = 0;
        z.sp_exch = 0;
        HIP_TRY(hipMemcpyAsync(s->d_ctr, &z, sizeof z, hipMemcpyHostToDevice, s->st));
        HIP_TRY(hipStreamSynchronize(s->st));
        s->sp_user = 0;
    }
    if (c.flags & (kFlagSpikeOverflow | kFlagEventOverflow))
        return fail(ARB_EOVERFLOW, (c.flags & kFlagSpikeOverflow) ? "spike buffer overflowed: spikes were lost"
                                                                  : "event buffer overflowed: events were lost");
    return ARB_OK;
}

int arb_set_probes(arb_sim s_, const int64_t* cv, int32_t n, int64_t max_steps) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s) return fail(ARB_EINVAL, "sim is NULL");
    if (n < 0 || (n > 0 && !cv) || max_steps < 0) return fail(ARB_EINVAL, "bad probe arguments");
    for (int32_t k = 0; k < n; ++k)
        if (cv[k] < 0 || cv[k] >= s->L.n_cv) return fail(ARB_EINVAL, "probe CV out of range");
    Lowered& L = s->L;
    const int np = int(L.packs.size());
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per(np);
    std::vector<int64_t> pack_of_slot_begin(np);
    for (int32_t k = 0; k < n; ++k) {
        const int64_t slot = L.perm[cv[k]];
        const int64_t pk = std::upper_bound(L.packs.begin(), L.packs.end(), slot,
                                            [](int64_t x, const PackDesc& D) { return x < D.slot0; }) -
                           L.packs.begin() - 1;
        per[pk].push_back({int32_t(slot - L.packs[pk].slot0), k});
    }
    std::vector<int32_t> ps, pid;
    for (int k = 0; k < np; ++k) {
        L.packs[k].pr0 = int32_t(ps.size());
        L.packs[k].npr = int32_t(per[k].size());
        for (auto& q : per[k]) {
            ps.push_back(q.first);
            pid.push_back(q.second);
        }
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    // the previous probe table and trace are no longer read by any kernel
    s->release(s->own_pr_slot);
    s->release(s->own_pr_id);
    s->release(s->own_trace);
    s->own_pr_slot = s->own_pr_id = nullptr;
    s->own_trace = nullptr;
    s->d_pr_slot = s->d_pr_id = nullptr;
    s->d_trace = nullptr;
    s->n_probe = 0;
    s->trace_cap = 0;
    int rc = ARB_OK;
    s->d_pr_slot = s->own_pr_slot = dupload(s, ps, rc);
    s->d_pr_id = s->own_pr_id = dupload(s, pid, rc);
    if (rc == ARB_OK) rc = s->upload(s->d_pk, L.packs.data(), L.packs.size() * sizeof(PackDesc));
    s->d_trace = s->own_trace =
        (n > 0 && max_steps > 0) ? dalloc<double>(s, size_t(n) * size_t(max_steps), rc) : nullptr;
    if (rc != ARB_OK) {
        // no probes rather than a half-made table
        for (PackDesc& D : L.packs) D.npr = 0;
        (void)s->upload(s->d_pk, L.packs.data(), L.packs.size() * sizeof(PackDesc));
        s->d_trace = nullptr;
        s->n_probe = 0;
        s->trace_cap = 0;
        s->graph_dirty = true;
        return rc;
    }
    s->n_probe = n;
    s->trace_cap = (n > 0) ? max_steps : 0;
    s->trace_step0 = s->step;
    s->graph_dirty = true;
    HIP_TRY(hipStreamSynchronize(s->st));
    return ARB_OK;
}

int arb_get_trace(arb_sim s_, double* dst, int64_t cap, int dst_on_device, int64_t* n_steps_out) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !n_steps_out) return fail(ARB_EINVAL, "null argument");
    *n_steps_out = 0;
    if (s->n_probe == 0) return ARB_OK;
    const int64_t rec = std::min(s->step - s->trace_step0, s->trace_cap);
    if (rec > cap) return fail(ARB_EOVERFLOW, "destination holds fewer steps than were recorded");
    if (rec > 0) {
        if (!dst) return fail(ARB_EINVAL, "dst is NULL");
        HIP_TRY(hipMemcpy2DAsync(dst, size_t(cap) * 8, s->d_trace, size_t(s->trace_cap) * 8, size_t(rec) * 8,
                                 size_t(s->n_probe), dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 s->st));
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    *n_steps_out = rec;
    s->trace_step0 = s->step;
    s->graph_dirty = true;
    return ARB_OK;
}

int arb_set_params(arb_sim s_, const double* theta, int64_t n) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !theta) return fail(ARB_EINVAL, "null argument");
    Lowered& L = s->L;
    if (n != 3 * int64_t(L.regions.size())) return fail(ARB_EINVAL, "theta must hold 3 values per region");
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(theta[k])) return fail(ARB_EINVAL, "theta not finite");
    for (size_t r = 0; r < L.regions.size(); ++r) {
        L.regions[r].gna = theta[3 * r + 0];
        L.regions[r].gk = theta[3 * r + 1];
        L.regions[r].gpas = theta[3 * r + 2];
    }
    recompute_coefficients(L);
    HIP_TRY(hipStreamSynchronize(s->st));
    int rc = s->upload(s->d_alpha, L.alpha.data(), L.alpha.size() * 8);
    if (rc == ARB_OK) rc = s->upload(s->d_beta, L.beta.data(), L.beta.size() * 8);
    if (rc == ARB_OK) rc = s->upload(s->d_hh_gna, L.hh_gna.data(), L.hh_gna.size() * 8);
    if (rc == ARB_OK) rc = s->upload(s->d_hh_gk, L.hh_gk.data(), L.hh_gk.size() * 8);
    if (rc == ARB_OK && s->timed) rc = s->upload(s->d_gmem, L.gmem.data(), L.gmem.size() * 8);
    if (rc != ARB_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->st));
    s->grad_valid = false;
    return ARB_OK;
}

int arb_get_state(arb_sim s_, void* blob, int64_t cap, int64_t* n_out) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !n_out) return fail(ARB_EINVAL, "null argument");
    if (s->timed) return fail(ARB_EINVAL, "state blobs are not kept for the variable time step");
    const Lowered& L = s->L;
    const StateShape sh = s->state_shape();
    int64_t bytes[kStateParts];
    void* ptr[kStateParts];
    state_part_bytes(L, sh, bytes);
    s->state_part_ptrs(ptr);
    int64_t total = sizeof(StateHeader);
    for (int k = 0; k < kStateParts; ++k) total += bytes[k];
    *n_out = total;
    if (!blob) return ARB_OK;
    if (cap < total) return fail(ARB_EOVERFLOW, "state blob capacity too small");
    const int64_t np = int64_t(L.packs.size());
    StateHeader h{kStateMagic, s->step, L.n_slots, int64_t(L.hh_cv.size()), int64_t(L.syn_global.size()),
                  np, np, s->bk_cap, s->sp_cap, s->sp_user};
    char* out = static_cast<char*>(blob);
    std::memcpy(out, &h, sizeof h);
    int64_t at = sizeof h;
    for (int k = 0; k < kStateParts; ++k) {
        if (bytes[k]) HIP_TRY(hipMemcpyAsync(out + at, ptr[k], size_t(bytes[k]), hipMemcpyDeviceToHost, s->st));
        at += bytes[k];
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    return ARB_OK;
}

int arb_set_state(arb_sim s_, const void* blob, int64_t n) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !blob) return fail(ARB_EINVAL, "null argument");
    if (s->timed) return fail(ARB_EINVAL, "state blobs are not kept for the variable time step");
    const Lowered& L = s->L;
    const StateShape sh = s->state_shape();
    // every value a kernel indexes with must lie in range before it reaches
    // the device (the blob is the caller's memory)
    const std::string bad = check_state_blob(L, sh, blob, n);
    if (!bad.empty()) return fail(ARB_EINVAL, bad);
    StateHeader h;
    std::memcpy(&h, blob, sizeof h);
    int64_t bytes[kStateParts];
    void* ptr[kStateParts];
    state_part_bytes(L, sh, bytes);
    s->state_part_ptrs(ptr);
    const char* in = static_cast<const char*>(blob);
    int64_t at = sizeof h;
    HIP_TRY(hipStreamSynchronize(s->st));
    for (int k = 0; k < kStateParts; ++k) {
        if (bytes[k]) HIP_TRY(hipMemcpyAsync(ptr[k], in + at, size_t(bytes[k]), hipMemcpyHostToDevice, s->st));
        at += bytes[k];
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    s->step = h.step;
    s->sp_user = uint32_t(h.sp_user);
    s->trace_step0 = s->step;
    s->graph_dirty = true;
    s->grad_valid = false;
    return ARB_OK;
}

int arb_get_info(arb_sim s_, arb_info* info) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !info) return fail(ARB_EINVAL, "null argument");
    const Lowered& L = s->L;
    arb_info I{};
    I.n_cells = L.n_cells;
    I.n_packs = int32_t(L.packs.size());
    I.n_cv = L.n_cv;
    I.n_slots = L.n_slots;
    I.n_hh = int64_t(L.hh_cv.size());
    I.n_syn = int64_t(L.syn_pack_index.size());  // the model's synapses (pack order may pad)
    I.n_conn = int64_t(L.cr_src.size());
    I.step = s->step;
    I.epoch_steps = s->K;
    I.block_threads = s->cfg.block_threads;
    I.coef_mode = s->cfg.coef_mode;
    I.lds_bytes = s->cfg.lds_bytes;
    I.device_bytes = s->device_bytes;
    // algorithmic bytes of one step in the SoA model: per CV V read+write,
    // c, sigma, parent index, pas conductance (44 B); per hh instance three
    // gates read+write plus a weight (56 B); per synapse g read+write plus
    // its CV index (20 B)
    I.bytes_per_step = 44 * L.n_cv + 56 * I.n_hh + 20 * I.n_syn;
    I.reg_slots = s->cfg.coef_mode == 3 ? s->cfg.reg_slots : 0;
    I.reg_len = s->cfg.coef_mode == 3 ? s->cfg.reg_len : 0;
    I.syn_hbm = s->cfg.syn_hbm;
    I.n_classes = int32_t(std::max<size_t>(1, s->classes.size()));
    *info = I;
    return ARB_OK;
}

int arb_get_kernel_time(arb_sim s_, double* ms_total, int64_t* n_launches) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !ms_total || !n_launches) return fail(ARB_EINVAL, "null argument");
    HIP_TRY(hipStreamSynchronize(s->st));
    double tot = 0.0;
    for (auto& pr : s->timer_pending) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
        s->timer_free.push_back(pr.first);
        s->timer_free.push_back(pr.second);
    }
    *ms_total = tot;
    *n_launches = int64_t(s->timer_pending.size());
    s->timer_pending.clear();
    return ARB_OK;
}

int arb_sync(arb_sim s_) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s) return fail(ARB_EINVAL, "sim is NULL");
    HIP_TRY(hipStreamSynchronize(s->st));
    bool sl = false, el = false;
    int rc = s->check_flags(sl, el);
    if (rc != ARB_OK) return rc;
    if (sl) return fail(ARB_EOVERFLOW, "spike buffer overflowed: spikes were lost");
    if (el) return fail(ARB_EOVERFLOW, "event buffer overflowed: events were lost");
    return ARB_OK;
}

int arb_free(arb_sim s_) {
    destroy_sim(static_cast<Sim*>(s_));
    return ARB_OK;
}

const char* arb_last_error(void) { return g_err.c_str(); }

int arb_grad_forward(arb_sim s_, int64_t n_steps, int32_t ckpt_every, double* trace_dev) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s) return fail(ARB_EINVAL, "sim is NULL");
    return grad_forward(s, n_steps, ckpt_every, trace_dev);
}

int arb_grad_backward(arb_sim s_, const double* dL_dtrace_dev, double* dL_dtheta_dev) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s) return fail(ARB_EINVAL, "sim is NULL");
    return grad_backward(s, dL_dtrace_dev, dL_dtheta_dev);
}

}  // extern "C"

namespace arbmi {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
int set_hip_error(hipError_t e, const char* where) { return hip_fail(e, where); }
}  // namespace arbmi
