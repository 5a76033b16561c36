// adjoint.cpp -- gradients of a soma-trace loss by the discrete adjoint:
// a forward pass with state checkpoints every k steps, then, segment by
// segment from the last, a recompute that records every forward state and a
// reverse sweep over it (adjoint_kernels.hip).  Input events, external and
// network, are replayed exactly by the recompute (the checkpoints hold the
// event queues), so they act as fixed inputs.
#include "adjoint.hpp"

#include <algorithm>
#include <vector>

#include "adjoint_kernels.hpp"
#include "sim.hpp"

namespace arbmi {

struct GradState {
    int64_t n_steps = 0, k = 0, step_begin = 0, n_seg = 0;
    std::vector<char*> ckpt;  // state copies at segment starts, plus the end state
    int64_t state_bytes = 0;
    // two sets of segment records: the recompute of segment j - 1 fills one
    // (on the auxiliary stream) while the adjoint of segment j reads the other
    double *rec_V[2] = {}, *rec_m[2] = {}, *rec_h[2] = {}, *rec_n[2] = {}, *rec_g[2] = {};
    hipStream_t aux = nullptr;
    hipEvent_t ev_rec[2] = {}, ev_adj[2] = {}, ev_join = nullptr;
    double *lamV = nullptr, *lamM = nullptr, *lamH = nullptr, *lamN = nullptr;
    double *accP1 = nullptr, *accP0 = nullptr, *accNa = nullptr, *accK = nullptr;
    int64_t *rp_off = nullptr, *rp_slot = nullptr, *rp_hh = nullptr;
    double *rp_area = nullptr, *reg_epas = nullptr;
    uint32_t* reg_mech = nullptr;
    int32_t *pr_slot = nullptr, *pr_id = nullptr;
    int adj_lds = 0;
    bool reg = false;  // register-resident adjoint (the sim's layout is the register one)
    bool ready = false;
};

namespace {

#define HIP_TRY(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return set_hip_error(e_, #expr); \
    } while (0)

struct Part {
    void* d;
    int64_t bytes;
};

std::vector<Part> state_parts(Sim* s) {
    int64_t bytes[kStateParts];
    void* ptr[kStateParts];
    state_part_bytes(s->L, s->state_shape(), bytes);
    s->state_part_ptrs(ptr);
    std::vector<Part> out;
    for (int k = 0; k < kStateParts; ++k) out.push_back({ptr[k], bytes[k]});
    return out;
}

// The dynamic state into (save) or out of (load) a checkpoint, in one
// launch on stream st.
int copy_state(Sim* s, char* ckpt, bool save, hipStream_t st) {
    CopyList c{};
    int64_t at = 0;
    for (const Part& q : state_parts(s)) {
        if (q.bytes) {
            if (c.n == kCopyParts) return set_error(ARB_EINVAL, "internal: too many state parts");
            uint32_t* dev = static_cast<uint32_t*>(q.d);
            uint32_t* cp = reinterpret_cast<uint32_t*>(ckpt + at);
            c.src[c.n] = save ? dev : cp;
            c.dst[c.n] = save ? cp : dev;
            c.words[c.n] = q.bytes / 4;
            ++c.n;
        }
        at += (q.bytes + 255) & ~int64_t(255);
    }
    HIP_TRY(launch_copy_parts(c, st));
    return ARB_OK;
}

int save_state(Sim* s, char* dst) { return copy_state(s, dst, true, s->st); }
int load_state(Sim* s, const char* src, hipStream_t st) { return copy_state(s, const_cast<char*>(src), false, st); }

template <class T>
T* galloc(Sim* s, size_t n, int& rc) {
    if (rc != ARB_OK) return nullptr;
    T* ptr = static_cast<T*>(s->raw_alloc(std::max<size_t>(n, 1) * sizeof(T)));
    if (!ptr) rc = set_error(ARB_ENOMEM, "device allocation failed (gradient buffers)");
    return ptr;
}

// (Re)allocate the gradient buffers for n steps with checkpoints every k.
int setup(Sim* s, int64_t n, int64_t k) {
    if (!s->grad) s->grad = new GradState();
    GradState& G = *s->grad;
    const Lowered& L = s->L;
    const int64_t nhh = int64_t(L.hh_cv.size()), nsyn = int64_t(L.syn_global.size());
    const int64_t n_seg = (n + k - 1) / k;
    int rc = ARB_OK;
    if (G.state_bytes == 0) {
        for (const Part& q : state_parts(s)) G.state_bytes += (q.bytes + 255) & ~int64_t(255);
        // adjoint LDS must fit
        G.reg = s->cfg.coef_mode == 3;
        if (G.reg && !s->cfg.rec)
            return set_error(ARB_ESTATE, "gradients of a register-layout sim need ARB_FLAG_GRADIENTS at build");
        int64_t lds = 0;
        for (const PackDesc& D : L.packs) lds = std::max(lds, G.reg ? reg_adjoint_lds_bytes(D) : adjoint_lds_bytes(D));
        if (lds > s->lds_max - 256)
            return set_error(ARB_EINVAL, "packs too large for the adjoint kernel: build with ARB_FLAG_GRADIENTS");
        G.adj_lds = int(std::max<int64_t>(lds, 8));
        const hipError_t pe =
            G.reg ? prepare_reg_adjoint_kernels(int(s->lds_max)) : prepare_adjoint_kernels(int(s->lds_max));
        if (pe != hipSuccess) return set_error(ARB_EHIP, "adjoint kernels");
        G.lamV = galloc<double>(s, L.n_slots, rc);
        G.accP1 = galloc<double>(s, L.n_slots, rc);
        G.accP0 = galloc<double>(s, L.n_slots, rc);
        G.lamM = galloc<double>(s, nhh, rc);
        G.lamH = galloc<double>(s, nhh, rc);
        G.lamN = galloc<double>(s, nhh, rc);
        G.accNa = galloc<double>(s, nhh, rc);
        G.accK = galloc<double>(s, nhh, rc);
        // membrane pieces grouped by region
        const int64_t nreg = int64_t(L.regions.size());
        std::vector<int64_t> hh_of_cv(L.n_cv, -1);
        for (size_t q = 0; q < L.hh_cv.size(); ++q) hh_of_cv[L.hh_cv[q]] = int64_t(q);
        std::vector<int64_t> off(nreg + 1, 0);
        for (int32_t r : L.piece_reg) off[r + 1]++;
        for (int64_t r = 0; r < nreg; ++r) off[r + 1] += off[r];
        std::vector<int64_t> slot(off[nreg]), hh(off[nreg]);
        std::vector<double> area(off[nreg]);
        std::vector<int64_t> fill(nreg, 0);
        for (int64_t i = 0; i < L.n_cv; ++i)
            for (int64_t p = L.piece_off[i]; p < L.piece_off[i + 1]; ++p) {
                const int32_t r = L.piece_reg[p];
                const int64_t at = off[r] + fill[r]++;
                slot[at] = L.perm[i];
                hh[at] = hh_of_cv[i];
                area[at] = L.piece_area[p];
            }
        std::vector<uint32_t> mech(nreg);
        std::vector<double> epas(nreg);
        for (int64_t r = 0; r < nreg; ++r) {
            mech[r] = L.regions[r].mech;
            epas[r] = L.regions[r].epas;
        }
        G.rp_off = galloc<int64_t>(s, off.size(), rc);
        G.rp_slot = galloc<int64_t>(s, slot.size(), rc);
        G.rp_hh = galloc<int64_t>(s, hh.size(), rc);
        G.rp_area = galloc<double>(s, area.size(), rc);
        G.reg_mech = galloc<uint32_t>(s, mech.size(), rc);
        G.reg_epas = galloc<double>(s, epas.size(), rc);
        // soma probes, [pack][cell] order, id = gid
        std::vector<int32_t> ps, pid;
        for (const PackDesc& D : L.packs)
            for (int32_t c = 0; c < D.ncell; ++c) {
                ps.push_back(L.pc_soma[D.cell0 + c]);
                pid.push_back(L.pc_gid[D.cell0 + c]);
            }
        G.pr_slot = galloc<int32_t>(s, ps.size(), rc);
        G.pr_id = galloc<int32_t>(s, pid.size(), rc);
        if (rc != ARB_OK) return rc;
        if ((rc = s->upload(G.rp_off, off.data(), off.size() * 8)) != ARB_OK) return rc;
        if ((rc = s->upload(G.rp_slot, slot.data(), slot.size() * 8)) != ARB_OK) return rc;
        if ((rc = s->upload(G.rp_hh, hh.data(), hh.size() * 8)) != ARB_OK) return rc;
        if ((rc = s->upload(G.rp_area, area.data(), area.size() * 8)) != ARB_OK) return rc;
        if ((rc = s->upload(G.reg_mech, mech.data(), mech.size() * 4)) != ARB_OK) return rc;
        if ((rc = s->upload(G.reg_epas, epas.data(), epas.size() * 8)) != ARB_OK) return rc;
        if ((rc = s->upload(G.pr_slot, ps.data(), ps.size() * 4)) != ARB_OK) return rc;
        if ((rc = s->upload(G.pr_id, pid.data(), pid.size() * 4)) != ARB_OK) return rc;
    }
    if (!G.aux) {
        HIP_TRY(hipStreamCreateWithFlags(&G.aux, hipStreamNonBlocking));
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(hipEventCreateWithFlags(&G.ev_rec[b], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&G.ev_adj[b], hipEventDisableTiming));
        }
        HIP_TRY(hipEventCreateWithFlags(&G.ev_join, hipEventDisableTiming));
    }
    if (G.k != k) {
        for (int b = 0; b < 2; ++b) {
            for (double* q : {G.rec_V[b], G.rec_m[b], G.rec_h[b], G.rec_n[b], G.rec_g[b]}) s->release(q);
            G.rec_V[b] = galloc<double>(s, size_t(k + 1) * L.n_slots, rc);
            G.rec_m[b] = galloc<double>(s, size_t(k) * nhh, rc);
            G.rec_h[b] = galloc<double>(s, size_t(k) * nhh, rc);
            G.rec_n[b] = galloc<double>(s, size_t(k) * nhh, rc);
            G.rec_g[b] = galloc<double>(s, size_t(k) * nsyn, rc);
        }
        if (rc != ARB_OK) {
            G.k = 0;
            return rc;
        }
        G.k = k;
    }
    while (int64_t(G.ckpt.size()) < n_seg + 1) {
        char* c = galloc<char>(s, size_t(G.state_bytes), rc);
        if (rc != ARB_OK) return rc;
        G.ckpt.push_back(c);
    }
    G.n_steps = n;
    G.n_seg = n_seg;
    return ARB_OK;
}

}  // namespace

int grad_forward(Sim* s, int64_t n_steps, int32_t ckpt_every, double* trace_dev) {
    if (n_steps <= 0 || ckpt_every <= 0) return set_error(ARB_EINVAL, "n_steps and ckpt_every must be positive");
    if (!trace_dev) return set_error(ARB_EINVAL, "trace_dev is NULL");
    if (s->timed) return set_error(ARB_EINVAL, "the variable time step has no gradients");
    if (s->step + n_steps >= (int64_t(1) << 31)) return set_error(ARB_EINVAL, "step count beyond 2^31");
    s->grad_valid = false;
    int rc = setup(s, n_steps, std::min<int64_t>(ckpt_every, n_steps));
    if (rc != ARB_OK) return rc;
    GradState& G = *s->grad;
    Lowered& L = s->L;
    // the caller's probes (arb_set_probes) are suspended during the forward
    // and resume afterwards, recording from the step the forward ends at
    std::vector<std::pair<int32_t, int32_t>> user_pr(L.packs.size());
    for (size_t k = 0; k < L.packs.size(); ++k) user_pr[k] = {L.packs[k].pr0, L.packs[k].npr};
    int32_t* const user_slot = s->d_pr_slot;
    int32_t* const user_id = s->d_pr_id;
    double* const user_trace = s->d_trace;
    const int64_t user_np = s->n_probe, user_cap = s->trace_cap;
    auto restore_probes = [&]() -> int {
        for (size_t k = 0; k < L.packs.size(); ++k) {
            L.packs[k].pr0 = user_pr[k].first;
            L.packs[k].npr = user_pr[k].second;
        }
        s->d_pr_slot = user_slot;
        s->d_pr_id = user_id;
        s->d_trace = user_trace;
        s->n_probe = user_np;
        s->trace_cap = user_cap;
        s->trace_step0 = s->step;
        s->graph_dirty = true;
        return s->upload(s->d_pk, L.packs.data(), L.packs.size() * sizeof(PackDesc));
    };
    // probes: the soma of every cell, written straight into the caller's trace
    {
        int32_t at = 0;
        for (PackDesc& D : L.packs) {
            D.pr0 = at;
            D.npr = D.ncell;
            at += D.ncell;
        }
        if ((rc = s->upload(s->d_pk, L.packs.data(), L.packs.size() * sizeof(PackDesc))) != ARB_OK) {
            (void)restore_probes();
            return rc;
        }
        s->d_pr_slot = G.pr_slot;
        s->d_pr_id = G.pr_id;
        s->d_trace = trace_dev;
        s->n_probe = L.n_cells;
        s->trace_cap = n_steps;
        s->trace_step0 = s->step;
        s->graph_dirty = true;
    }
    G.step_begin = s->step;
    for (int64_t j = 0; j < G.n_seg && rc == ARB_OK; ++j) {
        if ((rc = save_state(s, G.ckpt[j])) != ARB_OK) break;
        const int64_t len = std::min(G.k, n_steps - j * G.k);
        rc = s->advance(len, nullptr);
    }
    if (rc == ARB_OK) rc = save_state(s, G.ckpt[G.n_seg]);
    if (rc == ARB_OK) {
        const hipError_t e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) rc = set_hip_error(e, "hipStreamSynchronize");
    }
    // the gradient trace (the caller's buffer) is not written again
    const int rc2 = restore_probes();
    if (rc != ARB_OK) return rc;
    if (rc2 != ARB_OK) return rc2;
    HIP_TRY(hipStreamSynchronize(s->st));
    G.ready = true;
    s->grad_valid = true;
    return ARB_OK;
}

int grad_backward(Sim* s, const double* dL_dtrace_dev, double* dL_dtheta_dev) {
    if (!s->grad || !s->grad_valid || !s->grad->ready)
        return set_error(ARB_ESTATE, "arb_grad_backward needs a preceding arb_grad_forward");
    if (!dL_dtrace_dev || !dL_dtheta_dev) return set_error(ARB_EINVAL, "null gradient buffer");
    GradState& G = *s->grad;
    const Lowered& L = s->L;
    const int64_t nhh = int64_t(L.hh_cv.size());
    const int64_t saved_step = s->step;
    hipStream_t const main = s->st;
    for (double* p : {G.lamV, G.accP1, G.accP0}) HIP_TRY(hipMemsetAsync(p, 0, size_t(L.n_slots) * 8, main));
    for (double* p : {G.lamM, G.lamH, G.lamN, G.accNa, G.accK})
        if (nhh) HIP_TRY(hipMemsetAsync(p, 0, size_t(nhh) * 8, main));
    // Segments from the last: the recompute of segment j (auxiliary stream)
    // restores its checkpoint and records every step into record set j % 2;
    // the adjoint of segment j (the sim's stream) waits for it and runs
    // backwards over it, while the recompute of segment j - 1 fills the
    // other set once the adjoint of segment j + 1 has finished reading it.
    // The adjoint reads only the records and the step-invariant
    // coefficients, so the recompute may change the sim's state meanwhile.
    HIP_TRY(hipEventRecord(G.ev_join, main));
    HIP_TRY(hipStreamWaitEvent(G.aux, G.ev_join, 0));
    auto recompute = [&](int64_t j) -> int {
        const int b = int(j & 1);
        s->st = G.aux;
        int rc = load_state(s, G.ckpt[j], G.aux);
        if (rc == ARB_OK) {
            s->step = G.step_begin + j * G.k;
            RecordArgs rec{G.rec_V[b], G.rec_m[b], G.rec_h[b], G.rec_n[b], G.rec_g[b]};
            rc = s->advance(std::min(G.k, G.n_steps - j * G.k), &rec);
        }
        s->st = main;
        if (rc != ARB_OK) return rc;
        HIP_TRY(hipEventRecord(G.ev_rec[b], G.aux));
        return ARB_OK;
    };
    auto join_aux = [&]() -> int {  // the sim's stream waits for the auxiliary one
        HIP_TRY(hipEventRecord(G.ev_join, G.aux));
        HIP_TRY(hipStreamWaitEvent(main, G.ev_join, 0));
        return ARB_OK;
    };
    int rc = recompute(G.n_seg - 1);
    for (int64_t j = G.n_seg - 1; j >= 0 && rc == ARB_OK; --j) {
        const int b = int(j & 1);
        const int64_t begin = G.step_begin + j * G.k;
        const int64_t len = std::min(G.k, G.n_steps - j * G.k);
        HIP_TRY(hipStreamWaitEvent(main, G.ev_rec[b], 0));
        AdjArgs a{};
        a.pk = s->d_pk;
        a.rd = s->d_rd;
        a.tk = s->d_tk;
        a.ch_slot = s->d_ch;
        a.nl = s->d_nl;
        a.pc_gid = s->d_pc_gid;
        a.pc_soma = s->d_pc_soma;
        a.alpha = s->d_alpha;
        a.F = s->d_F;
        a.invd = s->d_invd;
        a.hh_gna = s->d_hh_gna;
        a.hh_gk = s->d_hh_gk;
        a.rec_V = G.rec_V[b];
        a.rec_m = G.rec_m[b];
        a.rec_h = G.rec_h[b];
        a.rec_n = G.rec_n[b];
        a.rec_g = G.rec_g[b];
        a.n_slots_total = L.n_slots;
        a.n_hh_total = nhh;
        a.n_syn_total = int64_t(L.syn_global.size());
        a.lamV = G.lamV;
        a.lamM = G.lamM;
        a.lamH = G.lamH;
        a.lamN = G.lamN;
        a.accP1 = G.accP1;
        a.accP0 = G.accP0;
        a.accNa = G.accNa;
        a.accK = G.accK;
        a.dLdtrace = dL_dtrace_dev;
        a.trace_len = G.n_steps;
        a.trace_step0 = G.step_begin;
        a.dt = L.dt;
        a.step0 = begin;
        a.nsteps = int32_t(len);
        if (G.reg)
            HIP_TRY(launch_reg_adjoint(s->step_args(), a, s->cfg, G.adj_lds, int(L.packs.size()), main));
        else
            HIP_TRY(launch_adjoint(a, s->cfg.block_threads, G.adj_lds, int(L.packs.size()), main));
        HIP_TRY(hipEventRecord(G.ev_adj[b], main));
        if (j > 0) {
            // set (j - 1) % 2 was last read by the adjoint of segment j + 1
            if (j + 1 < G.n_seg) HIP_TRY(hipStreamWaitEvent(G.aux, G.ev_adj[(j - 1) & 1], 0));
            rc = recompute(j - 1);
        }
    }
    const int rcj = join_aux();
    if (rc != ARB_OK) return rc;
    if (rcj != ARB_OK) return rcj;
    if ((rc = load_state(s, G.ckpt[G.n_seg], main)) != ARB_OK) return rc;
    s->step = saved_step;
    GradReduceArgs r{};
    r.n_reg = int64_t(L.regions.size());
    r.rp_off = G.rp_off;
    r.rp_slot = G.rp_slot;
    r.rp_hh = G.rp_hh;
    r.rp_area = G.rp_area;
    r.reg_mech = G.reg_mech;
    r.reg_epas = G.reg_epas;
    r.accP1 = G.accP1;
    r.accP0 = G.accP0;
    r.accNa = G.accNa;
    r.accK = G.accK;
    r.out = dL_dtheta_dev;
    HIP_TRY(launch_grad_reduce(r, main));
    HIP_TRY(hipStreamSynchronize(main));
    return ARB_OK;
}

void grad_release(Sim* s) {
    if (s->grad) {
        GradState& G = *s->grad;
        if (G.aux) (void)hipStreamSynchronize(G.aux);
        for (int b = 0; b < 2; ++b) {
            if (G.ev_rec[b]) (void)hipEventDestroy(G.ev_rec[b]);
            if (G.ev_adj[b]) (void)hipEventDestroy(G.ev_adj[b]);
        }
        if (G.ev_join) (void)hipEventDestroy(G.ev_join);
        if (G.aux) (void)hipStreamDestroy(G.aux);
    }
    delete s->grad;
    s->grad = nullptr;
}

}  // namespace arbmi
