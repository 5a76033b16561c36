// autotune.cpp -- choose the step kernel's launch shape by measurement.
//
// Candidates are (coefficient mode, threads per workgroup, cells per pack):
// register-resident coefficients for every workgroup size where the branches
// fit the registers, streamed coefficients at two pack sizes, and
// LDS-resident coefficients.  Each candidate is built for a strided sample of
// the model's cells (connections dropped, everything else kept), run for a
// few warm-up steps, then timed over a fixed number of steps with HIP events
// on the sim's stream; the fastest in CV-updates per second wins.  With the
// environment variable ARB_AUTOTUNE_CACHE naming a file, results are stored
// there keyed by the model's shape and the device, and reused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sim.hpp"

namespace arbmi {

namespace {

struct Candidate {
    int coef_mode, threads, cells_per_pack;
};

// FNV-1a over the quantities that decide the best launch shape (a sim built
// for gradients runs the recording variants and packs for the adjoint's LDS,
// so it has keys of its own)
uint64_t shape_key(const ModelView& m, const DeviceLimits& d, const arb_params& p) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
        for (int i = 0; i < 8; ++i) {
            h ^= (x >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix(uint64_t(m.n_cells));
    mix(uint64_t(m.n_br));
    mix(uint64_t(m.n_syn));
    std::vector<uint64_t> len_hist(20, 0), cv_hist(20, 0);
    for (int64_t b = 0; b < m.n_br; ++b) len_hist[std::min<int64_t>(19, m.br[b].n_cv)]++;
    for (int32_t c = 0; c < m.n_cells; ++c) {
        int64_t n = 1;
        for (int32_t b = 0; b < m.cells[c].n_branch; ++b) n += m.br[m.cells[c].branch_begin + b].n_cv;
        int lg = 0;
        while ((int64_t(1) << lg) < n && lg < 19) ++lg;
        cv_hist[lg]++;
    }
    for (uint64_t x : len_hist) mix(x);
    for (uint64_t x : cv_hist) mix(x);
    mix(uint64_t(d.n_cu));
    mix(uint64_t(d.lds_max));
    mix(uint64_t((p.flags & ARB_FLAG_GRADIENTS) ? 1 : 0));
    mix(6);  // version of the candidate set and kernels
    return h;
}

bool cache_lookup(uint64_t key, Candidate& c) {
    const char* path = std::getenv("ARB_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    unsigned long long k;
    int a, b, e;
    bool found = false;
    while (std::fscanf(f, "%llx %d %d %d", &k, &a, &b, &e) == 4)
        if (k == key) {
            c = Candidate{a, b, e};
            found = true;
        }
    std::fclose(f);
    return found;
}

void cache_store(uint64_t key, const Candidate& c) {
    const char* path = std::getenv("ARB_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%llx %d %d %d\n", (unsigned long long)key, c.coef_mode, c.threads, c.cells_per_pack);
    std::fclose(f);
}

// A strided sample of cells with their branches, synapses, input events and
// clamps (connections are dropped: the sample's timing is that of the step).
struct Sample {
    std::vector<arb_cell> cells;
    std::vector<arb_branch> br;
    std::vector<arb_synapse> syn;
    std::vector<arb_event> ev;
    std::vector<arb_iclamp> ic;
    int64_t n_cv = 0;
    ModelView view() const {
        return ModelView{cells.data(), int32_t(cells.size()), br.data(), int64_t(br.size()),
                         syn.data(), int64_t(syn.size()), nullptr, 0, ev.data(), int64_t(ev.size()),
                         ic.data(), int32_t(ic.size())};
    }
};

Sample make_sample(const ModelView& m, int32_t n_sample) {
    Sample s;
    const int32_t n = std::min(n_sample, m.n_cells);
    std::vector<int32_t> new_id(m.n_cells, -1);
    // a strided sample plus the cells with the most branches (the layouts'
    // limits bind there)
    std::vector<int32_t> pick;
    for (int32_t k = 0; k < n; ++k) pick.push_back(int32_t((int64_t(k) * m.n_cells) / n));
    std::vector<int32_t> by_size(m.n_cells);
    for (int32_t c = 0; c < m.n_cells; ++c) by_size[c] = c;
    const int32_t top = std::min<int32_t>(8, m.n_cells);
    std::partial_sort(by_size.begin(), by_size.begin() + top, by_size.end(),
                      [&](int32_t a, int32_t b) { return m.cells[a].n_branch > m.cells[b].n_branch; });
    for (int32_t k = 0; k < top; ++k) pick.push_back(by_size[k]);
    std::sort(pick.begin(), pick.end());
    pick.erase(std::unique(pick.begin(), pick.end()), pick.end());
    for (int32_t k = 0; k < int32_t(pick.size()); ++k) {
        const int32_t c = pick[k];
        new_id[c] = k;
        arb_cell C = m.cells[c];
        const int64_t b0 = int64_t(s.br.size());
        for (int32_t b = 0; b < C.n_branch; ++b) {
            s.br.push_back(m.br[C.branch_begin + b]);
            s.n_cv += m.br[C.branch_begin + b].n_cv;
        }
        s.n_cv += 1;
        C.branch_begin = b0;
        s.cells.push_back(C);
    }
    std::vector<int64_t> new_syn(m.n_syn, -1);
    for (int64_t q = 0; q < m.n_syn; ++q) {
        const int32_t c = m.syn[q].cell;
        if (c < 0 || c >= m.n_cells || new_id[c] < 0) continue;
        arb_synapse S = m.syn[q];
        S.cell = new_id[c];
        new_syn[q] = int64_t(s.syn.size());
        s.syn.push_back(S);
    }
    for (int64_t q = 0; q < m.n_ev; ++q) {
        if (int64_t(m.ev[q].syn) >= m.n_syn || new_syn[m.ev[q].syn] < 0) continue;
        arb_event E = m.ev[q];
        E.syn = uint32_t(new_syn[m.ev[q].syn]);
        s.ev.push_back(E);
    }
    for (int32_t q = 0; q < m.n_ic; ++q) {
        const int32_t c = m.ic[q].cell;
        if (c < 0 || c >= m.n_cells || new_id[c] < 0) continue;
        arb_iclamp I = m.ic[q];
        I.cell = new_id[c];
        s.ic.push_back(I);
    }
    return s;
}

// CV-updates per second of one candidate on the sample, or 0 if it fails
double time_candidate(const Sample& smp, const arb_params& base, const DeviceLimits& d, const Candidate& c) {
    arb_params p = base;
    p.flags &= ~(ARB_FLAG_AUTOTUNE | ARB_FLAG_TIME_KERNELS | ARB_FLAG_GRAPH);
    p.coef_mode = c.coef_mode;
    p.block_threads = c.threads;
    p.cells_per_pack = c.cells_per_pack;
    p.epoch_steps = 0;
    Sim* s = nullptr;
    std::string err;
    if (build_sim(smp.view(), p, d, &s, err) != ARB_OK || !s) return 0.0;
    if (s->cfg.coef_mode != c.coef_mode) {  // fell back to another mode
        destroy_sim(s);
        return 0.0;
    }
    const int warm = 10, timed = 100;
    double rate = 0.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        s->advance(warm, nullptr) == ARB_OK && hipEventRecord(e0, s->st) == hipSuccess &&
        s->advance(timed, nullptr) == ARB_OK && hipEventRecord(e1, s->st) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f)
            rate = double(smp.n_cv) * timed / (double(ms) * 1e-3);
    }
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    destroy_sim(s);
    return rate;
}

}  // namespace

arb_params autotune(const ModelView& m, const arb_params& p, const DeviceLimits& d) {
    arb_params out = p;
    const uint64_t key = shape_key(m, d, p);
    Candidate best{0, 0, 0};
    if (!cache_lookup(key, best)) {
        // enough cells for several waves of workgroups on every CU, so that
        // the last, partial wave weighs about as much as in the full model;
        // at most about 8M synapses, which bounds the trial builds' time
        const int64_t syn_per_cell = m.n_cells > 0 ? std::max<int64_t>(1, m.n_syn / m.n_cells) : 1;
        const int32_t n_sample =
            int32_t(std::max<int64_t>(64, std::min<int64_t>(int64_t(d.n_cu) * 32, 8000000 / syn_per_cell)));
        const Sample smp = make_sample(m, n_sample);
        int64_t max_width = 1;
        for (const arb_cell& C : smp.cells) {
            std::vector<int> depth(C.n_branch, 0), count(C.n_branch + 2, 0);
            for (int32_t b = 0; b < C.n_branch; ++b) {
                const arb_branch& B = smp.br[C.branch_begin + b];
                depth[b] = (B.parent < 0 || B.parent >= b) ? 1 : depth[B.parent] + 1;
                count[depth[b]]++;
            }
            for (int v : count) max_width = std::max<int64_t>(max_width, v);
        }
        const int fill256 = int(std::max<int64_t>(1, 256 / max_width));
        const std::vector<Candidate> cands = {
            {3, 256, 0}, {3, 128, 0}, {3, 64, 0}, {3, 64, 1}, {3, 128, 1},
            {2, 256, fill256}, {2, 256, std::max(1, fill256 / 2)}, {2, 128, std::max(1, fill256 / 2)},
            {2, 64, 1}, {1, 64, 1}, {1, 256, 0}};
        double best_rate = 0.0;
        for (const Candidate& c : cands) {
            const double r = time_candidate(smp, p, d, c);
            if (r > best_rate) {
                best_rate = r;
                best = c;
            }
        }
        if (best_rate > 0.0) cache_store(key, best);
    }
    if (best.coef_mode > 0) {
        out.coef_mode = best.coef_mode;
        out.block_threads = best.threads;
        out.cells_per_pack = best.cells_per_pack;
    }
    return out;
}

}  // namespace arbmi
