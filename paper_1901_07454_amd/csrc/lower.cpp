// lower.cpp -- validation, discretisation and packing of a model (host).
//
// Discretisation follows Sec. II of the Arbor paper (vertex-centred finite
// volumes with first-order axial flux, eq. 2a) with these choices for what
// the paper leaves open: a branch of length L split into n CVs has nodes at
// k L/n (k = 1..n) from its proximal end; node k's CV is [x_k - h/2, x_k +
// h/2] clipped to the branch, so a branch end without children is a sealed
// half-CV and the parent node owns the first half-segment; the soma is one
// isopotential node of the given area; a mechanism acts on the part of a CV's
// membrane that carries it.
//
// The implicit-Euler matrix (Sec. II) is c_i/dt on the diagonal plus the
// weighted Laplacian of the CV tree.  The membrane current is explicit in
// the scheme, so for a fixed dt the matrix never changes: its leaves-to-root
// elimination (extended Thomas / Hines) is done here once, and the kernels
// only replay the right-hand-side part of the elimination and the
// substitution every step, using
//   F_i = u_i / d'_i  (u_i = -sigma_i, d'_i the eliminated diagonal)
//   rhs'_p -= F_c rhs'_c     (elimination, children c of p)
//   x_i = rhs'_i / d'_i - F_i x_parent(i)  (substitution).
#include "lower.hpp"

#include "gen/mechanisms_desc.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <sstream>

namespace arbmi {

namespace {

const double kPi = 3.14159265358979323846;

struct CellCV {
    int ncv = 0;
    std::vector<int> parent;        // local parent, -1 at the soma
    std::vector<double> cap, sig;   // pF, nS to parent
    std::vector<int> first;         // first local CV of each branch
    std::vector<int> depth;         // per branch (soma = 0, root branch = 1)
    std::vector<int> pnode;         // per branch: local CV the branch hangs from
    // solver segments: the branches, each cut into a chain of segments of at
    // most the register layout's rows (one segment per branch otherwise);
    // the CVs and their tree are the same, the solve's tasks are segments
    std::vector<int> sfirst, slen, sparent, sdepth, spnode;  // sparent -1: the soma
    int nseg() const { return int(sfirst.size()); }
};

template <class... A>
std::string fmt(const char* f, A... a) {
    char buf[512];
    std::snprintf(buf, sizeof buf, f, a...);
    return buf;
}

// local CV index of (branch, cv) in a cell, or -1 if out of range
int64_t locate(const arb_cell& c, const arb_branch* br, const std::vector<int>& first, int32_t b,
               int32_t k) {
    if (b == -1) return k == 0 ? 0 : -1;
    if (b < -1 || b >= c.n_branch) return -1;
    if (k < 0 || k >= br[c.branch_begin + b].n_cv) return -1;
    return first[b] + k;
}

// One candidate pack: which cells, and the slot layout that results.
struct PackPlan {
    std::vector<int32_t> cells;
    int64_t nslot = 0;
    int64_t nsyn = 0, nhh = 0, nbr = 0, nic = 0, nin = 0;
    bool hhg = false;  // hh conductances and nonlinear right-hand sides in HBM
};

}  // namespace

int lower_model(const arb_cell* cells, int32_t n_cells, const arb_branch* br, int64_t n_br,
                const arb_synapse* syn, int64_t n_syn, const arb_connection* conn, int64_t n_conn,
                const arb_event* ev, int64_t n_ev, const arb_iclamp* ic, int32_t n_ic,
                const arb_params& p, const LowerOptions& opt, Lowered& L, std::string& err) {
    // ---------------------------------------------------------------- checks
    if (n_cells < 1) { err = "n_cells must be >= 1"; return ARB_EINVAL; }
    if (!cells || (n_br > 0 && !br)) { err = "null cell or branch array"; return ARB_EINVAL; }
    if (n_br < 0 || n_syn < 0 || n_conn < 0 || n_ev < 0 || n_ic < 0) { err = "negative count"; return ARB_EINVAL; }
    if ((n_syn && !syn) || (n_conn && !conn) || (n_ev && !ev) || (n_ic && !ic)) {
        err = "null array with a positive count"; return ARB_EINVAL;
    }
    if (!(p.dt_ms > 0) || !std::isfinite(p.dt_ms)) { err = "dt must be positive"; return ARB_EINVAL; }
    if (!std::isfinite(p.threshold_mV) || !std::isfinite(p.v_init_mV)) { err = "threshold/v_init not finite"; return ARB_EINVAL; }
    if (p.epoch_steps < 0) { err = "epoch_steps must be >= 0"; return ARB_EINVAL; }
    L.dt = p.dt_ms;
    L.threshold = p.threshold_mV;
    L.v_init = p.v_init_mV;
    L.n_cells = n_cells;
    const double dt = p.dt_ms;

    std::vector<CellCV> geo(n_cells);
    L.cell_cv0.assign(n_cells + 1, 0);
    L.cell_reg0.assign(n_cells + 1, 0);
    int64_t br_seen = 0;
    for (int32_t c = 0; c < n_cells; ++c) {
        const arb_cell& C = cells[c];
        if (C.n_branch < 0 || C.branch_begin < 0 || C.branch_begin + C.n_branch > n_br) {
            err = fmt("cell %d: branch range out of bounds", c); return ARB_EINVAL;
        }
        if (!(C.soma_area_um2 > 0) || !(C.cm_uF_cm2 > 0) || !(C.Ra_ohm_cm > 0) ||
            !std::isfinite(C.soma_area_um2) || !std::isfinite(C.cm_uF_cm2) || !std::isfinite(C.Ra_ohm_cm)) {
            err = fmt("cell %d: soma area, cm and Ra must be positive", c); return ARB_EINVAL;
        }
        const double sg[5] = {C.soma_gbar_na, C.soma_gbar_k, C.soma_gl_hh, C.soma_g_pas, C.soma_e_pas};
        for (double x : sg) if (!std::isfinite(x)) { err = fmt("cell %d: soma parameter not finite", c); return ARB_EINVAL; }
        if (C.soma_mech & ~(ARB_MECH_HH | ARB_MECH_PAS)) { err = fmt("cell %d: unknown soma mechanism bits", c); return ARB_EINVAL; }
        int64_t ncv = 1;
        for (int32_t b = 0; b < C.n_branch; ++b) {
            const arb_branch& B = br[C.branch_begin + b];
            if (B.parent < -1 || B.parent >= b) { err = fmt("cell %d branch %d: parent %d must be -1 or a lower index", c, b, B.parent); return ARB_EINVAL; }
            if (B.n_cv < 1) { err = fmt("cell %d branch %d: n_cv < 1", c, b); return ARB_EINVAL; }
            if (!(B.length_um > 0) || !(B.diam_um > 0) || !std::isfinite(B.length_um) || !std::isfinite(B.diam_um)) {
                err = fmt("cell %d branch %d: length and diameter must be positive", c, b); return ARB_EINVAL;
            }
            const double bg[5] = {B.gbar_na, B.gbar_k, B.gl_hh, B.g_pas, B.e_pas};
            for (double x : bg) if (!std::isfinite(x)) { err = fmt("cell %d branch %d: parameter not finite", c, b); return ARB_EINVAL; }
            if (B.mech & ~(ARB_MECH_HH | ARB_MECH_PAS)) { err = fmt("cell %d branch %d: unknown mechanism bits", c, b); return ARB_EINVAL; }
            ncv += B.n_cv;
        }
        if (ncv > (1 << 24)) { err = fmt("cell %d: too many CVs", c); return ARB_EINVAL; }
        br_seen += C.n_branch;
        L.cell_cv0[c + 1] = L.cell_cv0[c] + ncv;
        L.cell_reg0[c + 1] = L.cell_reg0[c] + 1 + C.n_branch;
    }
    (void)br_seen;
    L.n_cv = L.cell_cv0[n_cells];
    const int64_t n_reg = L.cell_reg0[n_cells];

    // ------------------------------------------------- discretisation (eq. 2a)
    L.regions.resize(n_reg);
    L.piece_off.assign(L.n_cv + 1, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> pieces(L.n_cv);
    for (int32_t c = 0; c < n_cells; ++c) {
        const arb_cell& C = cells[c];
        CellCV& G = geo[c];
        const int64_t cv0 = L.cell_cv0[c], r0 = L.cell_reg0[c];
        G.ncv = int(L.cell_cv0[c + 1] - cv0);
        G.parent.assign(G.ncv, -1);
        G.cap.assign(G.ncv, 0.0);
        G.sig.assign(G.ncv, 0.0);
        G.first.assign(C.n_branch, 0);
        G.depth.assign(C.n_branch, 0);
        G.pnode.assign(C.n_branch, 0);
        L.regions[r0] = Region{C.soma_mech, C.soma_gbar_na, C.soma_gbar_k, C.soma_gl_hh, C.soma_g_pas, C.soma_e_pas};
        pieces[cv0].push_back({int32_t(r0), C.soma_area_um2});
        int next = 1;
        for (int32_t b = 0; b < C.n_branch; ++b) { G.first[b] = next; next += br[C.branch_begin + b].n_cv; }
        for (int32_t b = 0; b < C.n_branch; ++b) {
            const arb_branch& B = br[C.branch_begin + b];
            const int32_t r = int32_t(r0 + 1 + b);
            L.regions[r] = Region{B.mech, B.gbar_na, B.gbar_k, B.gl_hh, B.g_pas, B.e_pas};
            const double h = B.length_um / B.n_cv;
            const int pn = (B.parent < 0) ? 0 : G.first[B.parent] + br[C.branch_begin + B.parent].n_cv - 1;
            G.pnode[b] = pn;
            G.depth[b] = (B.parent < 0) ? 1 : G.depth[B.parent] + 1;
            // the parent node's CV reaches h/2 into this branch
            pieces[cv0 + pn].push_back({r, kPi * B.diam_um * 0.5 * h});
            // axial conductance between consecutive nodes, cylinder of length h:
            // pi d^2 / (4 Ra h) S  ==  2.5e4 pi d^2 / (Ra h) nS  (d, h in um)
            const double sigma = 2.5e4 * kPi * B.diam_um * B.diam_um / (C.Ra_ohm_cm * h);
            for (int k = 0; k < B.n_cv; ++k) {
                const int i = G.first[b] + k;
                G.parent[i] = (k == 0) ? pn : i - 1;
                G.sig[i] = sigma;
                const double len = (k + 1 < B.n_cv) ? h : 0.5 * h;  // sealed half at the far end
                pieces[cv0 + i].push_back({r, kPi * B.diam_um * len});
            }
        }
        // solver segments, in branch order (a parent's before its children's):
        // a branch of n CVs becomes ceil(n / seg_max) segments of nearly equal
        // length, each hanging from the previous one's last CV
        const int seg_max = (opt.reg_slots > 0 && opt.reg_len > 0) ? opt.reg_len : INT32_MAX;
        std::vector<int> last_seg(C.n_branch, -1);
        for (int32_t b = 0; b < C.n_branch; ++b) {
            const arb_branch& B = br[C.branch_begin + b];
            const int parts = (B.n_cv <= seg_max) ? 1 : (B.n_cv + seg_max - 1) / seg_max;
            const int base = B.n_cv / parts, rem = B.n_cv % parts;
            int prev = (B.parent < 0) ? -1 : last_seg[B.parent];
            int off = 0;
            for (int k = 0; k < parts; ++k) {
                const int len = base + (k < rem ? 1 : 0);
                G.sfirst.push_back(G.first[b] + off);
                G.slen.push_back(len);
                G.sparent.push_back(prev);
                G.sdepth.push_back(prev < 0 ? 1 : G.sdepth[prev] + 1);
                G.spnode.push_back(k == 0 ? G.pnode[b] : G.first[b] + off - 1);
                prev = G.nseg() - 1;
                off += len;
            }
            last_seg[b] = prev;
        }
    }
    for (int64_t i = 0; i < L.n_cv; ++i) L.piece_off[i + 1] = L.piece_off[i] + int64_t(pieces[i].size());
    L.piece_reg.resize(L.piece_off[L.n_cv]);
    L.piece_area.resize(L.piece_off[L.n_cv]);
    for (int64_t i = 0; i < L.n_cv; ++i)
        for (size_t k = 0; k < pieces[i].size(); ++k) {
            L.piece_reg[L.piece_off[i] + k] = pieces[i][k].first;
            L.piece_area[L.piece_off[i] + k] = pieces[i][k].second;
        }
    pieces.clear();
    pieces.shrink_to_fit();

    std::vector<double> cap_user(L.n_cv, 0.0);
    std::vector<char> has_hh(L.n_cv, 0);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i) {
            double a = 0.0;
            for (int64_t k = L.piece_off[i]; k < L.piece_off[i + 1]; ++k) {
                a += L.piece_area[k];
                if (L.regions[L.piece_reg[k]].mech & ARB_MECH_HH) has_hh[i] = 1;
            }
            cap_user[i] = 0.01 * cells[c].cm_uF_cm2 * a;  // uF/cm^2 x um^2 -> pF
            geo[c].cap[i - L.cell_cv0[c]] = cap_user[i];
        }

    // ------------------------------------------- generated density mechanisms
    const int64_t n_den = p.n_densities;
    if (n_den < 0 || (n_den > 0 && !p.densities)) { err = "densities: bad count or NULL array"; return ARB_EINVAL; }
    std::vector<std::vector<int64_t>> den_of_reg(n_den ? n_reg : 0);
    std::map<std::vector<double>, int32_t> gen_row_of;  // (parameters, mechanism) -> parameter row
    for (int64_t q = 0; q < n_den; ++q) {
        const arb_density& D = p.densities[q];
        if (D.cell < 0 || D.cell >= n_cells || D.branch < -1 || D.branch >= cells[D.cell].n_branch) {
            err = fmt("density %lld: cell or branch out of range", (long long)q); return ARB_EINVAL;
        }
        if (D.mech < 0 || D.mech >= gen::kNumMechs) { err = fmt("density %lld: unknown mechanism", (long long)q); return ARB_EINVAL; }
        if (D.n_param < 0 || D.n_param > gen::kMechs[D.mech].n_params) {
            err = fmt("density %lld: %s takes at most %d parameters", (long long)q, gen::kMechs[D.mech].name,
                      gen::kMechs[D.mech].n_params);
            return ARB_EINVAL;
        }
        for (int32_t k = 0; k < D.n_param; ++k)
            if (!std::isfinite(D.param[k])) { err = fmt("density %lld: parameter not finite", (long long)q); return ARB_EINVAL; }
        den_of_reg[L.cell_reg0[D.cell] + 1 + D.branch].push_back(q);
    }
    if (n_den > 0) {
        if (opt.grads) { err = "generated mechanisms have no gradients"; return ARB_EINVAL; }
        if (opt.conn_delay_ms || opt.ev_t_ms) { err = "generated mechanisms do not run with the variable time step"; return ARB_EINVAL; }
        if (opt.coef_mode != 3) { err = "generated mechanisms need the register layout (coef_mode 3)"; return ARB_EINVAL; }
    }
    std::vector<char> has_gen(L.n_cv, 0);
    if (n_den > 0)
        for (int64_t i = 0; i < L.n_cv; ++i)
            for (int64_t k = L.piece_off[i]; k < L.piece_off[i + 1]; ++k)
                if (!den_of_reg[L.piece_reg[k]].empty()) has_gen[i] = 1;

    // ------------------------------------------------ synapses, clamps, events
    std::vector<int64_t> syn_cv(n_syn);
    for (int64_t q = 0; q < n_syn; ++q) {
        const arb_synapse& S = syn[q];
        if (S.cell < 0 || S.cell >= n_cells) { err = fmt("synapse %lld: cell out of range", (long long)q); return ARB_EINVAL; }
        int64_t i = locate(cells[S.cell], br, geo[S.cell].first, S.branch, S.cv);
        if (i < 0) { err = fmt("synapse %lld: branch/cv out of range", (long long)q); return ARB_EINVAL; }
        if (!(S.tau_ms > 0) || !std::isfinite(S.tau_ms) || !std::isfinite(S.e_rev_mV)) {
            err = fmt("synapse %lld: tau must be positive", (long long)q); return ARB_EINVAL;
        }
        syn_cv[q] = L.cell_cv0[S.cell] + i;
    }
    std::vector<int64_t> ic_cv(n_ic);
    for (int32_t q = 0; q < n_ic; ++q) {
        const arb_iclamp& I = ic[q];
        if (I.cell < 0 || I.cell >= n_cells) { err = fmt("clamp %d: cell out of range", q); return ARB_EINVAL; }
        int64_t i = locate(cells[I.cell], br, geo[I.cell].first, I.branch, I.cv);
        if (i < 0) { err = fmt("clamp %d: branch/cv out of range", q); return ARB_EINVAL; }
        if (!std::isfinite(I.amp_nA)) { err = fmt("clamp %d: amplitude not finite", q); return ARB_EINVAL; }
        ic_cv[q] = L.cell_cv0[I.cell] + i;
    }
    for (int64_t q = 0; q < n_ev; ++q) {
        if (int64_t(ev[q].syn) >= n_syn) { err = fmt("event %lld: synapse out of range", (long long)q); return ARB_EINVAL; }
        if (ev[q].step < 0 || ev[q].step >= (int64_t(1) << 31)) { err = fmt("event %lld: step out of range", (long long)q); return ARB_EINVAL; }
        if (!std::isfinite(ev[q].w_uS)) { err = fmt("event %lld: weight not finite", (long long)q); return ARB_EINVAL; }
    }
    if (p.dry_run_ranks < 0 || p.dry_run_ranks > (1 << 20) ||
        int64_t(std::max(1, p.dry_run_ranks)) * n_cells >= (int64_t(1) << 31)) {
        err = "dry_run_ranks out of range (at most 2^20, and ranks x cells below 2^31)";
        return ARB_EINVAL;
    }
    L.dry_run_ranks = std::max(1, p.dry_run_ranks);
    L.n_src = int64_t(L.dry_run_ranks) * n_cells;
    L.min_delay = 0;
    L.max_delay = 0;
    for (int64_t q = 0; q < n_conn; ++q) {
        const arb_connection& K = conn[q];
        if (int64_t(K.src) >= L.n_src || K.dst >= uint32_t(n_cells)) { err = fmt("connection %lld: cell out of range", (long long)q); return ARB_EINVAL; }
        if (int64_t(K.syn) >= n_syn || syn[K.syn].cell != int32_t(K.dst)) {
            err = fmt("connection %lld: synapse not on the destination cell", (long long)q); return ARB_EINVAL;
        }
        if (K.delay_steps < 1) { err = fmt("connection %lld: delay_steps must be >= 1", (long long)q); return ARB_EINVAL; }
        if (!std::isfinite(K.w_uS)) { err = fmt("connection %lld: weight not finite", (long long)q); return ARB_EINVAL; }
        L.min_delay = q == 0 ? K.delay_steps : std::min(L.min_delay, K.delay_steps);
        L.max_delay = std::max(L.max_delay, K.delay_steps);
    }
    L.timed = opt.conn_delay_ms != nullptr || opt.ev_t_ms != nullptr;
    if (L.timed) {
        // the variable step runs one cell per workgroup in the register
        // layout; clamps, gradients and the dry run are fixed-step features
        if (n_ic > 0) { err = "the variable time step takes no current clamps"; return ARB_EINVAL; }
        if (opt.grads) { err = "the variable time step has no gradients"; return ARB_EINVAL; }
        if (p.dry_run_ranks > 1) { err = "the variable time step has no dry-run mode"; return ARB_EINVAL; }
        if (opt.coef_mode != 3 || opt.max_cells_per_pack != 1) {
            err = "the variable time step needs the register layout with one cell per pack"; return ARB_EINVAL;
        }
        if ((n_ev && !opt.ev_t_ms) || (n_conn && !opt.conn_delay_ms)) { err = "missing event times or delays"; return ARB_EINVAL; }
        // continuous times: an epoch of K grid steps must end before any
        // event of its spikes can arrive (K dt <= the minimum delay)
        for (int64_t q = 0; q < n_ev; ++q)
            if (!(opt.ev_t_ms[q] >= 0.0) || !(opt.ev_t_ms[q] < double(int64_t(1) << 31) * dt)) {
                err = fmt("event %lld: time out of range", (long long)q); return ARB_EINVAL;
            }
        for (int64_t q = 0; q < n_conn; ++q) {
            const double dm = opt.conn_delay_ms[q];
            if (!(dm >= dt) || !std::isfinite(dm)) { err = fmt("connection %lld: delay_ms must be at least dt", (long long)q); return ARB_EINVAL; }
            L.min_delay_ms = q == 0 ? dm : std::min(L.min_delay_ms, dm);
            L.max_delay_ms = std::max(L.max_delay_ms, dm);
        }
        if (n_conn) {
            int64_t k = int64_t(L.min_delay_ms / dt);
            while (double(k + 1) * dt <= L.min_delay_ms) ++k;
            while (k > 1 && double(k) * dt > L.min_delay_ms) --k;
            L.min_delay = int32_t(std::min<int64_t>(k, INT32_MAX));
            L.max_delay = int32_t(std::min<double>(std::ceil(L.max_delay_ms / dt) + 1.0, double(INT32_MAX)));
        }
    }
    if (n_conn && p.epoch_steps > L.min_delay) {
        err = fmt("epoch_steps %d exceeds the minimum delay %d", p.epoch_steps, L.min_delay); return ARB_EINVAL;
    }

    // per-CV markers for the nonlinear list
    std::vector<int32_t> nsyn_cv(L.n_cv, 0), nic_cv(L.n_cv, 0);
    for (int64_t q = 0; q < n_syn; ++q) nsyn_cv[syn_cv[q]]++;
    for (int32_t q = 0; q < n_ic; ++q) nic_cv[ic_cv[q]]++;
    std::vector<int32_t> nhh_cell(n_cells, 0), nsyn_cell(n_cells, 0), nic_cell(n_cells, 0);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i) {
            nhh_cell[c] += has_hh[i];
            nsyn_cell[c] += nsyn_cv[i];
            nic_cell[c] += nic_cv[i];
        }
    std::vector<int64_t> nin_cell(n_cells, 0);  // incoming connections
    for (int64_t q = 0; q < n_conn; ++q) nin_cell[conn[q].dst]++;

    // -------------------------------------------------------------- packing
    const int T = opt.block_threads;
    L.block_threads = T;
    // Rounds of a set of cells: the branches of one depth level (deepest
    // first; the soma is level 0) split into rounds of at most T.  In the
    // register-resident layout (S > 0) every thread has S register slots and
    // each round takes one slot index j on a contiguous run of threads that
    // have not used slot j yet; it fails when the slots run out or a branch
    // is longer than the registers hold.
    struct Item { int32_t c, b; int len; };
    struct RoundPlan { std::vector<Item> items; int t0 = 0, j = 0, len = 0; };
    const int S = opt.reg_slots;
    auto build_rounds = [&](const std::vector<int32_t>& cs, std::vector<RoundPlan>& out) -> bool {
        out.clear();
        int maxd = 0;
        for (int32_t c : cs) for (int d : geo[c].sdepth) maxd = std::max(maxd, d);
        // The items of each level in top-down order: the somas in cell order,
        // then at each deeper level every parent's first child in the order
        // of the parents, then every second child, and so on.  Consecutive
        // threads of a round then read consecutive entries for their
        // children and grandchildren in the tree passes (no LDS bank
        // conflicts in a full binary tree); the arithmetic of every branch
        // is the same in any order.
        std::vector<std::vector<Item>> lev(maxd + 1);
        {
            std::vector<std::vector<int32_t>> pos(cs.size()), rank(cs.size());
            for (size_t ci = 0; ci < cs.size(); ++ci) {
                const auto& G = geo[cs[ci]];
                lev[0].push_back({cs[ci], -1, 1});
                pos[ci].assign(G.nseg(), -1);
                rank[ci].assign(G.nseg(), 0);
                std::vector<int32_t> seen(G.nseg() + 1, 0);  // [0] = soma, [b + 1] = segment b
                for (int32_t b = 0; b < G.nseg(); ++b) rank[ci][b] = seen[G.sparent[b] + 1]++;
            }
            struct Key { int32_t k; int64_t ppos; size_t ci; int32_t b; };
            std::vector<Key> keys;
            for (int d = 1; d <= maxd; ++d) {
                keys.clear();
                for (size_t ci = 0; ci < cs.size(); ++ci) {
                    const auto& G = geo[cs[ci]];
                    for (int32_t b = 0; b < G.nseg(); ++b)
                        if (G.sdepth[b] == d) {
                            const int32_t p = G.sparent[b];
                            keys.push_back({rank[ci][b], p < 0 ? int64_t(ci) : int64_t(pos[ci][p]), ci, b});
                        }
                }
                std::sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
                    return x.k != y.k ? x.k < y.k : x.ppos < y.ppos;
                });
                for (size_t i = 0; i < keys.size(); ++i) {
                    pos[keys[i].ci][keys[i].b] = int32_t(i);
                    lev[d].push_back({cs[keys[i].ci], keys[i].b, geo[cs[keys[i].ci]].slen[keys[i].b]});
                }
            }
        }
        std::vector<int> next_free(std::max(S, 1), 0);
        for (int d = maxd; d >= 0; --d) {
            const std::vector<Item>& items = lev[d];
            size_t s0 = 0;
            while (s0 < items.size()) {
                int jb = 0;
                size_t room = size_t(T);
                if (S > 0) {
                    // the first slot that takes the rest of the level whole,
                    // else the one with the most free threads: few slots in
                    // use let the kernel keep fewer registers
                    jb = -1;
                    const size_t rest = items.size() - s0;
                    for (int j = 0; j < S && jb < 0; ++j)
                        if (size_t(T - next_free[j]) >= rest) jb = j;
                    if (jb < 0) {
                        int best = 0;
                        for (int j = 0; j < S; ++j)
                            if (T - next_free[j] > best) { best = T - next_free[j]; jb = j; }
                    }
                    if (jb < 0) return false;
                    room = size_t(T - next_free[jb]);
                }
                const size_t m = std::min(items.size() - s0, room);
                RoundPlan rp;
                rp.items.assign(items.begin() + s0, items.begin() + s0 + m);
                rp.t0 = (S > 0) ? next_free[jb] : 0;
                rp.j = jb;
                for (const Item& it : rp.items) rp.len = std::max(rp.len, it.len);
                if (S > 0) {
                    if (rp.len > opt.reg_len) return false;
                    next_free[jb] += int(m);
                }
                out.push_back(std::move(rp));
                s0 += m;
            }
        }
        return true;
    };
    // most children of any task (soma or segment) of each cell
    std::vector<int32_t> max_children(n_cells, 0);
    for (int32_t c = 0; c < n_cells; ++c) {
        std::vector<int32_t> nch(geo[c].nseg() + 1, 0);  // [0] = soma, [b + 1] = segment b
        for (int32_t b = 0; b < geo[c].nseg(); ++b) nch[geo[c].sparent[b] + 1]++;
        for (int32_t v : nch) max_children[c] = std::max(max_children[c], v);
    }
    struct Shape { int64_t nslot = 0, nrd = 0; bool ok = true, has_pad = false; int slots = 1; };
    auto plan_shape = [&](const std::vector<int32_t>& cs) -> Shape {
        std::vector<RoundPlan> rps;
        Shape sh;
        sh.ok = build_rounds(cs, rps);
        for (const RoundPlan& rp : rps) {
            sh.nslot += int64_t(S > 0 ? opt.reg_len : rp.len) * int64_t(rp.items.size());
            for (const Item& it : rp.items) sh.has_pad = sh.has_pad || (S > 0 && it.len < opt.reg_len);
            sh.slots = std::max(sh.slots, rp.j + 1);
        }
        sh.nrd = int64_t(rps.size());
        return sh;
    };
    // CVs carrying hh or synapses, per cell
    std::vector<int32_t> nnl_cell(n_cells, 0);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i)
            nnl_cell[c] += (has_hh[i] || nsyn_cv[i] || nic_cv[i] || has_gen[i]) ? 1 : 0;
    auto exact_lds = [&](const PackPlan& pp, int mode) -> int64_t {
        const Shape sh = plan_shape(pp.cells);
        if (!sh.ok) return int64_t(1) << 40;  // does not fit the register slots
        PackDesc D{};
        D.nslot = int32_t(sh.nslot);
        D.spare = sh.has_pad ? 0 : D.nslot;
        D.binary = 1;
        for (int32_t c : pp.cells) D.binary = D.binary && max_children[c] <= 2;
        D.syn_global = (S > 0 && 24 * pp.nsyn > kSynLdsMax) ? 1 : 0;
        D.nrd = int32_t(sh.nrd);
        D.ntk = int32_t(pp.nbr + int64_t(pp.cells.size()));
        D.nch = int32_t(pp.nbr);
        D.nsyn = int32_t(pp.nsyn);
        D.nhh = int32_t(pp.nhh);
        int64_t nnl = 0;
        for (int32_t c : pp.cells) nnl += nnl_cell[c];
        D.nnl = int32_t(nnl);
        D.hh_global = pp.hhg ? 1 : 0;
        if (opt.grads && mode == 3) {
            // the adjoint reads the synapses' recorded conductances from LDS
            if (D.syn_global) return int64_t(1) << 40;
            return std::max(pack_lds_bytes(D, mode), reg_adjoint_lds_bytes(D));
        }
        return pack_lds_bytes(D, mode);
    };
    std::vector<int32_t> order(n_cells);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return geo[a].ncv > geo[b].ncv; });
    const int64_t max_cells = std::max<int64_t>(1, std::min<int64_t>(T, opt.max_cells_per_pack));
    std::vector<PackPlan> plans;
    int coef_mode = opt.coef_mode;
    {
        PackPlan cur;
        for (int32_t c : order) {
            PackPlan trial = cur;
            trial.cells.push_back(c);
            trial.nsyn += nsyn_cell[c];
            trial.nhh += nhh_cell[c];
            trial.nbr += geo[c].nseg();
            trial.nic += nic_cell[c];
            trial.nin += nin_cell[c];
            // a cell alone always makes a pack
            bool fits = cur.cells.empty() || (int64_t(trial.cells.size()) <= max_cells && trial.nin <= kPackInMax);
            if (fits && !cur.cells.empty()) fits = exact_lds(trial, coef_mode) <= opt.lds_budget;
            if (!fits) {
                if (!cur.cells.empty()) plans.push_back(cur);
                cur = PackPlan();
                cur.cells.push_back(c);
                cur.nsyn = nsyn_cell[c];
                cur.nhh = nhh_cell[c];
                cur.nbr = geo[c].nseg();
                cur.nic = nic_cell[c];
                cur.nin = nin_cell[c];
            } else {
                cur = trial;
            }
            // a cell too large for the register layout's LDS alone keeps its
            // hh conductances and nonlinear right-hand sides in HBM
            if (cur.cells.size() == 1 && S > 0 && !opt.grads && !L.timed && coef_mode == 3 &&
                exact_lds(cur, coef_mode) > opt.lds_hard_max) {
                cur.hhg = true;
                if (exact_lds(cur, coef_mode) > opt.lds_hard_max) cur.hhg = false;
            }
        }
        if (!cur.cells.empty()) plans.push_back(cur);
    }
    if (S > 1) {
        // Packs that need the same kernel variant (register slots in use,
        // state in HBM) next to each other, most slots first, each group
        // largest LDS first: the host launches each run of them as one class
        // with the registers and LDS it needs.
        struct Key { int slots, hbm; int64_t lds; };
        std::vector<Key> key(plans.size());
        for (size_t k = 0; k < plans.size(); ++k) {
            const Shape sh = plan_shape(plans[k].cells);
            key[k] = Key{sh.slots, (plans[k].hhg || 24 * plans[k].nsyn > kSynLdsMax) ? 1 : 0,
                         exact_lds(plans[k], coef_mode)};
        }
        std::vector<size_t> idx(plans.size());
        std::iota(idx.begin(), idx.end(), size_t(0));
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
            if (key[a].slots != key[b].slots) return key[a].slots > key[b].slots;
            if (key[a].hbm != key[b].hbm) return key[a].hbm > key[b].hbm;
            return key[a].lds > key[b].lds;
        });
        std::vector<PackPlan> sorted;
        sorted.reserve(plans.size());
        for (size_t k : idx) sorted.push_back(std::move(plans[k]));
        plans.swap(sorted);
    }
    for (const PackPlan& pp : plans)
        if (S > 0 && !plan_shape(pp.cells).ok) {
            err = "a cell does not fit the register-resident layout";
            return ARB_EINVAL;
        }
    for (const PackPlan& pp : plans)
        if (exact_lds(pp, coef_mode) > opt.lds_hard_max) {
            err = fmt("a cell needs %lld bytes of LDS, more than the %lld available",
                      (long long)exact_lds(pp, coef_mode), (long long)opt.lds_hard_max);
            return ARB_EINVAL;
        }
    L.coef_mode = coef_mode;
    L.reg_slots = opt.reg_slots;
    L.reg_len = opt.reg_slots > 0 ? opt.reg_len : 0;

    // ------------------------------------------------- slot layout per pack
    const int64_t n_packs = int64_t(plans.size());
    L.packs.resize(n_packs);
    L.perm.assign(L.n_cv, -1);
    std::vector<int64_t> pack_of_cell(n_cells), slot_of_user(L.n_cv, -1);
    int64_t slot_base = 0;
    for (int64_t pk = 0; pk < n_packs; ++pk) {
        const PackPlan& pp = plans[pk];
        PackDesc& D = L.packs[pk];
        D = PackDesc{};
        D.slot0 = slot_base;
        D.rd0 = int32_t(L.rounds.size());
        D.cell0 = int32_t(L.pc_gid.size());
        D.ncell = int32_t(pp.cells.size());
        int maxd = 0;
        for (int32_t c : pp.cells) {
            pack_of_cell[c] = pk;
            for (int d : geo[c].sdepth) maxd = std::max(maxd, d);
        }
        // rounds, deepest first; a task is (cell, branch) with branch -1 = soma
        std::vector<RoundPlan> rps;
        if (!build_rounds(pp.cells, rps)) { err = "a cell does not fit the register-resident layout"; return ARB_EINVAL; }
        int64_t ns = 0;
        std::vector<RoundDesc> rds;
        for (const RoundPlan& rp : rps) {
            const std::vector<Item>& ri = rp.items;
            RoundDesc R{int32_t(ns), int32_t(ri.size()), rp.len, 0, rp.t0, rp.j};
            // slots of every CV of the round
            for (size_t t = 0; t < ri.size(); ++t) {
                const Item& it = ri[t];
                const int64_t cv0 = L.cell_cv0[it.c];
                if (it.b < 0) {
                    slot_of_user[cv0] = slot_base + ns + int64_t(t);
                } else {
                    for (int k = 0; k < it.len; ++k)
                        slot_of_user[cv0 + geo[it.c].sfirst[it.b] + k] = slot_base + ns + int64_t(k) * int64_t(ri.size()) + int64_t(t);
                }
            }
            // the register-resident kernel gives every branch reg_len rows: a
            // shorter branch's spare rows take its pad CVs
            ns += int64_t(S > 0 ? opt.reg_len : rp.len) * int64_t(ri.size());
            rds.push_back(R);
        }
        D.nslot = int32_t(ns);
        D.nrd = int32_t(rds.size());
        D.nlev = maxd + 1;
        D.binary = 1;
        for (int32_t c : pp.cells) D.binary = D.binary && max_children[c] <= 2;
        D.syn_global = (S > 0 && 24 * pp.nsyn > kSynLdsMax) ? 1 : 0;
        D.hh_global = pp.hhg ? 1 : 0;
        if (L.timed && D.syn_global) {
            err = "the variable time step keeps every synapse in LDS: a cell has too many synapses";
            return ARB_EINVAL;
        }
        // the register-resident kernel's empty slots write to a slot no CV
        // uses: the first pad row if there is one, else one past the end
        D.spare = D.nslot;
        if (S > 0) {
            int64_t at = 0;
            for (const RoundPlan& rp : rps) {
                const int64_t w = int64_t(rp.items.size());
                for (int64_t t = 0; t < w && D.spare == D.nslot; ++t)
                    if (rp.items[t].len < opt.reg_len) D.spare = int32_t(at + int64_t(rp.items[t].len) * w + t);
                at += int64_t(opt.reg_len) * w;
            }
        }
        D.tk0 = int32_t(L.tasks.size());
        D.ch0 = int32_t(L.ch_slot.size());
        // tasks (need every slot assigned first, for parents and children).
        // Rounds run deepest first, so a task's children already have their
        // pack-local task index when the task is made; parents get theirs in
        // a second pass.
        std::map<std::pair<int32_t, int32_t>, int32_t> task_of;  // (cell, branch) -> pack-local task
        std::vector<std::pair<int32_t, int32_t>> item_of;        // pack-local task -> (cell, branch)
        for (size_t r = 0; r < rds.size(); ++r) {
            rds[r].task0 = int32_t(L.tasks.size()) - D.tk0;  // pack-local task
            for (const Item& it : rps[r].items) {
                const int64_t cv0 = L.cell_cv0[it.c];
                TaskDesc T_{};
                T_.len = it.len;
                T_.par = (it.b < 0) ? -1 : int32_t(slot_of_user[cv0 + geo[it.c].spnode[it.b]] - slot_base);
                T_.ch0 = int32_t(L.ch_slot.size()) - D.ch0;  // pack-local child entry
                T_.nch = 0;
                for (int32_t b2 = 0; b2 < geo[it.c].nseg(); ++b2)
                    if (geo[it.c].sparent[b2] == it.b) {
                        L.ch_slot.push_back(int32_t(slot_of_user[cv0 + geo[it.c].sfirst[b2]] - slot_base));
                        L.ch_task.push_back(task_of.at({it.c, b2}));
                        T_.nch++;
                    }
                task_of[{it.c, it.b}] = int32_t(L.tasks.size()) - D.tk0;
                item_of.push_back({it.c, it.b});
                L.tasks.push_back(T_);
            }
            L.rounds.push_back(rds[r]);
        }
        for (const auto& cb : item_of) {
            const int32_t b = cb.second;
            const int32_t pb = (b < 0) ? -2 : geo[cb.first].sparent[b];
            L.tk_ptask.push_back(pb == -2 ? -1 : task_of.at({cb.first, pb}));
            L.tk_lev.push_back(b < 0 ? 0 : geo[cb.first].sdepth[b]);
        }
        D.ntk = int32_t(L.tasks.size()) - D.tk0;
        D.nch = int32_t(L.ch_slot.size()) - D.ch0;
        for (int32_t c : pp.cells) {
            L.pc_gid.push_back(c);
            L.pc_soma.push_back(int32_t(slot_of_user[L.cell_cv0[c]] - slot_base));
        }
        slot_base += ns;
    }
    L.n_slots = slot_base;
    L.perm = slot_of_user;
    L.slot_cell.assign(L.n_slots, -1);
    for (int32_t c = 0; c < n_cells; ++c)
        for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i) L.slot_cell[L.perm[i]] = c;

    // --------------------------------------- coefficients and factorisation
    L.cap.assign(L.n_slots, 0.0);
    L.alpha.assign(L.n_slots, 0.0);
    L.beta.assign(L.n_slots, 0.0);
    L.F.assign(L.n_slots, 0.0);
    L.invd.assign(L.n_slots, 0.0);
    L.d_elim.assign(L.n_slots, 0.0);
    L.sigsum.assign(L.n_slots, 0.0);
    L.uoff.assign(L.n_slots, 0.0);
    for (int32_t c = 0; c < n_cells; ++c) {
        const CellCV& G = geo[c];
        const int64_t cv0 = L.cell_cv0[c];
        std::vector<double> d(G.ncv);
        std::vector<double> ss(G.ncv, 0.0);
        for (int i = 1; i < G.ncv; ++i) { ss[i] += G.sig[i]; ss[G.parent[i]] += G.sig[i]; }
        for (int i = 0; i < G.ncv; ++i) d[i] = G.cap[i] / dt;
        for (int i = 1; i < G.ncv; ++i) { d[i] += G.sig[i]; d[G.parent[i]] += G.sig[i]; }
        std::vector<double> Fl(G.ncv, 0.0);
        for (int i = G.ncv - 1; i >= 1; --i) {
            const double u = -G.sig[i];
            Fl[i] = u / d[i];
            d[G.parent[i]] -= Fl[i] * u;
        }
        for (int i = 0; i < G.ncv; ++i) {
            const int64_t s = L.perm[cv0 + i];
            L.cap[s] = G.cap[i];
            L.sigsum[s] = ss[i];
            L.uoff[s] = (i == 0) ? 0.0 : -G.sig[i];
            L.F[s] = Fl[i];
            L.d_elim[s] = d[i];
            L.invd[s] = 1.0 / d[i];
        }
    }
    // per task: Z = prod_k (-F_k) over its CVs, proximal to distal
    L.tk_Z.assign(L.tasks.size(), 1.0);
    for (const PackDesc& D : L.packs)
        for (int32_t r = 0; r < D.nrd; ++r) {
            const RoundDesc& R = L.rounds[D.rd0 + r];
            for (int32_t i = 0; i < R.w; ++i) {
                const int64_t t = int64_t(D.tk0) + R.task0 + i;
                double z = 1.0;
                for (int32_t k = 0; k < L.tasks[t].len; ++k) z *= -L.F[D.slot0 + R.slot0 + int64_t(k) * R.w + i];
                L.tk_Z[t] = z;
            }
        }

    // ------------------------------------------- nonlinear CVs per pack
    std::vector<std::vector<int64_t>> syn_at(L.n_cv), ic_at(L.n_cv);
    for (int64_t q = 0; q < n_syn; ++q) syn_at[syn_cv[q]].push_back(q);
    for (int32_t q = 0; q < n_ic; ++q) ic_at[ic_cv[q]].push_back(q);
    L.syn_pack_index.assign(n_syn, -1);
    for (int64_t pk = 0; pk < n_packs; ++pk) {
        PackDesc& D = L.packs[pk];
        D.nl0 = int32_t(L.nl.size());
        D.hh0 = int32_t(L.hh_cv.size());
        D.syn0 = int32_t(L.syn_global.size());
        D.ic0 = int32_t(L.ic_on.size());
        std::vector<std::pair<int64_t, int64_t>> here;  // (slot, user cv)
        for (int32_t k = 0; k < D.ncell; ++k) {
            const int32_t c = L.pc_gid[D.cell0 + k];
            for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i)
                if (has_hh[i] || nsyn_cv[i] || nic_cv[i] || has_gen[i]) here.push_back({L.perm[i], i});
        }
        std::sort(here.begin(), here.end());
        if (D.syn_global)  // CVs with similar synapse counts share a group: little padding
            std::stable_sort(here.begin(), here.end(), [&](const std::pair<int64_t, int64_t>& a,
                                                           const std::pair<int64_t, int64_t>& b) {
                return syn_at[a.second].size() > syn_at[b.second].size();
            });
        const size_t nl_first = L.nl.size();
        if (n_den > 0) L.gen_pk.push_back(int32_t(L.gen_mech.size()));
        // (the instances' states are gathered instance-major in gen_st0 and
        // made state-major after the last pack)
        for (auto& sc : here) {
            const int64_t i = sc.second;
            NlDesc N{};
            N.slot = int32_t(sc.first - D.slot0);
            N.hh = -1;
            if (has_hh[i]) { N.hh = int32_t(L.hh_cv.size()) - D.hh0; L.hh_cv.push_back(i); }
            N.nsyn = int32_t(syn_at[i].size());
            L.nl.push_back(N);
            if (n_den > 0) {  // this CV's instances: its pieces in order, each region's entries in order
                L.gen_off.push_back(int32_t(L.gen_mech.size()));
                for (int64_t k = L.piece_off[i]; k < L.piece_off[i + 1]; ++k)
                    for (int64_t q : den_of_reg[L.piece_reg[k]]) {
                        const arb_density& E = p.densities[q];
                        const gen::MechDesc& M = gen::kMechs[E.mech];
                        double prm[gen::kMaxParams] = {}, st[gen::kMaxStates] = {};
                        for (int32_t j = 0; j < M.n_params; ++j) prm[j] = (j < E.n_param) ? E.param[j] : M.defaults[j];
                        gen::steady(E.mech, L.v_init, prm, st);
                        std::vector<double> key(prm, prm + gen::kMaxParams);
                        key.push_back(double(E.mech));
                        auto row = gen_row_of.find(key);
                        if (row == gen_row_of.end()) {
                            static_assert(gen::kNumMechs <= 127, "a catalogue index fits the row word's high bits");
                            if (L.gen_rmech.size() >= (size_t(1) << 24)) {
                                err = "more than 2^24 distinct generated-mechanism parameter sets";
                                return ARB_EINVAL;
                            }
                            row = gen_row_of.emplace(key, int32_t(L.gen_rmech.size())).first;
                            L.gen_rmech.push_back(E.mech);
                            L.gen_prm.insert(L.gen_prm.end(), prm, prm + gen::kMaxParams);
                        }
                        L.gen_mech.push_back(E.mech);
                        L.gen_row.push_back(row->second | (E.mech << 24));  // the mechanism rides along
                        L.gen_slot.push_back(N.slot);
                        L.gen_w.push_back(10.0 * L.piece_area[k]);  // S/cm^2 x um^2 -> nS
                        L.gen_st0.insert(L.gen_st0.end(), st, st + gen::kMaxStates);
                    }
            }
        }
        // Synapses in pack order.  In LDS they are contiguous per CV.  A pack
        // that keeps them in HBM interleaves them over the threads that take
        // the CVs (thread t takes nonlinear entries t, t + T, ...): synapse k
        // of entry u T + t sits at group base + k w + t, w the group's
        // entries, so a wave's loads of one k are consecutive; shorter CVs
        // are padded with zero entries.
        auto put = [&](int64_t pos, int64_t q) {
            L.syn_pack_index[q] = pos;
            L.syn_global[pos] = q;
            L.syn_e[pos] = syn[q].e_rev_mV;
            L.syn_decay[pos] = std::exp(-dt / syn[q].tau_ms);
            L.syn_tau[pos] = syn[q].tau_ms;
        };
        const int64_t nhere = int64_t(here.size());
        const int64_t group = D.syn_global ? int64_t(T) : 1;
        for (int64_t u0 = 0; u0 < nhere; u0 += group) {
            const int64_t w = std::min(group, nhere - u0);
            int64_t mx = 0;
            for (int64_t t = 0; t < w; ++t) mx = std::max<int64_t>(mx, L.nl[nl_first + u0 + t].nsyn);
            const int64_t base = int64_t(L.syn_global.size());
            const int64_t len = D.syn_global ? mx * w : L.nl[nl_first + u0].nsyn;
            L.syn_global.resize(base + len, -1);
            L.syn_e.resize(base + len, 0.0);
            L.syn_decay.resize(base + len, 0.0);
            L.syn_tau.resize(base + len, 1.0);
            for (int64_t t = 0; t < w; ++t) {
                NlDesc& N = L.nl[nl_first + u0 + t];
                N.syn0 = int32_t(base + t - D.syn0);
                const std::vector<int64_t>& qs = syn_at[here[u0 + t].second];
                for (size_t k = 0; k < qs.size(); ++k) put(base + int64_t(k) * w + t, qs[k]);
            }
        }
        // one e_syn and decay for the whole pack, if its synapses share them
        D.syn_uniform = 0;
        D.syn_e = 0.0;
        D.syn_decay = 0.0;
        {
            bool first = true, same = true;
            for (int64_t pos = D.syn0; pos < int64_t(L.syn_global.size()) && same; ++pos) {
                if (L.syn_global[pos] < 0) continue;
                if (first) {
                    D.syn_e = L.syn_e[pos];
                    D.syn_decay = L.syn_decay[pos];
                    first = false;
                } else {
                    same = L.syn_e[pos] == D.syn_e && L.syn_decay[pos] == D.syn_decay;
                }
            }
            D.syn_uniform = (!first && same) ? 1 : 0;
        }
        // clamps of the pack, by slot then input order
        std::vector<std::pair<int64_t, int64_t>> cl;  // (slot, clamp)
        for (int32_t k = 0; k < D.ncell; ++k) {
            const int32_t c = L.pc_gid[D.cell0 + k];
            for (int64_t i = L.cell_cv0[c]; i < L.cell_cv0[c + 1]; ++i)
                for (int64_t q : ic_at[i]) cl.push_back({L.perm[i], q});
        }
        std::sort(cl.begin(), cl.end());
        for (auto& sq : cl) {
            L.ic_slot.push_back(int32_t(sq.first - D.slot0));
            L.ic_on.push_back(ic[sq.second].step_on);
            L.ic_off.push_back(ic[sq.second].step_off);
            L.ic_amp.push_back(1000.0 * ic[sq.second].amp_nA);  // nA -> pA
        }
        D.nnl = int32_t(L.nl.size()) - D.nl0;
        D.nic = int32_t(L.ic_on.size()) - D.ic0;
        D.nhh = int32_t(L.hh_cv.size()) - D.hh0;
        D.nsyn = int32_t(L.syn_global.size()) - D.syn0;
        if (n_den > 0 && (D.syn_global || D.hh_global) && L.gen_pk.back() != int32_t(L.gen_mech.size())) {
            err = "generated mechanisms do not run on a cell whose state is held in HBM (too large for LDS)";
            return ARB_EINVAL;
        }
    }
    if (n_den > 0) {
        L.gen_off.push_back(int32_t(L.gen_mech.size()));
        L.gen_pk.push_back(int32_t(L.gen_mech.size()));
        const size_t ni = L.gen_mech.size();
        std::vector<double> sm(L.gen_st0.size());
        for (size_t q = 0; q < ni; ++q)
            for (int k = 0; k < gen::kMaxStates; ++k) sm[size_t(k) * ni + q] = L.gen_st0[q * gen::kMaxStates + k];
        L.gen_st0.swap(sm);
    }
    L.n_hh_total = int64_t(L.hh_cv.size());
    L.hh_gna.assign(L.hh_cv.size(), 0.0);
    L.hh_gk.assign(L.hh_cv.size(), 0.0);
    L.glin_extra.assign(L.n_cv, 0.0);
    L.gmem.assign(L.n_slots, 0.0);
    recompute_coefficients(L);
    // the register-resident kernel needs only as many slots as the rounds use
    if (L.reg_slots > 0) {
        int used = 1;
        for (const RoundDesc& R : L.rounds) used = std::max(used, R.j + 1);
        L.reg_slots = used;
    }

    // external events, grouped per pack, ordered (step, pack synapse, input order)
    {
        std::vector<int64_t> idx(n_ev);
        std::iota(idx.begin(), idx.end(), 0);
        auto key_pack = [&](int64_t q) { return pack_of_cell[syn[ev[q].syn].cell]; };
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            const int64_t pa = key_pack(a), pb = key_pack(b);
            if (pa != pb) return pa < pb;
            if (opt.ev_t_ms && opt.ev_t_ms[a] != opt.ev_t_ms[b]) return opt.ev_t_ms[a] < opt.ev_t_ms[b];
            if (ev[a].step != ev[b].step) return ev[a].step < ev[b].step;
            const int64_t sa = L.syn_pack_index[ev[a].syn], sb = L.syn_pack_index[ev[b].syn];
            if (sa != sb) return sa < sb;
            return a < b;
        });
        L.xe_step.resize(n_ev);
        if (opt.ev_t_ms) L.xe_t.resize(n_ev);
        L.xe_syn.resize(n_ev);
        L.xe_w.resize(n_ev);
        for (auto& D : L.packs) { D.xe0 = 0; D.xe1 = 0; }
        int64_t at = 0;
        for (int64_t pk = 0; pk < n_packs; ++pk) {
            L.packs[pk].xe0 = at;
            while (at < n_ev && key_pack(idx[at]) == pk) {
                const int64_t q = idx[at];
                L.xe_step[at] = ev[q].step;
                if (opt.ev_t_ms) L.xe_t[at] = opt.ev_t_ms[q];
                L.xe_syn[at] = int32_t(L.syn_pack_index[ev[q].syn] - L.packs[pk].syn0);
                L.xe_w[at] = 1000.0 * ev[q].w_uS;  // uS -> nS
                ++at;
            }
            L.packs[pk].xe1 = at;
        }
    }

    // connections: rank by (dst pack, pack synapse, src, index).
    // A pack's synapse positions are contiguous and packs follow each other,
    // so ordering by position orders by pack: a counting sort by position
    // (stable, so by index within a position), then by source where several
    // connections share a synapse.
    {
        const size_t npos = L.syn_global.size();
        std::vector<int64_t> at(npos + 1, 0);
        for (int64_t q = 0; q < n_conn; ++q) at[size_t(L.syn_pack_index[conn[q].syn]) + 1]++;
        for (size_t k = 0; k < npos; ++k) at[k + 1] += at[k];
        std::vector<int64_t> idx(n_conn);
        {
            std::vector<int64_t> fill(at.begin(), at.end() - 1);
            for (int64_t q = 0; q < n_conn; ++q) idx[size_t(fill[size_t(L.syn_pack_index[conn[q].syn])]++)] = q;
        }
        for (size_t k = 0; k < npos; ++k)
            if (at[k + 1] - at[k] > 1)
                std::stable_sort(idx.begin() + at[k], idx.begin() + at[k + 1],
                                 [&](int64_t a, int64_t b) { return conn[a].src < conn[b].src; });
        if (n_conn >= (int64_t(1) << 32)) { err = "too many connections"; return ARB_EINVAL; }
        L.cr_pack.resize(n_conn);
        L.cr_syn.resize(n_conn);
        L.cr_delay.resize(n_conn);
        if (opt.conn_delay_ms) L.cr_delay_ms.resize(n_conn);
        L.cr_src.resize(n_conn);
        L.cr_w.resize(n_conn);
        std::vector<int64_t> in_per_pack(n_packs, 0);
        for (int64_t r = 0; r < n_conn; ++r) {
            const arb_connection& K = conn[idx[r]];
            const int64_t pk = pack_of_cell[K.dst];
            L.cr_pack[r] = int32_t(pk);
            L.cr_syn[r] = int32_t(L.syn_pack_index[K.syn] - L.packs[pk].syn0);
            L.cr_delay[r] = K.delay_steps;
            if (opt.conn_delay_ms) L.cr_delay_ms[r] = opt.conn_delay_ms[idx[r]];
            L.cr_src[r] = K.src;
            L.cr_w[r] = 1000.0 * K.w_uS;
            in_per_pack[pk]++;
        }
        L.max_in_per_pack = n_packs ? *std::max_element(in_per_pack.begin(), in_per_pack.end()) : 0;
        L.in_off.assign(n_packs + 1, 0);
        for (int64_t pk = 0; pk < n_packs; ++pk) L.in_off[pk + 1] = L.in_off[pk] + in_per_pack[pk];
    }
    return ARB_OK;
}

std::string verify_layout(const Lowered& L) {
    // every synapse at exactly one pack-order position, and back
    for (size_t q = 0; q < L.syn_pack_index.size(); ++q) {
        const int64_t pos = L.syn_pack_index[q];
        if (pos < 0 || pos >= int64_t(L.syn_global.size()) || L.syn_global[pos] != int64_t(q))
            return fmt("synapse %zu has no pack-order position", q);
    }
    // connection ranks grouped by destination pack, in pack order
    if (!L.cr_pack.empty()) {
        if (L.in_off.size() != L.packs.size() + 1 || L.in_off.back() != int64_t(L.cr_pack.size()))
            return "connection rank ranges do not cover the ranks";
        for (size_t r = 0; r < L.cr_pack.size(); ++r) {
            const int32_t pk = L.cr_pack[r];
            if (int64_t(r) < L.in_off[size_t(pk)] || int64_t(r) >= L.in_off[size_t(pk) + 1])
                return fmt("connection rank %zu outside its pack's range", r);
        }
    }
    // every user CV in exactly one slot, slots inside their pack
    std::vector<int32_t> hit(L.n_slots, 0);
    for (int64_t i = 0; i < L.n_cv; ++i) {
        const int64_t s = L.perm[i];
        if (s < 0 || s >= L.n_slots) return fmt("CV %lld has no slot", (long long)i);
        if (hit[s]++) return fmt("slot %lld holds two CVs", (long long)s);
    }
    for (size_t pk = 0; pk < L.packs.size(); ++pk) {
        const PackDesc& D = L.packs[pk];
        if (D.ncell < 1 || D.ncell > L.block_threads) return fmt("pack %zu has no cell or more cells than threads", pk);
        // round order: a task's children finished in earlier rounds (elimination
        // runs rounds in order); its parent's slot lies in a later round
        std::vector<int32_t> round_of_slot(D.nslot, -1);
        for (int32_t r = 0; r < D.nrd; ++r) {
            const RoundDesc& R = L.rounds[D.rd0 + r];
            if (R.w < 1 || R.t0 < 0 || R.t0 + R.w > L.block_threads) return fmt("pack %zu round %d: bad threads", pk, r);
            if (int64_t(R.slot0) + int64_t(R.len) * R.w > D.nslot) return fmt("pack %zu round %d: slots overflow", pk, r);
            for (int64_t q = R.slot0; q < int64_t(R.slot0) + int64_t(R.len) * R.w; ++q) round_of_slot[q] = r;
        }
        if (L.reg_slots > 0) {
            if (D.ntk + 2 > 65535) return fmt("pack %zu: too many tasks for the register layout", pk);
            for (int32_t t = 0; t < D.ntk && D.binary; ++t)
                if (L.tasks[D.tk0 + t].nch > 2) return fmt("pack %zu: binary flag with a wider branch point", pk);
            if (D.spare < 0 || D.spare > D.nslot) return fmt("pack %zu: spare slot out of range", pk);
            if (D.spare < D.nslot && round_of_slot[D.spare] >= 0) {
                // inside a round: it must be a pad row of that round's branch
                const RoundDesc& R = L.rounds[D.rd0 + round_of_slot[D.spare]];
                const int32_t i = (D.spare - R.slot0) % R.w, k = (D.spare - R.slot0) / R.w;
                if (k < L.tasks[D.tk0 + R.task0 + i].len) return fmt("pack %zu: spare slot holds a CV", pk);
            }
        }
        // first and last slot of every task of the pack
        std::vector<int32_t> task_slot0(D.ntk, -1), task_last(D.ntk, -1);
        for (int32_t r = 0; r < D.nrd; ++r) {
            const RoundDesc& R = L.rounds[D.rd0 + r];
            for (int i = 0; i < R.w; ++i) {
                const int32_t t = R.task0 + i;
                if (t < 0 || t >= D.ntk) return fmt("pack %zu round %d: task out of range", pk, r);
                task_slot0[t] = R.slot0 + i;
                task_last[t] = R.slot0 + (L.tasks[D.tk0 + t].len - 1) * R.w + i;
            }
        }
        std::vector<std::vector<char>> used(std::max(L.reg_slots, 1), std::vector<char>(L.block_threads, 0));
        for (int32_t r = 0; r < D.nrd; ++r) {
            const RoundDesc& R = L.rounds[D.rd0 + r];
            if (L.reg_slots > 0) {
                if (R.j < 0 || R.j >= L.reg_slots) return fmt("pack %zu round %d: register slot out of range", pk, r);
                if (R.len > L.reg_len) return fmt("pack %zu round %d: branch longer than the registers", pk, r);
                for (int t = R.t0; t < R.t0 + R.w; ++t)
                    if (used[R.j][t]++) return fmt("pack %zu: thread %d register slot %d used twice", pk, t, R.j);
            }
            for (int i = 0; i < R.w; ++i) {
                const TaskDesc& T = L.tasks[D.tk0 + R.task0 + i];
                if (T.len < 1 || T.len > R.len) return fmt("pack %zu round %d: bad task length", pk, r);
                if (T.par >= 0 && !(round_of_slot[T.par] > r)) return fmt("pack %zu round %d: parent not later", pk, r);
                for (int c = 0; c < T.nch; ++c) {
                    const int32_t cs = L.ch_slot[D.ch0 + T.ch0 + c];
                    if (cs < 0 || cs >= D.nslot || !(round_of_slot[cs] < r))
                        return fmt("pack %zu round %d: child not earlier", pk, r);
                    // the child's task starts at that slot and names this task as its parent
                    const int32_t ct = L.ch_task[D.ch0 + T.ch0 + c];
                    if (ct < 0 || ct >= D.ntk || task_slot0[ct] != cs || L.tk_ptask[D.tk0 + ct] != R.task0 + i)
                        return fmt("pack %zu round %d: child task does not match its slot", pk, r);
                }
                // the parent task's distal CV is the one this branch hangs from,
                // one level up
                const int32_t pt = L.tk_ptask[D.tk0 + R.task0 + i];
                const int32_t lv = L.tk_lev[D.tk0 + R.task0 + i];
                if (lv < 0 || lv >= D.nlev || (pt >= 0 && L.tk_lev[D.tk0 + pt] != lv - 1) || (pt < 0 && lv != 0))
                    return fmt("pack %zu round %d: bad task level", pk, r);
                if ((pt < 0) != (T.par < 0)) return fmt("pack %zu round %d: parent task and slot disagree", pk, r);
                if (pt >= 0 && (pt >= D.ntk || task_last[pt] != T.par))
                    return fmt("pack %zu round %d: parent task does not end at the parent slot", pk, r);
            }
        }
    }
    return "";
}

// alpha_i = c_i/dt - G_lin,i and beta_i = sum G e over the linear terms
// (pas and the hh leak), so that the right-hand side of the implicit-Euler
// system is  rhs_i = alpha_i V_i + beta_i - (nonlinear and point currents).
void recompute_coefficients(Lowered& L) {
    const double dt = L.dt;
    std::vector<double> gna(L.n_cv, 0.0), gk(L.n_cv, 0.0);
    for (int64_t i = 0; i < L.n_cv; ++i) {
        double G = 0.0, GE = 0.0, gl = 0.0;
        for (int64_t k = L.piece_off[i]; k < L.piece_off[i + 1]; ++k) {
            const Region& R = L.regions[L.piece_reg[k]];
            const double a10 = 10.0 * L.piece_area[k];  // S/cm^2 x um^2 -> nS
            if (R.mech & ARB_MECH_PAS) { G += a10 * R.gpas; GE += a10 * R.gpas * R.epas; }
            if (R.mech & ARB_MECH_HH) { gna[i] += a10 * R.gna; gk[i] += a10 * R.gk; gl += a10 * R.gl; }
        }
        const int64_t s = L.perm[i];
        L.alpha[s] = L.cap[s] / dt - G - gl;
        L.beta[s] = GE + gl * kEL;
        L.gmem[s] = G + gl;
        L.glin_extra[i] = gl;
    }
    for (size_t q = 0; q < L.hh_cv.size(); ++q) {
        L.hh_gna[q] = gna[L.hh_cv[q]];
        L.hh_gk[q] = gk[L.hh_cv[q]];
    }
}

void state_part_bytes(const Lowered& L, const StateShape& sh, int64_t b[kStateParts]) {
    const int64_t np = int64_t(L.packs.size());
    const int64_t nhh = int64_t(L.hh_cv.size()), nsyn = int64_t(L.syn_global.size());
    const int64_t nbk = sh.net ? np * (int64_t(sh.K) + 1) * 4 : 0;
    const int64_t v[kStateParts] = {L.n_slots * 8, nhh * 8, nhh * 8, nhh * 8, nsyn * 8, np * 8, nbk, nbk,
                                    np * sh.bk_cap * 4, np * sh.bk_cap * 8, int64_t(sizeof(Counters)),
                                    int64_t(sh.sp_cap) * 4, int64_t(sh.sp_cap) * 8, int64_t(sh.sp_cap) * 8,
                                    int64_t(sh.n_hist) * 4, int64_t(sh.n_hist) * sh.hist_cap * 4,
                                    int64_t(sh.n_hist) * sh.hist_cap * 8, int64_t(L.gen_st0.size()) * 8};
    for (int k = 0; k < kStateParts; ++k) b[k] = v[k];
}

std::string check_state_blob(const Lowered& L, const StateShape& sh, const void* blob, int64_t n) {
    if (!blob) return "null blob";
    if (n < int64_t(sizeof(StateHeader))) return "state blob too small";
    StateHeader h;
    std::memcpy(&h, blob, sizeof h);
    const int64_t np = int64_t(L.packs.size());
    const int64_t nhh = int64_t(L.hh_cv.size()), nsyn = int64_t(L.syn_global.size());
    if (h.magic != kStateMagic || h.n_slots != L.n_slots || h.n_hh != nhh || h.n_syn != nsyn || h.n_packs != np ||
        h.n_bk != np || h.bk_cap != sh.bk_cap || h.sp_cap != int64_t(sh.sp_cap))
        return "state blob does not belong to this model";
    int64_t bytes[kStateParts];
    state_part_bytes(L, sh, bytes);
    int64_t total = sizeof(StateHeader);
    for (int k = 0; k < kStateParts; ++k) total += bytes[k];
    if (n < total) return "state blob truncated";
    const char* in = static_cast<const char*>(blob);
    const char* part[kStateParts];
    int64_t off = sizeof h;
    for (int k = 0; k < kStateParts; ++k) {
        part[k] = in + off;
        off += bytes[k];
    }
    auto rd32 = [](const char* b, int64_t i) { uint32_t v; std::memcpy(&v, b + 4 * i, 4); return v; };
    auto rd64 = [](const char* b, int64_t i) { int64_t v; std::memcpy(&v, b + 8 * i, 8); return v; };
    Counters c;
    std::memcpy(&c, part[10], sizeof c);
    const uint32_t have = std::min(c.sp_count, sh.sp_cap);
    if (h.step < 0 || h.step >= (int64_t(1) << 31) || h.sp_user < 0 || h.sp_user > int64_t(have) || c.sp_exch > have)
        return "state blob: step or spike counters out of range";
    for (int64_t p = 0; p < np; ++p) {
        const int64_t x = rd64(part[5], p);
        if (x < L.packs[p].xe0 || x > L.packs[p].xe1) return "state blob: event cursor out of range";
    }
    for (uint32_t i = 0; i < have; ++i)
        if (rd32(part[11], i) >= uint32_t(L.n_cells)) return "state blob: spike gid out of range";
    if (sh.net) {
        const int64_t K = sh.K;
        for (int64_t p = 0; p < np; ++p) {
            uint32_t prev = 0;
            for (int64_t b = 0; b <= K; ++b) {
                const uint32_t o = rd32(part[6], p * (K + 1) + b), x = rd32(part[7], p * (K + 1) + b);
                if (o < prev || o > uint32_t(sh.bk_cap) || x > uint32_t(K))
                    return "state blob: event bucket offsets out of range";
                prev = o;
            }
            for (uint32_t i = 0; i < prev; ++i) {
                const uint32_t q = rd32(part[8], p * int64_t(sh.bk_cap) + i);
                if (q >= uint32_t(L.packs[p].nsyn)) return "state blob: event synapse out of range";
            }
        }
        for (int64_t k = 0; k < sh.n_hist; ++k) {
            const uint32_t m = rd32(part[14], k);
            if (m > sh.hist_cap) return "state blob: spike history count out of range";
            for (uint32_t i = 0; i < m; ++i)
                if (rd32(part[15], k * int64_t(sh.hist_cap) + i) >= uint32_t(L.n_cells))
                    return "state blob: spike history gid out of range";
        }
    }
    return "";
}

}  // namespace arbmi
