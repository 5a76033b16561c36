// plan.cpp -- launch shape and packing limits for a model.
#include <algorithm>
#include <vector>

#include "sim.hpp"

namespace arbmi {

Plan choose_plan(const arb_cell* cells, int32_t n_cells, const arb_branch* br, int64_t n_br, const arb_params& p,
                 int64_t lds_max, int n_cu) {
    (void)n_cu;
    Plan pl;
    lds_max -= 256;  // static LDS of the kernels
    // largest cell (CVs), widest branch level, longest branch, most branches
    int64_t max_cv = 1, max_width = 1, max_len = 1, max_tasks = 1, max_tasks8 = 1;
    std::vector<int> depth, count;
    for (int32_t c = 0; c < n_cells && cells; ++c) {
        const arb_cell& C = cells[c];
        if (C.branch_begin < 0 || C.n_branch < 0 || C.branch_begin + C.n_branch > n_br) continue;
        int64_t n = 1, seg8 = 1;
        depth.assign(C.n_branch, 0);
        count.assign(C.n_branch + 2, 0);
        for (int32_t b = 0; b < C.n_branch; ++b) {
            const arb_branch& B = br[C.branch_begin + b];
            n += std::max(0, B.n_cv);
            seg8 += (std::max(1, B.n_cv) + 7) / 8;
            max_len = std::max<int64_t>(max_len, B.n_cv);
            depth[b] = (B.parent < 0 || B.parent >= b) ? 1 : depth[B.parent] + 1;
            if (depth[b] <= C.n_branch) count[depth[b]]++;
        }
        for (int v : count) max_width = std::max<int64_t>(max_width, v);
        max_cv = std::max(max_cv, n);
        max_tasks = std::max<int64_t>(max_tasks, int64_t(C.n_branch) + 1);
        max_tasks8 = std::max(max_tasks8, seg8);
    }
    const bool grads = (p.flags & ARB_FLAG_GRADIENTS) != 0;

    // Streamed coefficients (mode 2): 16 B of LDS per CV, 256 threads, enough
    // cells per pack that the widest branch level fills the workgroup.  Also
    // the fallback of the other modes.
    const int T2 = p.block_threads ? p.block_threads : 256;
    pl.fallback_cells_per_pack = std::max<int64_t>(1, std::min<int64_t>(T2, T2 / max_width));
    pl.fallback_lds_budget = lds_max / 2;
    pl.fallback_lds_hard_max = lds_max;
    if (grads) {  // the streamed adjoint kernel keeps 32 B per CV (forward: 16 B)
        pl.fallback_lds_budget = lds_max / 3;
        pl.fallback_lds_hard_max = lds_max / 2 - 1024;
    }

    // Register-resident coefficients (mode 3) by default when every branch
    // fits the registers: L = 8 CVs with up to 3 branches per thread, or
    // L = 16 with 1.  On request (and for the autotuner) longer branches are
    // cut into chains of 8-CV segments.  An explicit request is honoured or
    // refused by the lowering, never changed.  With gradients the packs must
    // also fit the register-resident adjoint kernel (the lowering checks).
    const bool reg_ok = p.coef_mode == 3 || (p.coef_mode == 0 && max_len <= 16);
    if (reg_ok) {
        pl.coef_mode = 3;
        pl.block_threads = p.block_threads ? p.block_threads : 256;
        pl.reg_len = (max_len > 8 && max_len <= 16) ? 16 : 8;
        if (pl.reg_len == 8)
            pl.reg_slots = (std::max(max_tasks, max_tasks8) <= 2 * pl.block_threads) ? 2 : 3;
        else
            pl.reg_slots = 1;
        pl.lds_budget = lds_max / 2;
        pl.lds_hard_max = lds_max;
        pl.max_cells_per_pack = p.cells_per_pack > 0 ? std::min(p.cells_per_pack, pl.block_threads) : pl.block_threads;
        if (p.cells_per_pack > 0) pl.lds_budget = lds_max;
        return pl;
    }

    pl.block_threads = T2;
    const int64_t need_lds1 = (max_cv + max_cv / 4) * 6 * 8 + max_cv * 3 * 8;
    pl.coef_mode = (p.coef_mode == 1 || p.coef_mode == 2) ? p.coef_mode : 2;
    if (pl.coef_mode == 1 && need_lds1 > lds_max && p.coef_mode == 0) pl.coef_mode = 2;
    pl.lds_budget = lds_max / 2;
    pl.lds_hard_max = lds_max;
    if (grads) {
        // the adjoint kernel keeps 32 B per CV (forward, streamed: 16 B)
        pl.coef_mode = 2;
        pl.lds_budget = lds_max / 3;
        pl.lds_hard_max = lds_max / 2 - 1024;
    }
    if (p.cells_per_pack > 0) {
        pl.max_cells_per_pack = std::min(p.cells_per_pack, pl.block_threads);
        pl.lds_budget = lds_max;  // an explicit pack size wins over the LDS target
    } else {
        pl.max_cells_per_pack = pl.fallback_cells_per_pack;
    }
    return pl;
}

}  // namespace arbmi
