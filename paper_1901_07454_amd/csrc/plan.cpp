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
    // largest cell (CVs) and widest branch level over all cells
    int64_t max_cv = 1, max_width = 1;
    std::vector<int> depth, count;
    for (int32_t c = 0; c < n_cells && cells; ++c) {
        const arb_cell& C = cells[c];
        if (C.branch_begin < 0 || C.n_branch < 0 || C.branch_begin + C.n_branch > n_br) continue;
        int64_t n = 1;
        depth.assign(C.n_branch, 0);
        count.assign(C.n_branch + 2, 0);
        for (int32_t b = 0; b < C.n_branch; ++b) {
            const arb_branch& B = br[C.branch_begin + b];
            n += std::max(0, B.n_cv);
            depth[b] = (B.parent < 0 || B.parent >= b) ? 1 : depth[B.parent] + 1;
            if (depth[b] <= C.n_branch) count[depth[b]]++;
        }
        for (int v : count) max_width = std::max<int64_t>(max_width, v);
        max_cv = std::max(max_cv, n);
    }
    // Streamed coefficients (mode 2) keep 16 B of LDS per CV and allow several
    // workgroups per CU; measured faster than LDS-resident coefficients on
    // the 1017-CV ring cells.  256 threads, with enough cells per pack that
    // the widest branch level fills the workgroup.
    pl.block_threads = p.block_threads ? p.block_threads : 256;
    const int64_t need_lds1 = (max_cv + max_cv / 4) * 6 * 8 + max_cv * 3 * 8;
    pl.coef_mode = p.coef_mode ? p.coef_mode : 2;
    if (pl.coef_mode == 1 && need_lds1 > lds_max && p.coef_mode == 0) pl.coef_mode = 2;
    pl.lds_budget = lds_max / 2;
    pl.lds_hard_max = lds_max;
    if (p.flags & ARB_FLAG_GRADIENTS) {
        // the adjoint kernel keeps 32 B per CV (forward, streamed: 16 B)
        pl.coef_mode = 2;
        pl.lds_budget = lds_max / 3;
        pl.lds_hard_max = lds_max / 2 - 1024;
    }
    if (p.cells_per_pack > 0) {
        pl.max_cells_per_pack = std::min(p.cells_per_pack, pl.block_threads);
        pl.lds_budget = lds_max;  // an explicit pack size wins over the LDS target
    } else {
        pl.max_cells_per_pack = std::max<int64_t>(1, std::min<int64_t>(pl.block_threads, pl.block_threads / max_width));
    }
    return pl;
}

}  // namespace arbmi
