// plan.cpp -- launch shape and packing limits for a model.
#include <algorithm>

#include "sim.hpp"

namespace arbmi {

Plan choose_plan(const arb_cell* cells, int32_t n_cells, const arb_branch* br, int64_t n_br, const arb_params& p,
                 int64_t lds_max, int n_cu) {
    (void)n_cu;
    Plan pl;
    lds_max -= 256;  // static LDS of the kernels
    pl.block_threads = p.block_threads ? p.block_threads : 64;
    // largest cell, in slots (CVs plus round padding, bounded by 25%)
    int64_t max_cv = 1;
    for (int32_t c = 0; c < n_cells && cells; ++c) {
        int64_t n = 1;
        if (cells[c].branch_begin >= 0 && cells[c].branch_begin + cells[c].n_branch <= n_br)
            for (int32_t b = 0; b < cells[c].n_branch; ++b) n += std::max(0, br[cells[c].branch_begin + b].n_cv);
        max_cv = std::max(max_cv, n);
    }
    const int64_t need_lds = (max_cv + max_cv / 4) * 6 * 8 + max_cv * 3 * 8;
    pl.coef_mode = p.coef_mode ? p.coef_mode : (need_lds <= lds_max ? 1 : 2);
    // several workgroups per CU when cells are small; a large cell gets a pack
    // of its own, up to the whole LDS
    pl.lds_budget = lds_max / 3;
    pl.lds_hard_max = lds_max;
    pl.max_cells_per_pack = pl.block_threads;
    return pl;
}

}  // namespace arbmi
