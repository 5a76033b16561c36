"""The generator's network structure for the 10k-connectivity model
(Sec. V-A): every synapse of every cell takes exactly one connection, from
another cell, with the minimum delay; cells regenerate identically alone."""
import numpy as np

from workloads import gen


def test_ten_thousand_way_wiring():
    n, k = 24, 500
    m = gen.config7(n_cells=n, n_syn=k, n_steps=2000)
    assert len(m["con_src"]) == n * k
    assert np.array_equal(np.sort(m["con_syn"]), np.arange(n * k))
    assert np.all(m["syn_cell"][m["con_syn"]] == m["con_dst"])
    assert np.all(m["con_src"] != m["con_dst"])
    assert np.all(m["con_delay"] == 800) and np.all(m["con_w"] > 0)
    # sources spread over all other cells
    counts = np.bincount(m["con_src"], minlength=n)
    assert counts.min() > 0.5 * k and counts.max() < 1.5 * k
    # 50 Hz drive: synapse 0 of each cell at steps 0, 800, 1600
    first = np.searchsorted(m["syn_cell"], np.arange(n))
    assert np.array_equal(np.sort(m["ev_syn"]), np.repeat(first, 3))
    assert np.array_equal(np.unique(m["ev_step"]), [0, 800, 1600])
    # 10 ms variant
    assert np.all(gen.config7(n_cells=4, n_syn=10, min_delay_ms=10.0)["con_delay"] == 400)


def test_subsets_regenerate_identically():
    full = gen.config7(n_cells=12, n_syn=200, n_steps=10)
    sub = gen.config7(n_cells=12, cells=[3, 7], n_syn=200, n_steps=10)
    keep = np.isin(full["con_dst"], [3, 7]) & np.isin(full["con_src"], [3, 7])
    assert len(sub["con_src"]) == int(keep.sum())
    assert np.array_equal(sub["br_length"], np.concatenate(
        [full["br_length"][full["cell_branch_begin"][c]:full["cell_branch_begin"][c] + full["cell_n_branch"][c]]
         for c in (3, 7)]))
