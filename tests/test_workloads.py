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


def test_local_synapse_indices_are_checked():
    """A connection or external event names a synapse of its own cell."""
    import pytest
    from tests import models
    for field, entry in (("in_conn", (0, 1, 10, 1e-3)), ("ext", (1, 5, 0.05))):
        src, dst = models.bare_cell([], [], [], []), models.bare_cell([], [], [], [])
        dst.syn.append((-1, 0, 2.0, 0.0))
        getattr(dst, field).append(entry)  # synapse 1 of a cell with one synapse
        with pytest.raises(ValueError, match="cell 1"):
            gen.assemble([src, dst], n_steps=10)


def test_mixed_pull_chunks_event_counts():
    """The model behind the event pull's mixed-chunk parity test does what it
    claims, in the oracle: in every epoch window each kicked source fires
    exactly once and each clamped source at least twice, the two kicked
    groups at different steps, and the targets fire."""
    import oracle
    from tests import models
    m = models.mixed_pull_chunks()
    s = oracle.Sim(m)
    s.run(4000)
    g, st, _ = s.spikes()
    kicked = [k for k in range(106) if k not in (96, 97)]
    for e in range(4):  # spikes of [800 e, 800 e + 800) arrive in epoch e + 1
        inw = (st >= 800 * e) & (st < 800 * e + 800)
        per = np.bincount(g[inw], minlength=108)
        assert np.all(per[kicked] == 1) and per[96] >= 2 and per[97] >= 2
        assert len(np.unique(st[inw & np.isin(g, kicked)])) == 2
    assert np.sum(g == 106) >= 4 and np.sum(g == 107) >= 4
    # rank order on the targets: 96 kicked, 32 clamped, 8 kicked on synapse 0
    src = m["con_src"][(m["con_dst"] == 106) & (m["con_syn"] == m["con_syn"][m["con_dst"] == 106].min())]
    assert np.array_equal(np.sort(src)[:96], np.arange(96)) and np.all(np.sort(src)[96:128] >= 96)


def test_longest_epochs_model_in_the_oracle():
    """The spikes the longest-epoch parity test expects, from the oracle at
    its own epoch length and at the 16,384-step epochs of the library."""
    import oracle
    from tests import models
    m = models.longest_epochs()
    for K in (None, 16384):
        s = oracle.Sim(m, epoch_steps=K)
        s.run(33000)
        g, st, _ = s.spikes()
        assert sorted(zip(st.tolist(), g.tolist())) == [(7, 0), (12768, 3), (20014, 1), (32774, 2), (32775, 4)]
