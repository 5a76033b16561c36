"""GPU adjoint (through the C ABI and torch.autograd) against the oracle's
discrete adjoint and against central finite differences of the GPU forward."""
import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu


# The two adjoint kernels: the register-resident one (the default layout of
# these cells) and the streamed one (coefficient mode 2).
LAYOUTS = {"register": ({}, 3), "streamed": ({"coef_mode": 2}, 2)}


def _setup(n_cells, n_steps, layout="register", **kw):
    import torch

    from paper_1901_07454_amd import grad
    m0 = gen.config4(n_cells=n_cells, n_steps=n_steps)
    mh = gen.config4(n_cells=n_cells, hidden=True, n_steps=n_steps)
    th0 = gen.config4_theta(m0)
    ref = oracle.Sim(mh)
    tgt = ref.run(n_steps, probes=oracle.cell_cv_begin(mh)[:-1])
    extra, mode = LAYOUTS[layout]
    gs = grad.GradSim(m0, **extra, **kw)
    if "flags" not in kw:
        assert gs.sim.info["coef_mode"] == mode, gs.sim.info
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    return m0, th0, tgt, gs, theta


def model_theta(m):
    """Per-region [gNa, gK, g_pas] of any model (regions: each cell's soma,
    then its branches), flat [regions, 3]."""
    out = []
    b = 0
    for c, nb in enumerate(m["cell_n_branch"]):
        out.append((m["soma_gna"][c], m["soma_gk"][c], m["soma_gpas"][c]))
        for k in range(int(nb)):
            out.append((m["br_gna"][b + k], m["br_gk"][b + k], m["br_gpas"][b + k]))
        b += int(nb)
    return np.array(out, dtype=np.float64)


def _oracle_rel(g, og):
    return np.abs(g - og) / np.maximum(np.abs(og), 1e-3 * np.max(np.abs(og), axis=(1, 2), keepdims=True))


def _loss_grad(gs, theta, tgt, n_steps, k):
    import torch

    from paper_1901_07454_amd import grad
    theta = theta.detach().clone().requires_grad_(True)
    tr = grad.soma_trace(theta, gs, n_steps, k)
    loss = torch.mean((tr - torch.as_tensor(tgt, device=tr.device)) ** 2)
    loss.backward()
    return tr.detach().cpu().numpy(), loss.item(), theta.grad.detach().cpu().numpy()


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_adjoint_matches_oracle_adjoint(layout):
    n_cells, n_steps = 6, 800
    m0, th0, tgt, gs, theta = _setup(n_cells, n_steps, layout)
    tr, L, g = _loss_grad(gs, theta, tgt, n_steps, 100)
    s = oracle.Sim(m0)
    s.set_params(th0.reshape(-1, 3))
    dl = 2.0 * (tr - tgt) / tr.size
    otr, og = s.adjoint(n_steps, dl)
    og = og.reshape(th0.shape)
    assert np.max(np.abs(tr - otr)) <= 1e-8
    rel = np.abs(g - og) / np.maximum(np.abs(og), 1e-3 * np.max(np.abs(og), axis=(1, 2), keepdims=True))
    print(f"max rel |g_gpu - g_oracle| = {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-7
    gs.close()


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_adjoint_checkpoint_interval_invariant(layout):
    n_cells, n_steps = 3, 600
    m0, th0, tgt, gs, theta = _setup(n_cells, n_steps, layout)
    ref = _loss_grad(gs, theta, tgt, n_steps, 600)[2]
    for k in (1, 37, 100):
        g = _loss_grad(gs, theta, tgt, n_steps, k)[2]
        assert np.allclose(g, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
    gs.close()


def test_adjoint_matches_gpu_finite_differences():
    n_cells, n_steps = 4, 600
    m0, th0, tgt, gs, theta = _setup(n_cells, n_steps)
    _, _, g = _loss_grad(gs, theta, tgt, n_steps, 100)
    import torch
    h = 1e-5
    fd = np.zeros_like(th0)
    for r in range(th0.shape[1]):
        for q in range(3):
            vals = []
            for sgn in (1, -1):
                t = th0.copy()
                t[:, r, q] *= 1 + sgn * h
                tr, _, _ = _loss_grad(gs, torch.tensor(t, device="cuda"), tgt, n_steps, 600)
                vals.append(np.mean((tr - tgt) ** 2, axis=1) / n_cells)
            fd[:, r, q] = (vals[0] - vals[1]) / (2 * h * th0[:, r, q])
    for c in range(n_cells):
        for q in range(3):
            den = np.maximum(np.abs(fd[c, :, q]), 1e-3 * np.max(np.abs(fd[c, :, q])))
            rel = np.abs(g[c, :, q] - fd[c, :, q]) / den
            assert rel.max() <= 1e-5, (c, q, rel.max())
    gs.close()


def test_forward_state_restored_after_backward():
    n_cells, n_steps = 2, 300
    m0, th0, tgt, gs, theta = _setup(n_cells, n_steps)
    import torch

    from paper_1901_07454_amd import grad
    tr = grad.soma_trace(theta, gs, n_steps, 100)
    v_after_fwd = gs.sim.voltages_host()
    torch.mean(tr).backward()
    assert np.array_equal(gs.sim.voltages_host(), v_after_fwd)
    gs.close()


def _ring_of_c4_cells(n_steps):
    cells = [gen.cell_c4(i, False) for i in range(4)]
    for i, d in enumerate(cells):
        d.syn.append((-1, 0, 2.0, 0.0))
        d.in_conn.append(((i - 1) % 4, len(d.syn) - 1, 120, 0.02))
    return gen.assemble(cells, n_steps=n_steps)


def test_adjoint_through_network_events():
    """The config-4 cells on a ring (delay 120 steps, epochs of 120): the
    events the recompute replays come from the spike exchange, and
    checkpoints every 37 steps restore the state in the middle of epochs."""
    import torch

    from paper_1901_07454_amd import grad
    n = 600
    m0 = _ring_of_c4_cells(n)
    th0 = gen.config4_theta(m0)
    tgt = 0.9 * oracle.Sim(m0).run(n, probes=oracle.cell_cv_begin(m0)[:-1])
    gs = grad.GradSim(m0)
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    tr, L, g = _loss_grad(gs, theta, tgt, n, 100)
    s = oracle.Sim(m0)
    s.set_params(th0.reshape(-1, 3))
    otr, og = s.adjoint(n, 2.0 * (tr - tgt) / tr.size)
    og = og.reshape(th0.shape)
    assert np.max(np.abs(tr - otr)) <= 1e-8
    rel = np.abs(g - og) / np.maximum(np.abs(og), 1e-3 * np.max(np.abs(og), axis=(1, 2), keepdims=True))
    print(f"max rel |g_gpu - g_oracle| = {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-7
    g37 = _loss_grad(gs, theta, tgt, n, 37)[2]
    assert np.allclose(g37, g, rtol=1e-12, atol=1e-14 * np.abs(g).max())
    gs.close()


def test_autotuned_gradient_sim(tmp_path, monkeypatch):
    """A gradient sim built with the autotuner, with a cache that already
    holds the plain sim's choice for the same model: the gradient sim gets
    its own entry, and its backward matches the oracle's adjoint."""
    from paper_1901_07454_amd import arbmi
    monkeypatch.setenv("ARB_AUTOTUNE_CACHE", str(tmp_path / "cache.txt"))
    n_cells, n_steps = 8, 400
    m0 = gen.config4(n_cells=n_cells, n_steps=n_steps)
    plain = arbmi.Simulation(m0, flags=arbmi.ARB_FLAG_AUTOTUNE)
    plain.close()
    m0, th0, tgt, gs, theta = _setup(n_cells, n_steps, flags=arbmi.ARB_FLAG_AUTOTUNE)
    assert len((tmp_path / "cache.txt").read_text().splitlines()) == 2
    print("gradient sim", gs.sim.info, flush=True)
    tr, L, g = _loss_grad(gs, theta, tgt, n_steps, 100)
    s = oracle.Sim(m0)
    s.set_params(th0.reshape(-1, 3))
    otr, og = s.adjoint(n_steps, 2.0 * (tr - tgt) / tr.size)
    assert np.max(np.abs(tr - otr)) <= 1e-8
    rel = _oracle_rel(g, og.reshape(th0.shape))
    print(f"max rel |g_gpu - g_oracle| = {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-7
    gs.close()


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_adjoint_of_ring_cells_with_synapses(layout):
    """Cells of the 8192-cell ring (127 passive branches, hh soma, 10
    synapses) on a 4-cell ring with the kick: synapse conductances enter
    dI/dV, several cells share a workgroup, and few hh instances per pack."""
    import torch

    from paper_1901_07454_amd import arbmi
    n = 600
    m0 = gen.config2(n_cells=4, n_steps=n)
    th = model_theta(m0)
    sim = arbmi.Simulation(m0, flags=arbmi.ARB_FLAG_GRADIENTS, **LAYOUTS[layout][0])
    assert sim.info["coef_mode"] == LAYOUTS[layout][1], sim.info
    sim.set_params(th)
    cv0 = oracle.cell_cv_begin(m0)
    tgt = oracle.Sim(m0).run(n, probes=cv0[:-1]) + 1.0
    trace = torch.empty(4, n, dtype=torch.float64, device="cuda")
    arbmi.arb_grad_forward(sim.h, n, 100, trace)
    tr = trace.cpu().numpy()
    dl = 2.0 * (tr - tgt) / tr.size
    out = torch.empty(th.size, dtype=torch.float64, device="cuda")
    arbmi.arb_grad_backward(sim.h, torch.as_tensor(dl, device="cuda"), out)
    g = out.cpu().numpy().reshape(-1, 3)
    s = oracle.Sim(m0)
    s.set_params(th)
    otr, og = s.adjoint(n, dl)
    assert np.max(np.abs(tr - otr)) <= 1e-8
    den = np.maximum(np.abs(og), 1e-3 * np.max(np.abs(og), axis=0, keepdims=True))
    rel = np.abs(g - og) / den
    print(f"{layout}: max rel |g_gpu - g_oracle| = {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-7
    sim.close()
