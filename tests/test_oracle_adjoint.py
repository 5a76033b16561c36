"""Pins for the oracle's discrete adjoint (gradients of a soma-trace loss with
respect to per-region gNa, gK, g_pas): central finite differences on the
discrete scheme, and the Taylor remainder."""
import numpy as np

import oracle
from workloads import gen

N_STEPS = 600
N_CELLS = 2


def _models():
    m0 = gen.config4(n_cells=N_CELLS, n_steps=N_STEPS)
    mh = gen.config4(n_cells=N_CELLS, hidden=True, n_steps=N_STEPS)
    return m0, mh


def _loss_and_trace(m, theta):
    s = oracle.Sim(m)
    s.set_params(theta.reshape(-1, 3))
    tr = s.run(N_STEPS, probes=oracle.cell_cv_begin(m)[:-1])
    return tr


def _target():
    m0, mh = _models()
    return _loss_and_trace(mh, gen.config4_theta(mh))


def _loss(tr, tgt):
    return np.mean((tr - tgt) ** 2)


def test_adjoint_matches_central_fd():
    m0, _ = _models()
    tgt = _target()
    th0 = gen.config4_theta(m0)
    s = oracle.Sim(m0)
    s.set_params(th0.reshape(-1, 3))
    tr = _loss_and_trace(m0, th0)
    dL = 2.0 * (tr - tgt) / tr.size
    tr_adj, grad = s.adjoint(N_STEPS, dL)
    assert np.array_equal(tr_adj, tr)
    grad = grad.reshape(th0.shape)
    # relative step 1e-5: at 1e-6 the finite difference's own rounding error
    # already reaches ~2e-5 on the smallest entries (it grows as h shrinks)
    h = 1e-5
    fd = np.zeros_like(th0)
    for r in range(th0.shape[1]):
        for q in range(3):
            tp, tm = th0.copy(), th0.copy()
            tp[:, r, q] *= 1 + h
            tm[:, r, q] *= 1 - h
            # cells are independent: one pair of runs gives every cell's entry,
            # taken from that cell's part of the loss
            Lp = np.mean((_loss_and_trace(m0, tp) - tgt) ** 2, axis=1) / N_CELLS
            Lm = np.mean((_loss_and_trace(m0, tm) - tgt) ** 2, axis=1) / N_CELLS
            fd[:, r, q] = (Lp - Lm) / (2 * h * th0[:, r, q])
    for c in range(N_CELLS):
        for q in range(3):
            den = np.maximum(np.abs(fd[c, :, q]), 1e-3 * np.max(np.abs(fd[c, :, q])))
            rel = np.abs(grad[c, :, q] - fd[c, :, q]) / den
            assert rel.max() <= 1e-5, (c, q, rel.max())


def test_adjoint_taylor_remainder_second_order():
    m0, _ = _models()
    tgt = _target()
    th0 = gen.config4_theta(m0)
    s = oracle.Sim(m0)
    s.set_params(th0.reshape(-1, 3))
    tr = _loss_and_trace(m0, th0)
    L0 = _loss(tr, tgt)
    _, grad = s.adjoint(N_STEPS, 2.0 * (tr - tgt) / tr.size)
    rng = np.random.default_rng(1)
    dirn = rng.normal(size=th0.shape) * th0
    slope = np.sum(grad.reshape(th0.shape) * dirn)
    rems = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        L1 = _loss(_loss_and_trace(m0, th0 + eps * dirn), tgt)
        rems.append(abs(L1 - L0 - eps * slope))
    assert 3.0 < rems[0] / rems[1] < 5.0
    assert 3.0 < rems[1] / rems[2] < 5.0
