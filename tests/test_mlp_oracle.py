"""Pins of the learned-preconditioner oracle (CPU): the backward pass against
central finite differences of the loss, the partition of unity, and the
identity network reproducing its input through the cell extraction and
weighted assembly."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_oracle as mo
from oracle.fe_oracle import constrained_mask


def rand_params(rng, F, H):
    S = rng.standard_normal((F, F)) / np.sqrt(F)
    return [rng.standard_normal((H, F)) / np.sqrt(F), 0.1 * rng.standard_normal(H),
            rng.standard_normal((H, H)) / np.sqrt(H), 0.1 * rng.standard_normal(H),
            rng.standard_normal((F, H)) / np.sqrt(H), 0.1 * rng.standard_normal(F), S + S.T]


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    F, H, n = 7, 6, 11
    params = rand_params(rng, F, H)
    X = rng.standard_normal((n, F))
    T = rng.standard_normal((n, F))
    loss, grads = mo.loss_and_grads(params, X, T)
    h = 1e-6
    for pi, P in enumerate(params):
        flat = P.reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mo.loss_and_grads(params, X, T)
            flat[idx] = old - h
            lm, _ = mo.loss_and_grads(params, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (pi, idx, fd, g)


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
@pytest.mark.parametrize("n", [(1, 2, 1), (2, 2, 3)])
def test_partition_of_unity(bc, n):
    mesh = W.BoxMesh(n=n, bc=bc)
    p = 2
    w = mo.pou_weights(mesh, p)
    from oracle.fe_oracle import cell_dof_map
    cmap = cell_dof_map(mesh, p)
    tot = np.zeros(constrained_mask(mesh, p).size)
    np.add.at(tot, cmap.ravel(), w.ravel())
    cons = constrained_mask(mesh, p)
    np.testing.assert_allclose(tot[~cons], 1.0, rtol=0, atol=1e-15)
    assert np.all(tot[cons] == 0.0)


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
def test_identity_network_reproduces_the_input(bc):
    mesh = W.BoxMesh(n=(2, 1, 3), bc=bc)
    p, k = 3, 4
    cons = constrained_mask(mesh, p)
    R = np.random.default_rng(1).uniform(-1, 1, (cons.size, k))
    R[cons] = 0.0
    X, _, rho = mo.cell_inputs(mesh, p, R)
    np.testing.assert_allclose(np.sqrt((X * X).mean(axis=1)), 1.0, rtol=1e-12)
    Z = mo.cell_assemble(mesh, p, X, rho, k)
    np.testing.assert_allclose(Z, R, rtol=0, atol=1e-14)
    d = np.random.default_rng(2).uniform(1, 2, cons.size)
    Z2 = mo.cell_assemble(mesh, p, X, rho, k, R=R, diag=d)
    np.testing.assert_allclose(Z2, R + R / d[:, None], rtol=0, atol=1e-14)
    # symmetric weighting: identity cell map gives sum_e Q_e^T w Q_e r = r too
    Xs, _, rhos = mo.cell_inputs(mesh, p, R, pou_sqrt=True)
    np.testing.assert_allclose(mo.cell_assemble(mesh, p, Xs, rhos, k, pou_sqrt=True), R,
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
@pytest.mark.parametrize("scaled", [False, True])
def test_symmetric_weighting_gives_a_symmetric_operator(bc, scaled):
    """With sqrt(w) on both sides and a symmetric linear cell map S, the assembled
    map r -> z is a symmetric matrix (checked as u^T M v = v^T M u)."""
    mesh = W.BoxMesh(n=(2, 2, 1), bc=bc)
    p, k = 2, 1
    cons = constrained_mask(mesh, p)
    F = (p + 1) ** 3
    rng = np.random.default_rng(5)
    S = rng.standard_normal((F, F))
    S = S + S.T

    d = rng.uniform(0.5, 2.0, cons.size) if scaled else None

    def M(r):
        X, _, rho = mo.cell_inputs(mesh, p, r, pou_sqrt=True, dscale=d)
        return mo.cell_assemble(mesh, p, X @ S.T, rho, k, pou_sqrt=True, dscale=d)
    u = rng.standard_normal((cons.size, 1))
    v = rng.standard_normal((cons.size, 1))
    u[cons] = 0.0
    v[cons] = 0.0
    assert abs((u * M(v)).sum() - (v * M(u)).sum()) <= 1e-12 * np.abs(u * M(v)).sum()


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 is halfway between 1 and the next BF16 value 1 + 2^-7: ties to even (1)
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3])
    r = mo.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_adam_first_step_moves_by_lr():
    w, g = np.array([1.0, -2.0]), np.array([0.5, -3.0])
    w1, m1, m2 = mo.adam_step(w, g, np.zeros(2), np.zeros(2), 0.1, 0.9, 0.999, 1e-12, 1)
    np.testing.assert_allclose(w1, w - 0.1 * np.sign(g), rtol=1e-6)


def _adam_golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "adam_three_steps.json")) as f:
        return json.load(f)


def test_adam_three_steps_match_the_hand_derivation():
    """Moment decay and bias correction at t = 2, 3 (a zero gradient at step 2 or 3),
    against values derived by hand in exact arithmetic (tests/golden/adam_three_steps.json).
    A missing bias correction, swapped b1/b2 or a moment that is not decayed fails."""
    g = _adam_golden()
    w = np.array(g["w0"])
    m1, m2 = np.zeros(2), np.zeros(2)
    for t, grad in enumerate(g["grads"], start=1):
        w, m1, m2 = mo.adam_step(w, np.array(grad), m1, m2, g["lr"], g["b1"], g["b2"], g["eps"], t)
        np.testing.assert_allclose(w, [g["w_after"][0][t - 1], g["w_after"][1][t - 1]],
                                   rtol=2e-7, atol=0)


@pytest.mark.parametrize("bc", [W.BC_NONE, W.BC_DIRICHLET0, W.BC_PERIODIC])
def test_linear_map_is_definite_when_identity_plus_skip_is(bc):
    """The deployed preconditioner z = D^-1 r + sum_e Q_e^T W^1/2 D^-1/2 S D^-1/2 W^1/2 Q_e r,
    built densely on the free rows from the oracle's gather and assembly: with the
    partition of unity it equals D^-1/2 [sum_e Q_e^T W_e^1/2 (I + S) W_e^1/2 Q_e] D^-1/2, so
    the smallest eigenvalue of D^1/2 M D^1/2 is at least that of I + S (equality for
    S = s I, where the map is (1 + s) D^-1; s < -1 makes it negative definite).  The
    condition is sufficient, which is what the eigenvalue floor of the skip block relies
    on (an S with a direction below -1 that no cell excites, e.g. on constrained local
    nodes, can still give a definite M)."""
    mesh = W.BoxMesh(n=(2, 3, 2), bc=bc)
    p = 2
    cons = constrained_mask(mesh, p)
    free = ~cons
    F = (p + 1) ** 3
    rng = np.random.default_rng(31)
    d = rng.uniform(0.5, 2.0, cons.size)
    Q, _ = np.linalg.qr(rng.standard_normal((F, F)))

    def dense(S):
        n = cons.size
        eye = np.eye(n)[:, free]
        X, _, rho = mo.cell_inputs(mesh, p, eye, pou_sqrt=True, dscale=d)
        U = X * rho[:, None]                      # the linear map needs no scale
        Z = mo.cell_assemble(mesh, p, U @ S.T, np.ones(len(rho)), eye.shape[1], R=eye,
                             diag=d, pou_sqrt=True, dscale=d)
        M = Z[free]
        dh = np.sqrt(d[free])
        return dh[:, None] * M * dh[None, :]

    for lam in (np.linspace(-0.9, 3.0, F), np.linspace(-0.5, 0.5, F)):
        S = (Q * lam) @ Q.T
        B = dense(S)
        np.testing.assert_allclose(B, B.T, rtol=0, atol=1e-12)
        assert np.linalg.eigvalsh(B).min() >= (1.0 + lam.min()) - 1e-10
    for s in (-1.5, -0.7, 0.4):
        ev = np.linalg.eigvalsh(dense(s * np.eye(F)))
        np.testing.assert_allclose(ev, 1.0 + s, rtol=0, atol=1e-12)
