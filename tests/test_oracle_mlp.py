"""Pins of the oracle's learned lifting closure.

- back-propagated gradients equal central finite differences of the loss;
- one Adam step from zero moments moves each parameter by lr * sign(g)
  (up to eps), the closed form of the bias-corrected first update;
- a network whose output is identically zero turns the learned lifting into
  plain Grad lifting, step for step;
- features and targets: an equilibrium has zero targets, and the features of
  an equilibrium are its normalised Gaussian central moments.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs
from tests.test_oracle_lattice import product_feq


@pytest.mark.parametrize("F,H,O_", [(10, 16, 7), (10, 64, 27), (28, 8, 37)])
def test_gradient_matches_central_differences(F, H, O_):
    rng = np.random.default_rng(0)
    np_ = O.mlp_nparams(F, H, O_)
    p = rng.normal(0, 0.3, np_)
    X = rng.normal(0, 1, (7, F))
    T = rng.normal(0, 1, (7, O_))
    loss, g = O.mlp_loss_grad(p, F, H, O_, X, T)
    idx = rng.choice(np_, 40, replace=False)
    for k in idx:
        h = 1e-6
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        fd = (O.mlp_loss_grad(pp, F, H, O_, X, T)[0] - O.mlp_loss_grad(pm, F, H, O_, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * abs(fd) + 1e-9, (k, fd, g[k])
    # forward agrees with the loss
    Y = O.mlp_forward(p, F, H, O_, X)
    assert abs(np.mean((Y - T) ** 2) - loss) < 1e-14


def test_adam_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    O.adam(p, m, v, g, 1, lr=1e-3, eps=1e-12)
    assert np.allclose(p, np.array([1.0, -2.0, 0.5]) - 1e-3 * np.sign(g), atol=1e-12)


def test_features_and_targets_of_equilibrium():
    u = np.array([0.2, -0.1, 0.0])
    theta = 1.3
    fq = product_feq(2, 3, 1.1, u, theta)
    gq = (1.5 - 1.0) * theta * fq
    feat = O.mlp_features(2, 3, fq, gq, thermal=1, cv=1.5)
    assert abs(feat[0] - 1.1) < 1e-14
    assert np.allclose(feat[1:3], u[:2] / math.sqrt(theta), atol=1e-14)
    assert abs(feat[3] - theta) < 1e-13
    # normalised central moments of a Gaussian: (2,0) and (0,2) are 1, the rest 0,
    # except (2,2) = 1 (product of the two variances); order (2,0),(1,1),(2,1),(0,2),(1,2),(2,2)
    assert np.allclose(feat[4:], [1, 0, 0, 1, 0, 1], atol=1e-12)
    fQ = product_feq(2, 6, 1.1, u, theta)
    gQ = (1.5 - 1.0) * theta * fQ
    t = O.mlp_targets(2, 3, 6, fQ, gQ, thermal=1, cv=1.5)
    assert t.size == 27 and np.max(np.abs(t)) < 1e-10


def test_zero_network_equals_grad_lifting():
    nx = ny = 16
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=5)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=3, blob=4)
    base = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, tau=0.7)
    outs = []
    for mode in (inputs.LIFT_GRAD, inputs.LIFT_MLP):
        o = O.Oracle(dict(base, lift_mode=mode))
        if mode == inputs.LIFT_MLP:
            F, Od = O.mlp_dims(2, 3, 6)
            H = 16
            o.set_mlp(H, np.zeros(O.mlp_nparams(F, H, Od)), np.zeros(F), np.ones(F),
                      np.zeros(Od), np.ones(Od))
        o.set_mask(mask, convert=False)
        o.init(rho, u, T)
        o.step(5)
        outs.append((o.get_pops(0), o.get_pops(1)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_nonzero_network_changes_only_lifted_values():
    # a constant output b3 shifts the completed moments; projection back is unchanged
    F, Od = O.mlp_dims(2, 3, 4)
    H = 8
    p = np.zeros(O.mlp_nparams(F, H, Od))
    p[-Od:] = 0.01
    cfg = inputs.base_config(nx=8, ny=8, n_low=3, n_high=4, lift_mode=inputs.LIFT_MLP)
    o = O.Oracle(cfg)
    o.set_mlp(H, p, np.zeros(F), np.ones(F), np.zeros(Od), np.ones(Od), manual_check=True)
    u = np.array([0.1, 0.05, 0])
    fq = product_feq(2, 3, 1.0, u, 1.0)
    got = o.lift_cell(fq)
    feq = product_feq(2, 4, 1.0, u, 1.0)
    assert np.max(np.abs(got - feq)) > 1e-4
    back = O.project(2, 4, 3, got)
    assert np.max(np.abs(back - fq)) < 1e-14
    # the raw moments the low-order set cannot hold moved by exactly rho T^{|p|/2} * 0.01
    x, _ = O.gh_rule(4)
    cx = np.array([x[i % 4] for i in range(16)])
    cy = np.array([x[i // 4] for i in range(16)])
    for j in range(16):
        m, k = j % 4, j // 4
        d = np.sum((got - feq) * cx ** m * cy ** k)
        if m < 3 and k < 3:
            assert abs(d) < 1e-13
        else:
            assert abs(d - 0.01) < 1e-12
