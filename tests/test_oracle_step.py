"""Pins of the oracle's semi-Lagrangian step (Sec. II.C, III.D).

- the reconstruction weights interpolate quadratics exactly;
- with D2Q9 alone and CFL = 1 every departure point is a lattice node, so the
  step must equal a standard on-lattice stream-and-collide LBM, written out
  below from scratch with its own equilibrium (and D3Q27 in 3D);
- a single velocity set on a periodic box conserves mass and momentum (and
  energy in the thermal model) to rounding;
- a uniform equilibrium is a fixed point of the coupled step for any mask;
- the storage rounding matches numpy's float16 and torch's bfloat16.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def test_lagrange_weights_reproduce_quadratics():
    for xi in np.linspace(-0.5, 0.5, 11):
        a = O.lagrange3(xi)
        s = np.array([-1.0, 0.0, 1.0])
        for k in range(3):
            assert abs(np.sum(a * s ** k) - xi ** k) < 1e-15
        # and not cubics (unless xi is a node)
        if min(abs(xi), abs(abs(xi) - 1)) > 1e-9:
            assert abs(np.sum(a * s ** 3) - xi ** 3) > 1e-6


def test_stencil_offsets_follow_departure_points():
    cfg = inputs.base_config(nx=8, ny=8, n_low=3, n_high=6)
    o = O.Oracle(cfg)
    x6, _ = O.gh_rule(6)
    assert abs(o.dt - 1.0 / x6.max()) < 1e-15   # CFL = max|c| dt / dx = 1
    for which, n in ((0, 3), (1, 6)):
        n0, a = o.stencil(which)
        x, _ = O.gh_rule(n)
        for i in range(n * n):
            for ax in range(2):
                c = x[(i // n ** ax) % n]
                d = -c * o.dt
                assert n0[i, ax] == math.floor(d + 0.5)
                xi = d - n0[i, ax]
                assert np.allclose(a[i, ax], O.lagrange3(xi), atol=0)
                assert -0.5 <= xi < 0.5


def standard_d2q9(rho, ux, uy, tau, steps):
    """Textbook D2Q9 stream-and-collide with integer velocities e in {-1,0,1}^2,
    sound speed^2 = 1/3 in lattice units and the tensor-product equilibrium
    whose 1D factors match the moments rho, rho v, rho (v^2 + 1/3)."""
    e = [-1, 0, 1]

    def feq1d(k, v):
        cs2 = 1.0 / 3.0
        if k == 0:
            return 1.0 - cs2 - v * v
        return 0.5 * (cs2 + v * v + k * v)

    def equilibrium(r, vx, vy):
        f = np.zeros((9,) + r.shape)
        for b in range(3):
            for a in range(3):
                f[a + 3 * b] = r * feq1d(e[a], vx) * feq1d(e[b], vy)
        return f

    # our velocities are sqrt(3) e with T_L = 1, so lattice-unit velocity v = u / sqrt(3)
    f = equilibrium(rho, ux / math.sqrt(3), uy / math.sqrt(3))
    for _ in range(steps):
        for b in range(3):
            for a in range(3):
                f[a + 3 * b] = np.roll(np.roll(f[a + 3 * b], e[a], axis=1), e[b], axis=0)
        r = f.sum(axis=0)
        vx = sum(e[i % 3] * f[i] for i in range(9)) / r
        vy = sum(e[i // 3] * f[i] for i in range(9)) / r
        f = f + (equilibrium(r, vx, vy) - f) / tau
    return f


def test_d2q9_cfl1_equals_standard_lbm():
    nx, ny, tau, steps = 24, 16, 0.7, 30
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.15, seed=3, drho=0.02)
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=0, tau=tau)
    o = O.Oracle(cfg)
    assert abs(o.dt - 1 / math.sqrt(3)) < 1e-15
    # the reference starts from the post-collision equilibrium of the same fields;
    # the oracle's state is post-collision too
    o.init(rho, u, T)
    o.step(steps)
    ref = standard_d2q9(rho[0], u[0, 0], u[1, 0], tau, steps)
    got = o.get_pops(0).reshape(9, ny, nx)
    assert np.max(np.abs(got - ref)) < 1e-13


def standard_d3q27(rho, u, tau, steps):
    """Textbook D3Q27 stream-and-collide on integer velocities e in {-1,0,1}^3:
    the same 1D equilibrium factors as the D2Q9 reference above, one per axis;
    population index a + 3 b + 9 c for the x, y, z components (a, b, c)."""
    e = [-1, 0, 1]

    def feq1d(k, v):
        cs2 = 1.0 / 3.0
        if k == 0:
            return 1.0 - cs2 - v * v
        return 0.5 * (cs2 + v * v + k * v)

    def equilibrium(r, v):
        f = np.zeros((27,) + r.shape)
        for i in range(27):
            a, b, c = i % 3, (i // 3) % 3, i // 9
            f[i] = r * feq1d(e[a], v[0]) * feq1d(e[b], v[1]) * feq1d(e[c], v[2])
        return f

    f = equilibrium(rho, u / math.sqrt(3))
    for _ in range(steps):
        for i in range(27):
            a, b, c = i % 3, (i // 3) % 3, i // 9
            f[i] = np.roll(f[i], (e[c], e[b], e[a]), axis=(0, 1, 2))
        r = f.sum(axis=0)
        v = np.stack([sum(e[(i // 3 ** ax) % 3] * f[i] for i in range(27)) / r for ax in range(3)])
        f = f + (equilibrium(r, v) - f) / tau
    return f


def test_d3q27_cfl1_equals_standard_lbm():
    """3D counterpart: D3Q27 alone at CFL 1 on a ragged periodic box."""
    nx, ny, nz, tau, steps = 10, 7, 6, 0.8, 12
    rho, u, T = inputs.smooth_random_flow(nx, ny, nz, umax=0.15, seed=5, drho=0.02)
    cfg = inputs.base_config(dim=3, nx=nx, ny=ny, nz=nz, n_low=3, n_high=0, tau=tau)
    o = O.Oracle(cfg)
    assert abs(o.dt - 1 / math.sqrt(3)) < 1e-15
    o.init(rho, u, T)
    o.step(steps)
    ref = standard_d3q27(rho, u, tau, steps)
    got = o.get_pops(0).reshape(27, nz, ny, nx)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("n,thermal", [(3, 0), (4, 0), (6, 0), (3, 1), (4, 1)])
def test_single_lattice_periodic_conservation(n, thermal):
    nx, ny = 20, 14
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=n, drho=0.05,
                                          dT=0.1 if thermal else 0.0)
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=n, n_high=0, tau=0.8, thermal=thermal)
    o = O.Oracle(cfg)
    o.init(rho, u, T)
    c0 = o.conservation()
    o.step(15)
    c1 = o.conservation()
    scale = np.array([c0[0], c0[0], c0[0], 1, c0[4]])
    rel = np.abs(c1 - c0) / scale
    assert rel[0] < 1e-14 and rel[1] < 1e-14 and rel[2] < 1e-14
    if thermal:
        assert rel[4] < 1e-14


@pytest.mark.parametrize("nq,nQ,thermal", [(3, 4, 0), (3, 6, 0), (3, 4, 1)])
def test_uniform_equilibrium_is_fixed_point_for_any_mask(nq, nQ, thermal):
    nx, ny = 16, 12
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.7, thermal=thermal)
    o = O.Oracle(cfg)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=2, blob=3)
    o.set_mask(mask, convert=False)
    rho = np.full((1, ny, nx), 1.1)
    u = np.zeros((2, 1, ny, nx))
    u[0] = 0.23
    u[1] = -0.11
    T = np.full((1, ny, nx), 1.15 if thermal else 1.0)
    o.init(rho, u, T)
    f0 = [o.get_pops(k) for k in range(2)]
    o.step(3)
    for k in range(2):
        assert np.max(np.abs(o.get_pops(k) - f0[k])) < 1e-14


def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-5, 2000),
                        rng.normal(0, 3e4, 200)])
    # exact ties: halfway between neighbouring half-precision values
    h = np.arange(1, 2000, dtype=np.float16).astype(np.float64) / 1024.0
    ties = (h[:-1] + h[1:]) / 2
    v = np.concatenate([v, ties, -ties])
    ref = v.astype(np.float16).astype(np.float64)
    got = np.array([O.round_fp16(x) for x in v])
    assert np.array_equal(got, ref)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    v = rng.normal(0, 1, 20000).astype(np.float32).astype(np.float64)
    base = torch.arange(1, 3000, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    ties = ((base[:-1] + base[1:]) / 2)
    ties = ties[ties.astype(np.float32).astype(np.float64) == ties]
    v = np.concatenate([v, ties, -ties])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.round_bf16(x) for x in v])
    assert np.array_equal(got, ref)


def test_criteria():
    # Mach criterion on a uniform flow and the stress criterion on an equilibrium
    nx, ny = 8, 8
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=4, crit_kind=inputs.CRIT_MA,
                             crit_thr=0.3, crit_every=1)
    o = O.Oracle(cfg)
    rho = np.ones((1, ny, nx))
    u = np.zeros((2, 1, ny, nx))
    u[0, 0, :, : nx // 2] = 0.35
    u[0, 0, :, nx // 2:] = 0.25
    o.init(rho, u)
    m, v = o.eval_criterion()
    assert np.all(m[0, :, : nx // 2] == 1) and np.all(m[0, :, nx // 2:] == 0)
    assert np.allclose(v[0, :, :nx // 2], 0.35, atol=1e-14)
    cfg2 = dict(cfg, crit_kind=inputs.CRIT_PINEQ, crit_thr=1e-3)
    o2 = O.Oracle(cfg2)
    o2.init(rho, u)
    _, v2 = o2.eval_criterion()
    assert np.max(v2) < 1e-14


def test_switching_keeps_state_moments():
    # switching a region to the high order and back leaves the low-order state unchanged
    nx, ny = 12, 10
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, tau=0.7)
    o = O.Oracle(cfg)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=9)
    o.init(rho, u, T)
    o.step(4)  # non-equilibrium state
    f0 = o.get_pops(0)
    m = inputs.random_mask(nx, ny, frac=0.4, seed=4, blob=4)
    o.set_mask(m)
    o.set_mask(np.zeros_like(m))
    assert np.max(np.abs(o.get_pops(0) - f0)) < 1e-14
