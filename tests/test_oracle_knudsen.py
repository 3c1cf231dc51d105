"""Pins of the oracle's Knudsen-number criterion (Sec. IV.A.3: Kn = lambda / L,
L = |phi / (dphi/dx)| with phi the density, refinement where Kn exceeds the
threshold; lambda the hard-sphere mean free path of the same section).

Each pin sets a density field whose discrete gradient and mean free path are
known in closed form and compares the criterion value of every cell:
- a periodic sine: the central difference of sin(kx) is sin(k) cos(kx);
- a linear ramp between non-periodic faces: every difference, one-sided at
  the faces included, is the slope;
- a plane in 2D and a ramp along z in 3D: |grad rho| is the slopes' norm;
- the thermal hard-sphere gas (mu ~ T^0.5): the mean free path from the
  section's formula lambda = 16/(5 sqrt(2 pi gamma)) mu a / p with
  a = sqrt(gamma T), p = rho T and mu = mu_1 (T/T_1)^0.5, mu_1 the viscosity
  (tau - 1/2) rho_1 T_1 dt of the reference state;
- the mask flags exactly the cells above the threshold.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs

GAM = 5.0 / 3.0


def lam_hs(mu, rho, T):
    """hard-sphere mean free path as printed in Sec. IV.A.3"""
    return 16.0 / (5.0 * math.sqrt(2 * math.pi * GAM)) * mu * np.sqrt(GAM * T) / (rho * T)


def criterion(cfg, rho, u, T):
    o = O.Oracle(cfg)
    o.init(rho, u, T)
    return o, o.eval_criterion()


@pytest.mark.parametrize("nq", [3, 4])
def test_periodic_sine(nq):
    N, A, tau = 48, 0.05, 0.8
    cfg = inputs.base_config(nx=N, ny=4, n_low=nq, n_high=nq + 1, tau=tau, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.02)
    x = np.arange(N)[None, None, :].repeat(4, axis=1).astype(float)
    rho = 1 + A * np.sin(2 * np.pi * x / N)
    o, (m, v) = criterion(cfg, rho, np.zeros((2, 1, 4, N)), np.ones((1, 4, N)))
    mu = (tau - 0.5) * rho * 1.0 * o.dt
    want = lam_hs(mu, rho, 1.0) * np.abs(A * np.sin(2 * np.pi / N) * np.cos(2 * np.pi * x / N)) / rho
    assert np.max(np.abs(v - want)) < 1e-15
    assert np.max(v) > 5e-4   # not a trivially small field


def test_linear_ramp_open_faces():
    N, s, tau = 40, 0.01, 0.7
    cfg = inputs.base_config(nx=N, ny=3, n_low=3, n_high=4, tau=tau, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.02, bc=[inputs.BC_OUTFLOW_ZG] * 2 + [inputs.BC_PERIODIC] * 4)
    x = np.arange(N)[None, None, :].repeat(3, axis=1).astype(float)
    rho = 1 + s * x
    o, (m, v) = criterion(cfg, rho, np.zeros((2, 1, 3, N)), np.ones((1, 3, N)))
    want = lam_hs((tau - 0.5) * rho * o.dt, rho, 1.0) * s / rho
    assert np.max(np.abs(v - want)) < 1e-15


def test_plane_2d_and_ramp_3d():
    nx, ny, a, b, tau = 20, 16, 0.004, -0.003, 0.9
    open4 = [inputs.BC_OUTFLOW_ZG] * 4 + [inputs.BC_PERIODIC] * 2
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=4, tau=tau, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.02, bc=open4)
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    rho = (1 + a * x + b * y)[None].astype(float)
    o, (m, v) = criterion(cfg, rho, np.zeros((2, 1, ny, nx)), np.ones((1, ny, nx)))
    want = lam_hs((tau - 0.5) * rho * o.dt, rho, 1.0) * math.hypot(a, b) / rho
    assert np.max(np.abs(v - want)) < 1e-15
    # 3D: a ramp along z between open z faces, periodic x and y
    n, c = 6, 0.02
    cfg3 = inputs.base_config(dim=3, nx=n, ny=n, nz=n, n_low=3, n_high=4, tau=tau,
                              crit_kind=inputs.CRIT_KN, crit_thr=0.02,
                              bc=[inputs.BC_PERIODIC] * 4 + [inputs.BC_OUTFLOW_ZG] * 2)
    z = np.arange(n)[:, None, None] * np.ones((n, n, n))
    rho3 = 1 + c * z
    o3, (m3, v3) = criterion(cfg3, rho3, np.zeros((3, n, n, n)), np.ones((n, n, n)))
    want3 = lam_hs((tau - 0.5) * rho3 * o3.dt, rho3, 1.0) * c / rho3
    assert np.max(np.abs(v3 - want3)) < 1e-15


def test_hard_sphere_thermal_mean_free_path():
    N, tau, rho1, T1 = 32, 3.0, 1.0, 1.0
    cfg = inputs.base_config(nx=N, ny=2, n_low=4, n_high=5, tau=tau, thermal=1, cv=1.5, tau_mode=1,
                             mu_exp=0.5, tau_ref_rho=rho1, tau_ref_T=T1, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.02)
    x = np.arange(N)[None, None, :].repeat(2, axis=1).astype(float)
    T = 1 + 0.3 * np.cos(2 * np.pi * x / N)
    rho = 1.2 + 0.1 * np.sin(2 * np.pi * x / N)
    o, (m, v) = criterion(cfg, rho, np.zeros((2, 1, 2, N)), T)
    # the oracle's own macros of the initial state (the equilibrium moments
    # reproduce rho and T to rounding)
    mu = (tau - 0.5) * rho1 * T1 * o.dt * (T / T1) ** 0.5
    drho = 0.1 * np.sin(2 * np.pi / N) * np.cos(2 * np.pi * x / N)
    want = lam_hs(mu, rho, T) * np.abs(drho) / rho
    assert np.max(np.abs(v - want)) < 1e-13 * np.max(want)


def test_mask_is_threshold():
    N = 40
    cfg = inputs.base_config(nx=N, ny=2, n_low=3, n_high=4, tau=0.8, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.0, bc=[inputs.BC_OUTFLOW_ZG] * 2 + [inputs.BC_PERIODIC] * 4)
    x = np.arange(N)[None, None, :].repeat(2, axis=1).astype(float)
    rho = 1 + 0.5 * np.tanh((x - N / 2) / 2.0)
    o = O.Oracle(cfg)
    o.init(rho, np.zeros((2, 1, 2, N)), np.ones((1, 2, N)))
    _, v = o.eval_criterion()
    thr = float(np.median(v))
    o2 = O.Oracle(dict(cfg, crit_thr=thr))
    o2.init(rho, np.zeros((2, 1, 2, N)), np.ones((1, 2, N)))
    m, v2 = o2.eval_criterion()
    assert np.array_equal(v, v2)
    assert np.array_equal(m, (v > thr).astype(np.uint8))
    assert 0 < m.sum() < m.size
