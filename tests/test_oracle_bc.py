"""Pins of the oracle's relaxation time, thermal collision and boundary rules.

- a decaying shear wave loses amplitude at the rate nu k^2 with the kinematic
  viscosity nu = (tau - 1/2) T dt of the transport coefficients (Sec. II.B,
  mu = (1/omega - 1/2) rho R T dt), also with the temperature-dependent
  viscosity mu ~ T^s of the hard-sphere model (Sec. IV.A.3);
- a uniform state equal to a fixed-equilibrium face state, or any uniform state
  with zero-gradient faces, is a fixed point of the step.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def shear_decay_rate(cfg, T0=1.0, steps=200):
    nx, ny = cfg["nx"], cfg["ny"]
    A = 1e-3
    x = np.arange(nx)
    rho = np.ones((1, ny, nx))
    u = np.zeros((2, 1, ny, nx))
    u[1] = A * np.sin(2 * math.pi * x / nx)[None, None, :]
    T = np.full((1, ny, nx), T0)
    o = O.Oracle(cfg)
    o.init(rho, u, T)
    s = np.sin(2 * math.pi * x / nx)

    def amp():
        uy = o.macros()[1][1, 0].mean(axis=0)
        return 2 * np.mean(uy * s)

    o.step(20)  # let the initial non-equilibrium transient relax
    a0 = amp()
    o.step(steps)
    a1 = amp()
    k = 2 * math.pi / nx
    return -math.log(a1 / a0) / (steps * o.dt) / (k * k), o.dt


@pytest.mark.parametrize("n", [3, 4, 6])
def test_shear_wave_viscosity(n):
    tau = 0.9
    cfg = inputs.base_config(nx=48, ny=4, n_low=n, n_high=0, tau=tau)
    nu, dt = shear_decay_rate(cfg)
    ref = (tau - 0.5) * dt
    assert abs(nu - ref) < 0.02 * ref, (nu, ref)


def test_shear_wave_viscosity_hard_sphere_thermal():
    # mu = mu_ref (T/T_ref)^0.5 with tau_ref at (rho, T) = (1, 1); run at T = 1.6
    tau_ref, T0 = 0.9, 1.6
    cfg = inputs.base_config(nx=48, ny=4, n_low=4, n_high=0, tau=tau_ref, thermal=1,
                             tau_mode=1, mu_exp=0.5, tau_ref_rho=1.0, tau_ref_T=1.0)
    nu, dt = shear_decay_rate(cfg, T0=T0)
    mu = (tau_ref - 0.5) * 1.0 * 1.0 * dt * (T0 / 1.0) ** 0.5
    assert abs(nu - mu) < 0.02 * mu, (nu, mu)


def test_fixed_equilibrium_faces_hold_uniform_state():
    st = [1.2, 0.15, -0.05, 0.0, 1.1]
    cfg = inputs.base_config(nx=12, ny=10, n_low=3, n_high=4, thermal=1, tau=0.7)
    cfg["bc"] = [inputs.BC_FIXED_EQ] * 4 + [0, 0]
    cfg["bc_state"] = [list(st) for _ in range(6)]
    o = O.Oracle(cfg)
    o.set_mask(inputs.random_mask(12, 10, frac=0.3, seed=1, blob=3), convert=False)
    rho = np.full((1, 10, 12), st[0])
    u = np.zeros((2, 1, 10, 12))
    u[0], u[1] = st[1], st[2]
    T = np.full((1, 10, 12), st[4])
    o.init(rho, u, T)
    f0 = o.get_pops(0)
    o.step(3)
    assert np.max(np.abs(o.get_pops(0) - f0)) < 1e-14


def test_zero_gradient_faces_hold_uniform_state():
    cfg = inputs.base_config(nx=12, ny=10, n_low=3, n_high=6, tau=0.7)
    cfg["bc"] = [inputs.BC_OUTFLOW_ZG] * 4 + [0, 0]
    o = O.Oracle(cfg)
    o.set_mask(inputs.random_mask(12, 10, frac=0.3, seed=2, blob=3), convert=False)
    rho = np.full((1, 10, 12), 0.9)
    u = np.zeros((2, 1, 10, 12))
    u[0] = 0.2
    o.init(rho, u)
    f0 = o.get_pops(1)
    o.step(3)
    assert np.max(np.abs(o.get_pops(1) - f0)) < 1e-14


def test_inlet_slot_injects_momentum_only_through_slot():
    w = inputs.jet_c2(nx=32, ny=24, slot_w=6, ma=0.3, tau=0.6, store=inputs.STORE_FP64,
                      crit_every=0)
    cfg = dict(w["cfg"], crit_kind=0)
    o = O.Oracle(cfg)
    o.init(w["rho"], w["u"], w["T"])
    o.step(6)
    rho, u, T = o.macros()
    lo = 24 // 2 - 3
    ux0 = u[0, 0, :, 0]
    assert np.all(ux0[lo:lo + 6] > 0.02)
    far = np.r_[0:lo - 4, lo + 10:24]
    assert np.max(np.abs(ux0[far])) < 0.02
