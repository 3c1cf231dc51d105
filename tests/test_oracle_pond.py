"""Pins of the oracle's co-moving reference frames (PonD, Sec. II.C.1).

- Transfer (eq. fll): G from a frame to itself is the identity; transfers
  compose; the co-moving equilibrium rho W_i (eq. feqPond) transferred to the
  lattice frame is the lattice equilibrium f^L of eq. feqL, computed by the
  oracle's separately pinned product-form routine.
- A uniform flow faster than any lattice speed (D2Q9 at |u| = 1.65) is an
  exact fixed point: every cell keeps rho W_i in the flow's frame and the
  predictor-corrector stops after one pass; likewise thermal D2Q16 at T = 1.3,
  between fixed-equilibrium and zero-gradient faces.
- The paper's claim that the co-moving frame makes the D2Q9 lattice
  compressible: a standing acoustic wave of the thermal D2Q9 model (f and g,
  cv = 3/2, gamma = 5/3) oscillates at the adiabatic sound speed sqrt(gamma T)
  (0.1 %), and advected at U = 0.8 its envelope is the one at rest (Galilean
  invariance, 2 % of the amplitude), while the lattice frame's envelope grows.
- The shear-wave viscosity (tau - 1/2) T dt (Sec. II.B transport
  coefficients) holds at rest and on a flow at U = 1.2 (1 % on 96 cells per
  wavelength; the interpolation adds 1 % at 48).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def lat_feq(n, rho, u, T):
    out = np.zeros(n * n)
    uu = np.array([u[0], u[1], 0.0])
    O.lib().or_lattice_feq(2, n, rho, O._p(uu), T, O._p(out))
    return out


@pytest.mark.parametrize("n", [3, 4, 5])
def test_transfer_identities(n):
    rng = np.random.default_rng(n)
    Q = n * n
    f = 0.1 + rng.random(Q)
    a = (0.3, -0.2, 0.0, 1.1)
    b = (-0.5, 0.4, 0.0, 0.8)
    c = (0.9, 0.1, 0.0, 1.4)
    assert np.max(np.abs(O.pond_transfer(2, n, a, a, f) - f)) < 1e-14
    ab = O.pond_transfer(2, n, a, b, f)
    assert np.max(np.abs(O.pond_transfer(2, n, b, c, ab) - O.pond_transfer(2, n, a, c, f))) < 1e-12
    W = lat_feq(n, 1.0, (0.0, 0.0), 1.0)          # the weights
    for rho, u, T in ((1.2, (0.3, -0.4), 1.0), (0.9, (0.6, 0.2), 1.3)):
        fl = O.pond_transfer(2, n, (u[0], u[1], 0.0, T), (0.0, 0.0, 0.0, 1.0), rho * W)
        assert np.max(np.abs(fl - lat_feq(n, rho, u, T))) < 1e-13


@pytest.mark.parametrize("case", ["d2q9", "d2q16-thermal-faces"])
def test_uniform_flow_fixed_point(case):
    nx, ny = 12, 6
    if case == "d2q9":
        u0, T0 = (1.5, -0.7), 1.0
        cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, tau=0.7, cfl=0.4)
    else:
        u0, T0 = (0.9, 0.4), 1.3
        state = [1.1, u0[0], u0[1], 0.0, T0]
        cfg = inputs.base_config(nx=nx, ny=ny, n_low=4, tau=0.7, cfl=0.4, thermal=1, cv=1.5,
                                 bc=[inputs.BC_FIXED_EQ, inputs.BC_OUTFLOW_ZG] + [inputs.BC_PERIODIC] * 4)
        cfg["bc_state"][0] = state
    p = O.Pond(cfg)
    rho = np.full((1, ny, nx), 1.1)
    u = np.zeros((2, 1, ny, nx))
    u[0], u[1] = u0
    p.init(rho, u, np.full((1, ny, nx), T0))
    p.step(5)
    r, uu, TT = p.macros()
    assert np.max(np.abs(r - 1.1)) < 1e-14
    assert np.max(np.abs(uu[0] - u0[0])) < 1e-14 and np.max(np.abs(uu[1] - u0[1])) < 1e-14
    assert np.max(np.abs(TT - T0)) < 1e-14
    fr = p.get_frames()
    assert np.max(np.abs(fr[0] - u0[0])) < 1e-14 and np.max(np.abs(fr[3] - T0)) < 1e-14
    assert p.iterations()[1] == 1


def acoustic_envelope(cls, U, N=64, steps=300, every=5):
    eps, cv = 1e-3, 1.5
    gam = (cv + 1) / cv
    cfg = inputs.base_config(nx=N, ny=2, n_low=3, tau=0.6, cfl=0.5, thermal=1, cv=cv)
    o = cls(cfg)
    k = 2 * np.pi / N
    x = np.arange(N)[None, None, :].repeat(2, axis=1).astype(float)
    u = np.zeros((2, 1, 2, N))
    u[0] = U
    o.init(1 + eps * np.cos(k * x), u, 1 + (gam - 1) * eps * np.cos(k * x))
    ts, amp = [], []
    for s in range(0, steps + 1, every):
        if s:
            o.step(every)
        r = o.macros()[0][0, 0]
        ts.append(s * o.dt)
        amp.append(np.fft.rfft(r)[1] * 2 / N)
    return np.array(ts), np.array(amp), k, gam, eps


def test_acoustic_speed_and_galilean_invariance():
    from scipy.optimize import curve_fit
    ts, a0, k, gam, eps = acoustic_envelope(O.Pond, 0.0)
    fit = lambda t, A, w, g, ph: A * np.cos(w * t + ph) * np.exp(-g * t)
    popt, _ = curve_fit(fit, ts, a0.real, p0=[eps, math.sqrt(gam) * k, 1e-3, 0.0])
    assert abs(popt[1] / k / math.sqrt(gam) - 1) < 1e-3
    _, a1, _, _, _ = acoustic_envelope(O.Pond, 0.8)
    assert np.max(np.abs(np.abs(a1) - np.abs(a0))) < 0.02 * eps
    _, al, _, _, _ = acoustic_envelope(O.Oracle, 0.8)
    assert np.max(np.abs(al)) > 1.2 * eps     # the lattice frame is not Galilean invariant here


def shear_nu(U, n=3, tau=0.8, N=96, steps=300, every=50):
    cfg = inputs.base_config(nx=N, ny=2, n_low=n, tau=tau, cfl=0.4)
    p = O.Pond(cfg)
    k = 2 * np.pi / N
    x = np.arange(N)[None, None, :].repeat(2, axis=1).astype(float)
    u = np.zeros((2, 1, 2, N))
    u[0] = U
    u[1] = 1e-3 * np.sin(k * x)
    p.init(np.ones((1, 2, N)), u)
    ts, amps = [], []
    for s in range(0, steps + 1, every):
        if s:
            p.step(every)
        uy = p.macros()[1][1, 0, 0]
        ts.append(s * p.dt)
        amps.append(abs(np.fft.rfft(uy)[1]))
    slope = np.polyfit(np.array(ts[1:]), np.log(np.array(amps[1:])), 1)[0]
    return -slope / k ** 2 / ((tau - 0.5) * p.dt)


@pytest.mark.parametrize("U", [0.0, 1.2])
def test_shear_viscosity(U):
    assert abs(shear_nu(U) - 1) < 0.01
