"""Pins of the oracle's global constant reference frame (eq. veli) and of the
storage scale of reduced-precision deviations.

- In a frame moving at u_ref, the equilibrium at (u_ref, T_ref) is rho W_i
  exactly (the co-moving equilibrium of eq. feqPond, transferred to a frame
  equal to it).
- D2Q9 in the frame u_ref = (sqrt(3), 0) with dt = 1/sqrt(3) has integer
  departure offsets 0, 1, 2 along x; the step must then equal a textbook
  on-lattice D2Q9 LBM of the flow relative to the frame, shifted one cell per
  step along x (a Galilean shift written out independently below).
- The equilibrium in a shifted and heated frame reproduces the Gaussian's raw
  moments in the particle velocities v = sqrt(T_ref) c + u_ref below the
  lattice order.
- Lifting and projection in a frame keep the low-order raw moments, lift an
  equilibrium to the equilibrium, and project after lifting to the identity.
- The 16-bit storage scale of the storage reference state (rho0, s, T0) is
  rho0 prod_a w_a r(c_a), r the density ratio of N(s_a, T0) to N(0, 1) at the
  node, recomputed here from numpy's Gauss-Hermite rule.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2102_12559_amd import inputs
from tests.test_oracle_step import standard_d2q9


def frame_cfg(**kw):
    cfg = inputs.base_config(**kw)
    cfg.setdefault("u_ref", (0.0, 0.0, 0.0))
    cfg.setdefault("T_ref", 1.0)
    return cfg


def gauss_moment(m, mean, var):
    """E[X^m] for X ~ N(mean, var) by the binomial sum over the even central moments."""
    s = 0.0
    for k in range(0, m + 1, 2):
        s += math.comb(m, k) * mean ** (m - k) * var ** (k // 2) * math.prod(range(1, k, 2))
    return s


def test_frame_equilibrium_at_frame_state_is_weights():
    for n, ur, Tr in ((3, (0.4, -0.2), 1.0), (4, (1.1, 0.3), 1.7), (6, (-0.6, 0.9), 0.8)):
        # T = T_ref needs the thermal model unless T_ref = T_L = 1
        cfg = frame_cfg(nx=4, ny=4, n_low=n, u_ref=ur + (0.0,), T_ref=Tr, thermal=int(Tr != 1.0))
        o = O.Oracle(cfg)
        rho = np.full((1, 4, 4), 1.3)
        u = np.zeros((2, 1, 4, 4))
        u[0], u[1] = ur
        o.init(rho, u, np.full((1, 4, 4), Tr))
        _, w = O.gh_rule(n)
        W = np.array([w[i % n] * w[i // n] for i in range(n * n)])
        f = o.get_pops(0)
        assert np.max(np.abs(f - 1.3 * W[:, None])) < 1e-14


def test_frame_equilibrium_moments():
    """Sum_i f_i v_x^m v_y^k = rho E[(sqrt(T) Z + u_x)^m] E[(sqrt(T) Z + u_y)^k] for
    m, k < n, with v the frame's particle velocities."""
    for n in (3, 4, 5, 6):
        ur, Tr = (0.7, -0.4), 1.6
        cfg = frame_cfg(nx=4, ny=4, n_low=n, thermal=1, cv=1.5, u_ref=ur + (0.0,), T_ref=Tr)
        o = O.Oracle(cfg)
        rho, ux, uy, T = 0.9, 1.2, -0.1, 1.3
        o.init(np.full((1, 4, 4), rho), np.stack([np.full((1, 4, 4), ux), np.full((1, 4, 4), uy)]),
               np.full((1, 4, 4), T))
        f = o.get_pops(0)[:, 0]
        x, _ = O.gh_rule(n)
        vx = np.array([math.sqrt(Tr) * x[i % n] + ur[0] for i in range(n * n)])
        vy = np.array([math.sqrt(Tr) * x[i // n] + ur[1] for i in range(n * n)])
        for m in range(n):
            for k in range(n):
                got = np.sum(f * vx ** m * vy ** k)
                want = rho * gauss_moment(m, ux, T) * gauss_moment(k, uy, T)
                assert abs(got - want) < 1e-11 * max(1.0, abs(want)), (n, m, k, got, want)


def test_shifted_frame_d2q9_is_a_galilean_shift_of_textbook_lbm():
    nx, ny, tau, steps = 24, 12, 0.7, 20
    U = math.sqrt(3.0)
    rho, urel, _ = inputs.smooth_random_flow(nx, ny, umax=0.12, seed=21, drho=0.02)
    u = urel.copy()
    u[0] += U
    # v_x = c + U in {0, sqrt3, 2 sqrt3}: CFL 2 gives dt = 1/sqrt(3), offsets 0, 1, 2
    cfg = frame_cfg(nx=nx, ny=ny, n_low=3, tau=tau, cfl=2.0, u_ref=(U, 0.0, 0.0))
    o = O.Oracle(cfg)
    assert abs(o.dt - 1 / math.sqrt(3)) < 1e-15
    n0, a = o.stencil(0)
    for i in range(9):
        assert n0[i, 0] == -(i % 3) and np.allclose(a[i, 0], [0, 1, 0], atol=1e-15)
    o.init(rho, u)
    o.step(steps)
    ref = standard_d2q9(rho[0], urel[0, 0], urel[1, 0], tau, steps)
    ref = np.roll(ref, steps, axis=2)
    got = o.get_pops(0).reshape(9, ny, nx)
    assert np.max(np.abs(got - ref)) < 1e-13
    r, uu, _ = o.macros()
    rr = ref.sum(axis=0)
    ux_ref = U + math.sqrt(3) * sum((i % 3 - 1) * ref[i] for i in range(9)) / rr
    assert np.max(np.abs(uu[0, 0] - ux_ref)) < 1e-13


def test_lift_and_project_in_a_frame():
    """Two velocity sets sharing the frame u_ref = (0.5, 0.2), T_ref = 1.4: the
    lifted populations keep every low-order raw moment in v and take the
    equilibrium's higher ones; projecting them back returns the input."""
    for nq, nQ in ((3, 4), (3, 6), (4, 5)):
        ur, Tr = (0.5, 0.2), 1.4
        cfg = frame_cfg(nx=4, ny=4, n_low=nq, n_high=nQ, thermal=1, cv=1.5, u_ref=ur + (0.0,),
                        T_ref=Tr)
        o = O.Oracle(cfg)
        x, _ = O.gh_rule(nq)
        X, _ = O.gh_rule(nQ)
        vq = [(math.sqrt(Tr) * x[i % nq] + ur[0], math.sqrt(Tr) * x[i // nq] + ur[1])
              for i in range(nq * nq)]
        vQ = [(math.sqrt(Tr) * X[i % nQ] + ur[0], math.sqrt(Tr) * X[i // nQ] + ur[1])
              for i in range(nQ * nQ)]
        rng = np.random.default_rng(nq * 7 + nQ)
        # a non-equilibrium low-order state: equilibrium of a flow plus noise
        o.init(np.full((1, 4, 4), 1.05), np.stack([np.full((1, 4, 4), 0.3), np.full((1, 4, 4), -0.2)]),
               np.full((1, 4, 4), 1.2))
        fq = o.get_pops(0)[:, 0] * (1 + 0.05 * rng.uniform(-1, 1, nq * nq))
        gq = 0.5 * 1.2 * o.get_pops(0)[:, 0] * (1 + 0.05 * rng.uniform(-1, 1, nq * nq))
        fQ, gQ = o.lift_cell(fq, gq, tile=0)
        for m in range(nq):
            for k in range(nq):
                mq = sum(fq[i] * vq[i][0] ** m * vq[i][1] ** k for i in range(nq * nq))
                mQ = sum(fQ[i] * vQ[i][0] ** m * vQ[i][1] ** k for i in range(nQ * nQ))
                assert abs(mq - mQ) < 1e-12 * max(1.0, abs(mq))
                gm = sum(gq[i] * vq[i][0] ** m * vq[i][1] ** k for i in range(nq * nq))
                gM = sum(gQ[i] * vQ[i][0] ** m * vQ[i][1] ** k for i in range(nQ * nQ))
                assert abs(gm - gM) < 1e-12 * max(1.0, abs(gm))
        # project after lift: the state of the low set again (through the stepper's
        # conversion of a high-order cell)
        mask = np.zeros((1, 4, 4), np.uint8)
        mask[0, 0, 0] = 1
        o.set_mask(mask, convert=False)
        pQ = np.zeros((nQ * nQ, 16))
        pQ[:, 0] = fQ
        o.set_pops(1, pQ)
        gQa = np.zeros((nQ * nQ, 16))
        gQa[:, 0] = gQ
        o.set_pops(1, gQa, fg=1)
        back = o.get_pops(0)[:, 0]
        assert np.max(np.abs(back - fq)) < 1e-13
        assert np.max(np.abs(o.get_pops(0, fg=1)[:, 0] - gq)) < 1e-13
        # an equilibrium lifts to the equilibrium of the high set in the same frame
        st = (np.full((1, 4, 4), 0.95), np.stack([np.full((1, 4, 4), 0.1), np.full((1, 4, 4), 0.6)]),
              np.full((1, 4, 4), 1.1))
        o.set_mask(np.zeros((1, 4, 4), np.uint8), convert=False)
        o.init(*st)
        feq_q, geq_q = o.get_pops(0)[:, 0], o.get_pops(0, fg=1)[:, 0]
        o.set_mask(np.ones((1, 4, 4), np.uint8), convert=False)
        o.init(*st)
        feq_Q, geq_Q = o.get_pops(1)[:, 0], o.get_pops(1, fg=1)[:, 0]
        fl, gl = o.lift_cell(feq_q, geq_q, tile=0)
        assert np.max(np.abs(fl - feq_Q)) < 1e-13 and np.max(np.abs(gl - geq_Q)) < 1e-13


def test_tilted_storage_scale():
    """FP16 storage of a uniform flow with the storage reference velocity set:
    stored = s_i (1 + rne16(f_i / s_i - 1)) with s_i recomputed here."""
    n, su, T0 = 4, (0.45, -0.2), 1.25
    cfg = frame_cfg(nx=4, ny=4, n_low=n, store=inputs.STORE_FP16_DEV, rho0=1.1, T0=T0,
                    store_u=su + (0.0,), thermal=1, cv=1.5)
    o = O.Oracle(cfg)
    u = np.stack([np.full((1, 4, 4), 0.5), np.full((1, 4, 4), -0.15)])
    o.init(np.full((1, 4, 4), 1.02), u, np.full((1, 4, 4), 1.2))
    got = o.get_pops(0)[:, 0]
    z, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / w.sum()

    def ratio(c, m):   # N(m, T0) over N(0, 1) at c
        return math.exp(c * c / 2 - (c - m) ** 2 / (2 * T0)) / math.sqrt(T0)
    s = np.array([1.1 * w[i % n] * ratio(z[i % n], su[0]) * w[i // n] * ratio(z[i // n], su[1])
                  for i in range(n * n)])
    feq = O.lattice_feq(2, n, 1.02, np.array([0.5, -0.15]), 1.2)
    want = s * (1 + (feq / s - 1).astype(np.float16).astype(np.float64))
    assert np.max(np.abs(got - want) / s) < 1e-12
    gs = 0.5 * T0 * s
    want_g = gs * (1 + (0.5 * 1.2 * feq / gs - 1).astype(np.float16).astype(np.float64))
    assert np.max(np.abs(o.get_pops(0, fg=1)[:, 0] - want_g) / gs) < 1e-12
    # the deviations from the carried-over scale are far smaller than from rho0 W_i
    W = np.array([w[i % n] * w[i // n] for i in range(n * n)])
    assert np.max(np.abs(feq / s - 1)) < 0.25 * np.max(np.abs(feq / (1.1 * W) - 1))
