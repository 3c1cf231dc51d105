"""Closed-form pins of oracle parts that the parity tests alone cannot fix.

- The |Pi_neq|_F / p criterion on a state whose non-equilibrium central
  second moment is set by hand: sqrt(2 d^2 + 2 e^2) / (rho T) for an
  off-diagonal deviation d and a traceless diagonal deviation (e, -e).
- The learned closure's per-tile error check against errors computed by hand:
  a constant-output network (only the last bias non-zero) and high-order band
  cells whose missing-moment non-equilibrium parts are set exactly, so each
  tile's network and Grad errors are sums of |c - t|^2 and |t|^2; ties go to
  Grad lifting, and tiles without band cells follow the domain totals.
- The Rankine-Hugoniot end states of the shock inputs against the textbook
  jump ratios for gamma = 5/3 and against the conservation of mass,
  momentum and energy fluxes across the jump.
- App. A: the coupled D2Q9 / D2Q25 scheme (D2Q25 on a central disk) is second
  order in L2 on the Taylor-Green vortex (diffusive scaling: U ~ 1/N, steps
  ~ N^2), as is D2Q9 alone.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def moment_matrix_np(n, dim=2):
    """M[j][i] = prod_a c_ia^{p_a(j)}, nodes from numpy's Gauss-Hermite rule."""
    z, _ = np.polynomial.hermite_e.hermegauss(n)
    Q = n ** dim
    M = np.zeros((Q, Q))
    for j in range(Q):
        pj = [(j // n ** a) % n for a in range(dim)]
        for i in range(Q):
            pi = [(i // n ** a) % n for a in range(dim)]
            M[j, i] = np.prod([z[pi[a]] ** pj[a] for a in range(dim)])
    return M


def moment_index(n, px, py):
    return px + n * py


@pytest.mark.parametrize("thermal,T", [(0, 1.0), (1, 1.7)])
def test_pineq_criterion_closed_form(thermal, T):
    rho, u = 1.3, (0.25, -0.15)
    d, e = 0.021, -0.013
    cfg = inputs.base_config(nx=4, ny=4, n_low=3, n_high=6, thermal=thermal, cv=1.5,
                             crit_kind=inputs.CRIT_PINEQ, crit_thr=1e-3)
    o = O.Oracle(cfg)
    o.init(np.full((1, 4, 4), rho), np.stack([np.full((1, 4, 4), u[0]), np.full((1, 4, 4), u[1])]),
           np.full((1, 4, 4), T))
    f = o.get_pops(0)
    M = moment_matrix_np(3)
    delta = np.zeros(9)
    delta[moment_index(3, 1, 1)] = d          # Pi_xy
    delta[moment_index(3, 2, 0)] = e          # Pi_xx, and -e on Pi_yy: energy kept
    delta[moment_index(3, 0, 2)] = -e
    df = np.linalg.solve(M, delta)
    f = f + df[:, None]
    o.set_pops(0, f)
    _, val = o.eval_criterion()
    want = math.sqrt(2 * d * d + 2 * e * e) / (rho * T)
    assert np.max(np.abs(val - want)) < 1e-12 * want
    # the Mach criterion of the same state is unchanged by the stress deviation
    o2 = O.Oracle(dict(cfg, crit_kind=inputs.CRIT_MA))
    o2.init(np.full((1, 4, 4), rho), np.stack([np.full((1, 4, 4), u[0]), np.full((1, 4, 4), u[1])]),
            np.full((1, 4, 4), T))
    o2.set_pops(0, f)
    _, ma = o2.eval_criterion()
    cs = math.sqrt(5.0 / 3.0 * T) if thermal else 1.0
    assert np.max(np.abs(ma - math.hypot(*u) / cs)) < 1e-13


def _closure_case(scenarios, c):
    """Grid 128 x 128 (four 64 x 64 check tiles), D2Q9 / D2Q16, constant network
    output c.  scenarios: {tile: (x0, y0, w, h, s)} puts a w x h block of
    high-order cells at (x0, y0) whose missing-moment targets are s * c (s = None:
    an equilibrium state, targets 0).  Returns the oracle's flags, E_mlp, E_grad
    and the hand-computed ones."""
    N, nq, nQ = 128, 3, 4
    cfg = inputs.base_config(nx=N, ny=N, n_low=nq, n_high=nQ, tau=0.7, lift_mode=inputs.LIFT_MLP)
    o = O.Oracle(cfg)
    F, Ot = O.mlp_dims(2, nq, nQ)
    H = 8
    P = O.mlp_nparams(F, H, Ot)
    params = np.zeros(P)
    params[P - Ot:] = c
    mask = np.zeros((1, N, N), np.uint8)
    for (x0, y0, w, h, _) in scenarios.values():
        mask[0, y0:y0 + h, x0:x0 + w] = 1
    o.set_mask(mask, convert=False)
    rho = np.full((1, N, N), 1.02)
    u = np.stack([np.full((1, N, N), 0.12), np.full((1, N, N), -0.07)])
    o.init(rho, u)
    fQ = o.get_pops(1)
    MQ = moment_matrix_np(nQ)
    missing = [j for j in range(nQ * nQ) if j % nQ >= nq or j // nQ >= nq]
    assert len(missing) == Ot
    want_m = np.zeros(4)
    want_g = np.zeros(4)
    has = np.zeros(4, bool)
    for t, (x0, y0, w, h, s) in scenarios.items():
        targ = np.zeros(Ot) if s is None else s * np.asarray(c)
        delta = np.zeros(nQ * nQ)
        delta[missing] = 1.02 * targ          # rho T^{|p|/2} t with T = 1
        df = np.linalg.solve(MQ, delta)
        for yy in range(y0, y0 + h):
            for xx in range(x0, x0 + w):
                fQ[:, yy * N + xx] += df
        ncell = w * h                          # blocks at most 4 cells thick: all border cells
        want_m[t] += ncell * np.sum((np.asarray(c) - targ) ** 2)
        want_g[t] += ncell * np.sum(targ ** 2)
        has[t] = True
    o.set_pops(1, fQ)
    o.set_mlp(H, params, np.zeros(F), np.ones(F), np.zeros(Ot), np.ones(Ot), bf16=False,
              manual_check=True)
    o.mlp_check()
    flags, em, eg = o.mlp_flags()
    want_f = np.where(has, want_m < want_g, want_m.sum() < want_g.sum()).astype(np.uint8)
    return flags, em, eg, want_f, want_m, want_g


def test_closure_check_by_hand():
    c = np.array([0.03, -0.02, 0.05, 0.01, -0.04, 0.02, 0.015])
    # tile 0: targets = network output; tile 1: targets = -output;
    # tile 2: equilibrium (targets 0); tile 3: no band cells
    sc = {0: (10, 10, 20, 4, 1.0), 1: (80, 20, 3, 4, -1.0), 2: (20, 90, 4, 3, None)}
    flags, em, eg, wf, wm, wg = _closure_case(sc, c)
    assert list(wf) == [1, 0, 0, 1]           # tile 3: totals 0*80+4*12+1*12 < 80+12
    assert np.array_equal(flags, wf)
    assert np.allclose(em, wm, rtol=1e-9, atol=1e-15)
    assert np.allclose(eg, wg, rtol=1e-9, atol=1e-15)
    # fewer matching cells: the totals now favour Grad in the empty tile
    sc[0] = (10, 10, 2, 4, 1.0)
    flags, em, eg, wf, wm, wg = _closure_case(sc, c)
    assert list(wf) == [1, 0, 0, 0]
    assert np.array_equal(flags, wf)


def test_closure_check_ties_go_to_grad():
    """A zero network on equilibrium band cells: both errors are the same sum
    (of rounding-level targets) in every tile, and every tile keeps Grad."""
    c = np.zeros(7)
    sc = {0: (10, 10, 4, 4, None), 1: (80, 20, 3, 4, None)}
    flags, em, eg, _, _, _ = _closure_case(sc, c)
    assert np.array_equal(em, eg)
    assert list(flags) == [0, 0, 0, 0]


TEXTBOOK_RH = {1.4: (1.5806, 1.3918), 2.0: (2.2857, 2.0781), 3.0: (3.0000, 3.6667)}


@pytest.mark.parametrize("ma", sorted(TEXTBOOK_RH))
def test_rankine_hugoniot_inputs(ma):
    g = 5.0 / 3.0
    s = inputs.rankine_hugoniot(ma, g)
    r, t = TEXTBOOK_RH[ma]
    assert abs(s["rho2"] / s["rho1"] - r) < 6e-5
    assert abs(s["T2"] / s["T1"] - t) < 6e-5
    # fluxes across the jump (p = rho T, enthalpy g/(g-1) T)
    m1, m2 = s["rho1"] * s["u1"], s["rho2"] * s["u2"]
    assert abs(m1 - m2) < 1e-12 * m1
    p1, p2 = s["rho1"] * s["T1"], s["rho2"] * s["T2"]
    assert abs(m1 * s["u1"] + p1 - (m2 * s["u2"] + p2)) < 1e-12 * p2
    h1 = g / (g - 1) * s["T1"] + 0.5 * s["u1"] ** 2
    h2 = g / (g - 1) * s["T2"] + 0.5 * s["u2"] ** 2
    assert abs(h1 - h2) < 1e-12 * h1
    assert abs(s["u1"] - ma * math.sqrt(g * s["T1"])) < 1e-14


def taylor_green_error(N, disk, U16=0.04, s16=40, tau=0.8):
    """Relative L2 error of the velocity against the decaying Taylor-Green
    vortex u = U (sin kx cos ky, -cos kx sin ky) exp(-2 nu k^2 t), nu = (tau - 1/2) dt,
    with D2Q25 on the disk of radius N/4 (or nowhere)."""
    U = U16 * 16 / N
    steps = s16 * (N // 16) ** 2
    k = 2 * math.pi / N
    y, x = np.mgrid[0:N, 0:N].astype(float)
    ux = U * np.sin(k * x) * np.cos(k * y)
    uy = -U * np.cos(k * x) * np.sin(k * y)
    rho = 1 - U * U / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    o = O.Oracle(inputs.base_config(nx=N, ny=N, n_low=3, n_high=5, tau=tau))
    mask = ((x - N / 2) ** 2 + (y - N / 2) ** 2 <= (N / 4) ** 2).astype(np.uint8)[None]
    if not disk:
        mask[:] = 0
    o.set_mask(mask, convert=False)
    o.init(rho[None], np.stack([ux[None], uy[None]]))
    o.step(steps)
    dec = math.exp(-2 * (tau - 0.5) * o.dt * k * k * steps * o.dt)
    _, u, _ = o.macros()
    num = np.sum((u[0, 0] - ux * dec) ** 2) + np.sum((u[1, 0] - uy * dec) ** 2)
    return math.sqrt(num / ((np.sum(ux ** 2) + np.sum(uy ** 2)) * dec * dec))


@pytest.mark.parametrize("disk", [False, True])
def test_taylor_green_second_order(disk):
    e = [taylor_green_error(N, disk) for N in (16, 32, 64)]
    slopes = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.8 < s < 2.3 for s in slopes), (e, slopes)
