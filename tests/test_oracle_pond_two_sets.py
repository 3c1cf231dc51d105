"""Pins of the oracle's co-moving frames with two velocity sets (Sec. II.C.1
with the coupling of Sec. III).

- A two-set context whose cells all use the high-order set is the single-set
  step of that set, bit for bit (same dt: the larger set sets it).
- Lifting in a cell's own frame keeps every moment of the low-order set
  (per-axis degree below n_q, with the frame's particle velocities), and
  projection keeps those moments of the high-order state (Sec. III.B-C).
- A uniform flow is an exact fixed point on a random mask: every cell's state
  is the co-moving equilibrium, which lifting, projection and the transfer
  reproduce exactly.
- The Knudsen-number criterion of the co-moving state selects the same cells
  as the static oracle's criterion on the same fields (at the initial state
  both hold the same equilibria), and the Mach-1.4 shock with D2Q16 / D2Q25
  keeps its Rankine-Hugoniot end states far from the shock.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def frame_moments(f, fr, n, pw):
    """sum_i f_i v_ix^p v_iy^q with v = sqrt(T) c + u of each cell's frame"""
    x, _ = O.gh_rule(n)
    Q = n * n
    a = np.arange(Q) % n
    b = np.arange(Q) // n
    sT = np.sqrt(fr[3])
    vx = sT[None, :] * x[a][:, None] + fr[0][None, :]
    vy = sT[None, :] * x[b][:, None] + fr[1][None, :]
    return np.array([np.sum(f * vx ** p * vy ** q, axis=0) for p, q in pw])


def run(cfg, rho, u, T, mask, steps):
    p = O.Pond(cfg)
    p.set_mask(mask, convert=False)
    p.init(rho, u, T)
    p.step(steps)
    return p


def test_all_high_is_the_single_set_step():
    nx, ny = 24, 10
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.4, seed=3, drho=0.03, dT=0.05)
    two = inputs.base_config(nx=nx, ny=ny, n_low=4, n_high=5, tau=0.7, thermal=1, cfl=0.5, pond=1)
    one = inputs.base_config(nx=nx, ny=ny, n_low=5, tau=0.7, thermal=1, cfl=0.5, pond=1)
    a = run(two, rho, u, T, np.ones((1, ny, nx), np.uint8), 4)
    b = run(one, rho, u, T, np.zeros((1, ny, nx), np.uint8), 4)
    assert a.dt == b.dt
    for fg in (0, 1):
        assert np.array_equal(a.get_pops(1, fg), b.get_pops(0, fg))
    assert np.array_equal(a.get_frames(), b.get_frames())


@pytest.mark.parametrize("nq,nQ", [(3, 4), (4, 5), (3, 6)])
def test_conversion_keeps_the_low_order_moments(nq, nQ):
    nx, ny = 20, 12
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.65, thermal=1, cfl=0.5, pond=1)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.5, seed=nq + nQ, drho=0.04, dT=0.08)
    mask = inputs.random_mask(nx, ny, frac=0.4, seed=7, blob=4)
    p = run(cfg, rho, u, T, mask, 3)    # non-equilibrium states after three steps
    fr = p.get_frames()
    m = p.get_mask().reshape(-1)
    pw = [(i, j) for j in range(nq) for i in range(nq)]
    for fg in (0, 1):
        lo, hi = p.get_pops(0, fg), p.get_pops(1, fg)
        ml, mh = frame_moments(lo, fr, nq, pw), frame_moments(hi, fr, nQ, pw)
        scale = np.maximum(np.abs(ml), 1e-3)
        err = np.max(np.abs(mh - ml) / scale)
        assert err < 1e-11, (fg, err)
        # the two sets hold different states: the conversion is not the identity
        assert np.max(np.abs(hi[:, m == 0])) > 0 and np.max(np.abs(lo[:, m == 1])) > 0


def test_uniform_flow_fixed_point_on_a_mask():
    nx, ny = 16, 10
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=4, n_high=5, tau=0.7, thermal=1, cfl=0.5, pond=1)
    u0, T0 = (0.8, -0.35), 1.2
    rho = np.full((1, ny, nx), 1.1)
    u = np.zeros((2, 1, ny, nx))
    u[0], u[1] = u0
    T = np.full((1, ny, nx), T0)
    mask = inputs.random_mask(nx, ny, frac=0.4, seed=2, blob=4)
    p = run(cfg, rho, u, T, mask, 5)
    r, uu, TT = p.macros()
    assert np.max(np.abs(r - 1.1)) < 1e-13
    assert np.max(np.abs(uu[0] - u0[0])) < 1e-13 and np.max(np.abs(uu[1] - u0[1])) < 1e-13
    assert np.max(np.abs(TT - T0)) < 1e-13
    assert np.array_equal(p.get_mask(), mask.reshape(p.get_mask().shape))


def test_knudsen_selection_matches_the_static_criterion_and_shock_holds():
    probe = O.Pond(inputs.base_config(nx=4, ny=4, n_low=4, n_high=5, cfl=0.45, pond=1))
    w = inputs.shock_c3(ma1=1.4, nx=160, ny=4, dt=probe.dt, n_high=5)
    cfg = dict(w["cfg"], pond=1, n_low=4, cfl=0.45, crit_kind=inputs.CRIT_KN, crit_thr=0.02,
               crit_every=10)
    zero = np.zeros((1, 4, 160), np.uint8)
    st = O.Oracle(dict(cfg, pond=0))
    st.set_mask(zero, convert=False)
    st.init(w["rho"], w["u"], w["T"])
    ref = st.eval_criterion()[0].reshape(-1)
    p = O.Pond(cfg)
    assert p.dt == st.dt
    p.set_mask(zero, convert=False)
    p.init(w["rho"], w["u"], w["T"])
    p.step(1)                            # the criterion pass of step 0
    got = p.get_mask().reshape(-1)
    assert got.sum() > 0 and np.array_equal(got, ref)
    p.step(39)
    r, uu, TT = p.macros()
    r = r.reshape(4, 160)
    assert np.all(np.isfinite(r))
    # the end states hold far from the shock (the faces give them exactly)
    assert np.max(np.abs(r[:, :8] - w["rho"].reshape(4, 160)[:, :8])) < 1e-6
    assert np.max(np.abs(r[:, -8:] - w["rho"].reshape(4, 160)[:, -8:])) < 1e-6
    m = p.get_mask().reshape(4, 160)
    assert 0 < m.sum() < m.size
