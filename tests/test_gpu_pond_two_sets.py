"""GPU parity of the co-moving frames with two velocity sets (Sec. II.C.1 with
the coupling of Sec. III) against the oracle through the C-ABI.

The GPU converts every band cell into the other set in its own frame after
each step (lifting through the lattice's separable completion matrices with
the equilibria taken in the frame, projection through the Lagrange basis);
the oracle converts each collocation point of the other set on the fly with
the moment matrices at the frame's particle velocities.  Compared: the sets
of the cells (bit for bit), each cell's frame, each set's populations at its
own cells and at the band cells of the other set, FP64 1e-12 (populations
relative to the frame's rho W_i scale)."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs
from tests.gpu_util import band_cells, say, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def pond2_pair(cfg, rho, u, T, mask, steps, tag):
    from paper_2102_12559_amd import msl
    say(f"[case] pond two sets {tag} grid={cfg['nx']}x{cfg['ny']} n=({cfg['n_low']},{cfg['n_high']}) "
        f"thermal={cfg['thermal']} tau2={cfg.get('tau2', 0)} crit={cfg['crit_kind']} steps={steps}")
    t0 = time.time()
    s = msl.Solver(cfg)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(steps)
    s.torch.cuda.synchronize()
    o = O.Pond(cfg)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(steps)
    say(f"  done {time.time() - t0:.2f}s; iterations gpu {s.pond_iterations()} oracle {o.iterations()}")
    return s, o


def compare2(s, o, cfg, periodic, tol=1e-12):
    gm = s.get_mask().cpu().numpy().reshape(-1)
    om = o.get_mask().reshape(-1)
    assert np.array_equal(gm, om), f"sets differ at {int(np.sum(gm != om))} cells"
    fg = s.pond_frames().cpu().numpy()
    ef = float(np.max(np.abs(fg - o.get_frames())))
    b0, b1 = band_cells(gm.reshape(cfg["ny"], cfg["nx"]), periodic)
    rho = o.macros()[0].reshape(-1)
    worst = 0.0
    for which, n, band in ((0, cfg["n_low"], b1), (1, cfg["n_high"], b0)):
        sel = (gm == which) | band
        if not sel.any():
            continue
        W = weights(2, n)
        for g in range(2 if cfg["thermal"] else 1):
            pg = s.get_populations(which, fg=g).cpu().numpy()[:, sel]
            po = o.get_pops(which, g)[:, sel]
            scale = np.maximum(np.abs(po), 0.1 * W[:, None] * rho[None, sel])
            err = float(np.max(np.abs(pg - po) / scale))
            say(f"  set {which} fg {g}: {int((gm == which).sum())} own + {int(band.sum())} band cells, {err:.3e}")
            worst = max(worst, err)
    say(f"  frames {ef:.3e}")
    assert ef < tol and worst < tol, (ef, worst)


@pytest.mark.parametrize("nq,nQ,thermal,tau2", [(3, 4, 0, 0.0), (4, 5, 1, 0.0), (3, 6, 1, 0.9)])
def test_random_mask_advected(nq, nQ, thermal, tau2):
    nx, ny = 40, 24
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.7, thermal=thermal, tau2=tau2,
                             cfl=0.4, pond=1)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.3, seed=nq * 5 + nQ, drho=0.03,
                                          dT=0.05 if thermal else 0.0)
    u[0] += 0.4
    u[1] -= 0.2
    mask = inputs.random_mask(nx, ny, frac=0.35, seed=nQ, blob=5)
    s, o = pond2_pair(cfg, rho, u, T, mask, 6, f"{nq}/{nQ}")
    compare2(s, o, cfg, (True, True))


def test_hermite_lift_zero_gradient_faces():
    nx, ny = 36, 20
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=5, tau=0.65, cfl=0.4, pond=1,
                             lift_mode=inputs.LIFT_GRAD_HERMITE)
    cfg["bc"] = [inputs.BC_OUTFLOW_ZG, inputs.BC_OUTFLOW_ZG, inputs.BC_PERIODIC, inputs.BC_PERIODIC,
                 inputs.BC_PERIODIC, inputs.BC_PERIODIC]
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.3, seed=12, drho=0.03)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=9, blob=4)
    s, o = pond2_pair(cfg, rho, u, T, mask, 5, "hermite zg")
    compare2(s, o, cfg, (False, True))


def test_uniform_flow_fixed_point_on_a_mask():
    nx, ny = 32, 16
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=4, n_high=5, tau=0.7, thermal=1, cfl=0.4, pond=1)
    rho = np.full((1, ny, nx), 1.1)
    u = np.zeros((2, 1, ny, nx))
    u[0], u[1] = 0.8, -0.35
    T = np.full((1, ny, nx), 1.2)
    mask = inputs.random_mask(nx, ny, frac=0.4, seed=2, blob=4)
    s, o = pond2_pair(cfg, rho, u, T, mask, 5, "uniform")
    r, uu, TT = [a.cpu().numpy() for a in s.macros()]
    assert np.max(np.abs(r - 1.1)) < 1e-13 and np.max(np.abs(TT - 1.2)) < 1e-13
    assert np.max(np.abs(uu[0] - 0.8)) < 1e-13 and np.max(np.abs(uu[1] + 0.35)) < 1e-13
    compare2(s, o, cfg, (True, True))


def test_shock_knudsen_criterion_d2q16_d2q25():
    """The paper's shock-structure set-up in co-moving frames: D2Q16 / D2Q25,
    Pr = 2/3 (tau2), hard-sphere viscosity, the Knudsen-number criterion
    every 5 steps at Kn_thr = 0.02."""
    probe = O.Pond(inputs.base_config(nx=4, ny=4, n_low=4, n_high=5, cfl=0.45, pond=1))
    w = inputs.shock_c3(ma1=1.4, nx=160, ny=4, dt=probe.dt, n_high=5)
    cfg = dict(w["cfg"], pond=1, n_low=4, cfl=0.45, crit_kind=inputs.CRIT_KN, crit_thr=0.02,
               crit_every=5)
    cfg["tau2"] = 0.5 + 1.5 * (cfg["tau"] - 0.5)
    s, o = pond2_pair(cfg, w["rho"], w["u"], w["T"], np.zeros((1, 4, 160), np.uint8), 30, "shock Ma 1.4")
    m = s.get_mask().cpu().numpy()
    assert 0 < m.sum() < m.size
    compare2(s, o, cfg, (False, True))
