"""Band conversion inside the stream-collide launches (2D two-set contexts)
and the graph launch modes of msl_step.

The low-order launch lifts its band cells into the high-order set and the
high-order launch projects its band cells into the low-order set (Sec. III.B-C,
App. C), from the post-collision populations they hold.  Each set's values at
the band cells of the other order are compared with the oracle, which lifts or
projects those cells' native state when asked for them.  The graph modes
replay the same launches: the state after a run must match launch-by-launch
execution bit for bit.
"""
import numpy as np
import pytest

from paper_2102_12559_amd import inputs
from tests.gpu_util import band_cells, compare_pops, run_pair, say, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def compare_band(s, o, tol, fg=0, periodic=(True, True), absolute=False):
    gm = s.get_mask().cpu().numpy()
    assert np.array_equal(gm.reshape(-1), o.get_mask().reshape(-1))
    b0, b1 = band_cells(gm, periodic)
    assert b0.any() and b1.any(), "no band cells"
    worst = 0.0
    for which, sel in ((1, b0), (0, b1)):
        g = s.get_populations(which, fg).cpu().numpy()[:, sel]
        r = o.get_pops(which, fg)[:, sel]
        assert np.all(np.isfinite(g))
        if absolute:
            err = float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
        else:
            n = s.cfg["n_low"] if which == 0 else s.cfg["n_high"]
            W = weights(s.dim, n)[:, None]
            err = float(np.max(np.abs(g - r) / np.maximum(np.abs(r), W * (1.0 if fg == 0 else 0.5))))
        say(f"  set {which} fg {fg} at {int(sel.sum())} band cells of the other order: {err:.3e}")
        worst = max(worst, err)
    assert worst <= tol, f"band parity {worst:.3e} > {tol:.1e}"


@pytest.mark.parametrize("nq,nQ", [(3, 4), (3, 6), (4, 5), (5, 6)])
def test_band_values_fp64(nq, nQ):
    nx, ny = 131, 45
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.65)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.3, seed=nq * 7 + nQ, drho=0.02)
    mask = inputs.random_mask(nx, ny, frac=0.25, seed=nQ + 1, blob=7)
    s, o = run_pair(cfg, rho, u, T, mask, 9, tag=f"band values {nq}/{nQ}")
    compare_pops(s, o, 1e-12)
    compare_band(s, o, 1e-12)


def test_band_values_thermal_two_relaxation_fp64():
    """Thermal f + g with the two-relaxation collision (tau2 != tau): both
    population sets of the band, lifted and projected."""
    nx, ny = 96, 40
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=4, tau=0.7, thermal=1, tau2=0.9)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=21, drho=0.03, dT=0.05)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=5, blob=6)
    s, o = run_pair(cfg, rho, u, T, mask, 8, tag="band values thermal qe")
    for fg in (0, 1):
        compare_pops(s, o, 1e-12, fg=fg)
        compare_band(s, o, 1e-12, fg=fg)


def test_band_values_hermite_lift_open_faces_fp64():
    """Hermite completion, zero-gradient x faces (no wrap of the band)."""
    nx, ny = 70, 37
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, tau=0.7,
                             lift_mode=inputs.LIFT_GRAD_HERMITE)
    cfg["bc"] = [inputs.BC_OUTFLOW_ZG, inputs.BC_OUTFLOW_ZG, inputs.BC_PERIODIC, inputs.BC_PERIODIC,
                 inputs.BC_PERIODIC, inputs.BC_PERIODIC]
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=9)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=3, blob=5)
    s, o = run_pair(cfg, rho, u, T, mask, 7, tag="band values hermite zg")
    compare_pops(s, o, 1e-12)
    compare_band(s, o, 1e-12, periodic=(False, True))


def test_band_values_fp32():
    nx, ny = 131, 45
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, tau=0.65, store=inputs.STORE_FP32)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.3, seed=2, drho=0.02)
    mask = inputs.random_mask(nx, ny, frac=0.25, seed=4, blob=7)
    s, o = run_pair(cfg, rho, u, T, mask, 9, oracle_cfg=dict(cfg, store=inputs.STORE_FP64),
                    tag="band values fp32")
    compare_band(s, o, 1e-5, absolute=True)


def _strip_mask(nx, ny):
    """A horizontal strip of the high-order set across the whole width (its
    low-order band rows put 64 band cells in a wave) and a vertical strip
    (4 band cells per wave row)."""
    mask = np.zeros((ny, nx), np.uint8)
    mask[20:28, :] = 1
    mask[:, 100:108] = 1
    return mask


def _band_cells_per_wave_row(mask):
    """Low-order band cells in each 64-cell row segment that holds any (a wave
    of the 2D kernel covers whole 64-cell rows of its tile)."""
    ny, nx = mask.shape
    b0, _ = band_cells(mask, (True, True))
    b0 = b0.reshape(ny, nx)
    nxp = -(-nx // 64) * 64
    b = np.zeros((ny, nxp), bool)
    b[:, :nx] = b0
    c = b.reshape(ny, nxp // 64, 64).sum(-1).ravel()
    return c[c > 0]


@pytest.mark.parametrize("nq,nQ,th", [(3, 6, 0), (3, 4, 1), (4, 5, 0)])
def test_band_lift_both_wave_paths_fp64(nq, nQ, th):
    """Waves with at most 4 band cells lift them one cell at a time across
    their lanes; waves with more lift one cell per lane.  The strip mask gives
    waves of both kinds; both must match the oracle's lift."""
    nx, ny = 192, 48
    mask = _strip_mask(nx, ny)
    c = _band_cells_per_wave_row(mask)
    assert (c <= 4).any() and (c > 4).any()
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.7, thermal=th, crit_every=0)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.25, seed=31 + nQ, drho=0.02,
                                          dT=0.04 if th else 0.0)
    s, o = run_pair(cfg, rho, u, T, mask, 5, tag=f"lift wave paths {nq}/{nQ} thermal {th}")
    for fg in ((0, 1) if th else (0,)):
        compare_pops(s, o, 1e-12, fg=fg)
        compare_band(s, o, 1e-12, fg=fg)


def test_band_lift_both_wave_paths_fp16():
    """The same two kinds of waves with FP16 deviation storage: the lifted
    values go through the storage scale of each high-order node."""
    nx, ny = 192, 48
    mask = _strip_mask(nx, ny)
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, tau=0.7, crit_every=0,
                             store=inputs.STORE_FP16_DEV)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.25, seed=41, drho=0.02)
    s, o = run_pair(cfg, rho, u, T, mask, 5, tag="lift wave paths fp16")
    compare_band(s, o, 2e-3, absolute=True)


def test_graph_modes_bit_identical():
    """A jet with the Mach criterion every 5 steps: launch by launch, step
    graphs, and graphs with parallel branches, over calls of uneven length
    with sampled timing, end in the same bytes."""
    from paper_2102_12559_amd import msl
    w = inputs.jet_c2(nx=128, ny=64, slot_w=12, crit_every=5)
    states = []
    for mode in (0, 1, 2):
        say(f"[case] graph mode {mode}: jet 128x64 fp32, calls of 7, 13, 20, 1, 19 steps")
        s = msl.Solver(w["cfg"])
        s.set_graph(mode)
        s.set_mask(w["mask"])
        s.init(w["rho"], w["u"], w["T"])
        s.profile(True, every=7)
        for n in (7, 13, 20, 1, 19):
            s.step(n)
        s.profile_read()
        s.profile(False)
        s.step(25)
        s.torch.cuda.synchronize()
        assert s.step_count == 85
        assert int(s.get_mask().sum()) > 0
        states.append(s.get_state())
        s.close()
    assert states[1] == states[0], "graph mode 1 differs from launch-by-launch stepping"
    assert states[2] == states[0], "graph mode 2 differs from launch-by-launch stepping"


@pytest.mark.parametrize("lift", [inputs.LIFT_GRAD, inputs.LIFT_MLP])
def test_parallel_branches_3d_bit_identical(lift):
    """3D two-set context (D3Q27 + D3Q64, FP16 deviations, the column walks):
    with mode 2 the two stream-collide launches of each untimed step run on
    two streams (Grad lift, and the learned closure with a random network);
    the state after calls of uneven length, with sampled timing and criterion
    passes, matches launch-by-launch stepping byte for byte."""
    from paper_2102_12559_amd import closure, msl
    w = inputs.vortex_shear_3d(n=32, rc=4.0, store=inputs.STORE_FP16_DEV)
    cfg = dict(w["cfg"], crit_every=5, lift_mode=lift)
    states = []
    for mode in (0, 2):
        say(f"[case] parallel branches 3D mode {mode} lift {lift}: 32^3 fp16, calls of 7, 13, 1, 9 steps")
        s = msl.Solver(cfg)
        if lift == inputs.LIFT_MLP:
            F, Od, H, P = s.mlp_dims()
            p = (closure.init_params(F, H, Od, seed=3) * 0.3).astype(np.float32)
            s.mlp_set_weights(p, np.zeros(F, np.float32), np.ones(F, np.float32),
                              np.zeros(Od, np.float32), np.full(Od, 1e-3, np.float32))
        s.set_graph(mode)
        s.set_mask(w["mask"])
        s.init(w["rho"], w["u"], w["T"])
        s.profile(True, every=7)
        for n in (7, 13, 1, 9):
            s.step(n)
        s.profile_read()
        s.profile(False)
        s.step(6)
        s.torch.cuda.synchronize()
        assert s.step_count == 36
        assert int(s.get_mask().sum()) > 0
        states.append(s.get_state())
        s.close()
    assert states[1] == states[0], "parallel branches differ from launch-by-launch stepping"
