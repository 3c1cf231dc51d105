"""GPU parity of the criterion's margin (crit_margin) against the oracle: the
dilated selection (bit for bit) and the populations it leads to, in the
lattice frame (2D and 3D) and in co-moving frames."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs
from tests.gpu_util import compare_pops, run_pair, say
from tests.test_gpu_pond_two_sets import compare2, pond2_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def test_margin_thermal_jet_fp64():
    w = inputs.jet_c2(nx=96, ny=48, slot_w=8, ma=0.5, tau=0.6, store=inputs.STORE_FP64, crit_thr=0.12,
                      crit_every=5, thermal=1, n_high=4, edge=0.0)
    cfg = dict(w["cfg"], crit_margin=3)
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 30, tag="jet margin 3")
    assert int(s.get_mask().sum()) > 0
    compare_pops(s, o, 1e-12)
    compare_pops(s, o, 1e-12, fg=1)


def test_margin_3d_fp64():
    nx, ny, nz = 20, 12, 10
    cfg = inputs.base_config(dim=3, nx=nx, ny=ny, nz=nz, n_low=3, n_high=4, tau=0.7,
                             crit_kind=inputs.CRIT_MA, crit_thr=0.25, crit_every=4, crit_margin=2)
    rho, u, T = inputs.smooth_random_flow(nx, ny, nz, umax=0.35, seed=8, drho=0.02)
    # (the short-wavelength flow decays below the threshold after a few steps:
    # 3 steps keep the selection of step 0, 160 cells dilated to 1710)
    s, o = run_pair(cfg, rho, u, T, np.zeros((nz, ny, nx), np.uint8), 3, tag="3D margin 2")
    m = int(s.get_mask().sum())
    say(f"  high-order cells {m}")
    assert 0 < m < nx * ny * nz
    compare_pops(s, o, 1e-12)


def test_margin_comoving_shock():
    probe = O.Pond(inputs.base_config(nx=4, ny=4, n_low=4, n_high=5, cfl=0.45, pond=1))
    w = inputs.shock_c3(ma1=1.6, nx=192, ny=4, dt=probe.dt, n_high=5, lam=8.0)
    cfg = dict(w["cfg"], pond=1, n_low=4, cfl=0.45, crit_kind=inputs.CRIT_KN, crit_thr=0.02,
               crit_every=5, crit_margin=6, lift_mode=inputs.LIFT_GRAD_HERMITE)
    cfg["tau2"] = 0.5 + 1.5 * (cfg["tau"] - 0.5)
    s, o = pond2_pair(cfg, w["rho"], w["u"], w["T"], np.zeros((1, 4, 192), np.uint8), 25, "shock margin 6")
    compare2(s, o, cfg, (False, True))
