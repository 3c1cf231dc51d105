"""GPU parity of the Knudsen-number criterion (Sec. IV.A.3: Kn = lambda / L,
L = rho / |grad rho|, hard-sphere mean free path, refinement above Kn_thr)
against the oracle through the C-ABI: the masks after every criterion pass
must match bit for bit (compare_pops checks them) and the populations to the
usual bars (FP64 1e-12, FP32 1e-5 on rho, u, T)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2102_12559_amd import inputs
from tests.gpu_util import compare_macros, compare_pops, run_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def shock_kn(ma, nq, nQ, store, pr23=True, frame=False):
    probe = inputs.base_config(nx=4, ny=4, n_low=nq, n_high=nQ)
    if frame:
        probe["u_ref"], probe["T_ref"] = inputs.shock_frame(ma)
    dt = Oracle(probe).dt
    w = inputs.shock_c3(ma1=ma, nx=256, ny=4, n_high=nQ, dt=dt, crit_every=5, store=store, frame=frame)
    cfg = dict(w["cfg"], n_low=nq, crit_kind=inputs.CRIT_KN, crit_thr=0.02)
    if pr23:
        cfg["tau2"] = 0.5 + 1.5 * (cfg["tau"] - 0.5)
    return w, cfg


@pytest.mark.parametrize("nq,nQ,frame", [(4, 5, True), (3, 6, False)])
def test_shock_knudsen_fp64(nq, nQ, frame):
    """The Mach-1.4 shock from a step, refined where Kn > 0.02 (D2Q16 / D2Q25
    as in the paper's shock-structure runs, in the global frame of the two
    end states, where the lattice frame diverges within 60 steps; and D2Q9 /
    D2Q36), Pr = 2/3, 60 steps with the criterion every 5."""
    w, cfg = shock_kn(1.4, nq, nQ, inputs.STORE_FP64, frame=frame)
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 60, tag=f"shock Kn {nq}/{nQ}")
    nh = int(s.get_mask().sum())
    say(f"  high-order cells {nh}")
    assert 0 < nh < cfg["nx"] * cfg["ny"]
    compare_pops(s, o, 1e-12)
    compare_pops(s, o, 1e-12, fg=1)


def test_shock_knudsen_frame_fp32():
    """Mach 2 in the global frame, FP32 storage: masks equal, 1e-5."""
    w, cfg = shock_kn(2.0, 3, 6, inputs.STORE_FP32, frame=True)
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 40,
                    oracle_cfg=dict(cfg, store=inputs.STORE_FP64), tag="shock Kn Ma 2 frame fp32")
    assert np.array_equal(s.get_mask().cpu().numpy().reshape(-1), o.get_mask().reshape(-1))
    rh = w["rh"]
    compare_macros(s, o, 1e-5, uscale=rh["u1"], rscale=rh["rho1"], Tscale=rh["T1"])


def test_open_faces_random_flow_fp64():
    """Athermal random flow between open x faces (zero-gradient outflow):
    the one-sided differences at the faces, 2D gradient magnitude."""
    nx, ny = 96, 40
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=81, drho=0.08)
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=4, tau=0.8, crit_kind=inputs.CRIT_KN,
                             crit_thr=0.001, crit_every=4,
                             bc=[inputs.BC_OUTFLOW_ZG] * 2 + [inputs.BC_PERIODIC] * 4)
    mask = np.zeros((1, ny, nx), np.uint8)
    s, o = run_pair(cfg, rho, u, T, mask, 17, tag="open faces Kn")
    nh = int(s.get_mask().sum())
    say(f"  high-order cells {nh}")
    assert 0 < nh < nx * ny
    compare_pops(s, o, 1e-12)


def test_knudsen_3d_fp64():
    """3D vortex with a density dip, D3Q27 / D3Q64 where Kn exceeds the
    threshold, open z faces."""
    n = 20
    rho, u, T = inputs.smooth_random_flow(n, n, n, umax=0.1, seed=83, drho=0.08)
    cfg = inputs.base_config(dim=3, nx=n, ny=n, nz=n, n_low=3, n_high=4, tau=0.8,
                             crit_kind=inputs.CRIT_KN, crit_thr=0.0035, crit_every=3,
                             bc=[inputs.BC_PERIODIC] * 4 + [inputs.BC_OUTFLOW_ZG] * 2)
    mask = np.zeros((n, n, n), np.uint8)
    s, o = run_pair(cfg, rho, u, T, mask, 7, tag="3D Kn")
    nh = int(s.get_mask().sum())
    say(f"  high-order cells {nh}")
    assert 0 < nh < n ** 3
    compare_pops(s, o, 1e-12)
