"""GPU L2 / max error norms (msl_error_norms: FP64 sums with wave shuffles,
LDS and a second pass) against the oracle's definition, evaluated on the
GPU's own macroscopic fields (1e-13 relative; the sums run in another order)
and on the oracle's state after the same run (1e-9: the two states agree to
the 1e-12 population bar)."""
import math

import numpy as np
import pytest

from oracle.oracle import error_norms
from paper_2102_12559_amd import inputs
from tests.gpu_util import run_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def check(s, o, refs, tol_self=1e-13, tol_oracle=1e-9):
    got = s.error_norms(*refs)
    rg, ug, Tg = [a.cpu().numpy() for a in s.macros()]
    want = error_norms(rg, ug, Tg, *refs)
    ro, uo, To = o.macros()
    want_o = error_norms(ro, uo, To, *refs)
    for f in ("rho", "u", "T"):
        for j in range(2):
            a, b, c = got[f][j], want[f][j], want_o[f][j]
            say(f"  {f}[{'l2' if j == 0 else 'max'}] gpu {a:.6e} def {b:.6e} oracle {c:.6e}")
            assert abs(a - b) <= tol_self * max(abs(b), 1e-300)
            assert abs(a - c) <= tol_oracle * max(abs(c), 1e-300)


def test_vortex_c1_against_initial_fields():
    w = inputs.vortex_c1()
    s, o = run_pair(w["cfg"], w["rho"], w["u"], w["T"], w["mask"], 60, tag="C1 norms")
    check(s, o, (w["rho"], w["u"], w["T"]))


def test_thermal_3d_and_skipped_fields():
    n = 24
    rho, u, T = inputs.smooth_random_flow(n, n, n, umax=0.15, seed=91, drho=0.03, dT=0.05)
    cfg = inputs.base_config(dim=3, nx=n, ny=n, nz=n, n_low=3, n_high=4, tau=0.8, thermal=1, cv=2.5)
    mask = np.zeros((n, n, n), np.uint8)
    mask[8:16] = 1
    s, o = run_pair(cfg, rho, u, T, mask, 6, tag="3D norms")
    check(s, o, (rho, u, T))
    got = s.error_norms(None, u, None)
    assert got["rho"] == (0.0, 0.0) and got["T"] == (0.0, 0.0) and got["u"][0] > 0


def test_large_grid_fp32_and_nan():
    """4096 x 2048 FP32 (more cells than one pass of the 1024 x 256 grid of
    threads covers), then a NaN in the reference propagates to both norms."""
    nx, ny = 4096, 2048
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.1, seed=93, drho=0.02)
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=0, tau=0.7, store=inputs.STORE_FP32)
    from paper_2102_12559_amd import msl
    s = msl.Solver(cfg)
    s.set_mask(np.zeros((1, ny, nx), np.uint8))
    s.init(rho, u, T)
    s.step(3)
    ref = rho * (1 + 1e-3)
    got = s.error_norms(ref, None, None)
    rg = s.macros()[0].cpu().numpy()
    want = error_norms(rg, None, None, ref, None, None)
    say(f"  rho l2 {got['rho'][0]:.6e} vs {want['rho'][0]:.6e}")
    assert abs(got["rho"][0] - want["rho"][0]) <= 1e-12 * want["rho"][0]
    assert got["rho"][1] == want["rho"][1]
    bad = ref.copy()
    bad.reshape(-1)[12345] = np.nan
    nanres = s.error_norms(bad, None, None)
    assert math.isnan(nanres["rho"][0]) and math.isnan(nanres["rho"][1])
    s.close()
