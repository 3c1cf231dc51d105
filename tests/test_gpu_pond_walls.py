"""GPU parity of diffuse walls in co-moving frames (the paper's Couette
set-up) against the oracle through the C-ABI: the GPU computes each column's
wall density from the adjacent cell's populations transferred into the wall's
frame by the per-axis Lagrange rows; the oracle by the moment matrices.
FP64 1e-12 on the frames and on each set's populations (own cells and band
cells of the other set), sets bit for bit."""
import numpy as np
import pytest

from paper_2102_12559_amd import inputs
from tests.test_gpu_pond_two_sets import compare2, pond2_pair
from tests.test_oracle_pond_walls import couette

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def rest(cfg):
    ny, nx = cfg["ny"], cfg["nx"]
    return np.ones((1, ny, nx)), np.zeros((2, 1, ny, nx)), np.ones((1, ny, nx))


def test_couette_d2q16_athermal():
    """D2Q16 everywhere (the low set of a 4/5 context with no high-order cell)."""
    cfg, mask = couette(4, 5, 0, ny=24, nx=8)
    rho, u, T = rest(cfg)
    s, o = pond2_pair(cfg, rho, u, T, mask, 150, "couette d2q16")
    compare2(s, o, cfg, (True, False))


def test_couette_thermal_two_sets_prandtl():
    """D2Q9 bulk with D2Q16 wall layers, thermal, Pr = 2/3 (tau2), moving
    walls at -+0.1 (the paper's Couette layout)."""
    cfg, mask = couette(3, 4, 1, ny=24, nx=8, layer=4)
    cfg["tau2"] = 0.5 + 1.5 * (cfg["tau"] - 0.5)
    rho, u, T = rest(cfg)
    s, o = pond2_pair(cfg, rho, u, T, mask, 150, "couette thermal 3/4 Pr 2/3")
    compare2(s, o, cfg, (True, False))


def test_walls_with_zero_gradient_x_faces():
    cfg, mask = couette(3, 4, 1, ny=20, nx=12, layer=3)
    cfg["bc"][0] = cfg["bc"][1] = inputs.BC_OUTFLOW_ZG
    rho, u, T = inputs.smooth_random_flow(12, 20, umax=0.1, seed=4, drho=0.02, dT=0.03)
    s, o = pond2_pair(cfg, rho, u, T, mask, 40, "walls + zero-gradient x")
    compare2(s, o, cfg, (False, False))
