"""GPU parity of the global constant reference frame (eq. veli) and of the
16-bit storage scale carried over to a storage reference state, against the
oracle through the C-ABI.

Tolerances as in the other parity tests: FP64 1e-12 per population (floored
at the storage scale), FP32 1e-5 on rho, u, T, 16-bit deviations 2e-3 on the
same macroscopic norms against the oracle run with the same storage rounding.
"""
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


@pytest.mark.parametrize("nq,nQ,thermal", [(3, 4, 0), (3, 6, 1), (4, 5, 0)])
def test_frame_random_mask_ragged_fp64(nq, nQ, thermal):
    """A frame moving at (0.35, -0.2) with T_ref = 1.3 on a ragged grid with a
    random mask: every stencil, equilibrium, lift and projection in the frame."""
    nx, ny = 131, 45
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=nq, n_high=nQ, tau=0.7, thermal=thermal,
                             u_ref=(0.35, -0.2, 0.0), T_ref=1.3)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.3, seed=nq * 10 + nQ, drho=0.02,
                                          dT=0.04 if thermal else 0.0)
    u[0] += 0.35
    u[1] -= 0.2
    mask = inputs.random_mask(nx, ny, frac=0.25, seed=nQ + 3, blob=7)
    s, o = run_pair(cfg, rho, u, T, mask, 15, tag=f"frame random mask {nq}/{nQ} th={thermal}")
    compare_pops(s, o, 1e-12)
    if thermal:
        compare_pops(s, o, 1e-12, fg=1)


@pytest.mark.parametrize("store,tol", [(inputs.STORE_FP64, 1e-12), (inputs.STORE_FP32, 1e-5)])
def test_frame_3d(store, tol):
    """3D D3Q27 + D3Q64 slab in a frame moving along x and z, ragged box."""
    nx, ny, nz = 70, 12, 10
    rho, u, T = inputs.smooth_random_flow(nx, ny, nz, umax=0.15, seed=31, drho=0.02)
    u[0] += 0.4
    u[2] += 0.1
    cfg = inputs.base_config(dim=3, nx=nx, ny=ny, nz=nz, n_low=3, n_high=4, tau=0.75, store=store,
                             u_ref=(0.4, 0.0, 0.1), T_ref=1.1)
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 4:8, :] = 1
    s, o = run_pair(cfg, rho, u, T, mask, 8, oracle_cfg=dict(cfg, store=inputs.STORE_FP64),
                    tag=f"3D frame store={store}")
    if store == inputs.STORE_FP64:
        compare_pops(s, o, tol)
    else:
        compare_macros(s, o, tol, uscale=1.0)


def test_vortex_fp16_tilted_storage():
    """The convected vortex (64 x 64, D2Q9 with a D2Q16 disk, advected at
    Ma 0.5) stored as FP16 deviations from the weights carried over to the
    advection velocity: 2e-3 after 200 steps (the BF16 case sits with the
    other storage tests)."""
    w = inputs.vortex_c1()
    cfg = dict(w["cfg"], store=inputs.STORE_FP16_DEV, store_u=(0.5, 0.0, 0.0))
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 200, tag="C1 fp16 tilted")
    compare_macros(s, o, 2e-3, uscale=1.0)


@pytest.mark.parametrize("ma", [2.0, 3.0])
def test_shock_in_global_frame_fp64(ma):
    """The normal shock at Mach 2 and 3 (D2Q9 far field, D2Q36 where
    |Pi_neq|/p > 1e-3, hard-sphere viscosity), in the global frame moving at the
    mean of the two end states' velocities and heated to their mean
    temperature; the lattice frame diverges within 10 steps at these Mach
    numbers.  80 steps, 1e-12."""
    probe_cfg = inputs.base_config(nx=4, ny=4, n_low=3, n_high=6)
    probe_cfg["u_ref"], probe_cfg["T_ref"] = inputs.shock_frame(ma)
    dt = Oracle(probe_cfg).dt
    w = inputs.shock_c3(ma1=ma, nx=256, ny=4, dt=dt, crit_every=5, store=inputs.STORE_FP64,
                        frame=True)
    s, o = run_pair(w["cfg"], w["rho"], w["u"], w["T"], w["mask"], 80, tag=f"shock Ma {ma} frame fp64")
    nh = int(s.get_mask().sum())
    say(f"  high-order cells {nh}")
    assert nh > 0
    compare_pops(s, o, 1e-12)
    compare_pops(s, o, 1e-12, fg=1)


BF16_SHOCK = pytest.mark.xfail(
    reason="BF16 (8 significant bits) misses the 2e-3 bar on the shock: 10 steps at Mach 2 in the "
           "global frame measured rho/rho0 1.6e-3, u/u1 2.1e-3, T/T0 3.3e-3 against the oracle with "
           "the same storage rounding (FP16: within 2e-3)", strict=False)


@pytest.mark.parametrize("store", [inputs.STORE_FP16_DEV,
                                   pytest.param(inputs.STORE_BF16_DEV, marks=BF16_SHOCK)])
def test_shock_in_global_frame_16bit(store):
    """The Mach-2 shock in its global frame with 16-bit deviations stored from
    the frame's rest state at the mean density (so both end states deviate by
    about half the jump): 2e-3 on rho/rho0, u/u1, T/T0 after 10 steps."""
    ma = 2.0
    probe_cfg = inputs.base_config(nx=4, ny=4, n_low=3, n_high=6)
    probe_cfg["u_ref"], probe_cfg["T_ref"] = inputs.shock_frame(ma)
    dt = Oracle(probe_cfg).dt
    w = inputs.shock_c3(ma1=ma, nx=256, ny=4, dt=dt, crit_every=5, store=store, frame=True)
    rh = w["rh"]
    rho0 = 0.5 * (rh["rho1"] + rh["rho2"])
    cfg = dict(w["cfg"], store_u=w["cfg"]["u_ref"], T0=w["cfg"]["T_ref"], rho0=rho0)
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 10, tag=f"shock Ma 2 frame store={store}")
    compare_macros(s, o, 2e-3, uscale=rh["u1"], rscale=rho0, Tscale=cfg["T0"])


def test_jet_c2_as_configured_early_horizon():
    """The jet as configured (Ma 1.2 slot, thermal, D2Q9 + D2Q16 where Ma > 0.4,
    tau 0.52, sharp slot edges) on a 128 x 64 grid with an 8-cell slot: in the
    lattice frame its equilibrium turns negative at the slot speed and the
    run diverges at about 30 steps on the oracle as on the GPU; parity at 15
    steps, 1e-12."""
    w = inputs.jet_c2(nx=128, ny=64, slot_w=8, ma=1.2, thermal=1, n_high=4, edge=0.0,
                      store=inputs.STORE_FP64, crit_every=5)
    s, o = run_pair(w["cfg"], w["rho"], w["u"], w["T"], w["mask"], 15, tag="C2 as configured fp64")
    assert int(s.get_mask().sum()) > 0
    compare_pops(s, o, 1e-12)
    compare_pops(s, o, 1e-12, fg=1)
