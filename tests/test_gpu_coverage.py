"""GPU parity of launch configurations and workloads that the smaller cases
do not reach, through the C-ABI against the oracle.

- D2Q9 in 8-row tiles (grids of at least 2048 such tiles) with the
  non-temporal stores of buffers larger than the 256 MB last-level cache:
  FP64 on 2048 x 2048 compared on every cell (1e-12 per population), FP32 on
  3072 x 3072 with a D2Q16 disk compared on sampled cells over one step from
  the GPU state (1e-5 on rho, u).
- The learned lift with FP16 and BF16 deviation storage in 2D and 3D against
  the oracle running the same network with BF16 operands and the same storage
  rounding (2e-3 on rho, u).
- Planar Couette flow (C4) in its configured FP32 storage against the FP64
  oracle (1e-5 on rho, u, T).
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2102_12559_amd import closure, inputs
from tests.gpu_util import compare_macros, compare_pops, run_pair, say
from tests.test_gpu_fullsize import cell_macros, interface_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_12559_amd import msl
    msl.lib()


def test_d2q9_8row_tiles_nontemporal_fp64():
    """2048 x 2048 FP64 D2Q9: 4096 tiles of 64 x 8 (the 8-row kernel) and a
    302 MB plane buffer (non-temporal stores)."""
    n = 2048
    cfg = inputs.base_config(nx=n, ny=n, n_low=3, n_high=0, tau=0.6, store=inputs.STORE_FP64)
    rho, u, T = inputs.smooth_random_flow(n, n, umax=0.1, seed=41, drho=0.01, modes=2)
    s, o = run_pair(cfg, rho, u, T, np.zeros((1, n, n), np.uint8), 3, tag="D2Q9 2048^2 fp64 8-row")
    compare_pops(s, o, 1e-12)


def test_d2q9_8row_tiles_nontemporal_fp32_sampled():
    """3072 x 3072 FP32, D2Q9 with a D2Q16 disk of radius 300: the 8-row D2Q9
    kernel with non-temporal stores (340 MB of D2Q9 planes), the high-order
    set's live-tile list and the band conversion at that size."""
    from oracle import oracle as O
    from paper_2102_12559_amd import msl
    n = 3072
    cfg = inputs.base_config(nx=n, ny=n, n_low=3, n_high=4, tau=0.6, store=inputs.STORE_FP32)
    rho, u, T = inputs.smooth_random_flow(n, n, umax=0.1, seed=42, drho=0.01, modes=2)
    mask = inputs.disk_mask(n, n, radius=300.0)
    say(f"[case] D2Q9 + D2Q16 disk {n}^2 fp32, 4 steps then one compared step")
    s = msl.Solver(cfg)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(4)
    lo = s.get_populations(0).cpu().numpy()
    hi = s.get_populations(1).cpu().numpy()
    s.step(1)
    lo1 = s.get_populations(0).cpu().numpy()
    hi1 = s.get_populations(1).cpu().numpy()
    m2 = mask.reshape(n, n)
    rng = np.random.default_rng(1)
    x = np.arange(n)
    edges = np.concatenate([x, (n - 1) * n + x, x * n, x * n + n - 1])
    samples = np.unique(np.concatenate([rng.choice(n * n, 4000, replace=False), edges,
                                        interface_cells(m2, 3000, rng)]))
    o = Oracle(dict(cfg, store=inputs.STORE_FP64))
    o.set_mask(mask, convert=False)
    o.set_pops(0, lo)
    o.set_pops(1, hi)
    fo, _ = o.step_cells(samples)
    flat = m2.reshape(-1)
    worst_r = worst_u = 0.0
    for which, arr, nn in ((0, lo1, 3), (1, hi1, 4)):
        sel = samples[flat[samples] == which]
        c, _ = O.gh_rule(nn)
        rows = np.searchsorted(samples, sel)
        rg, ug = cell_macros(arr[:, sel].T, c, 2)
        ro, uo = cell_macros(fo[rows, :nn * nn], c, 2)
        worst_r = max(worst_r, float(np.max(np.abs(rg - ro))))
        worst_u = max(worst_u, float(np.max(np.abs(ug - uo))))
    say(f"  {samples.size} cells: max |drho| {worst_r:.2e}, max |du| {worst_u:.2e}")
    assert worst_r <= 1e-5 and worst_u <= 1e-5


def _learned_pair(cfg, rho, u, T, mask, steps, seed, tag):
    from paper_2102_12559_amd import msl
    say(f"[case] {tag}")
    s = msl.Solver(cfg)
    F, Od, H, P = s.mlp_dims()
    p = (closure.init_params(F, H, Od, seed=seed) * 0.5).astype(np.float32)
    xm = np.zeros(F, np.float32)
    xm[0] = 1.0
    xs = np.full(F, 0.5, np.float32)
    tm = np.zeros(Od, np.float32)
    ts = np.full(Od, 1e-3, np.float32)
    s.mlp_set_weights(p, xm, xs, tm, ts)
    flags = np.ones(s.num_check_tiles(), np.uint8)
    s.mlp_set_flags(flags)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(steps)
    o = Oracle(cfg)
    o.set_mlp(H, p.astype(np.float64), xm.astype(np.float64), xs.astype(np.float64),
              tm.astype(np.float64), ts.astype(np.float64), bf16=True, manual_check=True)
    o.set_mlp_flags(flags)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(steps)
    return s, o


@pytest.mark.parametrize("store", [inputs.STORE_FP16_DEV, inputs.STORE_BF16_DEV])
def test_learned_lift_16bit_2d(store):
    nx, ny = 80, 70
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, lift_mode=inputs.LIFT_MLP,
                             store=store, tau=0.7)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=19, drho=0.02)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=7, blob=8)
    s, o = _learned_pair(cfg, rho, u, T, mask, 20, 23, f"learned lift 2D store={store}")
    compare_macros(s, o, 2e-3, uscale=1.0)


@pytest.mark.parametrize("store", [inputs.STORE_FP16_DEV, inputs.STORE_BF16_DEV])
def test_learned_lift_16bit_3d(store):
    """The learned lift in the 3D configuration of the vortex and shear-slab
    workload (D3Q27 + D3Q64, 16-bit deviations), on a 20^3 box."""
    n = 20
    w = inputs.vortex_shear_3d(n=n, store=store, lift_mode=inputs.LIFT_MLP, rc=3.0)
    cfg = dict(w["cfg"])
    mask = np.zeros((n, n, n), np.uint8)
    mask[:, 6:12, :] = 1
    s, o = _learned_pair(cfg, w["rho"], w["u"], w["T"], mask, 8, 29, f"learned lift 3D store={store}")
    compare_macros(s, o, 2e-3, uscale=1.0)


def test_couette_c4_fp32():
    probe = Oracle(inputs.base_config(nx=4, ny=4, n_low=3, n_high=6))
    w = inputs.couette_c4(N=64, kn=0.5, band=4, dt=probe.dt, store=inputs.STORE_FP32)
    cfg = w["cfg"]
    s, o = run_pair(cfg, w["rho"], w["u"], w["T"], w["mask"], 300,
                    oracle_cfg=dict(cfg, store=inputs.STORE_FP64), tag="couette C4 fp32")
    compare_macros(s, o, 1e-5, uscale=1.0)
