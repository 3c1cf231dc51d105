"""Parity at the full workload sizes, in the configuration bench.py times.

The whole run cannot be repeated on the CPU at these sizes, so the GPU state
after a number of steps (masks switched by the criterion, band cells in
place) is handed to the oracle, one more step is taken on both sides, and the
new populations of sampled cells are compared.  The samples cover random
cells, every kind of face, and cells next to the other velocity set (whose
stencils read lifted or projected values).

- jet, 1024 x 512, FP32 storage, D2Q9 + D2Q36: the full oracle takes the
  state; bar 1e-5 on rho, u per sampled cell (relative to rho0 and c_s).
- 3D vortex and shear slab, 256^3, FP16 deviations, D3Q27 + D3Q64: a cell's
  update reads only its 5^3 neighbourhood, so the oracle steps that
  neighbourhood (periodic box of 5^3, no criterion) for each sampled cell;
  bar 2e-3 on rho, u.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2102_12559_amd import inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cell_macros(f, c, dim):
    """rho and u of populations f[..., Q] on the tensor lattice with 1D nodes c."""
    n = len(c)
    Q = f.shape[-1]
    idx = np.arange(Q)
    rho = f.sum(axis=-1)
    u = []
    for a in range(dim):
        ca = np.asarray(c)[(idx // n ** a) % n]
        u.append((f * ca).sum(axis=-1) / rho)
    return rho, np.stack(u, axis=-1)


def interface_cells(mask, count, rng):
    """Cells with a cell of the other order within Chebyshev distance 2."""
    m = mask.astype(np.int8)
    near = np.zeros(m.shape, bool)
    for sh in np.ndindex(*([5] * m.ndim)):
        off = [s - 2 for s in sh]
        near |= np.roll(m, off, axis=tuple(range(m.ndim))) != m
    idx = np.flatnonzero(near.reshape(-1))
    if idx.size > count:
        idx = rng.choice(idx, count, replace=False)
    return idx


def test_jet_full_size_fp32_sampled():
    from oracle import oracle as O
    from paper_2102_12559_amd import msl
    w = inputs.jet_c2()
    cfg = w["cfg"]
    nx, ny = cfg["nx"], cfg["ny"]
    say(f"[case] jet full size {nx}x{ny} fp32, 2001 steps then one compared step")
    s = msl.Solver(cfg)
    s.set_mask(w["mask"])
    s.init(w["rho"], w["u"], w["T"])
    s.step(2001)   # the criterion ran at step 2000; step 2001 has none
    mask = s.get_mask().cpu().numpy().reshape(ny, nx)
    lo = s.get_populations(0).cpu().numpy()
    hi = s.get_populations(1).cpu().numpy()
    s.step(1)
    lo1 = s.get_populations(0).cpu().numpy()
    hi1 = s.get_populations(1).cpu().numpy()
    nh = int(mask.sum())
    say(f"  high-order cells {nh}")
    assert nh > 1000
    rng = np.random.default_rng(0)
    x = np.arange(nx)
    y = np.arange(ny)
    edges = np.concatenate([y * nx, y * nx + nx - 1, x, (ny - 1) * nx + x,
                            y * nx + 1, y * nx + nx - 2])
    samples = np.unique(np.concatenate([rng.choice(nx * ny, 3000, replace=False), edges,
                                        interface_cells(mask, 3000, rng)]))
    ocfg = dict(cfg, store=inputs.STORE_FP64)
    o = Oracle(ocfg)
    o.set_mask(mask[None], convert=False)
    o.set_pops(0, lo)
    o.set_pops(1, hi)
    fo, _ = o.step_cells(samples)
    flat = mask.reshape(-1)
    worst_r = worst_u = 0.0
    for which, arr, n in ((0, lo1, 3), (1, hi1, 6)):
        sel = samples[flat[samples] == which]
        if sel.size == 0:
            continue
        Q = n * n
        c, _ = O.gh_rule(n)
        rows = np.searchsorted(samples, sel)
        rg, ug = cell_macros(arr[:, sel].T, c, 2)
        ro, uo = cell_macros(fo[rows, :Q], c, 2)
        worst_r = max(worst_r, float(np.max(np.abs(rg - ro))))
        worst_u = max(worst_u, float(np.max(np.abs(ug - uo))))
    say(f"  {samples.size} cells: max |drho| {worst_r:.2e}, max |du| {worst_u:.2e}")
    assert worst_r <= 1e-5 and worst_u <= 1e-5


def test_vortex_shear_3d_full_size_fp16_sampled():
    import torch
    from oracle import oracle as O
    from paper_2102_12559_amd import msl
    n = 256
    w = inputs.vortex_shear_3d(n=n)
    cfg = w["cfg"]
    say(f"[case] 3D vortex + shear {n}^3 fp16-dev, 21 steps then one compared step")
    s = msl.Solver(cfg)
    s.set_mask(w["mask"])
    s.init(w["rho"], w["u"], w["T"])
    s.step(21)    # criterion at steps 0 and 20
    mask_d = s.get_mask().reshape(n, n, n)
    mask = mask_d.cpu().numpy()
    nh = int(mask.sum())
    say(f"  high-order cells {nh}")
    assert nh > 10000
    rng = np.random.default_rng(1)
    samples = np.unique(np.concatenate([rng.choice(n ** 3, 600, replace=False),
                                        interface_cells(mask, 600, rng)]))
    # 5^3 neighbourhoods (periodic) of every sample, gathered on the device
    off = np.array(list(np.ndindex(5, 5, 5))) - 2          # [125][z, y, x]
    z0, y0, x0 = np.unravel_index(samples, (n, n, n))
    nb = (((z0[:, None] + off[None, :, 0]) % n) * n + (y0[:, None] + off[None, :, 1]) % n) * n \
        + (x0[:, None] + off[None, :, 2]) % n                  # [S][125]
    nbd = torch.as_tensor(nb.reshape(-1), device=s.device)
    before = [s.get_populations(l)[:, nbd].cpu().numpy().reshape(-1, nb.shape[0], 125)
              for l in (0, 1)]
    s.step(1)
    after = [s.get_populations(l)[:, torch.as_tensor(samples, device=s.device)].cpu().numpy()
             for l in (0, 1)]
    ocfg = dict(cfg, nx=5, ny=5, nz=5, store=inputs.STORE_FP64, crit_kind=inputs.CRIT_NONE,
                bc=[inputs.BC_PERIODIC] * 6)
    worst_r = worst_u = 0.0
    flat = mask.reshape(-1)
    for k in range(samples.size):
        o = Oracle(ocfg)
        o.set_mask(flat[nb[k]].reshape(1, 5, 5, 5)[0], convert=False)
        o.set_pops(0, before[0][:, k, :])
        o.set_pops(1, before[1][:, k, :])
        fo, _ = o.step_cells(np.array([62]))   # the centre of the 5^3 box
        which = int(flat[samples[k]])
        nn = 3 if which == 0 else 4
        c, _ = O.gh_rule(nn)
        rg, ug = cell_macros(after[which][:, k][None], c, 3)
        ro, uo = cell_macros(fo[:, :nn ** 3], c, 3)
        worst_r = max(worst_r, float(abs(rg[0] - ro[0])))
        worst_u = max(worst_u, float(np.max(np.abs(ug - uo))))
    say(f"  {samples.size} cells: max |drho| {worst_r:.2e}, max |du| {worst_u:.2e}")
    assert worst_r <= 2e-3 and worst_u <= 2e-3


@pytest.mark.parametrize("ma,store,steps", [
    (1.4, inputs.STORE_FP64, 80), (1.4, inputs.STORE_FP32, 30), (1.4, inputs.STORE_FP16_DEV, 10),
    pytest.param(1.4, inputs.STORE_BF16_DEV, 10, marks=pytest.mark.xfail(
        reason="BF16 (8 significant bits) misses the 2e-3 bar on the shock: measured 3.6e-3 on "
               "rho with rho0 = 1, and with the mean end state as the storage reference still "
               "above 2e-3 on u or T (FP16: within 2e-3)", strict=False))])
def test_shock_full_size(ma, store, steps):
    """Normal shock on the full 8192 x 4 grid (RH end states, hard-sphere
    viscosity, |Pi_neq|/p criterion every 5 steps), whole-grid comparison.
    FP64: 1e-12 per population; FP32: 1e-5 on rho, u/u1, T; FP16 and BF16
    deviations: 2e-3 on rho/rho0, u/u1, T/T0, stored from the weights carried
    over to the mean (rho0, u, T0) of the two end states, which keeps |h|
    well below its value with the lattice weights (with the mean velocity
    and temperature but rho0 = 1, BF16 measured 3.6e-3 on rho).  The inflow
    moves faster than the D2Q9 lattice speed
    sqrt(3) (Mach 1.4: u1 = 1.81), and the flow next to the inlet amplifies
    any difference by about a factor 10 every 35 steps (FP64 differences:
    1e-15 at step 1, 5e-13 at step 80, 1.5e-11 at step 120, 5e-4 at step 300,
    the same growth at 256 and at 8192 cells): the comparison is made at an
    early horizon: 80 steps in FP64, 30 in FP32, 10 with 16-bit deviations
    (one rounding decided differently on the two sides costs a unit in the
    last place of h).  At Mach 2 and 3 (u1 = 2.58, 3.87) the lattice-frame
    run produces non-finite values within 10 steps on both sides; those
    configurations run in a global constant frame (tests/test_gpu_frame.py)."""
    from tests.gpu_util import compare_macros, compare_pops, run_pair
    probe = Oracle(inputs.base_config(nx=4, ny=4, n_low=3, n_high=6))
    w = inputs.shock_c3(ma1=ma, dt=probe.dt, store=store)
    rh = w["rh"]
    rho0, T0 = 1.0, 1.0
    if store >= inputs.STORE_FP16_DEV:
        rho0, T0 = 0.5 * (rh["rho1"] + rh["rho2"]), 0.5 * (rh["T1"] + rh["T2"])
        w["cfg"] = dict(w["cfg"], store_u=(0.5 * (rh["u1"] + rh["u2"]), 0.0, 0.0), rho0=rho0, T0=T0)
    ocfg = dict(w["cfg"], store=inputs.STORE_FP64 if store == inputs.STORE_FP32 else store)
    s, o = run_pair(w["cfg"], w["rho"], w["u"], w["T"], w["mask"], steps, oracle_cfg=ocfg,
                    tag=f"shock Ma {ma} full size")
    say(f"  high-order cells: {int(s.get_mask().sum())}")
    if store == inputs.STORE_FP64:
        compare_pops(s, o, 1e-12)
        compare_pops(s, o, 1e-12, fg=1)
    else:
        tol = {inputs.STORE_FP32: 1e-5, inputs.STORE_FP16_DEV: 2e-3,
               inputs.STORE_BF16_DEV: 2e-3}[store]
        compare_macros(s, o, tol, uscale=w["rh"]["u1"], rscale=rho0, Tscale=T0)
