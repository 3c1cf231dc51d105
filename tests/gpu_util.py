"""Helpers shared by the GPU tests: run the same seeded case through the HIP
library and through the oracle, and compare them.  Test code only."""
import sys
import time

import numpy as np

from oracle.oracle import Oracle
from paper_2102_12559_amd import inputs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(cfg, rho, u, T, mask, steps, oracle_cfg=None, tag=""):
    from paper_2102_12559_amd import msl
    say(f"[case] {tag} grid={cfg['nx']}x{cfg['ny']}x{cfg['nz']} n=({cfg['n_low']},{cfg['n_high']}) "
        f"store={cfg['store']} thermal={cfg['thermal']} steps={steps}")
    t0 = time.time()
    s = msl.Solver(cfg)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(steps)
    s.torch.cuda.synchronize()
    say(f"  gpu done {time.time() - t0:.2f}s")
    o = Oracle(oracle_cfg or cfg)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(steps)
    say(f"  oracle done {time.time() - t0:.2f}s")
    return s, o


def weights(dim, n):
    from oracle import oracle as O
    _, w = O.gh_rule(n)
    Q = n ** dim
    W = np.ones(Q)
    for i in range(Q):
        r = i
        for a in range(dim):
            W[i] *= w[r % n]
            r //= n
    return W


def compare_pops(s, o, tol, fg=0, rho0=1.0):
    """max over native cells of |f_gpu - f_ref| / max(|f_ref|, rho0 W_i)"""
    gm = s.get_mask().cpu().numpy().reshape(-1)
    om = o.get_mask().reshape(-1)
    assert np.array_equal(gm, om), f"masks differ at {np.sum(gm != om)} cells"
    worst = 0.0
    for which in range(len(s.Q)):
        sel = gm == which
        if not sel.any():
            continue
        g = s.get_populations(which, fg).cpu().numpy()[:, sel]
        r = o.get_pops(which, fg)[:, sel]
        n = s.cfg["n_low"] if which == 0 else s.cfg["n_high"]
        W = weights(s.dim, n)[:, None]
        scale = np.maximum(np.abs(r), rho0 * W * (1.0 if fg == 0 else 0.5))
        assert np.all(np.isfinite(g)) and np.all(np.isfinite(r)), "non-finite populations"
        err = float(np.max(np.abs(g - r) / scale))
        say(f"  set {which} fg {fg}: max rel err {err:.3e} over {sel.sum()} cells")
        worst = max(worst, err)
    assert worst <= tol, f"population parity {worst:.3e} > {tol:.1e}"
    return worst


def compare_macros(s, o, tol, uscale, rscale=1.0, Tscale=1.0):
    """max over cells of |d rho| / rscale, |d u| / uscale and |d T| / Tscale
    (the reference density and temperature, and max(U, c_s))."""
    rg, ug, Tg = [a.cpu().numpy() for a in s.macros()]
    ro, uo, To = o.macros()
    assert all(np.all(np.isfinite(a)) for a in (rg, ug, Tg, ro, uo, To)), "non-finite macros"
    e_rho = np.max(np.abs(rg - ro)) / rscale
    e_u = np.max(np.abs(ug - uo)) / uscale
    e_T = np.max(np.abs(Tg - To)) / Tscale
    say(f"  macros: rho {e_rho:.3e} u {e_u:.3e} T {e_T:.3e}")
    assert e_rho <= tol and e_u <= tol and e_T <= tol, (e_rho, e_u, e_T)
    return e_rho, e_u, e_T


def band_cells(mask, periodic):
    """Cells with a cell of the other order within the 3-point stencil's reach
    (2 cells along each axis, a 5 x 5 box); periodic per axis (x, y)."""
    m = mask.reshape(mask.shape[-2:]).astype(np.int8)
    pad = [(2, 2), (2, 2)]
    p = m
    for ax, per in ((1, periodic[0]), (0, periodic[1])):
        w = [(0, 0), (0, 0)]
        w[ax] = pad[ax]
        p = np.pad(p, w, mode="wrap" if per else "edge")
    ny, nx = m.shape
    hi = np.zeros_like(m)
    lo = np.ones_like(m)
    for dy in range(5):
        for dx in range(5):
            v = p[dy:dy + ny, dx:dx + nx]
            hi = np.maximum(hi, v)
            lo = np.minimum(lo, v)
    return ((m == 0) & (hi == 1)).reshape(-1), ((m == 1) & (lo == 0)).reshape(-1)
