"""Pins of the criterion's margin (crit_margin): the high-order set also takes
every cell within `margin` cells, per axis, of a cell the criterion selects.

- or_dilate_mask against a brute-force box maximum (periodic faces wrap,
  other faces end the box), 2D and 3D, margins 0 to 3.
- The oracle's step applies it: after one step the mask is the dilated
  selection of the criterion at step 0, with the static frame and with
  co-moving frames.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import inputs


def brute(mask, m, periodic):
    nz, ny, nx = mask.shape
    out = np.zeros_like(mask)
    dims = (nx, ny, nz)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                v = 0
                for dz in range(-m, m + 1) if nz > 1 else (0,):
                    for dy in range(-m, m + 1):
                        for dx in range(-m, m + 1):
                            q = [x + dx, y + dy, z + dz]
                            ok = True
                            for a in range(3 if nz > 1 else 2):
                                if not 0 <= q[a] < dims[a]:
                                    if periodic[a]:
                                        q[a] %= dims[a]
                                    else:
                                        ok = False
                            if ok:
                                v |= mask[q[2], q[1], q[0]]
                out[z, y, x] = v
    return out


@pytest.mark.parametrize("m", [0, 1, 3])
@pytest.mark.parametrize("dim,bc", [(2, [0, 0, 0, 0, 0, 0]), (2, [2, 1, 0, 0, 0, 0]),
                                    (3, [0, 0, 2, 2, 0, 0])])
def test_dilation_is_a_box_maximum(m, dim, bc):
    nx, ny, nz = 13, 9, (6 if dim == 3 else 1)
    rng = np.random.default_rng(m + 7 * dim)
    mask = (rng.random((nz, ny, nx)) < 0.06).astype(np.uint8)
    cfg = inputs.base_config(dim=dim, nx=nx, ny=ny, nz=nz, n_low=3, n_high=4, crit_margin=m)
    cfg["bc"] = bc
    periodic = [bc[2 * a] == 0 and bc[2 * a + 1] == 0 for a in range(3)]
    got = O.dilate_mask(cfg, mask)
    assert np.array_equal(got, brute(mask, m, periodic))


def test_step_applies_the_margin_static_frame():
    w = inputs.jet_c2(nx=96, ny=48, slot_w=8, ma=0.5, tau=0.6, store=inputs.STORE_FP64, crit_thr=0.12,
                      crit_every=5, thermal=1, n_high=4, edge=0.0)
    cfg = dict(w["cfg"], crit_margin=3)
    o = O.Oracle(cfg)
    o.set_mask(w["mask"], convert=False)
    o.init(w["rho"], w["u"], w["T"])
    o.step(5)
    for _ in range(4):
        sel = o.eval_criterion()[0]     # the selection at a multiple of 5 steps
        o.step(1)                       # that step's criterion pass, then the step
        assert np.array_equal(o.get_mask(), O.dilate_mask(cfg, sel))
        o.step(4)
    assert o.get_mask().sum() > sel.sum() > 0


def test_step_applies_the_margin_comoving_frames():
    probe = O.Pond(inputs.base_config(nx=4, ny=4, n_low=4, n_high=5, cfl=0.45, pond=1))
    w = inputs.shock_c3(ma1=1.4, nx=96, ny=4, dt=probe.dt, n_high=5)
    cfg = dict(w["cfg"], pond=1, n_low=4, cfl=0.45, crit_kind=inputs.CRIT_KN, crit_thr=0.02,
               crit_every=5, crit_margin=4)
    st = O.Oracle(dict(cfg, pond=0, crit_margin=0))
    st.set_mask(w["mask"], convert=False)
    st.init(w["rho"], w["u"], w["T"])
    sel = st.eval_criterion()[0]          # the co-moving selection at the initial state
    p = O.Pond(cfg)
    p.set_mask(w["mask"], convert=False)
    p.init(w["rho"], w["u"], w["T"])
    p.step(1)
    assert np.array_equal(p.get_mask().reshape(sel.shape), O.dilate_mask(cfg, sel))
