"""Training and use of the learned lifting closure.

The network replaces the equilibrium completion of the lifting step (missing
raw moments set to their equilibrium values, Sec. III.B) by the equilibrium
values plus a learned estimate of their non-equilibrium part.  It is trained
on snapshots of runs that use the high-order velocity set everywhere: each
high-order cell's state is projected onto the low-order set (Sec. III.C), the
features are the normalised low-order moments of that projection, the
targets the normalised non-equilibrium parts of the missing raw moments of the
high-order state.  Collection, training (BF16 matrix cores, FP32 Adam) and
inference all run in libmsl; this module only orchestrates them.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs, msl


def init_params(F, H, O, seed=0):
    """Uniform Glorot initialisation from the seeded generator; zero biases."""
    sizes = [(F, H), (H,), (H, H), (H,), (H, O), (O,)]
    r = inputs.uniform_pm1(seed, F * H + H * H + H * O)
    out, k = [], 0
    for s in sizes:
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            out.append(lim * r[k:k + s[0] * s[1]])
            k += s[0] * s[1]
        else:
            out.append(np.zeros(s[0]))
    return np.concatenate(out).astype(np.float32)


XSTD_FLOOR = 1e-6   # spread below which a feature counts as constant
XCLIP = 8.0         # standardised features are limited to +-8 (as in the library)


def standardize(X, Y):
    """Column means and standard deviations.  A feature that hardly varies in
    the training data (u_z of a columnar flow) gets a spread of at least
    XSTD_FLOOR, so that a small change of it in use does not become a huge
    network input; targets with no spread get 1."""
    xm = X.mean(axis=0)
    xs = np.maximum(X.std(axis=0), XSTD_FLOOR)
    ym = Y.mean(axis=0)
    ys = Y.std(axis=0)
    ys[ys < 1e-12] = 1.0
    return (xm.astype(np.float32), xs.astype(np.float32), ym.astype(np.float32),
            ys.astype(np.float32))


def couette_case(N, kn, *, n_high=6, store=inputs.STORE_FP32, band=4, lift_mode=inputs.LIFT_GRAD,
                 nx=8, thermal=0, hidden=64):
    """A Couette configuration (with the time step of the D2Q9/high-order pair)."""
    probe = msl.Solver(inputs.base_config(nx=8, ny=8, n_low=3, n_high=n_high))
    dt = probe.dt
    probe.close()
    w = inputs.couette_c4(N=N, kn=kn, band=band, dt=dt, store=store, n_high=n_high,
                          lift_mode=lift_mode, nx=nx, thermal=thermal)
    w["cfg"]["mlp_hidden"] = hidden
    return w


def collect_snapshots(cases, times, n_high=6, hidden=64):
    """Snapshots of full high-order Couette runs: for each (N, Kn) case, the
    state after each number of steps in `times` (ascending).  Returns host
    float32 arrays X [rows][F], Y [rows][O]."""
    Xs, Ys = [], []
    for (N, kn) in cases:
        w = couette_case(N, kn, n_high=n_high, lift_mode=inputs.LIFT_MLP, hidden=hidden)
        s = msl.Solver(w["cfg"])
        s.set_mask(np.ones_like(w["mask"]))
        s.init(w["rho"], w["u"], w["T"])
        done = 0
        for t in times:
            s.step(t - done)
            done = t
            X, Y = s.collect_snapshots(s.ncell)
            Xs.append(X.cpu().numpy())
            Ys.append(Y.cpu().numpy())
        s.close()
    return np.concatenate(Xs), np.concatenate(Ys)


def snapshots_of_run(w, times, max_rows=None):
    """Snapshots of a run of workload `w` on the high-order set everywhere
    (its mask is replaced by all ones and its criterion switched off; the
    configuration must use the learned lift so that the closure buffers
    exist): features and targets of every
    cell after each number of steps in `times` (ascending), at most
    `max_rows` per time (every k-th cell in cell order).  Host float32."""
    s = msl.Solver(dict(w["cfg"], crit_kind=inputs.CRIT_NONE))   # stays on the high-order set
    s.set_mask(np.ones_like(w["mask"]))
    s.init(w["rho"], w["u"], w["T"])
    Xs, Ys = [], []
    done = 0
    for t in times:
        s.step(t - done)
        done = t
        X, Y = s.collect_snapshots(s.ncell)
        X, Y = X.cpu().numpy(), Y.cpu().numpy()
        if max_rows and X.shape[0] > max_rows:
            k = -(-X.shape[0] // max_rows)
            X, Y = X[::k], Y[::k]
        Xs.append(X)
        Ys.append(Y)
    s.close()
    return np.concatenate(Xs), np.concatenate(Ys)


def train(X, Y, *, epochs=50, batch=1024, lr=1e-3, hidden=64, seed=0, n_high=6, val_frac=0.1,
          schedule=None, cfg=None):
    """Train the closure on the GPU.  Rows are shuffled with the seeded
    generator and split into training and validation parts.  `schedule`, a
    list of (epochs, learning rate) phases run one after the other with the
    optimiser state carried over, replaces (epochs, lr).  `cfg` is the
    configuration whose network shape is trained (default: the 2D D2Q9/D2Q36
    Couette case).  Returns a dict with the parameters, standardisation
    statistics and loss history."""
    import torch
    rows = X.shape[0]
    order = np.argsort(inputs.uniform_pm1(seed + 17, rows), kind="stable")
    X = X[order]
    Y = Y[order]
    nval = int(round(val_frac * rows))
    Xt, Yt, Xv, Yv = X[nval:], Y[nval:], X[:nval], Y[:nval]
    xm, xs, ym, ys = standardize(Xt.astype(np.float64), Yt.astype(np.float64))
    if cfg is None:
        cfg = couette_case(32, 0.1, n_high=n_high, lift_mode=inputs.LIFT_MLP, hidden=hidden)["cfg"]
    s = msl.Solver(cfg)
    F, O, H, P = s.mlp_dims()
    p0 = init_params(F, H, O, seed=seed)
    s.mlp_set_weights(p0, xm, xs, ym, ys)
    dev = s.device
    Xn = torch.as_tensor(np.clip((Xt - xm) / xs, -XCLIP, XCLIP), dtype=torch.float32, device=dev)
    Yn = torch.as_tensor((Yt - ym) / ys, dtype=torch.float32, device=dev)
    phases = schedule if schedule else [(epochs, lr)]
    log = np.concatenate([s.mlp_train(Xn, Yn, batch=batch, epochs=e, lr=r) for e, r in phases])
    params = s.mlp_get_weights()
    val = None
    if nval:
        Xvn = torch.as_tensor(np.clip((Xv - xm) / xs, -XCLIP, XCLIP), dtype=torch.float32, device=dev)
        pred = s.mlp_forward(Xvn).cpu().numpy()
        val = float(np.mean((pred - (Yv - ym) / ys) ** 2))
    s.close()
    return dict(params=params, xmean=xm, xstd=xs, tmean=ym, tstd=ys, loss=log, val_mse=val,
                F=F, O=O, H=H)


def install(solver, net):
    solver.mlp_set_weights(net["params"], net["xmean"], net["xstd"], net["tmean"], net["tstd"])
