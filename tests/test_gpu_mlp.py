"""GPU checks of the learned lifting closure against the oracle.

- forward pass of the BF16 matrix-core network against the oracle's network
  with BF16-rounded operands (FP64 sums);
- gradients against the oracle's FP64 back-propagation: cosine >= 0.999 and
  relative error <= 2e-2;
- snapshot features and targets against the oracle's definitions;
- a multi-step run with the learned lift against the oracle with the same
  network (BF16-emulating), and the per-tile error check.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2102_12559_amd import closure, inputs
from tests.gpu_util import say, weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mlp_solver(n_high=6, hidden=64, nx=16, ny=16, store=inputs.STORE_FP64):
    from paper_2102_12559_amd import msl
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=n_high, lift_mode=inputs.LIFT_MLP,
                             store=store, mlp_hidden=hidden, tau=0.7)
    return msl.Solver(cfg), cfg


def random_net(F, H, Od, seed):
    rng = np.random.default_rng(seed)
    p = closure.init_params(F, H, Od, seed=seed).astype(np.float64)
    nb = O.mlp_nparams(F, H, Od)
    p = p + rng.normal(0, 0.05, nb)          # non-zero biases too
    return p.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n_high", [4, 6])
def test_forward_matches_oracle(n_high):
    import torch
    s, _ = mlp_solver(n_high)
    F, Od, H, P = s.mlp_dims()
    say(f"[case] mlp forward F={F} O={Od} H={H}")
    p = random_net(F, H, Od, 1)
    ones = np.ones(F, np.float32)
    s.mlp_set_weights(p.astype(np.float32), np.zeros(F, np.float32), ones,
                      np.zeros(Od, np.float32), np.ones(Od, np.float32))
    X = np.random.default_rng(2).normal(0, 1, (203, F)).astype(np.float32)
    Yg = s.mlp_forward(torch.as_tensor(X)).cpu().numpy()
    Yo = O.mlp_forward(p, F, H, Od, X.astype(np.float64), bf16=True)
    err = np.max(np.abs(Yg - Yo)) / np.max(np.abs(Yo))
    say(f"  forward max rel err {err:.2e}")
    assert err < 1e-2


@pytest.mark.parametrize("n", [64, 1000])
def test_gradient_matches_oracle(n):
    import torch
    s, _ = mlp_solver(6)
    F, Od, H, P = s.mlp_dims()
    say(f"[case] mlp gradient n={n}")
    p = random_net(F, H, Od, 3)
    ones = np.ones(F, np.float32)
    s.mlp_set_weights(p.astype(np.float32), np.zeros(F, np.float32), ones,
                      np.zeros(Od, np.float32), np.ones(Od, np.float32))
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (n, F)).astype(np.float32)
    Y = rng.normal(0, 1, (n, Od)).astype(np.float32)
    lg, gg = s.mlp_grad(torch.as_tensor(X), torch.as_tensor(Y))
    gg = gg.cpu().numpy().astype(np.float64)
    lo, go = O.mlp_loss_grad(p, F, H, Od, X.astype(np.float64), Y.astype(np.float64))
    cos = float(gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go)))
    rel = float(np.linalg.norm(gg - go) / np.linalg.norm(go))
    say(f"  loss gpu {lg:.6f} oracle {lo:.6f}; grad cosine {cos:.6f} rel {rel:.3e}")
    assert abs(lg - lo) < 2e-2 * lo
    assert cos >= 0.999 and rel <= 2e-2


def test_training_reduces_loss():
    import torch
    s, _ = mlp_solver(4)
    F, Od, H, P = s.mlp_dims()
    say("[case] mlp training on a smooth target")
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (4096, F)).astype(np.float32)
    A = rng.normal(0, 0.5, (F, Od))
    Y = np.tanh(X @ A).astype(np.float32)
    p0 = closure.init_params(F, H, Od, seed=0)
    ones = np.ones(F, np.float32)
    s.mlp_set_weights(p0, np.zeros(F, np.float32), ones, np.zeros(Od, np.float32),
                      np.ones(Od, np.float32))
    log = s.mlp_train(torch.as_tensor(X), torch.as_tensor(Y), batch=256, epochs=20, lr=3e-3)
    say(f"  loss first {log[:4].mean():.4f} last {log[-4:].mean():.4f}")
    assert log[-4:].mean() < 0.1 * log[:4].mean()


def test_snapshots_match_oracle_definitions():
    import torch
    from paper_2102_12559_amd import msl
    nx, ny = 16, 12
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, lift_mode=inputs.LIFT_MLP,
                             store=inputs.STORE_FP64, tau=0.7, thermal=1)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.2, seed=7, drho=0.03, dT=0.05)
    say("[case] snapshots")
    s = msl.Solver(cfg)
    s.set_mask(np.ones((1, ny, nx), np.uint8))
    s.init(rho, u, T)
    s.step(5)
    X, Y = s.collect_snapshots(nx * ny)
    X, Y = X.cpu().numpy(), Y.cpu().numpy()
    fQ = s.get_populations(1).cpu().numpy()
    gQ = s.get_populations(1, fg=1).cpu().numpy()
    for k in (0, 37, nx * ny - 1):
        fq, gq = O.project(2, 6, 3, fQ[:, k], gQ[:, k])
        fr = O.mlp_features(2, 3, fq, gq, thermal=1, cv=1.5)
        tr = O.mlp_targets(2, 3, 6, fQ[:, k], gQ[:, k], thermal=1, cv=1.5)
        assert np.allclose(X[k], fr, rtol=1e-5, atol=1e-6), (k, X[k], fr)
        assert np.allclose(Y[k], tr, rtol=1e-4, atol=1e-6 * np.max(np.abs(tr))), k


def test_learned_lift_step_matches_oracle():
    """Random-mask run with the learned lift (fixed flags: every tile uses the
    network) against the oracle running the same network with BF16 operands."""
    from paper_2102_12559_amd import msl
    from oracle.oracle import Oracle
    nx, ny = 80, 70
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, lift_mode=inputs.LIFT_MLP,
                             store=inputs.STORE_FP64, tau=0.7)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.25, seed=9, drho=0.02)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=5, blob=8)
    say("[case] learned lift run")
    s = msl.Solver(cfg)
    F, Od, H, P = s.mlp_dims()
    p = (closure.init_params(F, H, Od, seed=11) * 0.5).astype(np.float32)
    xm = np.zeros(F, np.float32); xm[0] = 1.0
    xs = np.full(F, 0.5, np.float32)
    tm = np.zeros(Od, np.float32)
    ts = np.full(Od, 1e-3, np.float32)
    s.mlp_set_weights(p, xm, xs, tm, ts)
    ntile = s.num_check_tiles()
    flags = np.ones(ntile, np.uint8)
    s.mlp_set_flags(flags)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(10)
    o = Oracle(cfg)
    o.set_mlp(H, p.astype(np.float64), xm.astype(np.float64), xs.astype(np.float64),
              tm.astype(np.float64), ts.astype(np.float64), bf16=True, manual_check=True)
    o.set_mlp_flags(flags)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(10)
    m = s.get_mask().cpu().numpy().reshape(-1)
    worst = 0.0
    for which in (0, 1):
        sel = m == which
        g = s.get_populations(which).cpu().numpy()[:, sel]
        r = o.get_pops(which)[:, sel]
        W = weights(2, 3 if which == 0 else 6)[:, None]
        e = np.max(np.abs(g - r) / np.maximum(np.abs(r), W))
        say(f"  set {which}: max rel err {e:.3e}")
        worst = max(worst, e)
    # the network itself runs in BF16 on both sides, its hidden activations are
    # rounded from FP32 (GPU) and FP64 (oracle) sums
    assert worst < 1e-4
    # the closure really acted: the plain-lift run differs
    cfg2 = dict(cfg, lift_mode=inputs.LIFT_GRAD)
    o2 = Oracle(cfg2)
    o2.set_mask(mask, convert=False)
    o2.init(rho, u, T)
    o2.step(10)
    d = np.max(np.abs(o2.get_pops(0)[:, m == 0] - o.get_pops(0)[:, m == 0]))
    say(f"  learned vs plain lift difference {d:.3e}")
    assert d > 1e-6


def test_error_check_flags_match_oracle():
    from paper_2102_12559_amd import msl
    from oracle.oracle import Oracle
    nx, ny = 150, 130   # several 64 x 64 check tiles
    cfg = inputs.base_config(nx=nx, ny=ny, n_low=3, n_high=6, lift_mode=inputs.LIFT_MLP,
                             store=inputs.STORE_FP64, tau=0.7)
    rho, u, T = inputs.smooth_random_flow(nx, ny, umax=0.25, seed=12, drho=0.02)
    mask = inputs.random_mask(nx, ny, frac=0.3, seed=6, blob=10)
    say("[case] error check flags")
    s = msl.Solver(cfg)
    F, Od, H, P = s.mlp_dims()
    p = (closure.init_params(F, H, Od, seed=21) * 0.3).astype(np.float32)
    xm = np.zeros(F, np.float32); xm[0] = 1.0
    xs = np.full(F, 0.5, np.float32)
    tm = np.zeros(Od, np.float32)
    ts = np.full(Od, 1e-3, np.float32)
    s.mlp_set_weights(p, xm, xs, tm, ts)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(21)   # checks at steps 0 and 20
    fg = s.mlp_get_flags().cpu().numpy()
    o = Oracle(cfg)
    o.set_mlp(H, p.astype(np.float64), xm.astype(np.float64), xs.astype(np.float64),
              tm.astype(np.float64), ts.astype(np.float64), bf16=True)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(21)
    fo, em, eg = o.mlp_flags()
    decisive = np.abs(em - eg) > 0.05 * np.maximum(eg, 1e-300)
    say(f"  flags gpu {fg.tolist()} oracle {fo.tolist()} decisive {decisive.sum()}/{fo.size}")
    assert np.array_equal(fg[decisive], fo[decisive])


def test_learned_lift_3d_matches_oracle():
    """3D (D3Q27 / D3Q64) run with the learned lift on every tile against the
    oracle running the same network with BF16 operands."""
    from paper_2102_12559_amd import msl
    from oracle.oracle import Oracle
    n = 14
    cfg = inputs.base_config(dim=3, nx=n, ny=n, nz=n, n_low=3, n_high=4, lift_mode=inputs.LIFT_MLP,
                             store=inputs.STORE_FP64, tau=0.7)
    rho, u, T = inputs.smooth_random_flow(n, n, n, umax=0.2, seed=13, drho=0.02)
    mask = np.zeros((n, n, n), np.uint8)
    mask[:, 4:9, :] = 1
    say("[case] learned lift 3D run")
    s = msl.Solver(cfg)
    F, Od, H, P = s.mlp_dims()
    assert (F, Od) == (28, 37)
    p = (closure.init_params(F, H, Od, seed=17) * 0.5).astype(np.float32)
    xm = np.zeros(F, np.float32); xm[0] = 1.0
    xs = np.full(F, 0.5, np.float32)
    tm = np.zeros(Od, np.float32)
    ts = np.full(Od, 1e-3, np.float32)
    s.mlp_set_weights(p, xm, xs, tm, ts)
    flags = np.ones(s.num_check_tiles(), np.uint8)
    s.mlp_set_flags(flags)
    s.set_mask(mask)
    s.init(rho, u, T)
    s.step(6)
    o = Oracle(cfg)
    o.set_mlp(H, p.astype(np.float64), xm.astype(np.float64), xs.astype(np.float64),
              tm.astype(np.float64), ts.astype(np.float64), bf16=True, manual_check=True)
    o.set_mlp_flags(flags)
    o.set_mask(mask, convert=False)
    o.init(rho, u, T)
    o.step(6)
    m = s.get_mask().cpu().numpy().reshape(-1)
    worst = 0.0
    for which in (0, 1):
        sel = m == which
        g = s.get_populations(which).cpu().numpy()[:, sel]
        r = o.get_pops(which)[:, sel]
        W = weights(3, 3 if which == 0 else 4)[:, None]
        e = np.max(np.abs(g - r) / np.maximum(np.abs(r), W))
        say(f"  set {which}: max rel err {e:.3e}")
        worst = max(worst, e)
    assert worst < 1e-4
