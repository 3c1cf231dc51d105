"""The allocation-free gradient entry point (msl_mlp_grad_noalloc) against
msl_mlp_grad through the C-ABI: the same kernels with the partials in the
library's static device array, so loss and gradient must agree exactly, on
two calls in a row (the second with fewer rows, so the array still holds the
first call's larger partials), and a request beyond the array's size is
refused before any GPU work."""
import ctypes as C

import numpy as np
import pytest

from paper_2102_12559_amd import closure, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dim,n_high", [(2, 6), (3, 4)])
def test_grad_noalloc_matches_workspace_entry(dim, n_high):
    import torch
    from paper_2102_12559_amd import msl
    n = 16
    cfg = inputs.base_config(dim=dim, nx=n, ny=n, nz=n if dim == 3 else 1, n_low=3, n_high=n_high,
                             lift_mode=inputs.LIFT_MLP, store=inputs.STORE_FP32, tau=0.7)
    s = msl.Solver(cfg)
    F, Od, H, P = s.mlp_dims()
    p = closure.init_params(F, H, Od, seed=5).astype(np.float32)
    s.mlp_set_weights(p, np.zeros(F, np.float32), np.ones(F, np.float32), np.zeros(Od, np.float32),
                      np.ones(Od, np.float32))
    rng = np.random.default_rng(dim)
    for rows in (2000, 333):
        print(f"[case] dim={dim} rows={rows} P={P}", flush=True)
        X = torch.as_tensor(rng.normal(0, 1, (rows, F)).astype(np.float32))
        Y = torch.as_tensor(rng.normal(0, 1, (rows, Od)).astype(np.float32))
        l1, g1 = s.mlp_grad(X, Y)
        l2, g2 = s.mlp_grad_noalloc(X, Y)
        g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
        print(f"  loss {l1:.7f} / {l2:.7f}, max |dg| {np.max(np.abs(g1 - g2)):.3e}", flush=True)
        assert np.isfinite(l1) and l1 == l2
        assert np.array_equal(g1, g2)
    # beyond the static array: refused on the host
    rows = 16384
    need = (rows // 64) * (P + 1) + 1
    assert need > (1 << 20)
    X = torch.zeros((rows, F), dtype=torch.float32, device="cuda")
    Y = torch.zeros((rows, Od), dtype=torch.float32, device="cuda")
    g = torch.empty(P, dtype=torch.float32, device="cuda")
    loss = C.c_float()
    rc = msl.lib().msl_mlp_grad_noalloc(s._ctx, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), rows,
                                        C.byref(loss), C.c_void_p(g.data_ptr()))
    assert rc == msl.MSL_EINVAL
    assert b"static array" in msl.lib().msl_last_error(s._ctx)
    s.close()
