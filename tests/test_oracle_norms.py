"""Pins of the oracle's error norms (the L2 / max norms of the reductions
row): closed forms on hand-made fields."""
import math

import numpy as np

from oracle.oracle import error_norms


def test_scaled_reference_gives_epsilon():
    rng = np.random.default_rng(1)
    rho = 1 + 0.1 * rng.random((1, 7, 9))
    u = rng.normal(size=(2, 1, 7, 9))
    T = 1 + 0.2 * rng.random((1, 7, 9))
    eps = 0.03
    n = error_norms(rho, u, T, rho / (1 + eps), u / (1 + eps), T / (1 + eps))
    for name, x in (("rho", rho), ("T", T)):
        assert abs(n[name][0] - eps) < 1e-14
        assert abs(n[name][1] - eps * np.max(np.abs(x)) / (1 + eps)) < 1e-15
    assert abs(n["u"][0] - eps) < 1e-14
    umag = np.sqrt(np.sum(u ** 2, axis=0))
    assert abs(n["u"][1] - eps * np.max(umag) / (1 + eps)) < 1e-14


def test_single_cell_and_vector_norm():
    N = 400
    rho = np.ones((1, 20, 20))
    ref = rho.copy()
    rho[0, 3, 4] += 1e-3
    u = np.zeros((2, 1, 20, 20))
    uref = np.full((2, 1, 20, 20), 0.5)
    u[:] = uref
    u[0, 0, 5, 5] += 3e-4
    u[1, 0, 5, 5] += 4e-4
    n = error_norms(rho, u, rho, ref, uref, None)
    assert abs(n["rho"][0] - 1e-3 / math.sqrt(N)) < 1e-17
    assert abs(n["rho"][1] - 1e-3) < 1e-15
    assert abs(n["u"][1] - 5e-4) < 1e-16
    assert abs(n["u"][0] - 5e-4 / math.sqrt(N * 0.5)) < 1e-17   # sum |u_ref|^2 = N * 2 * 0.25
    assert n["T"] == (0.0, 0.0)


def test_identical_and_zero_reference():
    x = np.linspace(0.5, 1.5, 30).reshape(1, 5, 6)
    n = error_norms(x, None, x, x, None, np.zeros_like(x))
    assert n["rho"] == (0.0, 0.0)
    # zero reference: the root mean square of the field itself
    assert abs(n["T"][0] - math.sqrt(np.mean(x ** 2))) < 1e-15
    assert n["T"][1] == 1.5
