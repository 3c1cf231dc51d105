"""Pins of the oracle's velocity sets and lattice equilibrium.

Each check is against something other than the oracle itself: the paper's
printed closed forms (Table I, eqs. QxxxL, RxxL, QxxxPonD, RxxPond, Fig. 1),
textbook Gaussian moments, a library polynomial root finder, and the Hermite
product form of the equilibrium derived independently below.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    for line in open(os.path.join(GOLD, "table1_gauss_hermite.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, cx, wx = line.split()
        env = {"sqrt": math.sqrt}
        rows.append((int(n), eval(cx, env), eval(wx, env)))
    return rows


def test_table1_nodes_and_weights():
    rows = _table1()
    for n in (3, 4, 5):
        x, w = O.gh_rule(n)
        ref = sorted([(c, wt) for (m, c, wt) in rows if m == n])
        # the printed nodes are the non-negative ones; the rule is symmetric
        pos = [(xv, wv) for xv, wv in zip(x, w) if xv >= -1e-15]
        assert len(pos) == len(ref)
        for (xv, wv), (c, wt) in zip(sorted(pos), ref):
            assert abs(xv - c) < 1e-14
            assert abs(wv - wt) < 1e-14
        assert np.allclose(x, -x[::-1], atol=1e-15)
        assert np.allclose(w, w[::-1], atol=1e-15)


def test_d1q6_nodes_are_hermite6_roots():
    # He_6(x) = x^6 - 15 x^4 + 45 x^2 - 15: x^2 are the roots of y^3 - 15y^2 + 45y - 15
    y = np.sort(np.roots([1.0, -15.0, 45.0, -15.0]).real)
    ref = np.sort(np.concatenate([-np.sqrt(y), np.sqrt(y)]))
    x, w = O.gh_rule(6)
    assert np.allclose(x, ref, atol=1e-13)


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_gauss_hermite_exactness(n):
    # sum_k w_k x_k^j = E[Z^j] (standard normal) for j <= 2n-1
    x, w = O.gh_rule(n)
    for j in range(2 * n):
        ez = 0.0 if j % 2 else float(np.prod(np.arange(j - 1, 0, -2))) if j else 1.0
        assert abs(np.sum(w * x ** j) - ez) < 1e-12 * max(1.0, ez)
    # and fails at degree 2n (so the rule is exactly of that order)
    j = 2 * n
    ez = float(np.prod(np.arange(j - 1, 0, -2)))
    assert abs(np.sum(w * x ** j) - ez) > 1e-3


def _hermite_table(c, nmax):
    # He_j(c) by the three-term recurrence, independent of the oracle
    H = np.zeros((nmax, len(c)))
    H[0] = 1.0
    if nmax > 1:
        H[1] = c
    for j in range(1, nmax - 1):
        H[j + 1] = c * H[j] - j * H[j - 1]
    return H


def product_feq(dim, n, rho, u, theta):
    """Closed product form of the lattice equilibrium.

    In 1D the lattice equilibrium must reproduce E[(sqrt(theta) Z + u)^m] for
    m < n; with Gauss-Hermite orthogonality its populations are
    w_a sum_{j<n} He_j(c_a) b_j / j!, with b_j = E[He_j(X)], X ~ N(u, theta),
    whose generating function is exp(u t + (theta-1) t^2 / 2).  The tensor
    product of the 1D factors reproduces every mixed moment with powers < n.
    """
    x, w = O.gh_rule(n)
    # b_j from the generating function: b_{j+1} = u b_j + j (theta - 1) b_{j-1}
    P = []
    H = _hermite_table(x, n)
    for a in range(dim):
        b = np.zeros(n)
        b[0] = 1.0
        if n > 1:
            b[1] = u[a]
        for j in range(1, n - 1):
            b[j + 1] = u[a] * b[j] + j * (theta - 1.0) * b[j - 1]
        fac = np.array([math.factorial(j) for j in range(n)], dtype=float)
        P.append(w * (H.T @ (b / fac)))
    out = np.zeros(n ** dim)
    for i in range(n ** dim):
        r, v = i, rho
        for a in range(dim):
            v *= P[a][r % n]
            r //= n
        out[i] = v
    return out


@pytest.mark.parametrize("dim,n", [(2, 3), (2, 4), (2, 5), (2, 6), (3, 3), (3, 4)])
@pytest.mark.parametrize("theta", [1.0, 1.7])
def test_transform_equilibrium_equals_product_form(dim, n, theta):
    u = np.array([0.31, -0.17, 0.09])[:dim]
    f = O.lattice_feq(dim, n, 1.13, u, theta)
    g = product_feq(dim, n, 1.13, u, theta)
    assert np.max(np.abs(f - g)) < 1e-14


def gaussian_moment(m, mu, var):
    # E[(sqrt(var) Z + mu)^m] by the binomial expansion and E[Z^k] = (k-1)!!
    s = 0.0
    for k in range(0, m + 1, 2):
        ez = float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0
        s += math.comb(m, k) * mu ** (m - k) * var ** (k / 2) * ez
    return s


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_lattice_reproduces_equilibrium_moments(n):
    # sum_i f^L_i c_x^m c_y^k = rho E[(sqrt(theta)Z+u_x)^m] E[(sqrt(theta)Z+u_y)^k], m,k < n
    rho, u, theta = 0.93, np.array([0.4, -0.25]), 1.3
    f = O.lattice_feq(2, n, rho, u, theta)
    x, _ = O.gh_rule(n)
    cx = np.array([x[i % n] for i in range(n * n)])
    cy = np.array([x[i // n] for i in range(n * n)])
    for m in range(n):
        for k in range(n):
            lhs = np.sum(f * cx ** m * cy ** k)
            rhs = rho * gaussian_moment(m, u[0], theta) * gaussian_moment(k, u[1], theta)
            assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))


def _gold_moments():
    d = {}
    for line in open(os.path.join(GOLD, "lattice_moments.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            d[k] = v
    return d


def _diag_moment(n, rho, u, order):
    f = O.lattice_feq(2, n, rho, np.array([u, 0.0]), 1.0)
    x, _ = O.gh_rule(n)
    cx = np.array([x[i % n] for i in range(n * n)])
    return np.sum(f * cx ** order)


@pytest.mark.parametrize("u", [0.1, 0.4, 0.9])
def test_printed_diagonal_moments(u):
    g = _gold_moments()
    env = dict(rho=1.2, u=u, T=1.0)
    # D2Q9: eqs. QxxxL, RxxL
    assert abs(_diag_moment(3, 1.2, u, 3) - eval(g["QxxxL9"], env)) < 1e-13
    assert abs(_diag_moment(3, 1.2, u, 4) - eval(g["RxxxxL9"], env)) < 1e-13
    # D2Q16 carries the Maxwell-Boltzmann third moment (eq. QxxxPonD) but not the fourth
    assert abs(_diag_moment(4, 1.2, u, 3) - eval(g["QxxxMB"], env)) < 1e-13
    assert abs(_diag_moment(4, 1.2, u, 4) - eval(g["RxxxxMB"], env)) > 1e-4 * u ** 4
    # D2Q25 and D2Q36 carry both (eq. RxxPond)
    for n in (5, 6):
        assert abs(_diag_moment(n, 1.2, u, 3) - eval(g["QxxxMB"], env)) < 1e-12
        assert abs(_diag_moment(n, 1.2, u, 4) - eval(g["RxxxxMB"], env)) < 1e-12


def test_fig1_deviation_three_percent():
    g = _gold_moments()
    ma = float(g["FIG1_MA"])
    env = dict(rho=1.0, u=ma, T=1.0)
    eps9 = (_diag_moment(3, 1.0, ma, 3) - eval(g["QxxxMB"], env)) / eval(g["QxxxMB"], env)
    assert abs(abs(eps9) * 100 - float(g["FIG1_EPS_PERCENT"])) < 0.2
    eps25 = (_diag_moment(5, 1.0, ma, 3) - eval(g["QxxxMB"], env)) / eval(g["QxxxMB"], env)
    assert abs(eps25) < 1e-13


def test_moment_matrix_rows_are_monomials():
    # row (m, k) of the D2Q16 moment matrix applied to f is sum_i c_x^m c_y^k f_i
    n = 4
    M, Mi = O.moment_matrix(2, n)
    x, _ = O.gh_rule(n)
    f = np.linspace(0.1, 1.0, n * n)
    cx = np.array([x[i % n] for i in range(n * n)])
    cy = np.array([x[i // n] for i in range(n * n)])
    for j in range(n * n):
        m, k = j % n, j // n
        assert abs(M[j] @ f - np.sum(cx ** m * cy ** k * f)) < 1e-12
    assert np.allclose(M @ Mi, np.eye(n * n), atol=1e-9)
