"""Pins of the oracle's lifting and projection (Sec. III.B, III.C, App. C).

The checks use the defining properties, evaluated with numpy on the outputs:
lifting keeps every low-order raw moment and sets the others to the
high-order equilibrium's (computed with the independent product form);
projection keeps the low-order raw moments; both conserve mass, momentum and
energy; projection undoes lifting; equilibria map to equilibria.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.test_oracle_lattice import product_feq


def lattice(dim, n):
    x, w = O.gh_rule(n)
    Q = n ** dim
    c = np.zeros((Q, dim))
    W = np.ones(Q)
    pw = np.zeros((Q, dim), dtype=int)
    for i in range(Q):
        r = i
        for a in range(dim):
            c[i, a] = x[r % n]
            W[i] *= w[r % n]
            pw[i, a] = r % n
            r //= n
    return c, W, pw


def raw_moment(c, f, p):
    v = f.copy()
    for a in range(c.shape[1]):
        v = v * c[:, a] ** p[a]
    return v.sum()


def noneq_state(dim, n, seed=0, amp=0.05, thermal=False, cv=1.5):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.3, 0.3, dim)
    T = 1.0 + (0.2 if thermal else 0.0)
    f = product_feq(dim, n, 1.05, np.pad(u, (0, 3 - dim)), T)
    f = f * (1.0 + amp * rng.uniform(-1, 1, f.size))
    g = None
    if thermal:
        g = (cv - dim / 2) * T * product_feq(dim, n, 1.05, np.pad(u, (0, 3 - dim)), T)
        g = g * (1.0 + amp * rng.uniform(-1, 1, g.size))
    return f, g


PAIRS = [(2, 3, 4), (2, 3, 5), (2, 3, 6), (2, 4, 6), (3, 3, 4)]


def macros(c, f, g=None, cv=1.5):
    rho = f.sum()
    j = c.T @ f
    E = 0.5 * np.sum((c ** 2).sum(axis=1) * f) + (g.sum() if g is not None else 0.0)
    return rho, j, E


@pytest.mark.parametrize("dim,nq,nQ", PAIRS)
def test_lift_keeps_low_moments_and_completes_with_equilibrium(dim, nq, nQ):
    fq, _ = noneq_state(dim, nq, seed=1)
    fQ = O.lift(dim, nq, nQ, fq)
    cq, _, _ = lattice(dim, nq)
    cQ, _, pwQ = lattice(dim, nQ)
    rho, j, _ = macros(cq, fq)
    u = np.pad(j / rho, (0, 3 - dim))
    feqQ = product_feq(dim, nQ, rho, u, 1.0)
    for jj in range(nQ ** dim):
        p = pwQ[jj]
        got = raw_moment(cQ, fQ, p)
        if np.all(p < nq):
            ref = raw_moment(cq, fq, p)
        else:
            ref = raw_moment(cQ, feqQ, p)
        assert abs(got - ref) < 1e-10 * max(1.0, abs(ref)), (p, got, ref)


@pytest.mark.parametrize("dim,nq,nQ", PAIRS)
def test_project_keeps_low_moments(dim, nq, nQ):
    fQ, _ = noneq_state(dim, nQ, seed=2)
    fq = O.project(dim, nQ, nq, fQ)
    cq, _, pwq = lattice(dim, nq)
    cQ, _, _ = lattice(dim, nQ)
    for jj in range(nq ** dim):
        p = pwq[jj]
        ref = raw_moment(cQ, fQ, p)
        assert abs(raw_moment(cq, fq, p) - ref) < 1e-11 * max(1.0, abs(ref))


@pytest.mark.parametrize("dim,nq,nQ", PAIRS)
def test_project_after_lift_is_identity(dim, nq, nQ):
    fq, _ = noneq_state(dim, nq, seed=3, amp=0.2)
    back = O.project(dim, nQ, nq, O.lift(dim, nq, nQ, fq))
    assert np.max(np.abs(back - fq)) < 1e-13


@pytest.mark.parametrize("dim,nq,nQ", PAIRS)
def test_equilibria_map_to_equilibria(dim, nq, nQ):
    u = np.array([0.2, -0.15, 0.1])
    fq = product_feq(dim, nq, 0.97, u, 1.0)
    fQ = product_feq(dim, nQ, 0.97, u, 1.0)
    assert np.max(np.abs(O.lift(dim, nq, nQ, fq) - fQ)) < 1e-14
    assert np.max(np.abs(O.lift(dim, nq, nQ, fq, mode=1) - fQ)) < 1e-14
    assert np.max(np.abs(O.project(dim, nQ, nq, fQ) - fq)) < 1e-14


@pytest.mark.parametrize("dim,nq,nQ", [(2, 3, 4), (2, 3, 6)])
def test_thermal_lift_and_project_conserve(dim, nq, nQ):
    cv = 1.5
    fq, gq = noneq_state(dim, nq, seed=4, thermal=True, cv=cv)
    fQ, gQ = O.lift(dim, nq, nQ, fq, gq, thermal=1, cv=cv)
    cq, _, _ = lattice(dim, nq)
    cQ, _, _ = lattice(dim, nQ)
    a = macros(cq, fq, gq)
    b = macros(cQ, fQ, gQ)
    assert abs(a[0] - b[0]) < 1e-14 and np.allclose(a[1], b[1], atol=1e-14)
    assert abs(a[2] - b[2]) < 1e-13
    fQ2, gQ2 = noneq_state(dim, nQ, seed=5, thermal=True, cv=cv)
    fq2, gq2 = O.project(dim, nQ, nq, fQ2, gQ2)
    a = macros(cQ, fQ2, gQ2)
    b = macros(cq, fq2, gq2)
    assert abs(a[0] - b[0]) < 1e-14 and np.allclose(a[1], b[1], atol=1e-14)
    assert abs(a[2] - b[2]) < 1e-13


def test_lift_after_project_keeps_stress():
    # the conserved and stress moments of a high-order state survive the round trip
    dim, nq, nQ = 2, 3, 6
    fQ, _ = noneq_state(dim, nQ, seed=6)
    f2 = O.lift(dim, nq, nQ, O.project(dim, nQ, nq, fQ))
    cQ, _, _ = lattice(dim, nQ)
    for p in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]:
        ref = raw_moment(cQ, fQ, p)
        assert abs(raw_moment(cQ, f2, p) - ref) < 1e-11 * max(1.0, abs(ref))


def test_hermite_variant_differs_off_equilibrium():
    # raw-moment and Hermite-coefficient completion agree on equilibria (above) but
    # not on non-equilibrium states: the He_4 coefficient mixes in the second moment
    fq, _ = noneq_state(2, 3, seed=7, amp=0.1)
    a = O.lift(2, 3, 4, fq, mode=0)
    b = O.lift(2, 3, 4, fq, mode=1)
    assert np.max(np.abs(a - b)) > 1e-5
    # both keep the low-order moments
    cq, _, pq = lattice(2, 3)
    cQ, _, _ = lattice(2, 4)
    for p in pq:
        assert abs(raw_moment(cQ, a, p) - raw_moment(cq, fq, p)) < 1e-12
        assert abs(raw_moment(cQ, b, p) - raw_moment(cq, fq, p)) < 1e-12
