"""Pins of the contact-solver oracle (projected Gauss-Seidel on the MLCP
a = A x + b, lo <= x <= hi, and its adjoint; Sec. 4.1, Eq. mlcp; App. C)
against what the mathematics fixes: the linear solve it converges to
without bounds, the exact complementarity solution found by enumerating
the active sets of small problems, a hand-computed sweep, complex-step
derivatives of the solve, and the implicit-function gradient of the
converged unbounded solve.  CPU only.
"""
import itertools

import numpy as np
import pytest

import oracle as O

BIG = 1e300


def _spd(n, rng, cond=10.0):
    """A random symmetric positive definite matrix (a Delassus-like
    operator J M^-1 J^T) with eigenvalues in [1, cond]."""
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return Q @ np.diag(np.linspace(1.0, cond, n)) @ Q.T


def test_unbounded_converges_to_the_linear_solve():
    """With no active bounds PGS is Gauss-Seidel on A x = -b, which converges
    for symmetric positive definite A."""
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 12):
        A, b = _spd(n, rng), rng.normal(size=n)
        x = O.pgs_solve(A, b, -BIG * np.ones(n), BIG * np.ones(n), np.zeros(n), 400)
        assert np.allclose(x, np.linalg.solve(A, -b), rtol=0, atol=1e-11)


def _lcp_by_enumeration(A, b, lo, hi):
    """The unique solution of the box-constrained MLCP with SPD A: every
    assignment of rows to {at lo, at hi, free} is tried; the free rows solve
    A_FF x_F = -(b_F + A_FC x_C); the assignment is kept if x respects the
    box and the residual a = A x + b has the sign its bound requires."""
    n = len(b)
    found = []
    for states in itertools.product((-1, 0, 1), repeat=n):
        if any((s == -1 and lo[i] <= -BIG) or (s == 1 and hi[i] >= BIG) for i, s in enumerate(states)):
            continue
        x = np.array([lo[i] if s == -1 else hi[i] if s == 1 else 0.0 for i, s in enumerate(states)])
        F = [i for i, s in enumerate(states) if s == 0]
        C = [i for i, s in enumerate(states) if s != 0]
        if F:
            x[F] = np.linalg.solve(A[np.ix_(F, F)], -(b[F] + A[np.ix_(F, C)] @ x[C]))
        a = A @ x + b
        ok = all((s == 0 and lo[i] - 1e-12 <= x[i] <= hi[i] + 1e-12) or (s == -1 and a[i] >= -1e-12) or
                 (s == 1 and a[i] <= 1e-12) for i, s in enumerate(states))
        if ok:
            found.append(x)
    assert found
    for x in found[1:]:
        assert np.allclose(x, found[0], atol=1e-9)
    return found[0]


@pytest.mark.parametrize("kind", ["lcp", "box"])
def test_converges_to_the_complementarity_solution(kind):
    """Small problems with active bounds: the solve after many sweeps equals
    the solution found by enumerating the active sets."""
    rng = np.random.default_rng(1 if kind == "lcp" else 2)
    for trial in range(40):
        n = int(rng.integers(1, 5))
        A, b = _spd(n, rng, 5.0), rng.normal(0, 2, n)
        if kind == "lcp":
            lo, hi = np.zeros(n), BIG * np.ones(n)
        else:
            lo, hi = -rng.uniform(0.1, 1.0, n), rng.uniform(0.1, 1.0, n)
        x = O.pgs_solve(A, b, lo, hi, np.zeros(n), 600)
        ref = _lcp_by_enumeration(A, b, lo, hi)
        assert np.allclose(x, ref, atol=1e-9), (trial, x, ref)
        if kind == "lcp":   # 0 <= a perp x >= 0
            a = A @ x + b
            assert np.all(x >= 0) and np.all(a >= -1e-9) and abs(a @ x) < 1e-9


def test_one_sweep_by_hand():
    """Two rows, one sweep: x1 = clamp(-(b1 + A12 x2_0)/A11), then x2 uses
    the new x1."""
    A = np.array([[2.0, 1.0], [0.5, 4.0]])
    b = np.array([1.0, -3.0])
    lo, hi = np.array([-0.2, -1.0]), np.array([1.0, 0.6])
    x0 = np.array([0.3, 0.7])
    x1 = min(max(-(1.0 + 1.0 * 0.7) / 2.0, -0.2), 1.0)   # -0.85 -> -0.2
    x2 = min(max(-(-3.0 + 0.5 * x1) / 4.0, -1.0), 0.6)   # 0.775 -> 0.6
    x, sw = O.pgs_solve(A, b, lo, hi, x0, 1, sweeps=True)
    assert np.array_equal(x, [x1, x2]) and np.array_equal(sw, [x0, [x1, x2]])
    # and the adjoint: both rows clamped, so every adjoint goes to a bound
    Ab, bb, lb, hb, x0b = O.pgs_adjoint(A, b, lo, hi, sw, np.array([1.5, -2.0]))
    assert np.array_equal(lb, [1.5, 0]) and np.array_equal(hb, [0, -2.0])
    assert not Ab.any() and not bb.any() and not x0b.any()


def _problem(seed, n, bounded=True):
    rng = np.random.default_rng(seed)
    A = _spd(n, rng, 6.0) + 0.3 * rng.normal(size=(n, n))   # not symmetric: every entry has its own adjoint
    A[np.diag_indices(n)] = np.abs(A[np.diag_indices(n)]) + 2.0
    b = rng.normal(0, 1.5, n)
    if bounded:
        lo, hi = -rng.uniform(0.05, 0.6, n), rng.uniform(0.05, 0.6, n)
    else:
        lo, hi = -BIG * np.ones(n), BIG * np.ones(n)
    x0 = rng.normal(0, 0.3, n)
    return A, b, lo, hi, x0, rng


@pytest.mark.parametrize("seed,niter", [(3, 12), (4, 12), (5, 12), (9, 2), (10, 3)])
def test_adjoint_against_complex_step(seed, niter):
    """Every input's adjoint (A, b, lo, hi, x0) after a few sweeps (far from
    converged, so every sweep's values matter), with bounds active on some
    rows, against complex-step derivatives of the solve along a random
    output weight."""
    n = 6
    A, b, lo, hi, x0, rng = _problem(seed, n)
    x, sw = O.pgs_solve(A, b, lo, hi, x0, niter, sweeps=True)
    w = rng.normal(size=n)
    Ab, bb, lb, hb, x0b = O.pgs_adjoint(A, b, lo, hi, sw, w)
    h = 1e-30

    def d(which, k):
        args = [A.astype(complex), b.astype(complex), lo.astype(complex), hi.astype(complex), x0.astype(complex)]
        args[which].reshape(-1)[k] += 1j * h
        return float((w @ O.pgs_solve_complex(*args, niter)).imag / h)

    for k in range(n * n):
        assert abs(d(0, k) - Ab.reshape(-1)[k]) < 1e-12, ("A", k)
    for which, ref in ((1, bb), (2, lb), (3, hb), (4, x0b)):
        for k in range(n):
            assert abs(d(which, k) - ref[k]) < 1e-12, (which, k)
    assert np.abs(lb).max() > 0 or np.abs(hb).max() > 0


def test_adjoint_of_the_converged_linear_solve():
    """Unbounded, many sweeps: x = -A^-1 b, so b_bar = -A^-T x_bar and
    A_bar = -(A^-T x_bar) x^T, and the start no longer matters."""
    n = 5
    A, b, lo, hi, x0, rng = _problem(6, n, bounded=False)
    x, sw = O.pgs_solve(A, b, lo, hi, x0, 400, sweeps=True)
    w = rng.normal(size=n)
    Ab, bb, lb, hb, x0b = O.pgs_adjoint(A, b, lo, hi, sw, w)
    lam = np.linalg.solve(A.T, w)
    assert np.allclose(bb, -lam, atol=1e-10)
    assert np.allclose(Ab, -np.outer(lam, x), atol=1e-10)
    assert np.abs(x0b).max() < 1e-10 and not lb.any() and not hb.any()
