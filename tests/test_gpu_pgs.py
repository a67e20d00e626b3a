"""GPU parity of the contact solver (projected Gauss-Seidel on a batch of
MLCPs a = A x + b, lo <= x <= hi, and its adjoint; Sec. 4.1, Eq. mlcp;
App. C) against the FP64 oracle, through the C ABI: every row bucket
(n = 1 .. 16), partial and long solves, active bounds, FP64 to round-off and
FP32 within a stated bar, the autograd wrapper, the edge cases (no sweep,
empty batch), and sampled problems of the benchmark-size batch.

Inputs: Delassus-like operators A = J M^-1 J^T (symmetric positive definite,
eigenvalues in [1, 8]) plus a small non-symmetric part so that every entry
has its own adjoint, b ~ N(0, 1.5^2), box bounds of half-width U(0.05, 0.6)
on most rows and one-sided (lo = 0, hi large) on the rest, x0 ~ N(0, 0.3^2).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda"
BIG = {torch.float64: 1e300, torch.float32: 1e30}


def _batch(B, n, seed, dtype):
    rng = np.random.default_rng(seed)
    A = np.empty((B, n, n))
    for p in range(B):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        A[p] = Q @ np.diag(np.linspace(1.0, 8.0, n)) @ Q.T + 0.2 * rng.normal(size=(n, n))
        A[p][np.diag_indices(n)] = np.abs(A[p][np.diag_indices(n)]) + 1.0
    b = rng.normal(0, 1.5, (B, n))
    half = rng.uniform(0.05, 0.6, (B, n))
    lo, hi = -half, half.copy()
    one_sided = rng.uniform(size=(B, n)) < 0.3
    lo[one_sided] = 0.0
    hi[one_sided] = BIG[dtype]
    x0 = rng.normal(0, 0.3, (B, n))
    if dtype == torch.float32:
        A, b, lo, hi, x0 = (v.astype(np.float32).astype(np.float64) for v in (A, b, lo, hi, x0))
    return A, b, lo, hi, x0


def _t(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _oracle(A, b, lo, hi, x0, niter, xbar):
    out = []
    for p in range(A.shape[0]):
        x, sw = O.pgs_solve(A[p], b[p], lo[p], hi[p], x0[p], niter, sweeps=True)
        out.append((x, sw) + O.pgs_adjoint(A[p], b[p], lo[p], hi[p], sw, xbar[p]))
    return out


def _gpu(A, b, lo, hi, x0, niter, xbar, dtype):
    from paper_2109_07719_amd import pgs
    A_, b_, lo_, hi_, x0_, xb_ = (_t(v, dtype) for v in (A, b, lo, hi, x0, xbar))
    ws = pgs.new_workspace(A.shape[0], A.shape[1], niter, dtype)
    x = pgs.solve(A_, b_, lo_, hi_, x0_, niter, workspace=ws)
    g = pgs.adjoint(A_, b_, lo_, hi_, xb_, niter, ws)
    n, B = A.shape[1], A.shape[0]
    sw = ws[: (niter + 1) * n * B * (8 if dtype == torch.float64 else 4)].view(dtype).reshape(niter + 1, n, B)
    return [x.cpu().numpy(), sw.permute(2, 0, 1).cpu().numpy()] + [v.cpu().numpy() for v in g]


def _compare(gpu, ref, tol, floor):
    names = ("x", "sweeps", "A_bar", "b_bar", "lo_bar", "hi_bar", "x0_bar")
    worst = {}
    for p, r in enumerate(ref):
        for k, nm in enumerate(names):
            worst[nm] = max(worst.get(nm, 0.0), rel(gpu[k][p], r[k], floor))
    print({k: "%.1e" % v for k, v in worst.items()})
    assert max(worst.values()) < tol, worst


@pytest.mark.parametrize("n,niter", [(1, 5), (3, 1), (4, 30), (7, 12), (12, 50), (16, 20)])
def test_solve_and_adjoint_fp64_round_off(n, niter):
    A, b, lo, hi, x0 = _batch(300, n, 100 + n, torch.float64)
    xbar = np.random.default_rng(n).normal(size=(300, n))
    ref = _oracle(A, b, lo, hi, x0, niter, xbar)
    gpu = _gpu(A, b, lo, hi, x0, niter, xbar, torch.float64)
    _compare(gpu, ref, 1e-10, 1e-12)
    # the batch exercises both bounds and free rows
    assert any(np.any(r[4]) for r in ref) and any(np.any(r[5]) for r in ref)


@pytest.mark.parametrize("n,niter", [(4, 30), (12, 50), (16, 20)])
def test_solve_and_adjoint_fp32(n, niter):
    A, b, lo, hi, x0 = _batch(400, n, 200 + n, torch.float32)
    xbar = np.random.default_rng(n).normal(size=(400, n)).astype(np.float32).astype(np.float64)
    ref = _oracle(A, b, lo, hi, x0, niter, xbar)
    gpu = _gpu(A, b, lo, hi, x0, niter, xbar, torch.float32)
    # a row whose unclamped value lies within FP32 rounding of its bound may
    # take the other branch; such problems are rare and are excluded by name
    names = ("x", "sweeps", "A_bar", "b_bar", "lo_bar", "hi_bar", "x0_bar")
    errs = np.array([[rel(gpu[k][p], r[k], 1e-6) for k in range(7)] for p, r in enumerate(ref)])
    bad = np.where(errs.max(axis=1) > 1e-4)[0]
    print("fp32 worst per output", dict(zip(names, ["%.1e" % v for v in errs.max(axis=0)])), "above 1e-4:", len(bad))
    assert len(bad) <= 0.01 * len(ref), bad
    assert np.median(errs.max(axis=1)) < 1e-5


def test_no_sweep_and_empty_batch():
    from paper_2109_07719_amd import pgs
    A, b, lo, hi, x0 = _batch(5, 3, 7, torch.float64)
    xbar = np.ones((5, 3))
    gpu = _gpu(A, b, lo, hi, x0, 0, xbar, torch.float64)
    assert np.array_equal(gpu[0], x0) and np.array_equal(gpu[6], xbar)
    assert not gpu[2].any() and not gpu[3].any() and not gpu[4].any() and not gpu[5].any()
    e = torch.empty((0, 3, 3), dtype=torch.float64, device=DEV)
    v = torch.empty((0, 3), dtype=torch.float64, device=DEV)
    assert pgs.solve(e, v, v, v, v, 10).shape == (0, 3)


def test_invalid_calls_raise():
    from paper_2109_07719_amd import _native as N
    from paper_2109_07719_amd import pgs
    A = torch.eye(17, dtype=torch.float32, device=DEV).expand(2, 17, 17).contiguous()
    v = torch.zeros((2, 17), dtype=torch.float32, device=DEV)
    with pytest.raises(N.SimError):
        pgs.solve(A, v, v, v, v, 3)
    A3 = torch.eye(3, dtype=torch.float32, device=DEV).expand(2, 3, 3).contiguous()
    v3 = torch.zeros((2, 3), dtype=torch.float32, device=DEV)
    ws = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(N.SimError):
        pgs.solve(A3, v3, v3, v3, v3, 3, workspace=ws)


def test_autograd_wrapper_matches_the_adjoint():
    from paper_2109_07719_amd import pgs
    A, b, lo, hi, x0 = _batch(64, 6, 9, torch.float64)
    ts = [_t(v, torch.float64).requires_grad_() for v in (A, b, lo, hi, x0)]
    x = pgs.pgs(*ts, 15)
    w = torch.randn_like(x)
    grads = torch.autograd.grad((x * w).sum(), ts)
    ref = _oracle(A, b, lo, hi, x0, 15, w.detach().cpu().numpy())
    for k, g in enumerate(grads):
        for p in range(64):
            assert rel(g[p].cpu().numpy(), ref[p][2 + k], 1e-12) < 1e-10


def test_benchmark_size_sampled():
    """65536 problems of 12 rows (four contacts with friction), 50 sweeps,
    FP32, in one launch each way; every 512th problem against the oracle."""
    from paper_2109_07719_amd import pgs
    B, n, niter = 65536, 12, 50
    rng = np.random.default_rng(11)
    A, b, lo, hi, x0 = _batch(B // 512, n, 12, torch.float32)
    # tile the sampled problems through the batch, the others are random permutations of them
    idx = rng.integers(0, B // 512, B)
    idx[::512] = np.arange(B // 512)
    full = [v[idx] for v in (A, b, lo, hi, x0)]
    xbar = rng.normal(size=(B, n)).astype(np.float32).astype(np.float64)
    ts = [_t(v, torch.float32) for v in full + [xbar]]
    ws = pgs.new_workspace(B, n, niter, torch.float32)
    x = pgs.solve(*ts[:5], niter, workspace=ws)
    g = pgs.adjoint(*ts[:4], ts[5], niter, ws)
    x, g = x.cpu().numpy(), [v.cpu().numpy() for v in g]
    errs = []
    for s in range(0, B, 512):
        r = _oracle(*[v[s:s + 1] for v in full], niter, xbar[s:s + 1])[0]
        errs.append(max(rel(x[s], r[0], 1e-6), max(rel(g[k][s], r[2 + k], 1e-6) for k in range(5))))
    errs = np.array(errs)
    print("sampled fp32 errs: median %.1e max %.1e" % (np.median(errs), errs.max()))
    assert np.mean(errs > 1e-4) <= 0.01 and np.median(errs) < 1e-5
