"""GPU: sim_backward_noalloc (the adjoint pass for callers that cannot
allocate; its K > 1 replay buffer is the library's static per-GPU array)
called through the C ABI gives the results of sim_backward, on two calls in
a row, the second smaller than the first, and rejects what it cannot do."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2109_07719_amd import _native as N
from paper_2109_07719_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(name, n, T, K, params):
    from paper_2109_07719_amd.sim import Sim
    b = synth.round_to_f32(synth.workload(name, n_systems=n, T=T))
    sim = Sim(b.systems, b.gravity, dtype=torch.float32)
    f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=torch.float32, device=DEV)
    q0, qd0, tau = f(b.q0), f(b.qd0), f(b.tau)
    ws = sim.new_workspace(T, K)
    qT, qdT, _ = sim.forward(q0, qd0, tau, b.dt, K=K, workspace=ws)
    gqT, gqdT = 2 * qT, torch.ones_like(qdT)
    ref = sim.backward(tau, b.dt, K, ws, gqT, gqdT, params=params)
    torch.cuda.synchronize()
    ref = [x.clone() for x in ref]
    nl = sim.info["n_links"]
    out = [torch.full_like(x, float("nan")) for x in ref]
    if not params:
        out += [None, None]
    # only the checkpoint part of the workspace is handed over
    ck_bytes = sim.workspace_bytes(T, K) - (0 if K <= 1 else _replay_bytes(sim, K))
    rc = N.lib().sim_backward_noalloc(sim._h, _p(tau), float(b.dt), T, K, _p(gqT), _p(gqdT), None,
                                      _p(out[0]), _p(out[1]), _p(out[2]), _p(out[3]), _p(out[4]),
                                      _p(ws), ck_bytes, _stream())
    N.check(rc)
    torch.cuda.synchronize()
    for x, y in zip(out, ref):
        assert torch.equal(x, y)
    assert sim.status() == 0
    return sim, b, tau, ws, gqT, gqdT, nl


def _replay_bytes(sim, K):
    # sim_workspace_bytes(T, K) - sim_workspace_bytes(T, K) of the checkpoints alone: the replay
    # buffer holds K state records, each the size of one checkpoint
    one = sim.workspace_bytes(K, K)   # T = K: one checkpoint + the replay buffer
    rec = sim.workspace_bytes(1, 1)   # one checkpoint record (256-byte aligned)
    return one - rec


def test_noalloc_backward_matches_backward_twice_second_smaller():
    # chains with K = 10 and parameter gradients, then a smaller batch with K = 7 and a shorter
    # horizon (the array keeps the first call's contents); then free roots and K = 1
    _case("chain7_4096", 96, 300, 10, True)
    _case("chain7_4096", 20, 120, 7, False)
    _case("quad_1024", 6, 90, 4, False)
    _case("trees_8192", 5, 40, 1, True)


def test_noalloc_backward_rejects_what_it_cannot_do():
    sim, b, tau, ws, gqT, gqdT, nl = _case("chain7_4096", 8, 50, 5, False)
    g = [torch.empty(sim.nq, device=DEV), torch.empty(sim.nv, device=DEV), torch.empty((50, sim.nu), device=DEV)]
    L = N.lib()
    rc = L.sim_backward_noalloc(sim._h, _p(tau), float(b.dt), 50, -3, _p(gqT), _p(gqdT), None, _p(g[0]), _p(g[1]),
                                _p(g[2]), None, None, _p(ws), ws.numel(), _stream())
    assert rc == N.SIM_ERR_INVALID_ARG
    # a replay buffer beyond the 64 MiB array
    rec = sim.workspace_bytes(2, 1) - sim.workspace_bytes(1, 1)   # one state record
    assert rec > 0
    big_K = (64 << 20) // rec + 10
    rc = L.sim_backward_noalloc(sim._h, _p(tau), float(b.dt), 50, big_K, _p(gqT), _p(gqdT), None, _p(g[0]),
                                _p(g[1]), _p(g[2]), None, None, _p(ws), ws.numel(), _stream())
    assert rc == N.SIM_ERR_WORKSPACE_TOO_SMALL
    assert b"64 MiB" in L.sim_last_error() or b"static scratch" in L.sim_last_error()
    # too small a checkpoint buffer
    rc = L.sim_backward_noalloc(sim._h, _p(tau), float(b.dt), 50, 5, _p(gqT), _p(gqdT), None, _p(g[0]),
                                _p(g[1]), _p(g[2]), None, None, _p(ws), 16, _stream())
    assert rc == N.SIM_ERR_WORKSPACE_TOO_SMALL
