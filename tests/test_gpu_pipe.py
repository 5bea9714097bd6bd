"""The pipelined windowed solvers for Lorenz-96 and Kuramoto (consecutive
Newton updates overlapping on separate workgroups) against the solver that
applies one update at a time, and against the oracle.  Both GPU solvers compute each
element and each fold step with the same arithmetic in the same order, so
the bar between them is bit for bit: same iteration count, same status,
identical trajectories.  Against the oracle: the same iterate to 1e-10 on
short horizons (the oracle's windowed Newton, same tol and window)."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _both(pint, w, T, dtype=torch.float64, system=None, **kw):
    """The same solve with the pipelined solver and with the other one."""
    out = {}
    system = pint.LORENZ96 if system is None else system
    try:
        for pipe in (True, False):
            pint.pint_set_dense_pipeline(pipe)
            out[pipe] = pint.solve(system, _t(w.x0, dtype), _t(w.params, dtype), w.dt, T, **kw)
            torch.cuda.synchronize()
    finally:
        pint.pint_set_dense_pipeline(True)
    return out[True], out[False]


@pytest.mark.parametrize("T,window,B", [(256, 32, 1), (300, 120, 1), (2048, 48, 1), (2048, 16, 2),
                                        (4096, 56, 16), (1000, 1000, 3), (777, 13, 5),
                                        (512, 24, 256), (600, 32, 100)])
def test_pipeline_equals_one_at_a_time(pint, T, window, B):
    # (B = 256 and 100 on a 256-CU device: one and two agents per instance)
    w = W.lorenz96(T=T, B=B)
    print(f"[pipe] T={T} W={window} B={B}", flush=True)
    (tp, ip, rp, sp), (to, io, ro, so) = _both(pint, w, T, tol=1e-10, window=window)
    assert torch.equal(sp, so) and bool((sp == 0).all())
    assert torch.equal(ip, io)
    assert torch.equal(tp, to)
    assert torch.equal(rp, ro)


@pytest.mark.parametrize("T,window", [(256, 32), (300, 120), (200, 7)])
def test_pipeline_same_iterate_as_oracle(pint, orc, T, window):
    w = W.lorenz96(T=T)
    ref = orc.newton(w.system, w.params[0], w.dt, T, w.x0[0], tol=1e-10, window=window,
                     max_iter=4 * T)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, T,
                                            tol=1e-10, window=window, max_iter=4 * T)
    torch.cuda.synchronize()
    assert int(status[0]) == ref["status"] == 0 and int(iters[0]) == ref["iters"]
    assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10
    assert abs(float(resid[0]) - ref["final_resid"]) <= 1e-14


def test_pipeline_fp32_equals_one_at_a_time(pint):
    w = W.lorenz96(T=1500, B=2)
    (tp, ip, rp, sp), (to, io, ro, so) = _both(pint, w, 1500, dtype=torch.float32, tol=2e-5,
                                               window=32)
    assert torch.equal(sp, so) and torch.equal(ip, io) and torch.equal(tp, to)


def test_pipeline_end_conditions(pint, orc):
    """The end of the iteration met by different agents: the update limit
    (NOT_CONVERGED with max_iter updates applied, the oracle's iterate), a
    guard that cuts updates, a non-finite start (NONFINITE, nothing
    applied), and a horizon shorter than one window."""
    w = W.lorenz96(T=400)
    for max_iter in (1, 5, 17):
        ref = orc.newton(w.system, w.params[0], w.dt, 400, w.x0[0], tol=1e-10, window=24,
                         max_iter=max_iter)
        traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 400,
                                                tol=1e-10, window=24, max_iter=max_iter)
        torch.cuda.synchronize()
        assert int(status[0]) == pint.NOT_CONVERGED == ref["status"]
        assert int(iters[0]) == max_iter == ref["iters"]
        assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10
    # a tight guard: updates are cut at the first state beyond it
    ref = orc.newton(w.system, w.params[0], w.dt, 400, w.x0[0], tol=1e-10, window=64,
                     guard=12.0, max_iter=4000)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 400,
                                            tol=1e-10, window=64, guard=12.0, max_iter=4000)
    torch.cuda.synchronize()
    assert int(status[0]) == ref["status"] and int(iters[0]) == ref["iters"]
    if ref["status"] == 0:
        assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10
    x0 = w.x0.copy()
    x0[0, 3] = np.nan
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(x0), _t(w.params), w.dt, 400,
                                            tol=1e-10, window=24)
    torch.cuda.synchronize()
    assert int(status[0]) == pint.NONFINITE and int(iters[0]) == 0
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 10,
                                            tol=1e-10, window=24)
    torch.cuda.synchronize()
    ref = orc.newton(w.system, w.params[0], w.dt, 10, w.x0[0], tol=1e-10, window=24, max_iter=100)
    assert int(status[0]) == 0 and int(iters[0]) == ref["iters"]


# ----------------------------------------------------------------- Kuramoto --
# The matrix-free pipeline: each agent's elements are Phi and the stage record,
# its fold applies J through the RK4 tangent; the same bar against the
# one-at-a-time solver (bit for bit) and the oracle (same iterate).

@pytest.mark.parametrize("T,window,B,d", [(64, 16, 2, 128), (256, 64, 2, 128), (200, 300, 3, 128),
                                          (512, 64, 8, 128), (333, 29, 4, 128), (300, 40, 2, 64)])
def test_kuramoto_pipeline_equals_one_at_a_time(pint, T, window, B, d):
    w = W.kuramoto(B=B, d=d, T=T)
    print(f"[pipe kuramoto] T={T} W={window} B={B} d={d}", flush=True)
    (tp, ip, rp, sp), (to, io, ro, so) = _both(pint, w, T, system=pint.KURAMOTO, tol=1e-10, window=window)
    assert torch.equal(sp, so) and bool((sp == 0).all())
    assert torch.equal(ip, io)
    assert torch.equal(tp, to)
    assert torch.equal(rp, ro)


def test_kuramoto_pipeline_fp32_equals_one_at_a_time(pint):
    w = W.kuramoto(B=2, T=600)
    (tp, ip, rp, sp), (to, io, ro, so) = _both(pint, w, 600, dtype=torch.float32, system=pint.KURAMOTO,
                                               tol=5e-5, window=64)
    assert torch.equal(sp, so) and torch.equal(ip, io) and torch.equal(tp, to)


@pytest.mark.parametrize("T,window", [(256, 64), (150, 11)])
def test_kuramoto_pipeline_same_iterate_as_oracle(pint, orc, T, window):
    w = W.kuramoto(B=1, T=T)
    ref = orc.newton(w.system, w.params[0], w.dt, T, w.x0[0], tol=1e-10, window=window,
                     max_iter=4 * T)
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, T,
                                            tol=1e-10, window=window, max_iter=4 * T)
    torch.cuda.synchronize()
    assert int(status[0]) == ref["status"] == 0 and int(iters[0]) == ref["iters"]
    assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10


def test_kuramoto_pipeline_end_conditions(pint, orc):
    """The update limit (the oracle's iterate after max_iter updates), a guard
    that cuts updates (the phases grow past it), and a non-finite start."""
    w = W.kuramoto(B=1, T=300)
    for max_iter in (1, 4):
        ref = orc.newton(w.system, w.params[0], w.dt, 300, w.x0[0], tol=1e-10, window=32,
                         max_iter=max_iter)
        traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, 300,
                                                tol=1e-10, window=32, max_iter=max_iter)
        torch.cuda.synchronize()
        assert int(status[0]) == pint.NOT_CONVERGED == ref["status"]
        assert int(iters[0]) == max_iter == ref["iters"]
        assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10
    guard = float(np.abs(w.x0).max()) + 0.5
    ref = orc.newton(w.system, w.params[0], w.dt, 300, w.x0[0], tol=1e-10, window=64,
                     guard=guard, max_iter=3000)
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, 300,
                                            tol=1e-10, window=64, guard=guard, max_iter=3000)
    torch.cuda.synchronize()
    assert int(status[0]) == ref["status"] and int(iters[0]) == ref["iters"]
    if ref["status"] == 0:
        assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10
    x0 = w.x0.copy()
    x0[0, 5] = np.nan
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(x0), _t(w.params), w.dt, 300,
                                            tol=1e-10, window=32)
    torch.cuda.synchronize()
    assert int(status[0]) == pint.NONFINITE and int(iters[0]) == 0


@pytest.mark.parametrize("system", ["lorenz96", "kuramoto"])
def test_pipeline_repeatable(pint, system):
    """The pipelined solvers' arithmetic does not depend on how the agents'
    timing interleaves: repeated solves give the same trajectory bit for bit."""
    if system == "lorenz96":
        w, T, win, sid = W.lorenz96(T=2048, B=4), 2048, 48, pint.LORENZ96
    else:
        w, T, win, sid = W.kuramoto(B=8, T=512), 512, 64, pint.KURAMOTO
    outs = []
    for _ in range(3):
        outs.append(pint.solve(sid, _t(w.x0), _t(w.params), w.dt, T, tol=1e-10, window=win))
        torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
        assert torch.equal(o[2], outs[0][2]) and torch.equal(o[3], outs[0][3])


@pytest.mark.parametrize("system", ["lorenz96", "kuramoto"])
@pytest.mark.parametrize("T", [1, 2, 3])
def test_pipeline_tiny_horizons(pint, orc, system, T):
    """Horizons of one to three steps (window 2): the first window start is
    step 1 and the state before it is x0; against the oracle."""
    w = W.lorenz96(T=T, B=2) if system == "lorenz96" else W.kuramoto(B=3, T=T)
    sid = pint.LORENZ96 if system == "lorenz96" else pint.KURAMOTO
    traj, iters, resid, status = pint.solve(sid, _t(w.x0), _t(w.params), w.dt, T, tol=1e-10, window=2)
    torch.cuda.synchronize()
    for b in range(w.B):
        ref = orc.newton(w.system, w.params[b], w.dt, T, w.x0[b], tol=1e-10, window=2, max_iter=100)
        assert int(status[b]) == ref["status"] == 0 and int(iters[b]) == ref["iters"]
        assert np.abs(traj[b].cpu().numpy() - ref["traj"]).max() <= 1e-10
