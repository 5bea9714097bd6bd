"""Error path of the cooperative solvers' bounded device-side waits.  The
host makes every cross-workgroup wait give up at once
(pint_set_wait_limit(0)): every kernel must still end, with the instances'
status PINT_ERR_DEVICE, and a solve after the default bound is restored must
be correct again.  No kernel is made to fault or hang: a wait that gives up
only sets the error word and leaves its loop."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _solve_limited(pint, *args, pipe=True, **kw):
    """A solve whose every cross-workgroup wait gives up at once; pipe picks
    the pipelined windowed solver (True) or the one-at-a-time one."""
    try:
        pint.pint_set_wait_limit(0)
        pint.pint_set_dense_pipeline(pipe)
        out = pint.solve(*args, **kw)
        torch.cuda.synchronize()
    finally:
        pint.pint_set_wait_limit(pint.WAIT_LIMIT_DEFAULT)
        pint.pint_set_dense_pipeline(True)
    return out


@pytest.mark.parametrize("pipe", [True, False])
def test_dense_banded_wait_gives_up(pint, orc, pipe):
    w = W.lorenz96(T=2048)
    print(f"[waits] lorenz96 T=2048 W=48 pipe={pipe}, wait limit 0", flush=True)
    _, _, _, status = _solve_limited(pint, pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 2048,
                                     tol=1e-10, window=48, pipe=pipe)
    assert int(status[0]) == pint.ERR_DEVICE
    print("[waits] lorenz96 T=2048 W=48, default bound", flush=True)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 2048,
                                            tol=1e-10, window=48)
    torch.cuda.synchronize()
    assert int(status[0]) == pint.OK
    h = orc.residual(w.system, w.params[0], w.dt, w.x0[0], traj[0].cpu().numpy())
    assert np.abs(h).max() < 1e-10


@pytest.mark.parametrize("pipe", [True, False])
def test_dense_kuramoto_wait_gives_up(pint, orc, pipe):
    w = W.kuramoto(B=2, T=512)
    print(f"[waits] kuramoto 2 x 512 W=64 pipe={pipe}, wait limit 0", flush=True)
    _, _, _, status = _solve_limited(pint, pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, 512,
                                     tol=1e-10, window=64, pipe=pipe)
    assert (status == pint.ERR_DEVICE).all()
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, 512,
                                            tol=1e-10, window=64)
    torch.cuda.synchronize()
    assert (status == pint.OK).all()


def test_small_cooperative_wait_gives_up(pint, orc):
    pin = next(p for p in W.paper_pins() if p["name"] == "logistic")
    T = 100000
    dt = pin["dt"] * pin["T"] / T
    guess = _t(np.full((T, 1), pin["guess"]))
    print("[waits] logistic T=1e5 plain (cooperative), wait limit 0", flush=True)
    _, _, _, status = _solve_limited(pint, pin["system"], _t(pin["x0"]), _t(pin["params"]), dt, T,
                                     tol=3e-14, max_iter=60, guess=guess)
    assert int(status) == pint.ERR_DEVICE
    traj, iters, resid, status = pint.solve(pin["system"], _t(pin["x0"]), _t(pin["params"]), dt,
                                            T, tol=3e-14, max_iter=60, guess=guess)
    torch.cuda.synchronize()
    assert int(status) == pint.OK
