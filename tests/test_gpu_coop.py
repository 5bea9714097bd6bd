"""GPU parity of the cooperative small-d solver: a few long instances in the
paper's plain mode, each spread over several workgroups (elements, residual
and scan fused per Newton iteration, the Jacobians never stored).  Same bar
as the one-workgroup solver: iteration counts equal to the oracle's, max-abs
1e-10 in FP64, 1e-4 relative in FP32."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PAPER_TOL = 3e-14


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("name,T", [("logistic", 100000), ("vdp", 100000), ("cartpole", 40000)])
def test_paper_explicit_problems_long(pint, orc, name, T):
    """The paper's explicit problems over their fixed horizons with the step
    counts of its runtime figure (Sec. 4.1, Figure 4: dt = horizon / T, so
    dt = 1e-4 here): same K and the same converged iterate as the oracle."""
    pin = next(p for p in W.paper_pins() if p["name"] == name)
    d = len(pin["x0"])
    dt = pin["dt"] * pin["T"] / T
    guess = np.full((T, d), pin["guess"], dtype=np.float64)
    print(f"[{name}] T={T} dt={dt} plain, cooperative", flush=True)
    ref = orc.newton(pin["system"], pin["params"], dt, T, pin["x0"], guess=guess,
                     tol=PAPER_TOL, max_iter=60)
    traj, iters, resid, status = pint.solve(pin["system"], _t(pin["x0"]), _t(pin["params"]),
                                            dt, T, tol=PAPER_TOL, max_iter=60,
                                            guess=_t(guess))
    torch.cuda.synchronize()
    assert int(status) == pint.OK == ref["status"]
    assert int(iters) == ref["iters"]
    scale = max(1.0, np.abs(ref["traj"]).max())
    assert np.abs(traj.cpu().numpy() - ref["traj"]).max() <= 1e-10 * scale
    assert float(resid) < PAPER_TOL


@pytest.mark.parametrize("method", [1, 2])
def test_several_instances_and_the_batched_solver_agree(pint, orc, method):
    """Three Robertson instances with their own rates (uniform T = 6000):
    the cooperative launch (pint_solve) and the one-workgroup batched launch
    (pint_solve_varlen on the same data) both equal the oracle."""
    w = W.robertson_batch(B=3, t_lo=6000, t_hi=6000)
    T = 6000
    x0, P = _t(w.x0), _t(w.params)
    traj, iters, resid, status = pint.solve(pint.ROBERTSON, x0, P, w.dt, T, tol=1e-12,
                                            method=method)
    trajv, _, itersv, residv, statusv = pint.solve_varlen(pint.ROBERTSON, x0, P, w.dt, [T] * 3,
                                                          tol=1e-12, method=method)
    torch.cuda.synchronize()
    om = orc.BEULER if method == 1 else orc.TRAP
    for b in range(3):
        ref = orc.newton_implicit(om, w.system, w.params[b], w.dt, T, w.x0[b], tol=1e-12,
                                  max_iter=T + 1)
        assert int(status[b]) == int(statusv[b]) == ref["status"] == 0
        assert int(iters[b]) == int(itersv[b]) == ref["iters"]
        assert np.abs(traj[b].cpu().numpy() - ref["traj"]).max() <= 1e-10
        assert np.abs(trajv[b * T:(b + 1) * T].cpu().numpy() - ref["traj"]).max() <= 1e-10
        assert float(resid[b]) < 1e-12 and abs(float(resid[b]) - ref["final_resid"]) <= 1e-13


def test_iteration_limit_and_nonfinite(pint, orc):
    """max_iter stops with NOT_CONVERGED and the iterate after exactly that
    many updates; a non-finite x0 stops with NONFINITE."""
    pin = next(p for p in W.paper_pins() if p["name"] == "vdp")
    T = 20000
    dt = 10.0 / T
    guess = np.ones((T, 2))
    ref = orc.newton(pin["system"], pin["params"], dt, T, pin["x0"], guess=guess,
                     tol=1e-12, max_iter=2)
    traj, iters, resid, status = pint.solve(pint.VDP, _t(pin["x0"]), _t(pin["params"]), dt,
                                            T, tol=1e-12, max_iter=2, guess=_t(guess))
    torch.cuda.synchronize()
    assert int(status) == pint.NOT_CONVERGED == ref["status"] and int(iters) == 2
    assert np.abs(traj.cpu().numpy() - ref["traj"]).max() <= 1e-10 * np.abs(ref["traj"]).max()
    assert abs(float(resid) - ref["final_resid"]) <= 1e-10 * ref["final_resid"]
    _, iters, resid, status = pint.solve(pint.VDP, _t([np.nan, 1.0]), _t(pin["params"]), dt, T)
    torch.cuda.synchronize()
    assert int(status) == pint.NONFINITE and int(iters) == 0


def test_fp32_long_logistic(pint, orc):
    """FP32 on the cooperative path (logistic over [0, 10], T = 8192, the
    paper's guess): status OK; the FP64 per-step defect of the FP32 iterate is
    below tol plus FP32 rounding; within 1e-4 relative of the FP64 sequential
    solution over the first 1000 steps (beyond that, per-step defects at the
    FP32 rounding floor accumulate with T; that error is printed)."""
    pin = next(p for p in W.paper_pins() if p["name"] == "logistic")
    T = 8192
    dt = 10.0 / T
    x0 = np.float32(pin["x0"][0])
    prm = np.asarray(pin["params"], dtype=np.float32)
    traj, iters, resid, status = pint.solve(pint.LOGISTIC, _t([x0], torch.float32),
                                            _t(prm, torch.float32), dt, T, tol=1e-6, max_iter=60,
                                            guess=_t(np.ones((T, 1)), torch.float32))
    torch.cuda.synchronize()
    assert int(status) == pint.OK
    got = traj.cpu().numpy().astype(np.float64)
    ref = orc.integrate(pin["system"], prm.astype(np.float64), dt, T, [float(x0)])
    scale = np.abs(ref).max()
    h = orc.residual(pin["system"], prm.astype(np.float64), dt, [float(x0)], got)
    assert np.abs(h).max() < 1e-6 + 8 * np.finfo(np.float32).eps * scale
    assert np.abs(got[:1000] - ref[:1000]).max() <= 1e-4 * scale
    print(f"fp32 logistic T={T}: K={int(iters) + 1}, max rel err over all steps "
          f"{np.abs(got - ref).max() / scale:.2e}")


@pytest.mark.parametrize("tile", [0, 1024, 4096])
def test_robertson_longest_horizon_any_range_size(pint, orc, tile):
    """The paper's longest implicit run (Robertson, dt = 5e-3, T = 1e5,
    Figures 7 and 9): K = 24 and the oracle's iterate, whatever the number
    of steps per workgroup (the tile option)."""
    pin = next(p for p in W.implicit_pins() if p["name"] == "robertson")
    T = 100000
    z = np.zeros((T, 3))
    ref = orc.newton_implicit(orc.BEULER, pin["system"], pin["params"], 5e-3, T, pin["x0"],
                              guess=z, tol=PAPER_TOL, max_iter=60)
    print(f"[robertson] T={T} tile={tile}", flush=True)
    traj, iters, resid, status = pint.solve(pint.ROBERTSON, _t(pin["x0"]), _t(pin["params"]), 5e-3,
                                            T, tol=PAPER_TOL, max_iter=60, guess=_t(z), tile=tile,
                                            method=pint.BACKWARD_EULER)
    torch.cuda.synchronize()
    assert int(status) == pint.OK == ref["status"]
    assert int(iters) + 1 == ref["iters"] + 1 == 24
    assert np.abs(traj.cpu().numpy() - ref["traj"]).max() <= 1e-10
