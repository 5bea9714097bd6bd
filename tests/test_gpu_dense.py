"""GPU parity, dense state dimension (Lorenz-96 d=40, Kuramoto d=128) through
the C ABI against the oracle on the same seeded inputs.

Bars: kernels that compute a plain function (RK4 step, residual, Jacobian
elements) match the oracle element by element to near rounding.  Newton
iterates match the oracle's iterate to 1e-10 max-abs in FP64 where the
problem allows it (short Lorenz-96 horizons, Kuramoto).  On long chaotic
Lorenz-96 horizons two correct implementations cannot agree to 1e-10 (a
difference of one rounding grows like exp(7.9 t) near x = F), so there the
checks are: equal iteration counts, every step's FP64 defect below tol, and
agreement with the sequential trajectory over the first 100 steps."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _near_attractor(orc, w, b, n):
    """A state reached after n sequential steps (off the equilibrium)."""
    return orc.integrate(w.system, w.params[b], w.dt, n, w.x0[b])[-1]


@pytest.mark.parametrize("kind", ["l96", "kur"])
def test_seq_integrate_defect(pint, orc, kind):
    """Each GPU step equals the oracle's RK4 step of the GPU's previous state."""
    w = W.lorenz96(T=600, B=3) if kind == "l96" else W.kuramoto(B=2, T=300)
    T = int(w.T[0])
    traj = pint.seq_integrate(w.system, _t(w.x0), _t(w.params), w.dt, T).cpu().numpy()
    traj = traj.reshape(w.B, T, w.d)
    for b in range(w.B):
        h = orc.residual(w.system, w.params[b], w.dt, w.x0[b], traj[b])
        assert np.abs(h).max() <= 1e-12 * max(1.0, np.abs(traj[b]).max())
        ref = orc.integrate(w.system, w.params[b], w.dt, 100, w.x0[b])
        assert np.abs(traj[b, :100] - ref).max() <= 1e-11


@pytest.mark.parametrize("kind", ["l96", "kur"])
def test_residual_and_elements(pint, orc, kind):
    """h, A_n = dPhi/dx(x_n) (row-major) and b_n = -h_{n+1} element by element."""
    rng = np.random.default_rng(17)
    if kind == "l96":
        w = W.lorenz96(T=8, B=2)
        start = [_near_attractor(orc, w, b, 400) for b in range(w.B)]
    else:
        w = W.kuramoto(B=2, T=8)
        start = [w.x0[b] for b in range(w.B)]
    T = 37
    x0 = np.stack(start)
    trajs = np.stack([orc.integrate(w.system, w.params[b], w.dt, T, x0[b])
                      + 1e-4 * rng.normal(size=(T, w.d)) for b in range(w.B)])
    h, hmax = pint.residual(w.system, _t(x0), _t(w.params), w.dt, _t(trajs))
    A, bb = pint.elements(w.system, _t(x0), _t(w.params), w.dt, _t(trajs))
    torch.cuda.synchronize()
    h, hmax, A, bb = h.cpu().numpy(), hmax.cpu().numpy(), A.cpu().numpy(), bb.cpu().numpy()
    for b in range(w.B):
        h_ref = orc.residual(w.system, w.params[b], w.dt, x0[b], trajs[b])
        assert np.abs(h[b] - h_ref).max() <= 1e-12
        assert abs(hmax[b] - np.abs(h_ref).max()) <= 1e-12
        assert np.abs(bb[b] + h_ref).max() <= 1e-12
        states = np.vstack([x0[b][None], trajs[b][:-1]])
        for n in range(T):
            J = orc.rk4_jac(w.system, w.params[b], w.dt, states[n])
            assert np.abs(A[b, n] - J).max() <= 1e-12 * max(1.0, np.abs(J).max()), (b, n)


@pytest.mark.parametrize("T,window,tol", [(96, 32, 1e-12), (128, 200, 1e-12), (64, 0, 1e-12),
                                          (256, 20, 1e-12), (256, 64, 1e-12), (256, 108, 1e-12),
                                          (300, 120, 1e-12)])
def test_lorenz96_same_iterate_short(pint, orc, T, window, tol):
    """Same iterate and iteration count as the oracle, for windows from 20 to
    200 steps (the fold walks them in chunks of 12 staged steps)."""
    w = W.lorenz96(T=T)
    print(f"[l96] T={T} W={window} tol={tol}", flush=True)
    ref = orc.newton(w.system, w.params[0], w.dt, T, w.x0[0], tol=tol, window=window,
                     max_iter=4 * T)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, T,
                                            tol=tol, window=window, max_iter=4 * T)
    torch.cuda.synchronize()
    assert int(status[0]) == ref["status"] == 0
    assert int(iters[0]) == ref["iters"]
    assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10


def test_lorenz96_long_horizon(pint, orc):
    """T=1024, W=32: iteration counts, FP64 defect and the early prefix."""
    w = W.lorenz96(T=1024, B=2)
    print("[l96] T=1024 W=32 B=2", flush=True)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 1024,
                                            tol=1e-10, window=32)
    torch.cuda.synchronize()
    traj = traj.cpu().numpy()
    for b in range(w.B):
        ref = orc.newton(w.system, w.params[b], w.dt, 1024, w.x0[b], tol=1e-10, window=32,
                         max_iter=4096)
        assert int(status[b]) == ref["status"] == 0
        dk = abs(int(iters[b]) - ref["iters"])
        assert dk <= max(2, ref["iters"] // 50), (int(iters[b]), ref["iters"])
        h = orc.residual(w.system, w.params[b], w.dt, w.x0[b], traj[b])
        assert np.abs(h).max() < 1e-10 and float(resid[b]) < 1e-10
        o1 = orc.integrate(w.system, w.params[b], w.dt, 100, w.x0[b])
        assert np.abs(traj[b, :100] - o1).max() <= 1e-8


@pytest.mark.parametrize("T,window", [(256, 64), (128, 0), (200, 300)])
def test_kuramoto_same_iterate(pint, orc, T, window):
    w = W.kuramoto(B=2, T=T)
    print(f"[kuramoto] T={T} W={window}", flush=True)
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, T,
                                            tol=1e-10, window=window, max_iter=4 * T)
    torch.cuda.synchronize()
    traj = traj.cpu().numpy()
    for b in range(w.B):
        ref = orc.newton(w.system, w.params[b], w.dt, T, w.x0[b], tol=1e-10, window=window,
                         max_iter=4 * T)
        assert int(status[b]) == ref["status"] == 0
        assert int(iters[b]) == ref["iters"]
        assert np.abs(traj[b] - ref["traj"]).max() <= 1e-10


def test_dense_edge_cases(pint, orc):
    w = W.lorenz96(T=16)
    # T = 0 and T = 1
    for T in (0, 1):
        traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, T,
                                                tol=1e-12, window=8)
        torch.cuda.synchronize()
        assert int(status[0]) == 0 and int(iters[0]) == T
    # non-finite parameter -> NONFINITE status, not a hang
    bad = w.params.copy()
    bad[0, 0] = np.inf
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(bad), w.dt, 16, window=8)
    torch.cuda.synchronize()
    assert int(status[0]) == pint.NONFINITE
    # max_iter reached
    ref = orc.newton(w.system, w.params[0], w.dt, 16, w.x0[0], tol=1e-14, window=8, max_iter=2)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 16,
                                            tol=1e-14, window=8, max_iter=2)
    torch.cuda.synchronize()
    assert int(status[0]) == pint.NOT_CONVERGED == ref["status"] and int(iters[0]) == 2
    assert np.abs(traj[0].cpu().numpy() - ref["traj"]).max() <= 1e-10


@pytest.mark.parametrize("kind", ["l96", "kur"])
def test_fp32_dense(pint, orc, kind):
    """FP32: FP64 defect of the FP32 iterate at FP32 rounding level and 1e-4
    relative agreement with the FP64 sequential trajectory over 50 steps."""
    w = W.lorenz96(T=400) if kind == "l96" else W.kuramoto(B=1, T=300)
    T = int(w.T[0])
    x0 = w.x0.astype(np.float32)
    P = w.params.astype(np.float32)
    traj, iters, resid, status = pint.solve(w.system, _t(x0, torch.float32), _t(P, torch.float32),
                                            w.dt, T, tol=2e-5 if kind == "l96" else 1e-5, window=32,
                                            max_iter=4 * T)
    torch.cuda.synchronize()
    got = traj[0].cpu().numpy().astype(np.float64)
    x064, P64 = x0[0].astype(np.float64), P[0].astype(np.float64)
    scale = max(1.0, np.abs(got).max())
    h = orc.residual(w.system, P64, w.dt, x064, got)
    assert int(status[0]) == 0
    assert np.abs(h).max() <= (2e-5 if kind == "l96" else 1e-5) + 16 * np.finfo(np.float32).eps * scale
    ref = orc.integrate(w.system, P64, w.dt, 50, x064)
    assert np.abs(got[:50] - ref).max() <= 1e-4 * scale


def test_lorenz96_large_batch_one_workgroup_path(pint, orc):
    """300 instances exceed the co-resident capacity for several workgroups
    per instance, so this runs the one-workgroup-per-instance solver."""
    w = W.lorenz96(T=48, B=300, window=16)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 48,
                                            tol=1e-12, window=16)
    torch.cuda.synchronize()
    traj = traj.cpu().numpy()
    for b in (0, 1, 150, 299):
        ref = orc.newton(w.system, w.params[b], w.dt, 48, w.x0[b], tol=1e-12, window=16, max_iter=200)
        assert int(status[b]) == ref["status"] == 0
        assert int(iters[b]) == ref["iters"]
        assert np.abs(traj[b] - ref["traj"]).max() <= 1e-10
