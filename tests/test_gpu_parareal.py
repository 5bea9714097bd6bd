"""GPU parity for Parareal (Sec. 2.2, eqs. parareal-init, fine-integrator,
coarse-integrator) through the C ABI, against the oracle's Parareal on the
same inputs.  Bars: the dense trajectory within 1e-10 max-abs in FP64 (states
of order one; the kernels contract multiply-adds, the oracle does not, so
the two differ by rounding only), the same number of fine sweeps K unless
the oracle's accepted R is within 10x of tol, every R of the history within
1e-9 relative plus a few ulps of the state; FP32 within 1e-4 relative of
the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = 2.220446049250313e-16


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _problems(orc, pint):
    out = {}
    for p in W.paper_pins():
        out[p["name"]] = (p["system"], p["params"], p["x0"], p["T"] * p["dt"], orc.RK4, pint.RK4)
    for p in W.implicit_pins():
        out[p["name"]] = (p["system"], p["params"], p["x0"], p["horizon"], orc.BEULER,
                          pint.BACKWARD_EULER)
    return out


def _compare(ref, traj, iters, resid, status, hist, tol, label):
    traj = traj.cpu().numpy()
    k_gpu = int(iters)
    assert int(status) == ref["status"], label
    if ref["status"] == 5:  # NONFINITE: the trajectory is not a result
        assert k_gpu == ref["iters"], (label, k_gpu, ref["iters"])
        return
    near = ref["final_resid"] > tol / 10 or (len(ref["hist"]) > 1 and ref["hist"][-2] < 10 * tol)
    if not near:
        assert k_gpu == ref["iters"], (label, k_gpu, ref["iters"])
    if k_gpu == ref["iters"]:
        scale = max(1.0, np.abs(ref["traj"]).max())
        err = np.abs(traj - ref["traj"]).max()
        assert err <= 1e-10 * scale, (label, err)
        h = hist.cpu().numpy()[:k_gpu]
        floor = 16 * EPS * scale
        assert np.all(np.abs(h - ref["hist"]) <= 1e-9 * ref["hist"] + floor), (label, h, ref["hist"])
        assert float(resid) == pytest.approx(ref["final_resid"], rel=1e-9, abs=floor)


@pytest.mark.parametrize("name,dt", [("logistic", 1e-2), ("vdp", 1e-2), ("cartpole", 1e-2),
                                     ("vdp", 1e-3), ("cartpole", 1e-4),
                                     ("dahlquist", 1e-1), ("robertson", 1e-1),
                                     ("robertson", 1e-2)])
def test_paper_problems(pint, orc, name, dt):
    """The paper's Parareal runs (Figures 5, 6, 8, 9): M = floor(sqrt(N))
    windows of floor(N/M) steps, the same error history and K as the oracle
    (tol 1e-12, above the rounding floor so the count is well defined)."""
    sys_, prm, x0, horizon, om, pm = _problems(orc, pint)[name]
    N = int(round(horizon / dt))
    M, S = orc.parareal_windows(N)
    tol = 1e-12
    print(f"[parareal {name}] dt={dt} N={N} M={M} S={S}", flush=True)
    ref = orc.parareal(sys_, prm, dt, M, S, x0, tol=tol, max_iter=40, method=om)
    out = pint.parareal(sys_, _t(x0), _t(prm), dt, M, S, tol=tol, max_iter=40, method=pm,
                        with_hist=True)
    torch.cuda.synchronize()
    assert int(out[3]) == pint.OK
    _compare(ref, *out, tol, name)


def test_batch_per_instance_params(pint, orc):
    """A batch of van der Pol instances with their own mu and x0 (one
    workgroup each), M above one workgroup's 256 threads so windows wrap
    around the 1024-thread launch, and a ragged M*S."""
    r = np.random.default_rng(11)
    B = 23
    mu = r.uniform(0.5, 3.0, size=(B, 1))
    x0 = r.uniform(-2, 2, size=(B, 2))
    dt, M, S, tol = 0.004, 300, 7, 1e-11
    traj, iters, resid, status, hist = pint.parareal(pint.VDP, _t(x0), _t(mu), dt, M, S, tol=tol,
                                                     max_iter=60, with_hist=True)
    torch.cuda.synchronize()
    for b in range(B):
        ref = orc.parareal(orc.VDP, mu[b], dt, M, S, x0[b], tol=tol, max_iter=60)
        _compare(ref, traj[b], iters[b], resid[b], status[b], hist[b], tol, f"inst {b}")


@pytest.mark.parametrize("method", ["trapezoidal", "backward_euler", "rk4"])
def test_lorenz63_and_robertson_rules(pint, orc, method):
    """Every one-step rule of the small solver as coarse and fine integrator:
    Lorenz-63 (chaotic: Parareal needs many sweeps) and Robertson (stiff)."""
    om = {"rk4": orc.RK4, "backward_euler": orc.BEULER, "trapezoidal": orc.TRAP}[method]
    r = np.random.default_rng(12)
    cases = [(orc.LORENZ63, [10.0, 28.0, 8.0 / 3.0], [1.0, 1.0, 1.0] + r.normal(0, 0.1, 3), 1e-3,
              45, 45),
             (orc.VDP, [2.0], [2.0, 0.0], 0.01, 31, 16)]
    if method == "backward_euler":
        # stiff; explicit RK4 is unstable at these steps, and the trapezoidal
        # rule's per-step Newton solve fails on the corrected states (the
        # oracle reports NONFINITE too)
        cases.append((orc.ROBERTSON, [0.04, 3e7, 1e4], [1.0, 0.0, 0.0], 0.05, 31, 33))
    for sys_, prm, x0, dt, M, S in cases:
        tol = 1e-11
        ref = orc.parareal(sys_, prm, dt, M, S, x0, tol=tol, max_iter=M + 1, method=om)
        out = pint.parareal(sys_, _t(x0), _t(prm), dt, M, S, tol=tol, max_iter=M + 1,
                            method=method, with_hist=True)
        torch.cuda.synchronize()
        _compare(ref, *out, tol, f"{sys_}/{method}")


def test_degenerate_and_error_paths(pint, orc):
    """S = 1 (coarse step = fine step: R = 0 at once, K = 1, the sequential
    trajectory); M = 1 (K = 2); M or S = 0; a NaN start (NONFINITE); a sweep
    limit (NOT_CONVERGED with K = max_iter)."""
    prm, x0 = _t([1.0]), _t([0.5, -0.3])
    traj, iters, resid, status = pint.parareal(pint.VDP, x0, prm, 0.01, 37, 1, tol=1e-15)
    seq = pint.seq_integrate(pint.VDP, x0[None], prm, 0.01, [37])
    torch.cuda.synchronize()
    assert int(status) == pint.OK and int(iters) == 1 and float(resid) == 0.0
    assert (traj - seq).abs().max().item() <= 1e-14
    traj, iters, resid, status = pint.parareal(pint.VDP, x0, prm, 0.01, 1, 50, tol=1e-14)
    torch.cuda.synchronize()
    assert int(status) == pint.OK and int(iters) == 2
    ref = orc.integrate(orc.VDP, [1.0], 0.01, 50, [0.5, -0.3])
    assert np.abs(traj.cpu().numpy() - ref).max() < 1e-13
    for M, S in ((0, 5), (5, 0)):
        traj, iters, resid, status = pint.parareal(pint.VDP, x0, prm, 0.01, M, S)
        torch.cuda.synchronize()
        assert int(status) == pint.OK and int(iters) == 0 and traj.numel() == 0
    _, iters, _, status = pint.parareal(pint.VDP, _t([float("nan"), 0.0]), prm, 0.01, 4, 4)
    torch.cuda.synchronize()
    assert int(status) == pint.NONFINITE and int(iters) == 1
    _, iters, _, status = pint.parareal(pint.VDP, x0, prm, 0.01, 8, 8, tol=1e-300, max_iter=3)
    torch.cuda.synchronize()
    assert int(status) == pint.NOT_CONVERGED and int(iters) == 3


def test_argument_checks(pint):
    """Host-side rejections: a dense dimension, options the method does not
    take, a missing workspace."""
    P = pint
    x0 = _t([[0.5, -0.3]])
    prm = _t([1.0])
    sysd = P.make_system(P.VDP, 2, prm, True)
    out = [torch.empty(1, dtype=t, device=DEV) for t in (torch.int64, torch.float64, torch.int32)]
    traj = torch.empty((1, 16, 2), dtype=torch.float64, device=DEV)
    opts = P.make_options(P.F64, 1e-10)
    assert P.pint_parareal(sysd, 1, x0, 0.01, 4, 4, opts, traj, *out, None, None) == P.ERR_WORKSPACE
    bad = P.make_options(P.F64, 1e-10, window=8)
    ws = torch.empty(P.pint_parareal_workspace_bytes(sysd, 1, 4, P.F64), dtype=torch.uint8, device=DEV)
    assert P.pint_parareal(sysd, 1, x0, 0.01, 4, 4, bad, traj, *out, None, ws) == P.ERR_INVALID_ARG
    assert P.pint_parareal(sysd, 1, x0, 0.01, -1, 4, opts, traj, *out, None, ws) == P.ERR_INVALID_ARG
    l96 = P.make_system(P.LORENZ96, 40, _t([8.0]), True)
    assert P.pint_parareal(l96, 1, _t(np.full((1, 40), 8.0)), 0.01, 4, 4, opts,
                           torch.empty((1, 16, 40), dtype=torch.float64, device=DEV), *out, None,
                           ws) == P.ERR_UNSUPPORTED


def test_fp32(pint, orc):
    """FP32 Parareal on van der Pol against the FP64 oracle: 1e-4 relative
    over the dense trajectory (tol at FP32 rounding)."""
    dt, N = 1e-3, 10000
    M, S = orc.parareal_windows(N)
    ref = orc.parareal(orc.VDP, [1.0], dt, M, S, [0.0, 1.0], tol=1e-13)
    traj, iters, resid, status = pint.parareal(pint.VDP, _t([0.0, 1.0], torch.float32),
                                               _t([1.0], torch.float32), dt, M, S, tol=2e-5)
    torch.cuda.synchronize()
    assert int(status) == pint.OK
    got = traj.cpu().numpy().astype(np.float64)
    rel = np.abs(got - ref["traj"]).max() / np.abs(ref["traj"]).max()
    print(f"fp32 parareal: K={int(iters)} rel err {rel:.2e}", flush=True)
    assert rel < 1e-4


def test_full_size_vdp(pint, orc):
    """The largest van der Pol run of Figure 6 (dt = 1e-5, N = 1e6, M = 1000
    windows of 1000 steps), sampled: K and the sweep history equal the
    oracle's, the trajectory within 1e-10 at every 997th state."""
    dt, N = 1e-5, 1000000
    M, S = orc.parareal_windows(N)
    tol = 1e-12
    ref = orc.parareal(orc.VDP, [1.0], dt, M, S, [0.0, 1.0], tol=tol, max_iter=40)
    out = pint.parareal(pint.VDP, _t([0.0, 1.0]), _t([1.0]), dt, M, S, tol=tol, max_iter=40,
                        with_hist=True)
    torch.cuda.synchronize()
    _compare(ref, *out, tol, "vdp 1e6")
