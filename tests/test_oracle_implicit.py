"""Pins for the oracle's implicit one-step rules (Sec. 3.4, eqs.
implicit-ode, root-finding-problem-implicit, jacobian-implicit,
newton-step-implicit-recursion): the residual histories and iteration counts
the paper prints for backward Euler (Sec. 4.2, Figures 8 and 9), closed forms
of both rules on linear systems, orders of accuracy, the Robertson
invariants, and agreement with step-by-step implicit integration."""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")

# Same reading of the unstated stopping tolerance as for the explicit
# figures; every printed implicit history ends below it and the entries
# before the last are far above it.
PAPER_TOL = 3e-14

ROB_P = [0.04, 3e7, 1e4]
ROB_X0 = [1.0, 0.0, 0.0]


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _problem(orc, name, dt):
    """(system, params, T, x0) of the paper's two implicit test problems."""
    if name == "dahlquist":
        return orc.LINEAR, [-1.0], int(round(4.0 / dt)), [1.0]
    return orc.ROBERTSON, ROB_P, int(round(500.0 / dt)), ROB_X0


@pytest.mark.parametrize("name", ["dahlquist", "robertson"])
def test_paper_implicit_residual_history(orc, name):
    """Figure 8: the printed histories at dt = 0.1 from the zero guess.  They
    fix the backward-Euler residual, the implicit Jacobian blocks, the
    inverse-diagonal scaling of the plotted quantity and full Newton steps."""
    gold = [(int(k), float(v)) for p, k, v in _read_table("implicit_residuals_dt1e-1.txt")
            if p == name]
    sys_, P, T, x0 = _problem(orc, name, 0.1)
    r = orc.newton_implicit(orc.BEULER, sys_, P, 0.1, T, x0, guess=np.zeros((T, len(x0))),
                            tol=PAPER_TOL, max_iter=60)
    assert r["status"] == orc.OK
    hist = r["hist"]
    assert len(hist) == len(gold)
    for k, v in gold:
        if v > 1e-12:
            assert abs(hist[k] - v) <= 1e-8 * v, (k, hist[k], v)
        else:  # rounding-floor values: same order of magnitude only
            assert hist[k] < 1e-12 and hist[k] < 20 * max(v, 1e-16)


@pytest.mark.parametrize("name", ["dahlquist", "robertson"])
def test_paper_implicit_iteration_counts(orc, name):
    """Figure 9: K (evaluations including the converged one) against dt."""
    for p, dt_s, K in _read_table("implicit_iterations.txt"):
        if p != name:
            continue
        dt = float(dt_s)
        sys_, P, T, x0 = _problem(orc, name, dt)
        r = orc.newton_implicit(orc.BEULER, sys_, P, dt, T, x0,
                                guess=np.zeros((T, len(x0))), tol=PAPER_TOL, max_iter=60)
        assert r["status"] == orc.OK
        assert r["iters"] + 1 == int(K), (dt, r["iters"] + 1, K)


def test_plotted_quantity_is_not_the_plain_residual(orc):
    """From the zero guess the Dahlquist residual is h_1 = -x_0 = -1 and zero
    elsewhere; the plotted 0.909... is (1 + dt)^{-1} |h_1|."""
    dt, T = 0.1, 40
    z = np.zeros((T, 1))
    h = orc.residual_implicit(orc.BEULER, orc.LINEAR, [-1.0], dt, [1.0], z)
    hs = orc.residual_implicit(orc.BEULER, orc.LINEAR, [-1.0], dt, [1.0], z, scaled=True)
    assert h[0, 0] == -1.0 and np.all(h[1:] == 0.0)
    assert hs[0, 0] == pytest.approx(-1.0 / 1.1, rel=1e-15) and np.all(hs[1:] == 0.0)


@pytest.mark.parametrize("method", ["be", "trap"])
def test_linear_system_closed_form_in_one_update(orc, method):
    """x' = M x: backward Euler gives x_n = (I - dt M)^{-n} x_0 and the
    trapezoidal rule x_n = ((I - dt/2 M)^{-1}(I + dt/2 M))^n x_0.  The
    Newton step of a linear problem is exact, so one update reaches them
    from any guess (a dropped dg/dx_{n-1} term would not)."""
    rng = np.random.default_rng(7)
    M = np.array([[-0.3, 1.2], [-1.1, -0.4]])
    dt, T = 0.05, 300
    x0 = np.array([1.0, -0.5])
    I = np.eye(2)
    if method == "be":
        R = np.linalg.inv(I - dt * M)
        m = orc.BEULER
    else:
        R = np.linalg.solve(I - 0.5 * dt * M, I + 0.5 * dt * M)
        m = orc.TRAP
    want = np.empty((T, 2))
    x = x0.copy()
    for n in range(T):
        x = R @ x
        want[n] = x
    guess = rng.standard_normal((T, 2))
    for window in (0, T):
        r = orc.newton_implicit(m, orc.LINEAR, M.ravel(), dt, T, x0, guess=guess,
                                tol=1e-13, max_iter=5, window=window)
        assert r["status"] == orc.OK and r["iters"] == 1
        np.testing.assert_allclose(r["traj"], want, rtol=1e-12, atol=1e-14)
    seq = orc.integrate_implicit(m, orc.LINEAR, M.ravel(), dt, T, x0)
    np.testing.assert_allclose(seq, want, rtol=1e-12, atol=1e-14)


def test_dahlquist_closed_form(orc):
    for dt in (0.1, 0.01, 1e-3):
        T = int(round(4.0 / dt))
        r = orc.newton_implicit(orc.BEULER, orc.LINEAR, [-1.0], dt, T, [1.0],
                                guess=np.zeros((T, 1)), tol=PAPER_TOL)
        n = np.arange(1, T + 1)
        np.testing.assert_allclose(r["traj"][:, 0], (1.0 + dt) ** (-n), rtol=1e-12)


def test_orders_of_accuracy_on_logistic(orc):
    """Backward Euler is first order, the trapezoidal rule second order:
    the error at t = 2 against the closed-form logistic solution shrinks by
    about 2 and 4 when dt halves."""
    r_, K = 1.0, 2.0
    x0 = 0.2

    def exact(t):
        return K * x0 * math.exp(r_ * t) / (K + x0 * (math.exp(r_ * t) - 1.0))

    for m, ratio in ((orc.BEULER, 2.0), (orc.TRAP, 4.0)):
        errs = []
        for dt in (0.02, 0.01, 0.005):
            T = int(round(2.0 / dt))
            x = orc.integrate_implicit(m, orc.LOGISTIC, [r_, K], dt, T, [x0])
            errs.append(abs(x[-1, 0] - exact(2.0)))
        for a, b in zip(errs, errs[1:]):
            assert a / b == pytest.approx(ratio, rel=0.06), (m, errs)


def test_robertson_vector_field(orc):
    """Mass conservation (the three rates sum to zero, so do the Jacobian's
    columns and the parameter derivative's columns) and finite differences."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.uniform(0.0, 1.0, 3) * np.array([1.0, 1e-4, 1.0])
        f = orc.f(orc.ROBERTSON, ROB_P, x)
        assert abs(f.sum()) <= 1e-12 * np.abs(f).max()
        J = orc.jf(orc.ROBERTSON, ROB_P, x)
        assert np.abs(J.sum(axis=0)).max() <= 1e-9 * np.abs(J).max()
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1e-7 * max(abs(x[j]), 1e-4)
            fd = (orc.f(orc.ROBERTSON, ROB_P, x + e) - orc.f(orc.ROBERTSON, ROB_P, x - e)) / (2 * e[j])
            np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-6 * np.abs(J).max())
        G = orc.ftheta(orc.ROBERTSON, ROB_P, x)
        assert np.abs(G.sum(axis=0)).max() <= 1e-12 * max(np.abs(G).max(), 1.0)
        for k in range(3):
            dp = np.array(ROB_P, dtype=float)
            h = 1e-6 * dp[k]
            dp[k] += h
            dm = np.array(ROB_P, dtype=float)
            dm[k] -= h
            fd = (orc.f(orc.ROBERTSON, dp, x) - orc.f(orc.ROBERTSON, dm, x)) / (2 * h)
            np.testing.assert_allclose(G[:, k], fd, rtol=1e-6, atol=1e-9)


def test_robertson_backward_euler_conserves_mass(orc):
    """A linear invariant of f is kept exactly by any implicit rule: the
    concentrations sum to one at every step, and the fast species stays
    tiny and positive (the stiff quasi-steady state)."""
    dt, T = 0.1, 5000
    x = orc.integrate_implicit(orc.BEULER, orc.ROBERTSON, ROB_P, dt, T, ROB_X0)
    np.testing.assert_allclose(x.sum(axis=1), 1.0, rtol=0, atol=1e-13)
    assert np.all(x[:, 1] > 0) and x[:, 1].max() < 1e-4
    r = orc.newton_implicit(orc.BEULER, orc.ROBERTSON, ROB_P, dt, T, ROB_X0,
                            guess=np.zeros((T, 3)), tol=1e-13)
    np.testing.assert_allclose(r["traj"], x, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("sysname", ["vdp", "lorenz63", "cartpole"])
@pytest.mark.parametrize("method", ["be", "trap"])
def test_implicit_newton_fixed_point_is_sequential(orc, sysname, method):
    """Plain and windowed Newton reach the step-by-step implicit trajectory."""
    m = orc.BEULER if method == "be" else orc.TRAP
    cfg = {
        "vdp": (orc.VDP, [1.0], [2.0, 0.0], 0.01, 600),
        "lorenz63": (orc.LORENZ63, [10.0, 28.0, 8.0 / 3.0], [1.0, 1.0, 1.0], 0.005, 150),
        "cartpole": (orc.CARTPOLE, [9.81, 1.0, 1.0, 0.1], [0.0, 0.5, 0.0, 0.0], 0.01, 300),
    }[sysname]
    s, P, x0, dt, T = cfg
    seq = orc.integrate_implicit(m, s, P, dt, T, x0)
    scale = np.abs(seq).max()
    for window in (0, 32):
        r = orc.newton_implicit(m, s, P, dt, T, x0, tol=1e-12, max_iter=400, window=window)
        assert r["status"] == orc.OK, (window, r["status"])
        np.testing.assert_allclose(r["traj"], seq, rtol=0, atol=1e-9 * scale)
        hs = orc.residual_implicit(m, s, P, dt, x0, r["traj"], scaled=True)
        assert np.abs(hs).max() < 1e-12


def test_implicit_quadratic_tail(orc):
    """Local quadratic convergence: near the solution the next residual is
    bounded by a constant times the square of the current one."""
    T, dt = 400, 0.01
    r = orc.newton_implicit(orc.TRAP, orc.VDP, [1.0], dt, T, [2.0, 0.0], tol=1e-15,
                            max_iter=60)
    h = r["hist"]
    tail = [(a, b) for a, b in zip(h, h[1:]) if 1e-12 < a < 1e-3]
    assert tail, h
    for a, b in tail:
        assert b <= 1e3 * a * a, (a, b)


def test_implicit_edge_cases(orc):
    z = orc.newton_implicit(orc.BEULER, orc.VDP, [1.0], 0.01, 0, [1.0, 0.0])
    assert z["status"] == orc.OK and z["iters"] == 0 and z["traj"].shape == (0, 2)
    r = orc.newton_implicit(orc.BEULER, orc.VDP, [1.0], 0.01, 50, [1.0, 0.0], max_iter=0)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 0
    # the sequential trajectory as the guess: already converged, no update
    seq = orc.integrate_implicit(orc.TRAP, orc.VDP, [1.0], 0.01, 50, [1.0, 0.0])
    r = orc.newton_implicit(orc.TRAP, orc.VDP, [1.0], 0.01, 50, [1.0, 0.0], guess=seq,
                            tol=1e-12)
    assert r["status"] == orc.OK and r["iters"] == 0
    # a window of one step is the sequential Newton iteration itself
    r = orc.newton_implicit(orc.BEULER, orc.VDP, [1.0], 0.01, 50, [1.0, 0.0], window=1,
                            tol=1e-12, max_iter=1000)
    assert r["status"] == orc.OK
    np.testing.assert_allclose(r["traj"],
                               orc.integrate_implicit(orc.BEULER, orc.VDP, [1.0], 0.01, 50,
                                                      [1.0, 0.0]), atol=1e-12)
