"""Pins for the oracle's Parareal (Sec. 2.2, eqs. parareal-init,
fine-integrator, coarse-integrator): the paper's printed error histories and
iteration counts, the closed form of Parareal on linear problems, the exact
windows after k corrections, and the degenerate splits."""
import math
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _problems(orc):
    """name -> (system, params, x0, horizon, method), the paper's problems."""
    out = {}
    for p in W.paper_pins():
        out[p["name"]] = (p["system"], p["params"], p["x0"], p["T"] * p["dt"], orc.RK4)
    for p in W.implicit_pins():
        out[p["name"]] = (p["system"], p["params"], p["x0"], p["horizon"], orc.BEULER)
    return out


def _tol(name):
    # the reading of the unstated Parareal tolerance (parareal_iterations.txt)
    return 1e-12 if name == "cartpole" else 1e-15


@pytest.mark.parametrize("name,dt", [("logistic", 1e-2), ("vdp", 1e-2), ("cartpole", 1e-2),
                                     ("dahlquist", 1e-1), ("robertson", 1e-1)])
def test_paper_parareal_history(orc, name, dt):
    """Figures 5 and 8: the printed Parareal error histories.  They fix the
    split (M = floor(sqrt(N)) windows of floor(N/M) fine steps, the coarse
    step S*dt), the single-step coarse integrator, the correction
    G(new) + F - G(old) and the error measure R."""
    gold = [(int(k), float(v)) for p, k, v in _read_table("parareal_residuals.txt") if p == name]
    sys_, prm, x0, horizon, method = _problems(orc)[name]
    N = int(round(horizon / dt))
    M, S = orc.parareal_windows(N)
    r = orc.parareal(sys_, prm, dt, M, S, x0, tol=_tol(name), max_iter=40, method=method)
    assert r["status"] == orc.OK
    assert r["iters"] == len(gold)
    # R is a difference of states of size up to |x|max, so besides 1e-7
    # relative it carries an absolute rounding of a few ulps of |x|max
    floor = 8 * 2.220446049250313e-16 * max(1.0, np.abs(r["traj"]).max())
    for k, v in gold:
        if v > 1e-11:
            assert abs(r["hist"][k] - v) <= 1e-7 * v + floor, (k, r["hist"][k], v)
        else:  # rounding-floor values: magnitude only
            assert r["hist"][k] < 1e-11 and r["hist"][k] < 20 * max(v, 1e-16), (k, r["hist"][k], v)


def test_paper_parareal_iteration_counts(orc):
    """Figures 6 and 9: K against dt, for the rows the tolerance reading
    reproduces (the fixture says which and why the others are unpinned)."""
    probs = _problems(orc)
    fast = bool(os.environ.get("PINT_FAST_TESTS"))
    for name, dt_s, K, tol_s, pinned in _read_table("parareal_iterations.txt"):
        if pinned != "1":
            continue
        dt = float(dt_s)
        sys_, prm, x0, horizon, method = probs[name]
        N = int(round(horizon / dt))
        if fast and N > 200000:
            continue
        M, S = orc.parareal_windows(N)
        r = orc.parareal(sys_, prm, dt, M, S, x0, tol=float(tol_s), max_iter=40, method=method)
        assert r["status"] == orc.OK, (name, dt)
        assert r["iters"] == int(K), (name, dt, r["iters"], K, r["hist"])


def _rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def _closed_form_iterates(Gm, Fm, x0, M, kmax):
    """Parareal on a linear problem with commuting coarse and fine
    propagators G, F (matrices): x_m^(k) = sum_{j<=k} C(m, j) (F - G)^j
    G^(m-j) x0 (Gander and Vandewalle 2007, Sec. 4)."""
    d = len(x0)
    D = Fm - Gm
    out = []
    for k in range(kmax):
        xs = []
        for m in range(M + 1):
            acc = np.zeros(d)
            for j in range(min(k, m) + 1):
                acc += math.comb(m, j) * (np.linalg.matrix_power(D, j)
                                          @ np.linalg.matrix_power(Gm, m - j) @ x0)
            xs.append(acc)
        out.append(np.array(xs))
    return out


@pytest.mark.parametrize("method", ["rk4", "beuler"])
def test_linear_closed_form(orc, method):
    """x' = A x: the coarse and fine maps are matrix functions of A, so the
    iterates have the binomial closed form; R^(k) and the final dense
    trajectory (fine steps from x^(K-1)) follow from it."""
    A = np.array([[-0.3, 1.0], [-1.0, -0.2]])
    x0 = np.array([1.0, -0.5])
    dt, M, S = 0.05, 6, 5
    H = S * dt
    I = np.eye(2)
    if method == "rk4":
        m_id = orc.RK4
        step = lambda h: I + h * A + (h * A) @ (h * A) / 2 + np.linalg.matrix_power(h * A, 3) / 6 \
            + np.linalg.matrix_power(h * A, 4) / 24
    else:
        m_id = orc.BEULER
        step = lambda h: np.linalg.inv(I - h * A)
    Gm, fm = step(H), step(dt)
    Fm = np.linalg.matrix_power(fm, S)
    kmax = 4
    iters = _closed_form_iterates(Gm, Fm, x0, M, kmax)
    r = orc.parareal(orc.LINEAR, A.ravel(), dt, M, S, x0, tol=0.0, max_iter=kmax, method=m_id)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == kmax
    for k in range(kmax):
        xk = iters[k]
        Rk = max(np.abs(xk[m + 1] - Fm @ xk[m]).max() for m in range(M))
        assert abs(r["hist"][k] - Rk) <= 1e-12 * max(Rk, 1e-3) + 1e-15, (k, r["hist"][k], Rk)
    # the returned trajectory: fine steps from the last iterate x^(kmax-1)
    last = iters[kmax - 1]
    for m in range(M):
        y = last[m]
        for j in range(S):
            y = fm @ y
            np.testing.assert_allclose(r["traj"][m * S + j], y, rtol=0, atol=1e-13)
    # and the scalar RK4 polynomial agrees with the matrix step (sanity of the test's own map)
    if method == "rk4":
        lam = -0.7
        r1 = orc.parareal(orc.LINEAR, [lam], dt, 1, S, [1.0], tol=0.0, max_iter=1)
        assert abs(r1["traj"][-1][0] - _rk4_poly(lam * dt) ** S) < 1e-15


@pytest.mark.parametrize("name", ["vdp", "cartpole", "robertson"])
def test_exact_windows_after_k_corrections(orc, name):
    """After k corrections the first k windows start from the exact fine
    states, so the dense trajectory of the next fine sweep equals the
    sequential integration there (the classic Parareal property); after M
    corrections it equals it everywhere."""
    sys_, prm, x0, horizon, method = _problems(orc)[name]
    dt = {"vdp": 1e-2, "cartpole": 1e-2, "robertson": 1e-1}[name]
    M, S = 12, 9
    if method == orc.RK4:
        seq = orc.integrate(sys_, prm, dt, M * S, x0)
    else:
        seq = orc.integrate_implicit(method, sys_, prm, dt, M * S, x0)
    scale = max(1.0, np.abs(seq).max())
    for k in (0, 1, 3, M):
        r = orc.parareal(sys_, prm, dt, M, S, x0, tol=0.0, max_iter=k + 1, method=method)
        exact = (k + 1) * S
        err = np.abs(r["traj"][:exact] - seq[:exact]).max()
        assert err <= 1e-12 * scale, (k, err)
        if k == 0:  # and not beyond, where the coarse error remains
            assert np.abs(r["traj"][exact:] - seq[exact:]).max() > 1e-9


def test_converged_equals_sequential(orc):
    """The fixed point is the sequential fine trajectory (Sec. 2.2): a
    converged run matches O1 to the tolerance's amplification."""
    for name in ("logistic", "vdp", "cartpole"):
        sys_, prm, x0, horizon, method = _problems(orc)[name]
        dt = 1e-2
        N = int(round(horizon / dt))
        M, S = orc.parareal_windows(N)
        r = orc.parareal(sys_, prm, dt, M, S, x0, tol=1e-13)
        seq = orc.integrate(sys_, prm, dt, M * S, x0)
        assert r["status"] == orc.OK
        assert np.abs(r["traj"] - seq).max() < 1e-11, name


def test_degenerate_splits(orc):
    """S = 1: the coarse step is the fine step, so R^(0) = 0 exactly and the
    trajectory is O1 bit for bit.  M = 1: one correction makes the single
    window exact.  M or S = 0: nothing to do.  A NaN start: NONFINITE."""
    sys_, prm, x0 = orc.VDP, [1.0], [0.5, -0.3]
    r = orc.parareal(sys_, prm, 0.01, 37, 1, x0, tol=1e-15)
    assert r["status"] == orc.OK and r["iters"] == 1 and r["hist"][0] == 0.0
    assert np.array_equal(r["traj"], orc.integrate(sys_, prm, 0.01, 37, x0))
    r = orc.parareal(sys_, prm, 0.01, 1, 50, x0, tol=1e-14)
    assert r["status"] == orc.OK and r["iters"] == 2 and r["hist"][0] > 1e-10
    np.testing.assert_allclose(r["traj"], orc.integrate(sys_, prm, 0.01, 50, x0), rtol=0, atol=1e-15)
    for M, S in ((0, 5), (5, 0)):
        r = orc.parareal(sys_, prm, 0.01, M, S, x0)
        assert r["status"] == orc.OK and r["iters"] == 0 and r["traj"].shape == (0, 2)
    r = orc.parareal(sys_, prm, 0.01, 4, 4, [np.nan, 0.0])
    assert r["status"] == orc.NONFINITE
    r = orc.parareal(sys_, prm, 0.01, 8, 8, x0, tol=0.0, max_iter=3)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 3
