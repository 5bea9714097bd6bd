"""Pins for the CPU oracle: values the paper prints, closed forms,
invariants and finite differences.  None of these retypes the oracle's
formulas; each is chosen so that a plausible mistake in it (a dropped term,
a wrong sign or index, a transposed operand) fails at least one test."""
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


def _pin(name):
    return next(p for p in W.paper_pins() if p["name"] == name)


# Reading of the paper's (unstated) stopping tolerance: the accepted final
# residuals of the printed histories go up to 1.38e-14 (cart-pole) and the
# rejected ones down to 4.85e-14 (logistic), so tol lies in (1.38e-14, 4.85e-14].
PAPER_TOL = 3e-14


# ---------------------------------------------------------------- P1, P2 --

@pytest.mark.parametrize("name", ["logistic", "vdp", "cartpole"])
def test_paper_residual_history(orc, name):
    """Figure 5 (Sec. 4.1): the printed Newton residual histories at dt=1e-2.
    They fix the RK4 tableau, the exact Jacobian of the step, the infinity
    norm over all entries, full Newton steps, the initial guess and the
    exclusion of x_0 from xi."""
    gold = [(int(k), float(v)) for p, k, v in _read_table("explicit_residuals_dt1e-2.txt") if p == name]
    pin = _pin(name)
    d = len(pin["x0"])
    guess = np.full((pin["T"], d), pin["guess"])
    r = orc.newton(pin["system"], pin["params"], pin["dt"], pin["T"], pin["x0"],
                   guess=guess, tol=PAPER_TOL, max_iter=50)
    assert r["status"] == orc.OK
    hist = r["hist"]
    # K = number of residual evaluations = updates + 1 (Figure 6 convention)
    assert len(hist) == len(gold)
    for k, v in gold:
        if v > 1e-11:
            assert abs(hist[k] - v) <= 1e-7 * v, (k, hist[k], v)
        else:  # rounding-floor values: same order of magnitude only
            assert hist[k] < 1e-11 and hist[k] < 20 * max(v, 1e-16)


@pytest.mark.parametrize("name", ["logistic", "vdp", "cartpole"])
def test_paper_iteration_counts(orc, name):
    """Figure 6 (Sec. 4.1): K against dt.  At dt=1e-2 K is exact.  At smaller
    dt the last evaluation sits at the rounding floor, whose size depends on
    the summation order of the implementation, so K may be one lower than
    printed (never higher)."""
    pin = _pin(name)
    horizon = pin["T"] * pin["dt"]
    d = len(pin["x0"])
    for p, dt_s, K in _read_table("explicit_iterations.txt"):
        if p != name:
            continue
        dt = float(dt_s)
        if dt < 1e-4 and os.environ.get("PINT_FAST_TESTS"):
            continue
        T = int(round(horizon / dt))
        r = orc.newton(pin["system"], pin["params"], dt, T, pin["x0"],
                       guess=np.full((T, d), pin["guess"]), tol=PAPER_TOL, max_iter=40)
        assert r["status"] == orc.OK
        ours = r["iters"] + 1
        if dt == 1e-2:
            assert ours == int(K)
        else:
            assert int(K) - 1 <= ours <= int(K), (dt, ours, K)


# ------------------------------------------------------- vector fields ----

def _fd_jac(fun, x, h=1e-3):
    """Fourth-order central differences, column by column."""
    x = np.asarray(x, float)
    cols = []
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = h
        cols.append((-fun(x + 2 * e) + 8 * fun(x + e) - 8 * fun(x - e) + fun(x - 2 * e)) / (12 * h))
    return np.stack(cols, axis=1)


def _systems(rng):
    """(system, params, x) samples with asymmetric Jacobians."""
    d8 = 8
    M = rng.normal(size=(3, 3))
    return [
        (W.LINEAR, M.ravel(), rng.normal(size=3)),
        (W.LOGISTIC, np.array([1.3, 2.1]), np.array([0.7])),
        (W.VDP, np.array([2.5]), rng.normal(size=2)),
        (W.CARTPOLE, np.array([9.81, 0.5, 10.0, 1.0]), np.array([0.3, 1.1, -0.4, 0.8])),
        (W.LORENZ63, np.array([10.0, 28.0, 8.0 / 3.0]), rng.normal(size=3) * 5),
        (W.LORENZ96, np.array([8.0]), 8 + rng.normal(size=d8)),
        (W.KURAMOTO, np.concatenate([[0.7], rng.normal(size=6)]), rng.uniform(0, 2 * np.pi, 6)),
    ]


def test_jf_matches_finite_differences(orc):
    rng = np.random.default_rng(11)
    for sysid, P, x in _systems(rng):
        J = orc.jf(sysid, P, x)
        Jfd = _fd_jac(lambda y: orc.f(sysid, P, y), x)
        assert np.allclose(J, Jfd, rtol=1e-8, atol=1e-8 * max(1.0, np.abs(J).max())), sysid


def test_ftheta_matches_finite_differences(orc):
    rng = np.random.default_rng(12)
    for sysid, P, x in _systems(rng):
        if sysid == W.CARTPOLE:
            with pytest.raises(ValueError):
                orc.ftheta(sysid, P, x)
            continue
        G = orc.ftheta(sysid, P, x)
        Gfd = _fd_jac(lambda q: orc.f(sysid, q, x), P)
        assert np.allclose(G, Gfd, rtol=1e-8, atol=1e-8), sysid


def test_lorenz63_equilibria(orc):
    s, rho, b = 10.0, 28.0, 8.0 / 3.0
    c = math.sqrt(b * (rho - 1))
    for x in ([0, 0, 0], [c, c, rho - 1], [-c, -c, rho - 1]):
        assert np.abs(orc.f(W.LORENZ63, [s, rho, b], x)).max() < 1e-13


def test_lorenz96_energy_equilibrium_and_spectrum(orc):
    rng = np.random.default_rng(3)
    d = 40
    x = rng.normal(size=d) * 3
    # with F = 0 the advection term conserves energy: sum x_i f_i = -sum x_i^2
    fx = orc.f(W.LORENZ96, [0.0], x)
    assert abs(np.dot(x, fx) + np.dot(x, x)) < 1e-10 * np.dot(x, x)
    # x = F 1 is an equilibrium
    assert np.abs(orc.f(W.LORENZ96, [8.0], np.full(d, 8.0))).max() == 0.0
    # circulant linearisation: eigenvalues F(w^k - w^{-2k}) - 1, w = e^{2 pi i/d}
    J = orc.jf(W.LORENZ96, [8.0], np.full(d, 8.0))
    w = np.exp(2j * np.pi * np.arange(d) / d)
    expect = 8.0 * (w - w ** -2) - 1.0
    got = np.linalg.eigvals(J)
    assert np.allclose(np.sort_complex(np.round(got, 9)), np.sort_complex(np.round(expect, 9)), atol=1e-7)
    assert abs(expect.real.max() - 7.94) < 0.01


def test_kuramoto_invariants(orc):
    rng = np.random.default_rng(5)
    d = 16
    om = rng.normal(size=d)
    P = np.concatenate([[0.3], om])
    th = rng.uniform(0, 2 * np.pi, d)
    fx = orc.f(W.KURAMOTO, P, th)
    assert abs(fx.sum() - om.sum()) < 1e-12          # coupling sums cancel
    assert np.allclose(orc.f(W.KURAMOTO, P, th + 1.234), fx, atol=1e-12)  # shift invariance
    J = orc.jf(W.KURAMOTO, P, th)
    assert np.abs(J.sum(axis=1)).max() < 1e-12       # J 1 = 0
    # two oscillators: phase difference phi' = (w2 - w1) - 2 K sin(phi)
    P2 = [0.4, 0.1, 0.9]
    th2 = np.array([0.2, 1.5])
    f2 = orc.f(W.KURAMOTO, P2, th2)
    phi = th2[1] - th2[0]
    assert abs((f2[1] - f2[0]) - ((0.9 - 0.1) - 2 * 0.4 * math.sin(phi))) < 1e-14


# ------------------------------------------------------------- RK4 step ---

def _rk4_poly(Z):
    I = np.eye(Z.shape[0])
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24


def test_rk4_linear_closed_form(orc):
    """For x' = M x every 4-stage order-4 RK method is x -> R(dt M) x with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24; dPhi/dx = R(dt M)."""
    rng = np.random.default_rng(7)
    d, dt = 5, 0.3
    M = rng.normal(size=(d, d))
    x = rng.normal(size=d)
    R = _rk4_poly(dt * M)
    assert np.allclose(orc.rk4_step(W.LINEAR, M.ravel(), dt, x), R @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(orc.rk4_jac(W.LINEAR, M.ravel(), dt, x), R, rtol=1e-13, atol=1e-13)


def test_rk4_fourth_order_on_logistic(orc):
    """Global error against the closed-form logistic solution shrinks 16x
    per halving of dt."""
    r_, K_, P0, t = 1.0, 1.0, 0.1, 2.0
    exact = K_ / (1 + (K_ / P0 - 1) * math.exp(-r_ * t))
    errs = []
    for n in (10, 20, 40):
        traj = orc.integrate(W.LOGISTIC, [r_, K_], t / n, n, [P0])
        errs.append(abs(traj[-1, 0] - exact))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


def test_rk4_jacobians_match_finite_differences(orc):
    rng = np.random.default_rng(13)
    dt = 0.02
    for sysid, P, x in _systems(rng):
        J = orc.rk4_jac(sysid, P, dt, x)
        Jfd = _fd_jac(lambda y: orc.rk4_step(sysid, P, dt, y), x)
        assert np.allclose(J, Jfd, rtol=1e-8, atol=1e-9), sysid
        if sysid == W.CARTPOLE:
            continue
        S = orc.rk4_ptheta(sysid, P, dt, x)
        Sfd = _fd_jac(lambda q: orc.rk4_step(sysid, q, dt, x), P)
        assert np.allclose(S, Sfd, rtol=1e-8, atol=1e-9), sysid


def test_residual_of_sequential_trajectory_is_zero(orc):
    w = W.lorenz63(T=300)
    traj = orc.integrate(w.system, w.params[0], w.dt, 300, w.x0[0])
    assert np.abs(orc.residual(w.system, w.params[0], w.dt, w.x0[0], traj)).max() == 0.0


# ------------------------------------------------- affine scan (P4) -------

def _augmented_chain(A, b, z0):
    """z via products of (d+1)x(d+1) augmented matrices [[A, b], [0, 1]]."""
    N, d, _ = A.shape
    out = np.empty((N, d))
    v = np.concatenate([z0, [1.0]])
    for n in range(N):
        G = np.eye(d + 1)
        G[:d, :d] = A[n]
        G[:d, d] = b[n]
        v = G @ v
        out[n] = v[:d]
    return out


def test_affine_seq_against_augmented_products(orc):
    for d in (1, 2, 3, 8):
        A, b = W.random_affine(50, d, seed=d, kind="gauss")
        z0 = np.random.default_rng(d).normal(size=d)
        assert np.allclose(orc.affine_seq(A, b, z0), _augmented_chain(A, b, z0), rtol=1e-12, atol=1e-12)


def test_affine_seq_constant_closed_form(orc):
    """Constant A, b and z_0 = 0: z_n = (I - A)^{-1} (I - A^n) b."""
    d, N = 3, 40
    rng = np.random.default_rng(2)
    A1 = 0.5 * rng.normal(size=(d, d)) / math.sqrt(d)
    b1 = rng.normal(size=d)
    z = orc.affine_seq(np.repeat(A1[None], N, 0), np.repeat(b1[None], N, 0))
    inv = np.linalg.inv(np.eye(d) - A1)
    for n in (1, 7, N):
        An = np.linalg.matrix_power(A1, n)
        assert np.allclose(z[n - 1], inv @ (np.eye(d) - An) @ b1, atol=1e-12)


def test_combine_is_associative_and_matches_recursion(orc):
    """Lemma (Sec. 3.1): any bracketing gives the same composition, and the
    composition of the first n elements maps z_0 to z_n."""
    d = 4
    A, b = W.random_affine(6, d, seed=9, kind="gauss")
    e = [(A[i], b[i]) for i in range(6)]
    left = e[0]
    for i in range(1, 6):             # ((e0 . e1) . e2) ... later on the left
        left = orc.combine(e[i], left)
    right = e[5]
    for i in range(4, -1, -1):        # e5 . (e4 . (... e0))
        right = orc.combine(right, e[i])
    mid = orc.combine(orc.combine(e[5], orc.combine(e[4], e[3])),
                      orc.combine(orc.combine(e[2], e[1]), e[0]))
    for F, c in (right, mid):
        assert np.allclose(F, left[0], atol=1e-12) and np.allclose(c, left[1], atol=1e-12)
    z0 = np.random.default_rng(1).normal(size=d)
    zN = orc.affine_seq(A, b, z0)[-1]
    assert np.allclose(left[0] @ z0 + left[1], zN, atol=1e-12)


# ------------------------------------------------------------- Newton -----

def test_linear_ode_converges_in_one_update(orc):
    """P3: Phi is linear for x' = M x, so h is affine and one Newton update
    lands on the root; the next evaluation is at rounding level."""
    rng = np.random.default_rng(4)
    d, T, dt = 3, 300, 0.05
    M = rng.normal(size=(d, d)) * 0.5
    x0 = rng.normal(size=d)
    guess = rng.normal(size=(T, d))
    r = orc.newton(W.LINEAR, M.ravel(), dt, T, x0, guess=guess, tol=1e-12)
    assert r["status"] == orc.OK and r["iters"] == 1
    R = _rk4_poly(dt * M)
    x = x0.copy()
    for n in range(T):
        x = R @ x
        assert np.allclose(r["traj"][n], x, rtol=1e-10, atol=1e-10)


def test_newton_fixed_point_is_sequential_trajectory(orc):
    """P5: H has identity diagonal blocks, so the root of h is O1."""
    w = W.lorenz63(T=512)
    ref = orc.integrate(w.system, w.params[0], w.dt, 512, w.x0[0])
    r = orc.newton(w.system, w.params[0], w.dt, 512, w.x0[0], tol=1e-13)
    assert r["status"] == orc.OK
    assert np.abs(r["traj"] - ref).max() < 1e-11


def test_exact_prefix_invariant(orc):
    """After k plain updates, x_1..x_k equal the sequential trajectory (to
    rounding), so Newton ends within T updates."""
    w = W.lorenz63(T=256)
    ref = orc.integrate(w.system, w.params[0], w.dt, 256, w.x0[0])
    for k in range(1, 6):
        r = orc.newton(w.system, w.params[0], w.dt, 256, w.x0[0], tol=1e-300, max_iter=k)
        assert r["status"] == orc.NOT_CONVERGED and r["iters"] == k
        assert np.abs(r["traj"][:k] - ref[:k]).max() < 1e-12
    # a tiny problem really terminates within T updates
    r = orc.newton(w.system, w.params[0], w.dt, 6, w.x0[0], tol=1e-14)
    assert r["status"] == orc.OK and r["iters"] <= 6


def test_quadratic_tail(orc):
    """P6 (Theorem 3.2): near the root r_{k+1} <= C r_k^2."""
    for name in ("logistic", "vdp", "cartpole"):
        pin = _pin(name)
        d = len(pin["x0"])
        r = orc.newton(pin["system"], pin["params"], pin["dt"], pin["T"], pin["x0"],
                       guess=np.full((pin["T"], d), pin["guess"]), tol=PAPER_TOL)
        h = r["hist"]
        tail = [(h[k], h[k + 1]) for k in range(len(h) - 1) if 1e-12 < h[k] < 1e-2 and h[k + 1] > 1e-15]
        assert tail, name
        for a, b in tail:
            assert b <= 1e3 * a * a, (name, a, b)


def test_windowed_newton_reaches_the_same_fixed_point(orc):
    w = W.lorenz63(T=2048)
    ref = orc.integrate(w.system, w.params[0], w.dt, 2048, w.x0[0])
    plain = orc.newton(w.system, w.params[0], w.dt, 2048, w.x0[0], tol=1e-10, max_iter=60)
    assert plain["status"] != orc.OK     # the plain method fails here (local theorem)
    r = orc.newton(w.system, w.params[0], w.dt, 2048, w.x0[0], tol=1e-13, window=128, max_iter=4096)
    assert r["status"] == orc.OK and r["final_resid"] < 1e-13
    assert np.abs(r["traj"] - ref).max() < 1e-10


def test_windowed_newton_defect_bound_on_lorenz96(orc):
    """Chaotic case: the converged windowed iterate has every step's defect
    below tol, and follows O1 over the first time unit."""
    w = W.lorenz96(T=1024, window=32)
    r = orc.newton(w.system, w.params[0], w.dt, 1024, w.x0[0], tol=1e-10, window=32, max_iter=2048)
    assert r["status"] == orc.OK
    h = orc.residual(w.system, w.params[0], w.dt, w.x0[0], r["traj"])
    assert np.abs(h).max() < 1e-10
    ref = orc.integrate(w.system, w.params[0], w.dt, 1024, w.x0[0])
    assert np.abs(r["traj"][:100] - ref[:100]).max() < 1e-8


def test_newton_edge_cases(orc):
    w = W.lorenz63()
    P, x0 = w.params[0], w.x0[0]
    r = orc.newton(w.system, P, w.dt, 0, x0)
    assert r["status"] == orc.OK and r["iters"] == 0
    r = orc.newton(w.system, P, w.dt, 1, x0, tol=1e-14)
    assert r["status"] == orc.OK and r["iters"] == 1
    assert np.array_equal(r["traj"][0], orc.rk4_step(w.system, P, w.dt, x0))
    r = orc.newton(w.system, P, w.dt, 64, x0, max_iter=1, tol=1e-14)
    assert r["status"] == orc.NOT_CONVERGED and r["iters"] == 1
    bad = x0.copy()
    bad[1] = np.nan
    for win in (0, 16):
        r = orc.newton(w.system, P, w.dt, 64, bad, window=win)
        assert r["status"] == orc.NONFINITE


# ------------------------------------------------------------ adjoint ------

def _loss_grad(traj, y, obs):
    """L = sum_j ||x_{n_j} - y_j||^2 and dL/dx_n."""
    g = np.zeros_like(traj)
    L = 0.0
    for j, n in enumerate(obs):
        diff = traj[n - 1] - y[j]
        L += float(diff @ diff)
        g[n - 1] += 2 * diff
    return L, g


def test_adjoint_dot_product_against_tangent(orc):
    rng = np.random.default_rng(21)
    cases = [(W.LORENZ63, [10.0, 28.0, 8 / 3], rng.normal(size=3) + 1, 1e-3, 300),
             (W.VDP, [2.0], rng.normal(size=2), 0.01, 400),
             (W.LORENZ96, [8.0], 8 + 0.5 * rng.normal(size=8), 0.005, 200),
             (W.KURAMOTO, np.concatenate([[0.4], rng.normal(size=5)]), rng.uniform(0, 6, 5), 0.01, 150)]
    for sysid, P, x0, dt, T in cases:
        traj = orc.integrate(sysid, P, dt, T, x0)
        g = rng.normal(size=traj.shape)
        gx0, gth = orc.adjoint(sysid, P, dt, x0, traj, g)
        dx0 = rng.normal(size=x0.size)
        dth = rng.normal(size=len(P))
        v = orc.tangent(sysid, P, dt, x0, traj, dx0, dth)
        lhs = float(np.sum(g * v))
        rhs = float(gx0 @ dx0 + gth @ dth)
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0), sysid


def test_adjoint_matches_central_differences(orc):
    """Short horizons, where finite differences of the loss are meaningful."""
    rng = np.random.default_rng(8)
    for sysid, P, x0, dt, T in [(W.LORENZ96, np.array([8.0]), 8 + 0.01 * rng.normal(size=40), 0.005, 200),
                                (W.LORENZ63, np.array([10.0, 28.0, 8 / 3]), 1 + 0.1 * rng.normal(size=3), 1e-3, 400),
                                (W.VDP, np.array([3.0]), rng.uniform(-2, 2, 2), 0.01, 300)]:
        d = x0.size
        obs = (np.arange(1, 9) * T) // 8
        y = rng.normal(size=(8, d))

        def L_of(x0_, P_):
            return _loss_grad(orc.integrate(sysid, P_, dt, T, x0_), y, obs)[0]

        traj = orc.integrate(sysid, P, dt, T, x0)
        _, g = _loss_grad(traj, y, obs)
        gx0, gth = orc.adjoint(sysid, P, dt, x0, traj, g)
        h = 1e-6
        for i in range(min(d, 6)):
            e = np.zeros(d)
            e[i] = h
            fd = (L_of(x0 + e, P) - L_of(x0 - e, P)) / (2 * h)
            assert abs(fd - gx0[i]) <= 1e-6 * max(1.0, abs(gx0[i])), (sysid, i, fd, gx0[i])
        for j in range(len(P)):
            e = np.zeros(len(P))
            e[j] = h * max(1.0, abs(P[j]))
            fd = (L_of(x0, P + e) - L_of(x0, P - e)) / (2 * e[j])
            assert abs(fd - gth[j]) <= 1e-6 * max(1.0, abs(gth[j])), (sysid, j, fd, gth[j])


def test_adjoint_linear_closed_form(orc):
    """x_n = R^n x0 for x' = M x, so dL/dx0 = sum_n (R^n)^T g_n."""
    rng = np.random.default_rng(31)
    d, T, dt = 4, 60, 0.05
    M = rng.normal(size=(d, d)) * 0.4
    x0 = rng.normal(size=d)
    traj = orc.integrate(W.LINEAR, M.ravel(), dt, T, x0)
    g = rng.normal(size=(T, d))
    gx0, _ = orc.adjoint(W.LINEAR, M.ravel(), dt, x0, traj, g)
    R = _rk4_poly(dt * M)
    expect = np.zeros(d)
    Rn = np.eye(d)
    for n in range(T):
        Rn = R @ Rn
        expect += Rn.T @ g[n]
    assert np.allclose(gx0, expect, rtol=1e-11, atol=1e-11)
