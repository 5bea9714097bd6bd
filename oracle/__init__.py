"""CPU oracle for the parallel-in-time Newton ODE solver (arXiv 2511.01465).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The HIP library never
links, loads or calls it, and it never calls the HIP library.

The arithmetic lives in ``oracle.c`` (plain C, double precision, built without
floating-point contraction).  This module only loads the shared object and
marshals numpy arrays.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# System identifiers (same numbering as the public C interface).
LINEAR, LOGISTIC, VDP, CARTPOLE, LORENZ63, LORENZ96, KURAMOTO, ROBERTSON = range(8)
OK, NOT_CONVERGED, NONFINITE = 0, 4, 5
# One-step rules: explicit RK4, backward Euler, trapezoidal (Sec. 3.4).
RK4, BEULER, TRAP = range(3)

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (IEEE semantics, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    i64p = C.POINTER(C.c_int64)
    i, i64, d = C.c_int, C.c_int64, C.c_double
    sig = {
        "orc_n_params": (i, [i, i]),
        "orc_f": (None, [i, i, dp, dp, dp]),
        "orc_jf": (None, [i, i, dp, dp, dp]),
        "orc_ftheta": (i, [i, i, dp, dp, dp]),
        "orc_rk4_step": (None, [i, i, dp, d, dp, dp]),
        "orc_rk4_jac": (None, [i, i, dp, d, dp, dp]),
        "orc_rk4_ptheta": (i, [i, i, dp, d, dp, dp]),
        "orc_integrate": (None, [i, i, dp, d, i64, dp, dp]),
        "orc_residual": (None, [i, i, dp, d, i64, dp, dp, dp]),
        "orc_affine_seq": (None, [i, i64, dp, dp, dp, dp]),
        "orc_combine": (None, [i, dp, dp, dp, dp, dp, dp]),
        "orc_newton": (i, [i, i, dp, d, i64, dp, dp, d, i64, i64, d, dp, i64p, dp]),
        "orc_residual_implicit": (None, [i, i, i, dp, d, i64, dp, dp, i, dp]),
        "orc_integrate_implicit": (i, [i, i, i, dp, d, i64, dp, dp]),
        "orc_newton_implicit": (i, [i, i, i, dp, d, i64, dp, dp, d, i64, i64, d, dp,
                                    i64p, dp]),
        "orc_adjoint": (i, [i, i, dp, d, i64, dp, dp, dp, dp, dp]),
        "orc_tangent": (i, [i, i, dp, d, i64, dp, dp, dp, dp, dp]),
        "orc_parareal": (i, [i, i, i, dp, d, i64, i64, dp, d, i64, dp, dp, i64p, dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def n_params(sys: int, d: int) -> int:
    return _load().orc_n_params(sys, d)


def f(sys, params, x):
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_f(sys, x.size, _p(_f64(params)), _p(x), _p(out))
    return out


def jf(sys, params, x):
    x = _f64(x)
    d = x.size
    J = np.empty((d, d))
    _load().orc_jf(sys, d, _p(_f64(params)), _p(x), _p(J))
    return J


def ftheta(sys, params, x):
    x = _f64(x)
    d = x.size
    G = np.empty((d, n_params(sys, d)))
    if _load().orc_ftheta(sys, d, _p(_f64(params)), _p(x), _p(G)) != 0:
        raise ValueError("no parameter derivative for this system")
    return G


def rk4_step(sys, params, dt, x):
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_rk4_step(sys, x.size, _p(_f64(params)), dt, _p(x), _p(out))
    return out


def rk4_jac(sys, params, dt, x):
    x = _f64(x)
    d = x.size
    J = np.empty((d, d))
    _load().orc_rk4_jac(sys, d, _p(_f64(params)), dt, _p(x), _p(J))
    return J


def rk4_ptheta(sys, params, dt, x):
    x = _f64(x)
    d = x.size
    S = np.empty((d, n_params(sys, d)))
    if _load().orc_rk4_ptheta(sys, d, _p(_f64(params)), dt, _p(x), _p(S)) != 0:
        raise ValueError("no parameter derivative for this system")
    return S


def integrate(sys, params, dt, T, x0):
    """O1: the sequential trajectory x_1..x_T as a [T, d] array."""
    x0 = _f64(x0)
    d = x0.size
    traj = np.empty((int(T), d))
    _load().orc_integrate(sys, d, _p(_f64(params)), dt, int(T), _p(x0), _p(traj))
    return traj


def residual(sys, params, dt, x0, traj):
    """h_n = x_n - Phi(x_{n-1}) for n = 1..T as a [T, d] array."""
    x0 = _f64(x0)
    d = x0.size
    traj = _f64(traj).reshape(-1, d)
    h = np.empty_like(traj)
    _load().orc_residual(sys, d, _p(_f64(params)), dt, traj.shape[0], _p(x0),
                         _p(traj), _p(h))
    return h


def affine_seq(F, c, z0=None):
    """z_{n+1} = F_n z_n + c_n; returns z_1..z_N as [N, d]."""
    F = _f64(F)
    N, d, _ = F.shape
    c = _f64(c).reshape(N, d)
    z = np.empty((N, d))
    _load().orc_affine_seq(d, N, _p(F), _p(c), _p(None if z0 is None else _f64(z0)),
                           _p(z))
    return z


def combine(later, earlier):
    """The operator of eq. (assoc-operator): later (x) earlier."""
    Fl, cl = _f64(later[0]), _f64(later[1])
    Fe, ce = _f64(earlier[0]), _f64(earlier[1])
    d = cl.size
    F = np.empty((d, d))
    c = np.empty(d)
    _load().orc_combine(d, _p(Fl), _p(cl), _p(Fe), _p(ce), _p(F), _p(c))
    return F, c


def newton(sys, params, dt, T, x0, guess=None, tol=1e-10, max_iter=None,
           window=0, guard=1e6):
    """O2.  Returns dict(traj, status, iters, final_resid, hist).

    guess: None for the constant guess x_n = x0, or a [T, d] array.
    window: 0 for the paper's plain method, else the window W (safeguarded
    form, also when W >= T).
    """
    x0 = _f64(x0)
    d = x0.size
    T = int(T)
    if guess is None:
        traj = np.tile(x0, (T, 1)) if T > 0 else np.empty((0, d))
    else:
        traj = _f64(guess).reshape(T, d).copy()
    if max_iter is None:
        max_iter = T + 1
    hist = np.full(int(max_iter) + 1, np.nan)
    iters = C.c_int64(0)
    fres = C.c_double(0.0)
    st = _load().orc_newton(sys, d, _p(_f64(params)), dt, T, _p(x0), _p(traj),
                            tol, int(max_iter), int(window), guard, _p(hist),
                            C.byref(iters), C.byref(fres))
    k = iters.value
    return dict(traj=traj, status=st, iters=k, final_resid=fres.value,
                hist=hist[: k + 1].copy())


def integrate_implicit(method, sys, params, dt, T, x0):
    """O1 for an implicit rule (BEULER or TRAP): each step solved by Newton's
    method to rounding; [T, d]."""
    x0 = _f64(x0)
    d = x0.size
    traj = np.empty((int(T), d))
    rc = _load().orc_integrate_implicit(method, sys, d, _p(_f64(params)), dt, int(T),
                                        _p(x0), _p(traj))
    if rc != 0:
        raise ArithmeticError("a step of the implicit integration did not converge")
    return traj


def residual_implicit(method, sys, params, dt, x0, traj, scaled=False):
    """h_n = x_n - x_{n-1} - g_{n-1}(x_{n-1}, x_n), n = 1..T, as [T, d]; with
    scaled, (I - dg_{n-1}/dx_n)^{-1} h_n."""
    x0 = _f64(x0)
    d = x0.size
    traj = _f64(traj).reshape(-1, d)
    h = np.empty_like(traj)
    _load().orc_residual_implicit(method, sys, d, _p(_f64(params)), dt, traj.shape[0],
                                  _p(x0), _p(traj), int(bool(scaled)), _p(h))
    return h


def newton_implicit(method, sys, params, dt, T, x0, guess=None, tol=1e-10,
                    max_iter=None, window=0, guard=1e6):
    """O2 for an implicit rule.  Same arguments and result as newton(); the
    residual in hist / final_resid is the scaled one."""
    x0 = _f64(x0)
    d = x0.size
    T = int(T)
    if guess is None:
        traj = np.tile(x0, (T, 1)) if T > 0 else np.empty((0, d))
    else:
        traj = _f64(guess).reshape(T, d).copy()
    if max_iter is None:
        max_iter = T + 1
    hist = np.full(int(max_iter) + 1, np.nan)
    iters = C.c_int64(0)
    fres = C.c_double(0.0)
    st = _load().orc_newton_implicit(method, sys, d, _p(_f64(params)), dt, T, _p(x0),
                                     _p(traj), tol, int(max_iter), int(window), guard,
                                     _p(hist), C.byref(iters), C.byref(fres))
    k = iters.value
    return dict(traj=traj, status=st, iters=k, final_resid=fres.value,
                hist=hist[: k + 1].copy())


def adjoint(sys, params, dt, x0, traj, g, with_theta=True):
    """O3.  Returns (dL/dx0, dL/dtheta or None)."""
    x0 = _f64(x0)
    d = x0.size
    traj = _f64(traj).reshape(-1, d)
    g = _f64(g).reshape(traj.shape)
    gx0 = np.empty(d)
    gth = np.empty(n_params(sys, d)) if with_theta else None
    rc = _load().orc_adjoint(sys, d, _p(_f64(params)), dt, traj.shape[0], _p(x0),
                             _p(traj), _p(g), _p(gx0), _p(gth))
    if rc != 0:
        raise ValueError("no parameter derivative for this system")
    return gx0, gth


def tangent(sys, params, dt, x0, traj, dx0, dtheta=None):
    x0 = _f64(x0)
    d = x0.size
    traj = _f64(traj).reshape(-1, d)
    v = np.empty_like(traj)
    rc = _load().orc_tangent(sys, d, _p(_f64(params)), dt, traj.shape[0], _p(x0),
                             _p(traj), _p(_f64(dx0)),
                             _p(None if dtheta is None else _f64(dtheta)), _p(v))
    if rc != 0:
        raise ValueError("no parameter derivative for this system")
    return v


def parareal_windows(N):
    """The paper's split of N steps for Parareal (Sec. 4.1): M = floor(sqrt(N))
    windows of S = floor(N / M) fine steps (a reading; it reproduces the
    printed R histories)."""
    import math
    M = math.isqrt(int(N))
    return (M, int(N) // M) if M > 0 else (0, 0)


def parareal(sys, params, dt, M, S, x0, tol=1e-10, max_iter=None, method=RK4):
    """Parareal of Sec. 2.2 with M windows of S fine steps.  Returns
    dict(traj [M*S, d], status, iters (K, fine sweeps), final_resid, hist)."""
    x0 = _f64(x0)
    d = x0.size
    M, S = int(M), int(S)
    if max_iter is None:
        max_iter = M + 1
    traj = np.empty((max(M * S, 0), d))
    hist = np.full(max(int(max_iter), 1), np.nan)
    iters = C.c_int64(0)
    fres = C.c_double(0.0)
    st = _load().orc_parareal(method, sys, d, _p(_f64(params)), dt, M, S, _p(x0), tol,
                              int(max_iter), _p(traj), _p(hist), C.byref(iters),
                              C.byref(fres))
    k = iters.value
    return dict(traj=traj, status=st, iters=k, final_resid=fres.value, hist=hist[:k].copy())


def map_instances(fn, items, threads=None):
    """Run fn over items on a thread pool (ctypes releases the GIL)."""
    threads = threads or min(len(items), os.cpu_count() or 1) or 1
    if threads == 1:
        return [fn(it) for it in items]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))
