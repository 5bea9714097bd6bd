"""Seeded synthetic inputs for the solver's workloads.

This module holds no arithmetic of the method: it only draws initial states,
parameters, horizons and loss targets with numpy's PCG64, so that the test
suite, the benchmark and the oracle checks all see the same arrays.  Each
workload is a closed-form ODE; no dataset is involved.

System identifiers follow the public C interface numbering.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LINEAR, LOGISTIC, VDP, CARTPOLE, LORENZ63, LORENZ96, KURAMOTO, ROBERTSON = range(8)
# One-step rules (public numbering).
RK4, BACKWARD_EULER, TRAPEZOIDAL = range(3)


@dataclass
class Workload:
    name: str
    system: int
    d: int
    dt: float
    x0: np.ndarray            # [B, d]
    params: np.ndarray        # [B, n_params]
    T: np.ndarray             # [B] steps per instance
    tol: float = 1e-10
    window: int = 0           # 0 = the paper's plain method
    extra: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return int(self.x0.shape[0])

    @property
    def uniform(self) -> bool:
        return bool(np.all(self.T == self.T[0]))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lorenz63(T: int = 2048, seed: int = 1, window: int = 128) -> Workload:
    """sigma=10, rho=28, beta=8/3, dt=1e-3, x0 = (1,1,1) + N(0, 0.1^2)."""
    r = _rng(seed)
    x0 = 1.0 + r.normal(0.0, 0.1, size=(1, 3))
    params = np.array([[10.0, 28.0, 8.0 / 3.0]])
    return Workload("lorenz63", LORENZ63, 3, 1e-3, x0, params,
                    np.array([T], dtype=np.int64), window=window)


def lorenz96(T: int = 65536, d: int = 40, B: int = 1, seed: int = 2,
             window: int = 64, F: float = 8.0) -> Workload:
    """Forcing F=8, dt=0.005, x0 = F + N(0, 0.01^2) per instance."""
    r = _rng(seed)
    x0 = F + r.normal(0.0, 0.01, size=(B, d))
    params = np.full((B, 1), F)
    return Workload("lorenz96", LORENZ96, d, 0.005, x0, params,
                    np.full(B, T, dtype=np.int64), window=window)


def vdp_batch(B: int = 4096, seed: int = 3, t_lo: int = 256, t_hi: int = 8192,
              window: int = 256) -> Workload:
    """mu ~ U[0.5, 5], x0 ~ U[-2, 2]^2, T ~ U{t_lo..t_hi} inclusive, dt=0.01."""
    r = _rng(seed)
    mu = r.uniform(0.5, 5.0, size=B)
    x0 = r.uniform(-2.0, 2.0, size=(B, 2))
    T = r.integers(t_lo, t_hi, size=B, endpoint=True).astype(np.int64)
    return Workload("vdp_batch", VDP, 2, 0.01, x0, mu.reshape(B, 1), T,
                    window=window)


def adjoint_l96(B: int = 256, T: int = 16384, d: int = 40, seed: int = 4,
                n_obs: int = 64, window: int = 64, F: float = 8.0) -> Workload:
    """Lorenz-96 batch for the adjoint: x0 = F + N(0, 0.01^2); targets
    y_j ~ N(0, I) at observation steps n_j = j*T/n_obs, j = 1..n_obs."""
    r = _rng(seed)
    x0 = F + r.normal(0.0, 0.01, size=(B, d))
    y = r.normal(0.0, 1.0, size=(B, n_obs, d))
    obs = (np.arange(1, n_obs + 1, dtype=np.int64) * T) // n_obs
    params = np.full((B, 1), F)
    return Workload("adjoint_l96", LORENZ96, d, 0.005, x0, params,
                    np.full(B, T, dtype=np.int64), window=window,
                    extra=dict(y=y, obs=obs))


def kuramoto(B: int = 8, d: int = 128, T: int = 4096, seed: int = 5,
             window: int = 256) -> Workload:
    """K = 2/d, omega ~ N(0,1)^d, theta0 ~ U[0, 2 pi)^d, dt=0.01; each
    instance draws its own omega and theta0 (omega first)."""
    r = _rng(seed)
    params = np.empty((B, d + 1))
    x0 = np.empty((B, d))
    for b in range(B):
        params[b, 0] = 2.0 / d
        params[b, 1:] = r.normal(0.0, 1.0, size=d)
        x0[b] = r.uniform(0.0, 2.0 * math.pi, size=d)
    return Workload("kuramoto", KURAMOTO, d, 0.01, x0, params,
                    np.full(B, T, dtype=np.int64), window=window)


def random_affine(N: int, d: int, seed: int = 0, kind: str = "rotation"):
    """Affine elements (A_n, b_n) for scan tests.

    kind="rotation": A_n a product of d-1 Givens rotations with U[0, 2 pi)
    angles (orthogonal, so long products stay bounded); b_n ~ N(0, 1).
    kind="gauss": A_n ~ N(0, 1/d) entries (products may grow or shrink).
    """
    r = _rng(seed)
    A = np.zeros((N, d, d))
    if kind == "rotation":
        A[:] = np.eye(d)
        for k in range(d - 1):
            th = r.uniform(0.0, 2.0 * math.pi, size=N)
            c, s = np.cos(th), np.sin(th)
            # left-multiply by the rotation in the (k, k+1) plane
            rk = A[:, k, :].copy()
            rk1 = A[:, k + 1, :].copy()
            A[:, k, :] = c[:, None] * rk - s[:, None] * rk1
            A[:, k + 1, :] = s[:, None] * rk + c[:, None] * rk1
    else:
        A = r.normal(0.0, 1.0 / math.sqrt(d), size=(N, d, d))
    b = r.normal(0.0, 1.0, size=(N, d))
    return A, b


def random_band_affine(N: int, d: int, bw: int, boff: int, seed: int = 0):
    """Cyclically banded orthogonal elements for the banded scan: A_n is the
    product of four layers of cyclic nearest-neighbour Givens rotations
    (pairs (0,1),(2,3),.. then (1,2),..,(d-1,0), twice; d even), so its
    nonzeros lie within offsets [-4, 4] of the diagonal, inside the band
    j - i in [-boff, bw - 1 - boff] (mod d) when boff >= 4 and
    bw - 1 - boff >= 4.  Returns (A [N,d,d] dense, band [N,d,bw] with
    A(i, (i + k - boff) mod d) = band[i, k], b [N,d])."""
    assert d % 2 == 0 and boff >= 4 and bw - 1 - boff >= 4
    r = _rng(seed)
    A = np.zeros((N, d, d))
    A[:] = np.eye(d)
    for layer in range(4):
        for p in range(layer % 2, d, 2):
            q = (p + 1) % d
            th = r.uniform(0.0, 2.0 * math.pi, size=N)
            c, s = np.cos(th), np.sin(th)
            rp, rq = A[:, p, :].copy(), A[:, q, :].copy()
            A[:, p, :] = c[:, None] * rp - s[:, None] * rq
            A[:, q, :] = s[:, None] * rp + c[:, None] * rq
    idx = (np.arange(d)[:, None] + np.arange(bw)[None, :] - boff) % d   # [d, bw] columns
    band = np.take_along_axis(A, np.broadcast_to(idx, (N, d, bw)), axis=2)
    b = r.normal(0.0, 1.0, size=(N, d))
    return A, band, b


def implicit_pins():
    """The two implicit problems of the paper's Sec. 4.2 (backward Euler,
    zero initial guess): Dahlquist (lambda = -1 on [0, 4]) and Robertson
    (k = (0.04, 3e7, 1e4) on [0, 500]); T = horizon / dt."""
    return [
        dict(name="dahlquist", system=LINEAR, params=[-1.0], x0=[1.0], horizon=4.0,
             dts=[1e-1, 1e-2, 1e-3, 1e-4]),
        dict(name="robertson", system=ROBERTSON, params=[0.04, 3e7, 1e4], x0=[1.0, 0.0, 0.0],
             horizon=500.0, dts=[1e-1, 1e-2, 5e-3]),
    ]


def robertson_batch(B: int = 1024, seed: int = 6, t_lo: int = 1000, t_hi: int = 5000,
                    window: int = 0) -> Workload:
    """Robertson instances around the paper's rates: k1, k2, k3 each times
    a log-uniform factor in [1/2, 2]; x0 = (1 - s, s, 0) with s ~ U[0, 1e-5];
    T ~ U{t_lo..t_hi} inclusive; dt = 0.1 (backward Euler)."""
    r = _rng(seed)
    base = np.array([0.04, 3e7, 1e4])
    params = base * np.exp(r.uniform(-math.log(2.0), math.log(2.0), size=(B, 3)))
    s = r.uniform(0.0, 1e-5, size=B)
    x0 = np.stack([1.0 - s, s, np.zeros(B)], axis=1)
    T = r.integers(t_lo, t_hi, size=B, endpoint=True).astype(np.int64)
    return Workload("robertson_batch", ROBERTSON, 3, 0.1, x0, params, T, window=window)


def paper_pins():
    """The three explicit problems of the paper's Sec. 4.1 at dt = 1e-2 with
    the paper's initial guesses (ones, ones, zeros)."""
    return [
        dict(name="logistic", system=LOGISTIC, params=[1.0, 1.0], x0=[0.1],
             dt=1e-2, T=1000, guess=1.0),
        dict(name="vdp", system=VDP, params=[1.0], x0=[0.0, 1.0], dt=1e-2,
             T=1000, guess=1.0),
        dict(name="cartpole", system=CARTPOLE, params=[9.81, 0.5, 10.0, 1.0],
             x0=[0.0, math.pi / 2, 0.0, 0.0], dt=1e-2, T=400, guess=0.0),
    ]
