"""GPU parity of the reverse-time adjoint scan (pint_adjoint) against the
oracle's sequential discrete adjoint on the same trajectory (FP64 bar 1e-10
relative to the gradient's magnitude), against central finite differences of
the loss on short horizons (1e-6 relative), and through SolveFn."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _loss_grad(traj, y, obs):
    g = np.zeros_like(traj)
    L = 0.0
    for j, n in enumerate(obs):
        diff = traj[n - 1] - y[j]
        L += float(diff @ diff)
        g[n - 1] += 2 * diff
    return L, g


CASES = [
    ("l63", W.LORENZ63, lambda r, B: (1 + 0.1 * r.normal(size=(B, 3)), np.tile([10.0, 28.0, 8 / 3], (B, 1))), 1e-3, 300),
    ("vdp", W.VDP, lambda r, B: (r.uniform(-2, 2, (B, 2)), r.uniform(0.5, 5, (B, 1))), 0.01, 400),
    ("logistic", W.LOGISTIC, lambda r, B: (r.uniform(0.1, 0.9, (B, 1)), np.tile([1.0, 1.0], (B, 1))), 0.01, 250),
    ("linear3", W.LINEAR, lambda r, B: (r.normal(size=(B, 3)), 0.4 * r.normal(size=(B, 9))), 0.05, 200),
    ("l96", W.LORENZ96, lambda r, B: (8 + 0.01 * r.normal(size=(B, 40)), np.full((B, 1), 8.0)), 0.005, 500),
]


@pytest.mark.parametrize("name,sysid,gen,dt,T", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("seg", [0, 37])
def test_adjoint_matches_sequential_adjoint(pint, orc, name, sysid, gen, dt, T, seg):
    rng = np.random.default_rng(3)
    B = 3
    x0, P = gen(rng, B)
    trajs = np.stack([orc.integrate(sysid, P[b], dt, T, x0[b]) for b in range(B)])
    g = rng.normal(size=trajs.shape)
    gx0, gth = pint.adjoint(sysid, _t(x0), _t(P), dt, _t(trajs), _t(g), seg=seg)
    torch.cuda.synchronize()
    gx0, gth = gx0.cpu().numpy(), gth.cpu().numpy()
    for b in range(B):
        rx0, rth = orc.adjoint(sysid, P[b], dt, x0[b], trajs[b], g[b])
        sx = max(1.0, np.abs(rx0).max())
        st = max(1.0, np.abs(rth).max())
        assert np.abs(gx0[b] - rx0).max() <= 1e-10 * sx, (name, b)
        assert np.abs(gth[b] - rth).max() <= 1e-10 * st, (name, b)


def test_adjoint_kuramoto_dx0(pint, orc):
    w = W.kuramoto(B=2, T=150)
    trajs = np.stack([orc.integrate(w.system, w.params[b], w.dt, 150, w.x0[b]) for b in range(2)])
    g = np.random.default_rng(1).normal(size=trajs.shape)
    gx0, gth = pint.adjoint(w.system, _t(w.x0), _t(w.params), w.dt, _t(trajs), _t(g),
                            with_params=False)
    torch.cuda.synchronize()
    for b in range(2):
        rx0, _ = orc.adjoint(w.system, w.params[b], w.dt, w.x0[b], trajs[b], g[b], with_theta=False)
        assert np.abs(gx0[b].cpu().numpy() - rx0).max() <= 1e-10 * max(1.0, np.abs(rx0).max())


def test_adjoint_finite_differences_lorenz96(pint, orc):
    """Loss over 8 evenly spaced observations, T = 200 (one time unit):
    central differences with h = 1e-6 on x0 components and on F."""
    w = W.adjoint_l96(B=2, T=200, n_obs=8)
    trajs = np.stack([orc.integrate(w.system, w.params[b], w.dt, 200, w.x0[b]) for b in range(w.B)])
    gs = np.stack([_loss_grad(trajs[b], w.extra["y"][b], w.extra["obs"])[1] for b in range(w.B)])
    gx0, gth = pint.adjoint(w.system, _t(w.x0), _t(w.params), w.dt, _t(trajs), _t(gs))
    torch.cuda.synchronize()
    gx0, gth = gx0.cpu().numpy(), gth.cpu().numpy()
    h = 1e-6
    for b in range(w.B):
        def L(x0, P):
            return _loss_grad(orc.integrate(w.system, P, w.dt, 200, x0), w.extra["y"][b], w.extra["obs"])[0]
        for i in (0, 7, 39):
            e = np.zeros(40)
            e[i] = h
            fd = (L(w.x0[b] + e, w.params[b]) - L(w.x0[b] - e, w.params[b])) / (2 * h)
            assert abs(fd - gx0[b, i]) <= 1e-6 * max(1.0, abs(gx0[b, i])), (b, i, fd, gx0[b, i])
        fd = (L(w.x0[b], w.params[b] + h) - L(w.x0[b], w.params[b] - h)) / (2 * h)
        assert abs(fd - gth[b, 0]) <= 1e-6 * max(1.0, abs(gth[b, 0])), (b, fd, gth[b, 0])


def test_adjoint_fp32(pint, orc):
    rng = np.random.default_rng(9)
    x0 = (8 + 0.01 * rng.normal(size=(2, 40))).astype(np.float32)
    P = np.full((2, 1), 8.0, dtype=np.float32)
    T = 150
    trajs = np.stack([orc.integrate(W.LORENZ96, P[b].astype(np.float64), 0.005, T,
                                    x0[b].astype(np.float64)) for b in range(2)]).astype(np.float32)
    g = rng.normal(size=trajs.shape).astype(np.float32)
    gx0, gth = pint.adjoint(W.LORENZ96, _t(x0, torch.float32), _t(P, torch.float32), 0.005,
                            _t(trajs, torch.float32), _t(g, torch.float32))
    torch.cuda.synchronize()
    for b in range(2):
        rx0, rth = orc.adjoint(W.LORENZ96, P[b].astype(np.float64), 0.005, x0[b].astype(np.float64),
                               trajs[b].astype(np.float64), g[b].astype(np.float64))
        assert np.abs(gx0[b].double().cpu().numpy() - rx0).max() <= 1e-4 * np.abs(rx0).max()
        assert abs(float(gth[b, 0]) - rth[0]) <= 1e-4 * abs(rth[0])


def test_solvefn_autograd(pint, orc):
    """Forward: Newton solve on the device; backward: the adjoint scan.  The
    gradient equals the oracle's adjoint on the returned trajectory."""
    w = W.adjoint_l96(B=2, T=256, n_obs=8, window=32)
    x0 = _t(w.x0).requires_grad_(True)
    P = _t(w.params).requires_grad_(True)
    traj, iters, resid, status = pint.SolveFn.apply(x0, P, pint.LORENZ96, w.dt, 256, 1e-12, 32, 0)
    obs = torch.tensor(w.extra["obs"] - 1, device=DEV)
    y = _t(w.extra["y"])
    loss = ((traj[:, obs, :] - y) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.all(status == 0)
    tr = traj.detach().cpu().numpy()
    for b in range(w.B):
        _, g = _loss_grad(tr[b], w.extra["y"][b], w.extra["obs"])
        rx0, rth = orc.adjoint(w.system, w.params[b], w.dt, w.x0[b], tr[b], g)
        assert np.abs(x0.grad[b].cpu().numpy() - rx0).max() <= 1e-10 * max(1.0, np.abs(rx0).max())
        assert abs(float(P.grad[b, 0]) - rth[0]) <= 1e-10 * max(1.0, abs(rth[0]))


def test_solvefn_x0_only_kuramoto(pint, orc):
    """Parameters that need no gradient are not differentiated: Kuramoto,
    whose parameter derivative is not built, gives dL/dx0 through SolveFn,
    equal to the oracle's adjoint on the returned trajectory."""
    w = W.kuramoto(B=2, T=128, window=64)
    x0 = _t(w.x0).requires_grad_(True)
    P = _t(w.params)
    traj, iters, resid, status = pint.SolveFn.apply(x0, P, pint.KURAMOTO, w.dt, 128, 1e-12, 64, 0)
    rng = np.random.default_rng(7)
    gt = rng.normal(size=traj.shape)
    (traj * _t(gt)).sum().backward()
    torch.cuda.synchronize()
    assert P.grad is None and torch.all(status == 0)
    tr = traj.detach().cpu().numpy()
    for b in range(w.B):
        rx0, _ = orc.adjoint(w.system, w.params[b], w.dt, w.x0[b], tr[b], gt[b], with_theta=False)
        assert np.abs(x0.grad[b].cpu().numpy() - rx0).max() <= 1e-10 * max(1.0, np.abs(rx0).max())
