"""Parity at the benchmark's full sizes, in the launch configurations that
bench.py times: properties that hold at any size (status, FP64 defect of
every step against the oracle's RK4, the early prefix against the oracle's
sequential trajectory, update counts against the oracle's windowed Newton on
the same workload) and sampled outputs the oracle computes one by one."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("window", [32, 48, 56, 64])
def test_lorenz96_full_horizon(pint, orc, window):
    """Lorenz-96 d=40, T=65536: every window the bench's tuner may pick."""
    w = W.lorenz96(T=65536)
    print(f"[full] lorenz96 T=65536 W={window}", flush=True)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, _t(w.x0), _t(w.params), w.dt, 65536,
                                            tol=w.tol, window=window)
    torch.cuda.synchronize()
    assert int(status[0]) == 0 and float(resid[0]) < w.tol
    tr = traj[0].cpu().numpy()
    h = orc.residual(w.system, w.params[0], w.dt, w.x0[0], tr)
    assert np.abs(h).max() < w.tol                         # FP64 defect, every step
    ref = orc.integrate(w.system, w.params[0], w.dt, 100, w.x0[0])
    assert np.abs(tr[:100] - ref).max() <= 1e-8            # the early prefix (same bar as T=1024)
    r = orc.newton(w.system, w.params[0], w.dt, 65536, w.x0[0], tol=w.tol, window=window,
                   max_iter=4 * 65536)
    assert r["status"] == 0
    assert abs(int(iters[0]) - r["iters"]) <= 0.02 * r["iters"]


def test_vdp_batch_tuned_graph(pint, orc, tmp_path):
    """4096 van der Pol instances, the autotuned launch shape, replayed from
    a HIP graph; sampled instances against the oracle's Newton."""
    from paper_2511_01465_amd import autotune
    w = W.vdp_batch()
    x0, prm = _t(w.x0), _t(w.params)
    print("[full] vdp batch 4096 tune", flush=True)
    cfg = autotune.tune_varlen(pint.VDP, x0, prm, w.dt, w.T, tol=1e-10, reps=1,
                               cache=str(tmp_path / "tune.json"))
    g = pint.SolveGraph(pint.VDP, x0, prm, w.dt, w.T, tol=1e-10, window=cfg["window"],
                        block=cfg["block"], wg_per_cu=cfg["wg_per_cu"], order=cfg["order"])
    for rep in range(2):
        print(f"[full] vdp batch graph launch {rep}", flush=True)
        g.launch()
        torch.cuda.synchronize()
    assert bool((g.status == 0).all()) and float(g.resid.max()) < 1e-10
    T_off = g.T_off.cpu().numpy()
    traj = g.traj.cpu().numpy()
    rng = np.random.default_rng(11)
    # six random instances plus the three longest with mu above 4.5 (the
    # stiffest, longest solves: the most updates)
    stiff = [b for b in np.argsort(-w.T) if w.params[b, 0] > 4.5][:3]
    pick = list(rng.choice(w.B, 6, replace=False)) + [int(b) for b in stiff]
    iters = g.iters.cpu().numpy()

    def run(b):
        return orc.newton(w.system, w.params[b], w.dt, int(w.T[b]), w.x0[b], tol=1e-10,
                          window=cfg["window"], max_iter=4 * int(w.T[b]))

    refs = orc.map_instances(run, pick)
    for b, r in zip(pick, refs):
        tb = traj[T_off[b]:T_off[b + 1]]
        h = orc.residual(w.system, w.params[b], w.dt, w.x0[b], tb)
        assert np.abs(h).max() < 1e-10, b
        assert r["status"] == 0
        dk = abs(int(iters[b]) - r["iters"])
        assert dk == 0 or (dk == 1 and np.min(r["hist"][-3:]) < 100 * 1e-10), \
            (b, int(iters[b]), r["iters"])
        # same iterate: 1e-10 max-abs, or within ||H^-1|| (r1 + r2) when the
        # neutral phase direction carries the two iterates apart
        err = float(np.abs(tb - r["traj"]).max())
        if err > 1e-10:
            from test_gpu_small import hinv_norm
            hn = hinv_norm(orc, w.system, w.params[b], w.dt, w.x0[b], r["traj"])
            bound = hn * (float(g.resid[b]) + r["final_resid"])
            assert err <= bound, (b, err, bound)
        print(f"[full] vdp b={b} T={int(w.T[b])} mu={w.params[b, 0]:.2f} updates "
              f"{int(iters[b])} (oracle {r['iters']}) max|gpu-oracle| {err:.2e}", flush=True)
    g.close()


@pytest.mark.timeout(900)
def test_kuramoto_full(pint, orc):
    """Kuramoto d=128, 8 x 4096, W=256 (the benchmark's launch): every
    instance against the oracle's windowed Newton on the same inputs (all
    eight on the host's cores at once): status and update count equal, the
    FP64 defect of every step below tol, and the iterates the same to 1e-10
    max-abs (the only neutral direction, the global phase, carries rounding
    additively, not exponentially)."""
    w = W.kuramoto()
    print("[full] kuramoto 8 x 4096", flush=True)
    traj, iters, resid, status = pint.solve(pint.KURAMOTO, _t(w.x0), _t(w.params), w.dt, 4096,
                                            tol=1e-10, window=256)
    torch.cuda.synchronize()
    assert bool((status == 0).all())
    tr = traj.cpu().numpy()

    def run(b):
        return orc.newton(w.system, w.params[b], w.dt, 4096, w.x0[b], tol=1e-10, window=256,
                          max_iter=4097)

    print("[full] kuramoto oracle, 8 instances", flush=True)
    refs = orc.map_instances(run, list(range(w.B)))
    for b, ref in enumerate(refs):
        h = orc.residual(w.system, w.params[b], w.dt, w.x0[b], tr[b])
        err = float(np.abs(tr[b] - ref["traj"]).max())
        print(f"[full] kuramoto b={b} updates {int(iters[b])} (oracle {ref['iters']}) "
              f"defect {np.abs(h).max():.2e} max|gpu-oracle| {err:.2e}", flush=True)
        assert ref["status"] == 0 and int(iters[b]) == ref["iters"], b
        assert np.abs(h).max() < 1e-10, b
        assert err <= 1e-10, b


def test_adjoint_full_sampled(pint, orc):
    """Adjoint on Lorenz-96, 256 x 16384: gradients of two sampled instances
    against the oracle's sequential discrete adjoint on the same trajectory."""
    w = W.adjoint_l96()
    print("[full] adjoint 256 x 16384", flush=True)
    x0, prm = _t(w.x0), _t(w.params)
    traj, iters, resid, status = pint.solve(pint.LORENZ96, x0, prm, w.dt, 16384, tol=1e-10, window=32)
    torch.cuda.synchronize()
    assert bool((status == 0).all())
    obs = torch.tensor(w.extra["obs"] - 1, device=DEV)
    y = _t(w.extra["y"])
    g = torch.zeros_like(traj)
    g[:, obs, :] = 2 * (traj[:, obs, :] - y)
    gx0, gth = pint.adjoint(pint.LORENZ96, x0, prm, w.dt, traj, g, seg=2048)
    torch.cuda.synchronize()
    for b in (0, 173):
        rx0, rth = orc.adjoint(w.system, w.params[b], w.dt, w.x0[b], traj[b].cpu().numpy(), g[b].cpu().numpy())
        sx = max(1.0, np.abs(rx0).max())
        assert np.abs(gx0[b].cpu().numpy() - rx0).max() <= 1e-10 * sx, b
        assert abs(float(gth[b, 0]) - rth[0]) <= 1e-10 * max(1.0, abs(rth[0])), b
