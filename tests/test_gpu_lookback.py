"""The decoupled lookback under forced timing, and what is and is not
repeatable bit for bit.

A tile of the scans composes its carry-in from whichever predecessors had
published when it looked (an inclusive prefix if one was there, else
aggregates applied in order), so two runs of pint_affine_scan on the same
input can differ in the last bits; the Newton solvers exchange compositions
in a fixed order and are repeatable bit for bit.  The delay hook
(pint_set_scan_delay) makes every third tile publish its aggregate late and
every third its inclusive prefix late, so successors wait for unpublished
predecessors and walk back over aggregate-only ones.  Bars: the scan's (FP64
1e-11 relative to the largest |z|, FP32 1e-4) against the oracle's
recursion, the lookback's error word clear, repeated scans within 1e-12 of
each other."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _elements(d, B, N, seed):
    A = np.empty((B, N, d, d))
    b = np.empty((B, N, d))
    for s in range(B):
        A[s], b[s] = W.random_affine(N, d, seed=seed + s, kind="rotation")
    return A, b


def _scan(P, A, b, z0, tile):
    B, N, d, _ = A.shape
    code = P.F64 if A.dtype == torch.float64 else P.F32
    z = torch.empty((B, N, d), dtype=A.dtype, device=DEV)
    ws = torch.zeros(P.pint_scan_workspace_bytes(d, B, N, tile, code), dtype=torch.uint8, device=DEV)
    assert P.pint_affine_scan(d, B, N, code, A, b, z0, z, tile, ws) == P.OK
    return z, ws


# (d, B, N, tile): small-d kernels at their own tile lengths (d <= 3: 1024 to
# 12288 elements per tile, d >= 4: 4096), dense d on MFMA at explicit tiles
CASES = [(2, 1, 70000, 0), (3, 2, 33000, 0), (5, 1, 30000, 0), (8, 1, 20000, 0),
         (40, 2, 1500, 32), (128, 2, 400, 16)]


@pytest.mark.parametrize("d,B,N,tile", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scan_with_injected_delays(pint, orc, d, B, N, tile, dtype):
    """Every third tile late with its aggregate, every third late with its
    inclusive prefix: the result still equals the sequential recursion, with
    and without a starting vector, and no wait gave up."""
    P = pint
    A, b = _elements(d, B, N, seed=700 + d)
    z0 = np.random.default_rng(d).normal(size=(B, d))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    At, bt, z0t = (torch.tensor(v, dtype=tdt, device=DEV) for v in (A, b, z0))
    if dtype == "f32":
        A, b, z0 = (v.astype(np.float32).astype(np.float64) for v in (A, b, z0))
    ref = np.stack([orc.affine_seq(A[s], b[s], z0[s]) for s in range(B)])
    scale = max(1.0, np.abs(ref).max())
    bar = 1e-11 if dtype == "f64" else 1e-4
    print(f"[lookback] d={d} B={B} N={N} tile={tile} {dtype}", flush=True)
    try:
        for delay in (0, 40, 200):
            P.pint_set_scan_delay(delay)
            z, ws = _scan(P, At, bt, z0t, tile)
            torch.cuda.synchronize()
            err_word = int(ws[4:8].view(torch.int32)[0])
            err = np.abs(z.double().cpu().numpy() - ref).max() / scale
            print(f"  delay {delay}: max rel err {err:.2e}, error word {err_word}", flush=True)
            assert err_word == 0
            assert err <= bar, (delay, err)
    finally:
        P.pint_set_scan_delay(0)


def test_scan_repeats_within_rounding(pint):
    """The same scan five times: equal to 1e-12 relative (the carry-in's
    composition order depends on timing, so not necessarily bit for bit)."""
    P = pint
    A, b = _elements(3, 1, 200000, seed=9)
    At, bt = torch.tensor(A, device=DEV), torch.tensor(b, device=DEV)
    outs = [_scan(P, At, bt, None, 0)[0] for _ in range(5)]
    torch.cuda.synchronize()
    scale = max(1.0, float(outs[0].abs().max()))
    distinct = 1 + sum(0 if torch.equal(o, outs[0]) else 1 for o in outs[1:])
    worst = max(float((o - outs[0]).abs().max()) for o in outs[1:]) / scale
    print(f"[lookback] 5 repeats: {distinct} distinct bit patterns, max rel diff {worst:.2e}",
          flush=True)
    assert worst <= 1e-12


def test_newton_solvers_repeat_bit_for_bit(pint):
    """The solvers combine their workgroups' compositions in a fixed order,
    so the same solve gives the same bits: the cooperative dense solver
    (Lorenz-96, Kuramoto), the cooperative small-d solver in plain mode and
    the batched small-d solver over uneven horizons."""
    P = pint
    w = W.lorenz96(T=3000)
    runs = [P.solve(P.LORENZ96, torch.tensor(w.x0, device=DEV), torch.tensor(w.params, device=DEV),
                    w.dt, 3000, tol=1e-10, window=48) for _ in range(3)]
    wk = W.kuramoto(B=2, T=600)
    runs_k = [P.solve(P.KURAMOTO, torch.tensor(wk.x0, device=DEV), torch.tensor(wk.params, device=DEV),
                      wk.dt, 600, tol=1e-10, window=256) for _ in range(2)]
    x0 = torch.tensor([[0.0, 1.0]], dtype=torch.float64, device=DEV)
    prm = torch.tensor([1.0], dtype=torch.float64, device=DEV)
    runs_c = [P.solve(P.VDP, x0, prm, 1e-4, 100000, tol=1e-12, guess=torch.ones((1, 100000, 2),
                      dtype=torch.float64, device=DEV)) for _ in range(2)]
    wv = W.vdp_batch(B=300, t_hi=3000)
    runs_v = [P.solve_varlen(P.VDP, torch.tensor(wv.x0, device=DEV), torch.tensor(wv.params, device=DEV),
                             wv.dt, wv.T, tol=1e-10, window=64) for _ in range(2)]
    torch.cuda.synchronize()
    for group in (runs, runs_k, runs_c):
        for r in group[1:]:
            assert torch.equal(r[0], group[0][0]) and torch.equal(r[1], group[0][1])
    assert torch.equal(runs_v[0][0], runs_v[1][0]) and torch.equal(runs_v[0][2], runs_v[1][2])
    assert int(runs[0][3][0]) == P.OK and bool((runs_k[0][3] == 0).all())
    assert int(runs_c[0][3][0]) == P.OK


def test_adjoint_repeats_within_rounding(pint):
    """One long Lorenz-96 instance: the adjoint's reverse scan runs over many
    tiles, so repeated gradients agree to rounding (1e-12 relative)."""
    P = pint
    w = W.adjoint_l96(B=1, T=4096)
    x0, prm = torch.tensor(w.x0, device=DEV), torch.tensor(w.params, device=DEV)
    traj, _, _, status = P.solve(P.LORENZ96, x0, prm, w.dt, 4096, tol=1e-10, window=48)
    obs = torch.tensor(w.extra["obs"] - 1, device=DEV)
    g = torch.zeros_like(traj)
    g[:, obs, :] = 2 * (traj[:, obs, :] - torch.tensor(w.extra["y"], device=DEV))
    outs = [P.adjoint(P.LORENZ96, x0, prm, w.dt, traj, g) for _ in range(3)]
    torch.cuda.synchronize()
    assert int(status[0]) == P.OK
    for gx, gth in outs[1:]:
        for a, b0 in ((gx, outs[0][0]), (gth, outs[0][1])):
            scale = max(1.0, float(b0.abs().max()))
            assert float((a - b0).abs().max()) <= 1e-12 * scale
