"""The fused Lorenz-96 reverse pass (elements built inside the reverse
recursion, never stored) against the two-kernel path (transposed bands
written per segment, then the banded scan) that pint_set_dense_pipeline(0)
selects, and against the oracle's sequential discrete adjoint.  Bars: FP64
1e-12 relative to the gradient's magnitude between the two GPU paths (same
recursion, different summation order), 1e-10 against the oracle; FP32 1e-4
relative to the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


def _both(pint, x0, P, dt, traj, g, seg=0):
    out = {}
    for fused in (True, False):
        pint.pint_set_dense_pipeline(fused)
        try:
            out[fused] = pint.adjoint(pint.LORENZ96, x0, P, dt, traj, g, seg=seg)
            torch.cuda.synchronize()
        finally:
            pint.pint_set_dense_pipeline(True)
    return out[True], out[False]


@pytest.mark.parametrize("B,T", [(1, 1), (2, 2), (3, 25), (2, 24), (5, 700), (300, 64)])
def test_fused_equals_two_kernel_path(pint, orc, B, T):
    """Short horizons around the ring size (24 slots), a horizon of several
    ring turns, and more instances than compute units."""
    rng = np.random.default_rng(B * 1000 + T)
    x0 = 8 + 0.01 * rng.normal(size=(B, 40))
    P = np.full((B, 1), 8.0) + 0.1 * rng.normal(size=(B, 1))
    dt = 0.005
    x0t, Pt = _t(x0), _t(P)
    traj = pint.seq_integrate(pint.LORENZ96, x0t, Pt, dt, T).reshape(B, T, 40)
    g = _t(rng.normal(size=(B, T, 40)))
    print(f"[adj fused] B={B} T={T}", flush=True)
    (fx, fth), (ox, oth) = _both(pint, x0t, Pt, dt, traj, g, seg=37)
    sx = max(1.0, float(ox.abs().max()))
    st = max(1.0, float(oth.abs().max()))
    assert float((fx - ox).abs().max()) <= 1e-12 * sx
    assert float((fth - oth).abs().max()) <= 1e-12 * st
    tr = traj.cpu().numpy()
    gn = g.cpu().numpy()
    for b in sorted({0, B - 1}):
        rx0, rth = orc.adjoint(W.LORENZ96, P[b], dt, x0[b], tr[b], gn[b])
        assert np.abs(fx[b].cpu().numpy() - rx0).max() <= 1e-10 * max(1.0, np.abs(rx0).max())
        assert abs(float(fth[b, 0]) - rth[0]) <= 1e-10 * max(1.0, abs(rth[0]))


def test_fused_fp32(pint, orc):
    rng = np.random.default_rng(21)
    B, T = 3, 300
    x0 = (8 + 0.01 * rng.normal(size=(B, 40))).astype(np.float32)
    P = np.full((B, 1), 8.0, dtype=np.float32)
    trajs = np.stack([orc.integrate(W.LORENZ96, P[b].astype(np.float64), 0.005, T,
                                    x0[b].astype(np.float64)) for b in range(B)]).astype(np.float32)
    g = rng.normal(size=trajs.shape).astype(np.float32)
    gx0, gth = pint.adjoint(W.LORENZ96, _t(x0, torch.float32), _t(P, torch.float32), 0.005,
                            _t(trajs, torch.float32), _t(g, torch.float32))
    torch.cuda.synchronize()
    for b in range(B):
        rx0, rth = orc.adjoint(W.LORENZ96, P[b].astype(np.float64), 0.005, x0[b].astype(np.float64),
                               trajs[b].astype(np.float64), g[b].astype(np.float64))
        assert np.abs(gx0[b].double().cpu().numpy() - rx0).max() <= 1e-4 * np.abs(rx0).max()
        assert abs(float(gth[b, 0]) - rth[0]) <= 1e-4 * abs(rth[0])


def test_fused_workspace_and_empty(pint):
    """The fused pass needs no element storage: the workspace query is small
    and independent of T and seg; T = 0 gives zero gradients."""
    P = pint
    sysd = P.make_system(P.LORENZ96, 40, _t([[8.0]]), False)
    assert P.pint_adjoint_workspace_bytes(sysd, 256, 16384, 2048, P.F64) <= 4096
    P.pint_set_dense_pipeline(False)
    try:
        assert P.pint_adjoint_workspace_bytes(sysd, 256, 16384, 2048, P.F64) > 1 << 30
    finally:
        P.pint_set_dense_pipeline(True)
    x0 = _t(np.full((2, 40), 8.0))
    gx0, gth = P.adjoint(P.LORENZ96, x0, _t([[8.0], [8.0]]), 0.005,
                         torch.empty((2, 0, 40), dtype=torch.float64, device=DEV),
                         torch.empty((2, 0, 40), dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    assert float(gx0.abs().max()) == 0.0 and float(gth.abs().max()) == 0.0
