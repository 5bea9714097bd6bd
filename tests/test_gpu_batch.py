"""Batched launch (uneven horizons, one persistent launch): the launch shape
(workgroup size, workgroups per compute unit) and the queue order do not
change any result (every instance is solved by one workgroup, the same
arithmetic in the same order), the HIP-graph replay equals the eager call on
every replay, and the autotuner returns a configuration under which every
instance converges, from its cache the second time."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch(B=96, seed=7):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-2, 2, (B, 2))
    mu = rng.uniform(0.5, 5.0, (B, 1))
    lengths = rng.integers(50, 601, B)
    return (torch.tensor(x0, device=DEV), torch.tensor(mu, device=DEV), lengths)


def _same(a, b):
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_launch_shape_and_order_do_not_change_results(pint):
    x0, mu, lengths = _batch()
    ref = pint.solve_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, window=64)
    torch.cuda.synchronize()
    assert bool((ref[4] == 0).all())
    perm = torch.randperm(len(lengths), generator=torch.Generator().manual_seed(1)).to(DEV)
    for kw in ({"block": 64}, {"block": 128, "wg_per_cu": 1}, {"wg_per_cu": 8},
               {"order": "longest_first"}, {"order": perm, "block": 64, "wg_per_cu": 16}):
        print(f"[batch] {kw if 'order' not in kw or isinstance(kw['order'], str) else 'perm'}", flush=True)
        got = pint.solve_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, window=64, **kw)
        torch.cuda.synchronize()
        _same(ref, got)


def test_order_entries_out_of_range_are_skipped(pint):
    x0, mu, lengths = _batch(B=8)
    B = len(lengths)
    order = torch.arange(B, dtype=torch.int64, device=DEV)
    order[3] = B + 5   # instance 3 is never taken
    T_off_h = torch.zeros(B + 1, dtype=torch.int64)
    T_off_h[1:] = torch.cumsum(torch.as_tensor(lengths), 0)
    traj = torch.empty((int(T_off_h[-1]), 2), dtype=torch.float64, device=DEV)
    iters = torch.full((B,), -7, dtype=torch.int64, device=DEV)
    resid = torch.empty(B, dtype=torch.float64, device=DEV)
    status = torch.full((B,), -7, dtype=torch.int32, device=DEV)
    sysd = pint.make_system(pint.VDP, 2, mu, False)
    opts = pint.make_options(pint.F64, tol=1e-10, window=64, order=order)
    ws = torch.empty(pint.pint_workspace_bytes(sysd, B, int(T_off_h[-1]), int(max(lengths)), opts),
                     dtype=torch.uint8, device=DEV)
    rc = pint.pint_solve_varlen(sysd, B, x0, 0.01, T_off_h.to(DEV), int(max(lengths)), opts, traj,
                                iters, resid, status, ws)
    torch.cuda.synchronize()
    assert rc == pint.OK
    assert int(status[3]) == -7 and int(iters[3]) == -7
    assert all(int(status[b]) == 0 for b in range(B) if b != 3)


def test_graph_replay_equals_eager(pint):
    x0, mu, lengths = _batch()
    eager = pint.solve_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, window=64,
                              order="longest_first")
    torch.cuda.synchronize()
    g = pint.SolveGraph(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, window=64,
                        order="longest_first", block=128)
    junk = torch.zeros(1 << 20, device=DEV)
    for rep in range(3):
        print(f"[batch] graph replay {rep}", flush=True)
        g.traj.fill_(float("nan"))
        g.status.fill_(-1)
        g.launch()
        torch.cuda.synchronize()
        _same((g.traj, g.iters, g.resid, g.status), (eager[0], eager[2], eager[3], eager[4]))
        junk.add_(1.0)   # eager work between replays
        torch.cuda.synchronize()
    # new initial states written in place, then one more replay
    x1 = x0.flip(0).contiguous()
    g.x0.copy_(x1)
    g.launch()
    torch.cuda.synchronize()
    eager1 = pint.solve_varlen(pint.VDP, x1, mu, 0.01, lengths, tol=1e-10, window=64)
    torch.cuda.synchronize()
    _same((g.traj, g.iters, g.resid, g.status), (eager1[0], eager1[2], eager1[3], eager1[4]))
    g.close()


def test_graph_dense_is_unsupported(pint):
    x0 = torch.full((2, 40), 8.0, dtype=torch.float64, device=DEV)
    with pytest.raises(pint.PintError):
        pint.SolveGraph(pint.LORENZ96, x0, torch.tensor([8.0], dtype=torch.float64, device=DEV),
                        0.005, [16, 16], window=8)


def test_autotune_varlen(pint, tmp_path):
    from paper_2511_01465_amd import autotune
    x0, mu, lengths = _batch(B=128, seed=3)
    cache = str(tmp_path / "tune.json")
    cfg = autotune.tune_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, windows=(32, 128),
                               blocks=(64, 256), wg_per_cu=(2, 4), reps=1, cache=cache)
    assert cfg["window"] in (32, 128) and cfg["block"] in (64, 256) and cfg["wg_per_cu"] in (2, 4)
    assert cfg["order"] in (None, "longest_first")
    assert all(t["ok"] for t in cfg["trials"] if t["window"] == cfg["window"])
    again = autotune.tune_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, windows=(32, 128),
                                 blocks=(64, 256), wg_per_cu=(2, 4), reps=1, cache=cache)
    assert again == cfg
    out = pint.solve_varlen(pint.VDP, x0, mu, 0.01, lengths, tol=1e-10, window=cfg["window"],
                            block=cfg["block"], wg_per_cu=cfg["wg_per_cu"], order=cfg["order"])
    torch.cuda.synchronize()
    assert bool((out[4] == 0).all())


def test_autotune_scan(pint, tmp_path):
    from paper_2511_01465_amd import autotune
    cfg = autotune.tune_scan(40, 2, 300, pint.F64, tiles=(16, 64), reps=1,
                             cache=str(tmp_path / "tune.json"))
    assert cfg["tile"] in (16, 64) and len(cfg["trials"]) == 2
    assert autotune.tune_scan(3, 1, 100)["tile"] == 0
