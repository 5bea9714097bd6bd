"""Autotuner for the batched solver and the dense scan.

The batched small-d solver (pint_solve_varlen) has four knobs that change
its speed but not what it converges to: the Newton window W (how far past
the first unconverged step one update reaches), the workgroup size (steps
per chunk of the in-workgroup scan), the number of persistent workgroups per
compute unit, and the order in which instances leave the work queue.  The
dense scan has one: the tile length.  `tune_varlen` and `tune_scan` time
candidates on the device with HIP events and keep the fastest whose every
instance converged; results are cached in a JSON file keyed by the workload
and the device, so a later call with the same key returns at once.

Search: coordinate descent, one knob at a time from the defaults, in the
order window, block, workgroups per CU, queue order (the window changes the
work by the largest factor, so it goes first).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional, Sequence

import torch

from . import (F64, F32, PintError, _dtype_code, _sys_id, longest_first, pint_affine_scan,
               pint_scan_workspace_bytes, solve_varlen)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pint", "autotune.json")


_BUILD_ID = None


def _build_id() -> str:
    """Digest of the loaded libpint.so: a rebuilt kernel invalidates old picks."""
    global _BUILD_ID
    if _BUILD_ID is None:
        from . import LIB_PATH
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as f:
            for blk in iter(lambda: f.read(1 << 20), b""):
                h.update(blk)
        _BUILD_ID = h.hexdigest()[:16]
    return _BUILD_ID


def _digest(*tensors) -> str:
    """Digest of tensor contents (initial states, parameters, horizons)."""
    h = hashlib.sha256()
    for t in tensors:
        t = torch.as_tensor(t)
        h.update(str((tuple(t.shape), str(t.dtype))).encode())
        h.update(t.detach().cpu().contiguous().numpy().tobytes())
    return h.hexdigest()[:16]


def _cands(values) -> str:
    return ",".join(str(v) for v in values)


def _device_name(device) -> str:
    try:
        return torch.cuda.get_device_name(device)
    except Exception:  # pragma: no cover
        return "unknown"


def _load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path: Optional[str], cache: dict) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(fn, reps: int, stream) -> float:
    fn()  # warm (and the first-call launch set-up)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def varlen_key(system, x0: torch.Tensor, lengths, dt: float, tol: float, guard: float,
               params=None, candidates=()) -> str:
    """Cache key: the workload (sizes, a digest of x0, params and the
    horizons), the candidate lists, the device and the library build."""
    lengths = torch.as_tensor(lengths, dtype=torch.int64)
    B, d = x0.shape
    data = _digest(x0, lengths, *(() if params is None else (params,)))
    cands = "|".join(_cands(c) for c in candidates)
    return "varlen|sys=%d|d=%d|dtype=%d|B=%d|sumT=%d|maxT=%d|dt=%g|tol=%g|guard=%g|data=%s|cand=%s|%s|lib=%s" % (
        _sys_id(system), d, _dtype_code(x0), B, int(lengths.sum()), int(lengths.max()) if B else 0,
        dt, tol, guard, data, cands, _device_name(x0.device), _build_id())


def tune_varlen(system, x0: torch.Tensor, params: torch.Tensor, dt: float, lengths, *,
                tol: float = 1e-10, guard: float = 1e6,
                windows: Sequence[int] = (64, 128, 256, 512),
                blocks: Sequence[int] = (64, 128, 256),
                wg_per_cu: Sequence[int] = (2, 4, 8),
                orders: Sequence[Optional[str]] = (None, "longest_first"),
                reps: int = 2, cache: Optional[str] = DEFAULT_CACHE, force: bool = False,
                stream=None) -> dict:
    """Pick (window, block, wg_per_cu, order) for this batch.  Returns a dict
    with those keys plus "ms" (the winner's time) and "trials" (every
    configuration timed, in order).  Plain mode (window 0) is not a
    candidate: on these workloads it does not converge in practice."""
    key = varlen_key(system, x0, lengths, dt, tol, guard, params,
                     (windows, blocks, wg_per_cu, orders))
    store = _load_cache(cache)
    if not force and key in store:
        return store[key]
    stream = stream if stream is not None else torch.cuda.current_stream()
    cur = {"window": int(windows[0]) if windows else 256, "block": 256, "wg_per_cu": 4, "order": None}
    trials = []

    def run(cfg):
        res = {}

        def fn():
            res["o"] = solve_varlen(system, x0, params, dt, lengths, tol=tol, guard=guard,
                                    window=cfg["window"], block=cfg["block"],
                                    wg_per_cu=cfg["wg_per_cu"], order=cfg["order"], stream=stream)

        ms = _time_ms(fn, reps, stream)
        ok = bool((res["o"][4] == 0).all())
        trials.append(dict(cfg, ms=ms, ok=ok))
        return ms if ok else float("inf")

    best = None
    for knob, values in (("window", windows), ("block", blocks), ("wg_per_cu", wg_per_cu),
                         ("order", orders)):
        scores = {}
        for v in values:
            cfg = dict(cur, **{knob: v})
            scores[v] = run(cfg)
        v_best = min(scores, key=lambda v: scores[v])
        cur[knob] = v_best
        best = scores[v_best]
    if best is None or best == float("inf"):
        raise PintError("autotune: no configuration converged on every instance")
    out = dict(cur, ms=best, trials=trials, key=key)
    store[key] = out
    _store_cache(cache, store)
    return out


def tune_scan(d: int, B: int, N: int, dtype: int = F64, *, tiles: Sequence[int] = (),
              reps: int = 3, cache: Optional[str] = DEFAULT_CACHE, force: bool = False,
              device="cuda:0", stream=None) -> dict:
    """Pick the tile length of the dense-d scan (d in 16..128) for B
    sequences of N elements, timed on random orthogonal-scaled elements
    (the scan's time does not depend on the values).  Small d has its tile
    fixed at compile time: returns {"tile": 0}."""
    if d <= 8:
        return {"tile": 0, "ms": None, "trials": []}
    tdt = torch.float64 if dtype == F64 else torch.float32
    key = "scan|d=%d|B=%d|N=%d|dtype=%d|cand=%s|%s|lib=%s" % (d, B, N, dtype, _cands(tiles),
                                                              _device_name(device), _build_id())
    store = _load_cache(cache)
    if not force and key in store:
        return store[key]
    stream = stream if stream is not None else torch.cuda.current_stream()
    g = torch.Generator(device="cpu").manual_seed(0)
    A = (torch.randn((B, N, d, d), generator=g, dtype=tdt) / d ** 0.5).to(device)
    b = torch.randn((B, N, d), generator=g, dtype=tdt).to(device)
    z = torch.empty((B, N, d), dtype=tdt, device=device)
    if not tiles:
        cus = torch.cuda.get_device_properties(device).multi_processor_count
        per = max(1, -(-cus // max(B, 1)))
        base = max(1, -(-N // per))
        tiles = sorted({max(1, base // 4), max(1, base // 2), base, base * 2})
    trials = []
    for t in tiles:
        ws = torch.empty(pint_scan_workspace_bytes(d, B, N, int(t), dtype), dtype=torch.uint8,
                         device=device)
        ms = _time_ms(lambda: pint_affine_scan(d, B, N, dtype, A, b, None, z, int(t), ws, stream),
                      reps, stream)
        trials.append({"tile": int(t), "ms": ms})
    best = min(trials, key=lambda r: r["ms"])
    out = {"tile": best["tile"], "ms": best["ms"], "trials": trials, "key": key}
    store[key] = out
    _store_cache(cache, store)
    return out


def tune_window(system, x0: torch.Tensor, params: torch.Tensor, dt: float, T: int, *,
                tol: float = 1e-10, guard: float = 1e6, windows: Sequence[int] = (32, 48, 56, 64),
                reps: int = 1, cache: Optional[str] = DEFAULT_CACHE, force: bool = False,
                stream=None) -> dict:
    """Pick the Newton window W of a uniform-horizon solve (pint_solve): the
    fastest candidate whose every instance converged.  A longer window
    costs more per update and needs fewer updates, up to the point where the
    linearisation across it fails and the guard keeps cutting updates."""
    from . import solve
    key = "window|sys=%d|d=%d|dtype=%d|B=%d|T=%d|dt=%g|tol=%g|guard=%g|data=%s|cand=%s|%s|lib=%s" % (
        _sys_id(system), x0.shape[-1], _dtype_code(x0), x0.shape[0] if x0.dim() > 1 else 1, T, dt,
        tol, guard, _digest(x0, params), _cands(windows), _device_name(x0.device), _build_id())
    store = _load_cache(cache)
    if not force and key in store:
        return store[key]
    stream = stream if stream is not None else torch.cuda.current_stream()
    trials = []
    for wv in windows:
        res = {}

        def fn():
            res["o"] = solve(system, x0, params, dt, T, tol=tol, guard=guard, window=int(wv),
                             stream=stream)

        ms = _time_ms(fn, reps, stream)
        st = res["o"][3]
        trials.append({"window": int(wv), "ms": ms, "ok": bool((st == 0).all()),
                       "updates_max": int(res["o"][1].max())})
    ok = [t for t in trials if t["ok"]]
    if not ok:
        raise PintError("autotune: no window converged on every instance")
    best = min(ok, key=lambda t: t["ms"])
    out = {"window": best["window"], "ms": best["ms"], "trials": trials, "key": key}
    store[key] = out
    _store_cache(cache, store)
    return out
