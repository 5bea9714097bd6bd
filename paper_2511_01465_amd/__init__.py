"""Python binding of libpint, the parallel-in-time Newton ODE solver for
AMD MI355X (Iacob, Razavi, Sarkka, arXiv 2511.01465).

This module only marshals arguments: torch tensors provide device memory and
the current HIP stream, and every step of the computation runs in the HIP
kernels of ``libpint.so``.  There is no CPU fallback: if the library is not
built, ``load()`` raises.

The functions named ``pint_*`` mirror the C entry points of ``include/pint.h``
one to one (same names, same argument order, torch tensors for device
pointers).  ``solve``, ``solve_varlen``, ``seq_integrate``, ``affine_scan``,
``adjoint`` and ``SolveFn`` are conveniences that allocate outputs and the
workspace with torch and call them.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpint.so")

# pint_system_id
LINEAR, LOGISTIC, VDP, CARTPOLE, LORENZ63, LORENZ96, KURAMOTO, ROBERTSON = range(8)
SYSTEM_NAMES = {"linear": LINEAR, "logistic": LOGISTIC, "vdp": VDP, "cartpole": CARTPOLE,
                "lorenz63": LORENZ63, "lorenz96": LORENZ96, "kuramoto": KURAMOTO,
                "robertson": ROBERTSON}
# pint_method: the one-step rule
RK4, BACKWARD_EULER, TRAPEZOIDAL = range(3)
METHOD_NAMES = {"rk4": RK4, "backward_euler": BACKWARD_EULER, "trapezoidal": TRAPEZOIDAL}
# pint_status
OK, ERR_INVALID_ARG, ERR_DEVICE, ERR_WORKSPACE, NOT_CONVERGED, NONFINITE, ERR_UNSUPPORTED = range(7)
F64, F32 = 0, 1


class PintError(RuntimeError):
    pass


class pint_system(C.Structure):
    _fields_ = [("system", C.c_int32), ("d", C.c_int32), ("n_params", C.c_int32),
                ("params_shared", C.c_int32), ("params", C.c_void_p), ("method", C.c_int32),
                ("reserved", C.c_int32)]


class pint_options(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("guess", C.c_int32), ("max_iter", C.c_int64),
                ("window", C.c_int64), ("tol", C.c_double), ("guard", C.c_double),
                ("tile", C.c_int32), ("flags", C.c_int32), ("block", C.c_int32),
                ("wg_per_cu", C.c_int32), ("order", C.c_void_p)]


_lib = None

EXPORTS = ["pint_n_params", "pint_status_string", "pint_supported", "pint_workspace_bytes",
           "pint_solve_varlen", "pint_solve", "pint_seq_integrate", "pint_residual",
           "pint_elements", "pint_scan_workspace_bytes", "pint_affine_scan",
           "pint_scan_band_workspace_bytes", "pint_affine_scan_band",
           "pint_adjoint_workspace_bytes", "pint_adjoint", "pint_graph_capture_varlen",
           "pint_graph_launch", "pint_graph_destroy", "pint_set_wait_limit",
           "pint_parareal_workspace_bytes", "pint_parareal", "pint_affine_scan_noalloc",
           "pint_set_scan_delay", "pint_set_dense_pipeline"]

# include/pint.h: PINT_WAIT_LIMIT_DEFAULT
WAIT_LIMIT_DEFAULT = 268435456


def load(path: str = LIB_PATH):
    """Load libpint.so and declare its C signatures.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PintError(f"libpint.so is not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    SP, OP = C.POINTER(pint_system), C.POINTER(pint_options)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "pint_n_params": (C.c_int, [i32, i32]),
        "pint_status_string": (C.c_char_p, [i32]),
        "pint_supported": (C.c_int, [i32, i32, i32]),
        "pint_workspace_bytes": (sz, [SP, i64, i64, i64, OP]),
        "pint_solve_varlen": (C.c_int, [SP, i64, vp, dbl, vp, i64, OP, vp, vp, vp, vp, vp, sz, vp]),
        "pint_solve": (C.c_int, [SP, i64, vp, dbl, i64, OP, vp, vp, vp, vp, vp, sz, vp]),
        "pint_seq_integrate": (C.c_int, [SP, i64, vp, dbl, vp, i64, i32, vp, vp]),
        "pint_residual": (C.c_int, [SP, i64, vp, dbl, i64, i32, vp, vp, vp, vp]),
        "pint_elements": (C.c_int, [SP, i64, vp, dbl, i64, i32, vp, vp, vp, vp]),
        "pint_scan_workspace_bytes": (sz, [i32, i64, i64, i32, i32]),
        "pint_affine_scan": (C.c_int, [i32, i64, i64, i32, vp, vp, vp, vp, i32, vp, sz, vp]),
        "pint_scan_band_workspace_bytes": (sz, [i32, i32, i32, i64, i64, i32, i32]),
        "pint_affine_scan_band": (C.c_int, [i32, i32, i32, i64, i64, i32, vp, vp, vp, vp, i32, vp,
                                            sz, vp]),
        "pint_adjoint_workspace_bytes": (sz, [SP, i64, i64, i64, i32]),
        "pint_adjoint": (C.c_int, [SP, i64, vp, dbl, i64, i32, vp, vp, vp, vp, i64, vp, sz, vp]),
        "pint_graph_capture_varlen": (C.c_int, [SP, i64, vp, dbl, vp, i64, OP, vp, vp, vp, vp, vp, sz,
                                                C.POINTER(C.c_void_p)]),
        "pint_graph_launch": (C.c_int, [vp, vp]),
        "pint_graph_destroy": (C.c_int, [vp]),
        "pint_set_wait_limit": (None, [C.c_uint64]),
        "pint_set_scan_delay": (None, [C.c_uint32]),
        "pint_set_dense_pipeline": (None, [C.c_int]),
        "pint_parareal_workspace_bytes": (sz, [SP, i64, i64, i32]),
        "pint_affine_scan_noalloc": (C.c_int, [i32, i64, i64, i32, vp, vp, vp, vp, i32, vp, vp]),
        "pint_parareal": (C.c_int, [SP, i64, vp, dbl, i64, i64, OP, vp, vp, vp, vp, vp, vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ------------------------------------------------------------ marshalling --

def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise PintError("expected a device tensor")
    if not t.is_contiguous():
        raise PintError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise PintError(f"unsupported dtype {t.dtype}")


def _check(rc: int, what: str):
    if rc != OK:
        msg = load().pint_status_string(rc).decode()
        raise PintError(f"{what}: {msg} (status {rc})")


def status_string(rc: int) -> str:
    return load().pint_status_string(rc).decode()


def n_params(system: int, d: int) -> int:
    return load().pint_n_params(system, d)


def supported(system: int, d: int, dtype: int = F64) -> bool:
    return bool(load().pint_supported(system, d, dtype))


def make_system(system: int, d: int, params: torch.Tensor, shared: bool,
                method: int = RK4) -> pint_system:
    return pint_system(system, d, n_params(system, d), 1 if shared else 0, _ptr(params),
                       _method_id(method), 0)


def make_options(dtype: int, tol: float = 1e-10, window: int = 0, max_iter: int = 0,
                 guess: int = 0, guard: float = 1e6, tile: int = 0, block: int = 0,
                 wg_per_cu: int = 0, order: Optional[torch.Tensor] = None) -> pint_options:
    """`order` (device int64 [B]) must stay alive while the options are used."""
    return pint_options(dtype, guess, int(max_iter), int(window), float(tol), float(guard),
                        int(tile), 0, int(block), int(wg_per_cu), _ptr(order))


def _sys_id(system) -> int:
    return SYSTEM_NAMES[system] if isinstance(system, str) else int(system)


def _method_id(method) -> int:
    return METHOD_NAMES[method] if isinstance(method, str) else int(method)


def _params_2d(params: torch.Tensor, B: int, np_: int):
    if params.dim() == 1:
        if params.numel() != np_:
            raise PintError("params has the wrong size")
        return params.contiguous(), True
    if params.shape != (B, np_):
        raise PintError("params must be [n_params] or [B, n_params]")
    return params.contiguous(), False


# --------------------------------------------- C entry points, one to one --

def pint_workspace_bytes(sysd, B, T_total, T_max, opts) -> int:
    return load().pint_workspace_bytes(C.byref(sysd), B, T_total, T_max, C.byref(opts))


def pint_solve(sysd, B, x0, dt, T, opts, traj, iters, resid, status, ws, stream=None) -> int:
    return load().pint_solve(C.byref(sysd), B, _ptr(x0), dt, T, C.byref(opts), _ptr(traj),
                             _ptr(iters), _ptr(resid), _ptr(status), _ptr(ws),
                             0 if ws is None else ws.numel(), _stream(stream))


def pint_solve_varlen(sysd, B, x0, dt, T_off, T_max, opts, traj, iters, resid, status, ws,
                      stream=None) -> int:
    return load().pint_solve_varlen(C.byref(sysd), B, _ptr(x0), dt, _ptr(T_off), T_max,
                                    C.byref(opts), _ptr(traj), _ptr(iters), _ptr(resid),
                                    _ptr(status), _ptr(ws), 0 if ws is None else ws.numel(),
                                    _stream(stream))


def pint_seq_integrate(sysd, B, x0, dt, T_off, T_max, dtype, traj, stream=None) -> int:
    return load().pint_seq_integrate(C.byref(sysd), B, _ptr(x0), dt, _ptr(T_off), T_max, dtype,
                                     _ptr(traj), _stream(stream))


def pint_residual(sysd, B, x0, dt, T, dtype, traj, h, hmax, stream=None) -> int:
    return load().pint_residual(C.byref(sysd), B, _ptr(x0), dt, T, dtype, _ptr(traj), _ptr(h),
                                _ptr(hmax), _stream(stream))


def pint_elements(sysd, B, x0, dt, T, dtype, traj, A, b, stream=None) -> int:
    return load().pint_elements(C.byref(sysd), B, _ptr(x0), dt, T, dtype, _ptr(traj), _ptr(A),
                                _ptr(b), _stream(stream))


def pint_scan_workspace_bytes(d, B, N, tile, dtype) -> int:
    return load().pint_scan_workspace_bytes(d, B, N, tile, dtype)


def pint_affine_scan(d, B, N, dtype, A, b, z0, z, tile, ws, stream=None) -> int:
    return load().pint_affine_scan(d, B, N, dtype, _ptr(A), _ptr(b), _ptr(z0), _ptr(z), tile,
                                   _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream))


def pint_affine_scan_noalloc(d, B, N, dtype, A, b, z0, z, tile, err=None, stream=None) -> int:
    return load().pint_affine_scan_noalloc(d, B, N, dtype, _ptr(A), _ptr(b), _ptr(z0), _ptr(z),
                                           tile, _ptr(err), _stream(stream))


# include/pint.h: PINT_NOALLOC_SCRATCH_BYTES
NOALLOC_SCRATCH_BYTES = 16 << 20


def pint_scan_band_workspace_bytes(d, bw, boff, B, N, tile, dtype) -> int:
    return load().pint_scan_band_workspace_bytes(d, bw, boff, B, N, tile, dtype)


def pint_affine_scan_band(d, bw, boff, B, N, dtype, band, b, z0, z, tile, ws, stream=None) -> int:
    return load().pint_affine_scan_band(d, bw, boff, B, N, dtype, _ptr(band), _ptr(b), _ptr(z0),
                                        _ptr(z), tile, _ptr(ws), 0 if ws is None else ws.numel(),
                                        _stream(stream))


def pint_adjoint_workspace_bytes(sysd, B, T, seg, dtype) -> int:
    return load().pint_adjoint_workspace_bytes(C.byref(sysd), B, T, seg, dtype)


def pint_adjoint(sysd, B, x0, dt, T, dtype, traj, g, dL_dx0, dL_dtheta, seg, ws,
                 stream=None) -> int:
    return load().pint_adjoint(C.byref(sysd), B, _ptr(x0), dt, T, dtype, _ptr(traj), _ptr(g),
                               _ptr(dL_dx0), _ptr(dL_dtheta), seg, _ptr(ws),
                               0 if ws is None else ws.numel(), _stream(stream))


def pint_graph_capture_varlen(sysd, B, x0, dt, T_off, T_max, opts, traj, iters, resid, status,
                              ws):
    """Returns (status, handle); handle is None unless status is OK."""
    h = C.c_void_p()
    rc = load().pint_graph_capture_varlen(C.byref(sysd), B, _ptr(x0), dt, _ptr(T_off), T_max,
                                          C.byref(opts), _ptr(traj), _ptr(iters), _ptr(resid),
                                          _ptr(status), _ptr(ws), 0 if ws is None else ws.numel(),
                                          C.byref(h))
    return rc, (h.value if rc == OK else None)


def pint_graph_launch(handle, stream=None) -> int:
    return load().pint_graph_launch(handle, _stream(stream))


def pint_graph_destroy(handle) -> int:
    return load().pint_graph_destroy(handle)


def pint_set_wait_limit(polls: int) -> None:
    load().pint_set_wait_limit(int(polls))


def pint_set_scan_delay(sleeps: int) -> None:
    load().pint_set_scan_delay(int(sleeps))


def pint_set_dense_pipeline(on: bool) -> None:
    load().pint_set_dense_pipeline(1 if on else 0)


def pint_parareal_workspace_bytes(sysd, B, M, dtype) -> int:
    return load().pint_parareal_workspace_bytes(C.byref(sysd), B, M, dtype)


def pint_parareal(sysd, B, x0, dt, M, S, opts, traj, iters, resid, status, hist, ws,
                  stream=None) -> int:
    return load().pint_parareal(C.byref(sysd), B, _ptr(x0), dt, M, S, C.byref(opts), _ptr(traj),
                                _ptr(iters), _ptr(resid), _ptr(status), _ptr(hist), _ptr(ws),
                                0 if ws is None else ws.numel(), _stream(stream))


# ---------------------------------------------------------- conveniences --

def _workspace(nbytes: int, device) -> Optional[torch.Tensor]:
    if nbytes <= 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def solve(system, x0: torch.Tensor, params: torch.Tensor, dt: float, T: int, *,
          tol: float = 1e-10, window: int = 0, max_iter: int = 0, guess: Optional[torch.Tensor] = None,
          guard: float = 1e6, tile: int = 0, method=RK4, stream=None):
    """Newton solve of a uniform batch.  x0 [B, d] (or [d]); params [n_params]
    (shared) or [B, n_params]; method: "rk4", "backward_euler",
    "trapezoidal" (or the pint_method code).  Returns (traj [B, T, d],
    iters [B] int64, resid [B] float64, status [B] int32), all on x0's
    device."""
    sid = _sys_id(system)
    single = x0.dim() == 1
    x0 = (x0[None] if single else x0).contiguous()
    B, d = x0.shape
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    dt_code = _dtype_code(x0)
    if guess is not None:
        traj = guess.reshape(B, T, d).to(x0.dtype).clone().contiguous()
    else:
        traj = torch.empty((B, T, d), dtype=x0.dtype, device=x0.device)
    iters = torch.empty(B, dtype=torch.int64, device=x0.device)
    resid = torch.empty(B, dtype=torch.float64, device=x0.device)
    status = torch.empty(B, dtype=torch.int32, device=x0.device)
    sysd = make_system(sid, d, prm, shared, method)
    opts = make_options(dt_code, tol, window, max_iter, 1 if guess is not None else 0, guard, tile)
    ws = _workspace(pint_workspace_bytes(sysd, B, B * T, T, opts), x0.device)
    _check(pint_solve(sysd, B, x0, float(dt), int(T), opts, traj, iters, resid, status, ws, stream),
           "pint_solve")
    if single:
        return traj[0], iters[0], resid[0], status[0]
    return traj, iters, resid, status


def parareal_windows(N: int):
    """The paper's split of N steps (Sec. 4.1): M = floor(sqrt(N)) windows
    of S = floor(N / M) fine steps."""
    import math
    M = math.isqrt(int(N))
    return (M, int(N) // M) if M > 0 else (0, 0)


def parareal(system, x0: torch.Tensor, params: torch.Tensor, dt: float, M: int, S: int, *,
             tol: float = 1e-10, max_iter: int = 0, method=RK4, with_hist: bool = False,
             stream=None):
    """Parareal of a uniform batch (pint_parareal).  x0 [B, d] (or [d]);
    params [n_params] or [B, n_params].  Returns (traj [B, M*S, d], iters
    [B] int64 (fine sweeps K), resid [B] float64 (last R), status [B] int32)
    and, with with_hist, hist [B, max_iter] float64 (NaN past K)."""
    sid = _sys_id(system)
    single = x0.dim() == 1
    x0 = (x0[None] if single else x0).contiguous()
    B, d = x0.shape
    M, S = int(M), int(S)
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    dt_code = _dtype_code(x0)
    dev = x0.device
    traj = torch.empty((B, M * S, d), dtype=x0.dtype, device=dev)
    iters = torch.empty(B, dtype=torch.int64, device=dev)
    resid = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    kmax = int(max_iter) if max_iter > 0 else M + 1
    hist = torch.full((B, kmax), float("nan"), dtype=torch.float64, device=dev) if with_hist else None
    sysd = make_system(sid, d, prm, shared, method)
    opts = make_options(dt_code, tol, 0, kmax)
    ws = _workspace(pint_parareal_workspace_bytes(sysd, B, M, dt_code), dev)
    _check(pint_parareal(sysd, B, x0, float(dt), M, S, opts, traj, iters, resid, status, hist, ws,
                         stream), "pint_parareal")
    out = (traj, iters, resid, status)
    if single:
        out = tuple(t[0] for t in out)
    if with_hist:
        out = out + ((hist[0] if single else hist),)
    return out


def longest_first(lengths, device) -> torch.Tensor:
    """Instance order for the work queue: longest horizon first (a stable
    sort), so the longest solves start early and the batch ends evenly."""
    lengths = torch.as_tensor(lengths, dtype=torch.int64).cpu()
    return torch.argsort(-lengths, stable=True).to(device)


def solve_varlen(system, x0: torch.Tensor, params: torch.Tensor, dt: float, lengths, *,
                 tol: float = 1e-10, window: int = 0, max_iter: int = 0, guess=None,
                 guard: float = 1e6, tile: int = 0, block: int = 0, wg_per_cu: int = 0,
                 order=None, method=RK4, stream=None):
    """Newton solve of B instances with their own horizons `lengths` [B].
    `order`: None, "longest_first", or a device int64 permutation [B].
    Returns (traj [sum T, d] packed, T_off [B+1], iters, resid, status)."""
    sid = _sys_id(system)
    if isinstance(order, str):
        if order != "longest_first":
            raise PintError(f"unknown order {order!r}")
        order = longest_first(lengths, x0.device)
    x0 = x0.contiguous()
    B, d = x0.shape
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    lengths = torch.as_tensor(lengths, dtype=torch.int64)
    T_off_h = torch.zeros(B + 1, dtype=torch.int64)
    T_off_h[1:] = torch.cumsum(lengths.cpu(), 0)
    total, T_max = int(T_off_h[-1]), int(lengths.max()) if B else 0
    T_off = T_off_h.to(x0.device)
    if guess is not None:
        traj = guess.reshape(total, d).to(x0.dtype).clone().contiguous()
    else:
        traj = torch.empty((total, d), dtype=x0.dtype, device=x0.device)
    iters = torch.empty(B, dtype=torch.int64, device=x0.device)
    resid = torch.empty(B, dtype=torch.float64, device=x0.device)
    status = torch.empty(B, dtype=torch.int32, device=x0.device)
    sysd = make_system(sid, d, prm, shared, method)
    opts = make_options(_dtype_code(x0), tol, window, max_iter, 1 if guess is not None else 0,
                        guard, tile, block, wg_per_cu, order)
    ws = _workspace(pint_workspace_bytes(sysd, B, total, T_max, opts), x0.device)
    _check(pint_solve_varlen(sysd, B, x0, float(dt), T_off, T_max, opts, traj, iters, resid,
                             status, ws, stream), "pint_solve_varlen")
    return traj, T_off, iters, resid, status


class SolveGraph:
    """A batched solve captured once as an executable HIP graph
    (pint_graph_capture_varlen) and replayed with `launch()`.  The buffers
    are owned here and fixed for the graph's life: write new initial states
    into `x0`, `params` (or `traj` with guess=True) in place between
    launches; results are in `traj`, `iters`, `resid`, `status`."""

    def __init__(self, system, x0: torch.Tensor, params: torch.Tensor, dt: float, lengths, *,
                 tol: float = 1e-10, window: int = 0, max_iter: int = 0, guess: bool = False,
                 guard: float = 1e6, block: int = 0, wg_per_cu: int = 0, order=None,
                 method=RK4):
        sid = _sys_id(system)
        self.x0 = x0.contiguous().clone()
        B, d = self.x0.shape
        self.params, shared = _params_2d(params.to(x0.dtype).clone(), B, n_params(sid, d))
        lengths = torch.as_tensor(lengths, dtype=torch.int64).cpu()
        T_off_h = torch.zeros(B + 1, dtype=torch.int64)
        T_off_h[1:] = torch.cumsum(lengths, 0)
        self.T_off = T_off_h.to(x0.device)
        total, T_max = int(T_off_h[-1]), int(lengths.max()) if B else 0
        if isinstance(order, str):
            if order != "longest_first":
                raise PintError(f"unknown order {order!r}")
            order = longest_first(lengths, x0.device)
        self.order = order
        self.traj = torch.empty((total, d), dtype=x0.dtype, device=x0.device)
        self.iters = torch.empty(B, dtype=torch.int64, device=x0.device)
        self.resid = torch.empty(B, dtype=torch.float64, device=x0.device)
        self.status = torch.empty(B, dtype=torch.int32, device=x0.device)
        self._sysd = make_system(sid, d, self.params, shared, method)
        self._opts = make_options(_dtype_code(x0), tol, window, max_iter, 1 if guess else 0, guard,
                                  0, block, wg_per_cu, order)
        self.ws = _workspace(pint_workspace_bytes(self._sysd, B, total, T_max, self._opts), x0.device)
        torch.cuda.synchronize(x0.device)
        rc, self._h = pint_graph_capture_varlen(self._sysd, B, self.x0, float(dt), self.T_off, T_max,
                                                self._opts, self.traj, self.iters, self.resid,
                                                self.status, self.ws)
        _check(rc, "pint_graph_capture_varlen")

    def launch(self, stream=None):
        if self._h is None:
            raise PintError("graph destroyed")
        _check(pint_graph_launch(self._h, stream), "pint_graph_launch")

    def close(self):
        if self._h is not None:
            pint_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def seq_integrate(system, x0: torch.Tensor, params: torch.Tensor, dt: float, lengths,
                  method=RK4, stream=None):
    """Sequential comparator (RK4, or a per-step Newton solve for the
    implicit rules).  lengths: int (uniform) or [B].  Returns the packed
    trajectory [sum T, d] (reshape to [B, T, d] for uniform T)."""
    sid = _sys_id(system)
    x0 = x0.contiguous()
    B, d = x0.shape
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    if isinstance(lengths, int):
        lengths = torch.full((B,), lengths, dtype=torch.int64)
    lengths = torch.as_tensor(lengths, dtype=torch.int64).cpu()
    T_off_h = torch.zeros(B + 1, dtype=torch.int64)
    T_off_h[1:] = torch.cumsum(lengths, 0)
    traj = torch.empty((int(T_off_h[-1]), d), dtype=x0.dtype, device=x0.device)
    sysd = make_system(sid, d, prm, shared, method)
    _check(pint_seq_integrate(sysd, B, x0, float(dt), T_off_h.to(x0.device),
                              int(lengths.max()) if B else 0, _dtype_code(x0), traj, stream),
           "pint_seq_integrate")
    return traj


def residual(system, x0, params, dt, traj, method=RK4, stream=None):
    """h [B, T, d] and ||h||_inf per instance for a uniform batch (the scaled
    residual for the implicit rules)."""
    sid = _sys_id(system)
    x0 = x0.contiguous()
    B, d = x0.shape
    T = traj.shape[1]
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    h = torch.empty_like(traj)
    hmax = torch.empty(B, dtype=torch.float64, device=x0.device)
    sysd = make_system(sid, d, prm, shared, method)
    _check(pint_residual(sysd, B, x0, float(dt), T, _dtype_code(x0), traj.contiguous(), h, hmax,
                         stream), "pint_residual")
    return h, hmax


def elements(system, x0, params, dt, traj, method=RK4, stream=None):
    """Newton-step elements A [B, T, d, d], b [B, T, d] of a uniform batch."""
    sid = _sys_id(system)
    x0 = x0.contiguous()
    B, d = x0.shape
    T = traj.shape[1]
    prm, shared = _params_2d(params.to(x0.dtype), B, n_params(sid, d))
    A = torch.empty((B, T, d, d), dtype=x0.dtype, device=x0.device)
    b = torch.empty((B, T, d), dtype=x0.dtype, device=x0.device)
    sysd = make_system(sid, d, prm, shared, method)
    _check(pint_elements(sysd, B, x0, float(dt), T, _dtype_code(x0), traj.contiguous(), A, b,
                         stream), "pint_elements")
    return A, b


def affine_scan(A: torch.Tensor, b: torch.Tensor, z0: Optional[torch.Tensor] = None, tile: int = 0,
                stream=None):
    """z_{n+1} = A_n z_n + b_n for each sequence: A [B, N, d, d], b [B, N, d]."""
    B, N, d, _ = A.shape
    dtc = _dtype_code(A)
    z = torch.empty((B, N, d), dtype=A.dtype, device=A.device)
    ws = _workspace(pint_scan_workspace_bytes(d, B, N, tile, dtc), A.device)
    _check(pint_affine_scan(d, B, N, dtc, A.contiguous(), b.contiguous(),
                            None if z0 is None else z0.contiguous(), z, tile, ws, stream),
           "pint_affine_scan")
    return z


def affine_scan_band(band: torch.Tensor, b: torch.Tensor, boff: int, z0: Optional[torch.Tensor] = None,
                     tile: int = 0, stream=None):
    """As affine_scan for cyclically banded A: band [B, N, d, bw] with
    A_n(i, (i + k - boff) mod d) = band[b, n, i, k]."""
    B, N, d, bw = band.shape
    dtc = _dtype_code(band)
    z = torch.empty((B, N, d), dtype=band.dtype, device=band.device)
    ws = _workspace(pint_scan_band_workspace_bytes(d, bw, boff, B, N, tile, dtc), band.device)
    _check(pint_affine_scan_band(d, bw, boff, B, N, dtc, band.contiguous(), b.contiguous(),
                                 None if z0 is None else z0.contiguous(), z, tile, ws, stream),
           "pint_affine_scan_band")
    return z


def adjoint(system, x0, params, dt, traj, g, seg: int = 0, with_params: bool = True,
            stream=None):
    """dL/dx0 [B, d] and dL/dtheta [B, n_params] (or None) through the
    reverse-time adjoint scan."""
    sid = _sys_id(system)
    x0 = x0.contiguous()
    B, d = x0.shape
    T = traj.shape[1]
    np_ = n_params(sid, d)
    prm, shared = _params_2d(params.to(x0.dtype), B, np_)
    dtc = _dtype_code(x0)
    gx0 = torch.empty((B, d), dtype=x0.dtype, device=x0.device)
    gth = torch.empty((B, np_), dtype=x0.dtype, device=x0.device) if with_params else None
    sysd = make_system(sid, d, prm, shared)
    ws = _workspace(pint_adjoint_workspace_bytes(sysd, B, T, seg, dtc), x0.device)
    _check(pint_adjoint(sysd, B, x0, float(dt), T, dtc, traj.contiguous(), g.contiguous(), gx0,
                        gth, int(seg), ws, stream), "pint_adjoint")
    return gx0, gth


class SolveFn(torch.autograd.Function):
    """traj = SolveFn.apply(x0 [B,d], params [B,np], system, dt, T, tol, window, seg).

    Forward: Newton solve (pint_solve); raises PintError unless every
    instance converged (the adjoint is that of the discrete solution map, so
    it is only meaningful at a root of h).  Backward: the reverse-time adjoint
    scan (pint_adjoint) through the discrete RK4 map at the returned
    trajectory, giving dL/dx0, and dL/dparams when params requires a
    gradient."""

    @staticmethod
    def forward(ctx, x0, params, system, dt, T, tol=1e-10, window=0, seg=0):
        traj, iters, resid, status = solve(system, x0.detach(), params.detach(), dt, T, tol=tol,
                                           window=window)
        st = status.reshape(-1)
        bad = (st != OK).nonzero()
        if bad.numel():
            b = int(bad[0, 0])
            raise PintError(f"SolveFn: instance {b} ended with status {int(st[b])} "
                            f"({status_string(int(st[b]))}); no gradient at a non-root")
        ctx.save_for_backward(x0.detach(), params.detach(), traj)
        ctx.system, ctx.dt, ctx.seg = system, dt, seg
        ctx.mark_non_differentiable(iters, resid, status)
        return traj, iters, resid, status

    @staticmethod
    def backward(ctx, g_traj, *_):
        x0, params, traj = ctx.saved_tensors
        g = torch.zeros_like(traj) if g_traj is None else g_traj.contiguous()
        want_th = bool(ctx.needs_input_grad[1])
        gx0, gth = adjoint(ctx.system, x0, params, ctx.dt, traj, g, seg=ctx.seg,
                           with_params=want_th)
        if gth is not None and params.dim() == 1:
            gth = gth.sum(0)
        return gx0, gth, None, None, None, None, None, None
