"""The C-ABI library loads and exports every function include/pint.h declares
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pint.h")
LIB = os.path.join(ROOT, "paper_2511_01465_amd", "libpint.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pint_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["pint_solve", "pint_solve_varlen", "pint_seq_integrate", "pint_adjoint",
              "pint_affine_scan", "pint_workspace_bytes", "pint_status_string"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_host_side_queries_without_gpu():
    import paper_2511_01465_amd as P
    lib = P.load()
    assert P.n_params(P.LORENZ96, 40) == 1 and P.n_params(P.KURAMOTO, 128) == 129
    assert P.n_params(P.VDP, 3) == -1
    assert P.status_string(P.NONFINITE).startswith("non-finite")
    assert P.supported(P.LORENZ63, 3) and P.supported(P.VDP, 2, P.F32)
    assert not P.supported(P.VDP, 3)
    # argument errors are caught on the host before anything is launched
    sysd = P.pint_system(P.LORENZ63, 3, 3, 1, None)
    opts = P.make_options(P.F64, tol=-1.0)
    rc = lib.pint_solve(ctypes.byref(sysd), 1, None, 1e-3, 16, ctypes.byref(opts),
                        None, None, None, None, None, 0, None)
    assert rc == P.ERR_INVALID_ARG
    opts = P.make_options(P.F64)
    bad = P.pint_system(P.LORENZ63, 3, 2, 1, None)   # wrong n_params
    rc = lib.pint_solve(ctypes.byref(bad), 1, None, 1e-3, 16, ctypes.byref(opts),
                        None, None, None, None, None, 0, None)
    assert rc == P.ERR_INVALID_ARG
    rc = lib.pint_solve(ctypes.byref(sysd), 0, None, 1e-3, 16, ctypes.byref(opts),
                        None, None, None, None, None, 0, None)
    assert rc == P.OK   # empty batch: nothing to do


@pytest.mark.parametrize("struct", ["pint_options", "pint_system"])
def test_struct_layout_matches_the_header(tmp_path, struct):
    """The ctypes mirrors of pint_options and pint_system have the C layout
    (size and field offsets from a program compiled against include/pint.h)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    import paper_2511_01465_amd as P
    cls = getattr(P, struct)
    src = tmp_path / "layout.c"
    fields = [f[0] for f in cls._fields_]
    body = " ".join('printf("%%zu ", offsetof(%s, %s));' % (struct, f) for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pint.h"\n'
                   'int main(void){printf("%%zu ", sizeof(%s)); %s return 0;}\n' % (struct, body))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(cls)] + [getattr(cls, f).offset for f in fields]
    assert got == want


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_small_scan_tile_lengths():
    """The tile lengths that size the small-d scan parity cases are the
    library's: sequences of one tile take the workspace of one-element
    sequences, and one element more takes a second tile each."""
    import paper_2511_01465_amd as P
    from test_gpu_scan import SMALL_TILE
    P.load()
    B = 1000
    for dt, code in (("f64", P.F64), ("f32", P.F32)):
        for d, L in SMALL_TILE[dt].items():
            one = P.pint_scan_workspace_bytes(d, B, 1, 0, code)
            assert P.pint_scan_workspace_bytes(d, B, L, 0, code) == one, (dt, d, L)
            assert P.pint_scan_workspace_bytes(d, B, L + 1, 0, code) > one, (dt, d, L)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_step_rule_argument_checks():
    """The one-step rule is checked on the host: unknown codes and a non-zero
    reserved word are invalid; the implicit rules exist for the small
    dimensions only and not for the adjoint."""
    import paper_2511_01465_amd as P
    lib = P.load()
    assert P.n_params(P.ROBERTSON, 3) == 3 and P.n_params(P.ROBERTSON, 2) == -1
    assert P.supported(P.ROBERTSON, 3)
    opts = P.make_options(P.F64)

    def solve_rc(system, d, method, reserved=0):
        sysd = P.pint_system(system, d, P.n_params(system, d), 1, None, method, reserved)
        return lib.pint_solve(ctypes.byref(sysd), 0, None, 1e-2, 16, ctypes.byref(opts),
                              None, None, None, None, None, 0, None)

    assert solve_rc(P.VDP, 2, P.BACKWARD_EULER) == P.OK
    assert solve_rc(P.ROBERTSON, 3, P.TRAPEZOIDAL) == P.OK
    assert solve_rc(P.VDP, 2, 3) == P.ERR_INVALID_ARG
    assert solve_rc(P.VDP, 2, -1) == P.ERR_INVALID_ARG
    assert solve_rc(P.VDP, 2, P.RK4, reserved=1) == P.ERR_INVALID_ARG
    assert solve_rc(P.LORENZ96, 40, P.BACKWARD_EULER) == P.ERR_UNSUPPORTED
    assert solve_rc(P.KURAMOTO, 64, P.TRAPEZOIDAL) == P.ERR_UNSUPPORTED
    sysd = P.pint_system(P.VDP, 2, 1, 1, None, P.BACKWARD_EULER, 0)
    assert lib.pint_adjoint(ctypes.byref(sysd), 0, None, 1e-2, 16, P.F64, None, None, None,
                            None, 0, None, 0, None) == P.ERR_UNSUPPORTED


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_launch_shape_and_graph_argument_checks():
    import paper_2511_01465_amd as P
    lib = P.load()
    sysd = P.pint_system(P.VDP, 2, 1, 1, None)
    for kw in ({"block": 96}, {"wg_per_cu": 17}, {"wg_per_cu": -1}):
        opts = P.make_options(P.F64, **kw)
        rc = lib.pint_solve(ctypes.byref(sysd), 0, None, 1e-2, 16, ctypes.byref(opts),
                            None, None, None, None, None, 0, None)
        assert rc == P.ERR_INVALID_ARG, kw
    # graph capture: a missing handle pointer or offsets is refused before any HIP call
    opts = P.make_options(P.F64)
    assert lib.pint_graph_capture_varlen(ctypes.byref(sysd), 0, None, 1e-2, None, 0,
                                         ctypes.byref(opts), None, None, None, None, None, 0,
                                         None) == P.ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.pint_graph_capture_varlen(ctypes.byref(sysd), 0, None, 1e-2, None, 0,
                                         ctypes.byref(opts), None, None, None, None, None, 0,
                                         ctypes.byref(h)) == P.ERR_INVALID_ARG
    assert h.value is None
    assert lib.pint_graph_launch(None, None) == P.ERR_INVALID_ARG
    assert lib.pint_graph_destroy(None) == P.ERR_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_affine_scan_argument_checks():
    """pint_affine_scan's error returns, each decided before any HIP call
    (the pointers below are never dereferenced)."""
    import paper_2511_01465_amd as P
    lib = P.load()
    fake = ctypes.c_void_p(256)
    scan = lambda d, B, N, dtype, A, b, z, tile, ws, nbytes: lib.pint_affine_scan(
        d, B, N, dtype, A, b, None, z, tile, ws, nbytes, None)
    assert scan(3, 0, 16, P.F64, None, None, None, 0, None, 0) == P.OK        # empty batch
    assert scan(3, 1, 0, P.F64, None, None, None, 0, None, 0) == P.OK        # empty sequences
    assert scan(0, 1, 16, P.F64, fake, fake, fake, 0, None, 0) == P.ERR_INVALID_ARG
    assert scan(3, -1, 16, P.F64, fake, fake, fake, 0, None, 0) == P.ERR_INVALID_ARG
    assert scan(3, 1, 16, P.F64, fake, fake, fake, -1, None, 0) == P.ERR_INVALID_ARG
    assert scan(3, 1, 16, 7, fake, fake, fake, 0, None, 0) == P.ERR_INVALID_ARG
    assert scan(3, 1, 16, P.F64, None, fake, fake, 0, None, 0) == P.ERR_INVALID_ARG
    assert scan(9, 1, 16, P.F64, fake, fake, fake, 0, fake, 1 << 20) == P.ERR_UNSUPPORTED
    assert lib.pint_scan_workspace_bytes(9, 1, 16, 0, P.F64) == 0
    need = lib.pint_scan_workspace_bytes(3, 1, 16, 0, P.F64)
    assert need > 0
    assert scan(3, 1, 16, P.F64, fake, fake, fake, 0, None, need) == P.ERR_WORKSPACE
    assert scan(3, 1, 16, P.F64, fake, fake, fake, 0, fake, need - 1) == P.ERR_WORKSPACE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpint.so not built")
def test_parareal_argument_checks():
    """pint_parareal's error returns, each decided before any HIP call (the
    pointers below are never dereferenced)."""
    import paper_2511_01465_amd as P
    lib = P.load()
    fake = ctypes.c_void_p(256)
    vdp = P.pint_system(P.VDP, 2, 1, 1, fake)
    opts = P.make_options(P.F64, 1e-10)

    def call(sysd, B, M, S, o, ws=None, nbytes=0, x0=fake):
        return lib.pint_parareal(ctypes.byref(sysd), B, x0, 1e-2, M, S, ctypes.byref(o), fake,
                                 fake, fake, fake, None, ws, nbytes, None)

    assert call(vdp, 0, 4, 4, opts) == P.OK                                  # empty batch
    assert call(vdp, 1, -1, 4, opts) == P.ERR_INVALID_ARG
    assert call(vdp, 1, 4, -1, opts) == P.ERR_INVALID_ARG
    assert call(vdp, 1, 4, 4, P.make_options(P.F64, 0.0)) == P.ERR_INVALID_ARG   # tol must be > 0
    assert call(vdp, 1, 4, 4, P.make_options(P.F64, 1e-10, window=4)) == P.ERR_INVALID_ARG
    assert call(vdp, 1, 4, 4, P.make_options(7, 1e-10)) == P.ERR_INVALID_ARG
    assert call(vdp, 1, 4, 4, opts, x0=None) == P.ERR_INVALID_ARG
    l96 = P.pint_system(P.LORENZ96, 40, 1, 1, fake)
    assert call(l96, 1, 4, 4, opts) == P.ERR_UNSUPPORTED                     # small d only
    need = lib.pint_parareal_workspace_bytes(ctypes.byref(vdp), 1, 4, P.F64)
    assert need >= 13 * 2 * 8                                              # (3M + 1) states
    assert call(vdp, 1, 4, 4, opts, None, need) == P.ERR_WORKSPACE
    assert call(vdp, 1, 4, 4, opts, fake, need - 1) == P.ERR_WORKSPACE
