"""pint_affine_scan_noalloc (the scan with the library's fixed device
scratch) through the C ABI, against pint_affine_scan with a caller
workspace on the same inputs: two calls in a row on one stream, the second
smaller, and a size beyond the fixed scratch refused before any launch.
Bar: the scan's FP64 bar (the lookback composes a tile's carry-in from
whichever predecessors had published, so two runs differ by rounding):
1e-12 relative to the largest |z| per sequence; FP32 1e-5."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(N, d, B, seed, dtype):
    A, b = W.random_affine(N * B, d, seed=seed, kind="rotation")
    A = torch.from_numpy(A.reshape(B, N, d, d)).to(DEV, dtype)
    b = torch.from_numpy(b.reshape(B, N, d)).to(DEV, dtype)
    z0 = torch.from_numpy(np.random.default_rng(seed).normal(size=(B, d))).to(DEV, dtype)
    return A, b, z0


def _with_ws(P, d, B, N, code, A, b, z0, tile):
    z = torch.empty((B, N, d), dtype=A.dtype, device=DEV)
    ws = torch.empty(P.pint_scan_workspace_bytes(d, B, N, tile, code), dtype=torch.uint8, device=DEV)
    assert P.pint_affine_scan(d, B, N, code, A, b, z0, z, tile, ws) == P.OK
    return z


def _no_alloc(P, d, B, N, code, A, b, z0, tile):
    z = torch.empty((B, N, d), dtype=A.dtype, device=DEV)
    err = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    lib = P.load()
    rc = lib.pint_affine_scan_noalloc(d, B, N, code, A.data_ptr(), b.data_ptr(), z0.data_ptr(),
                                      z.data_ptr(), tile, err.data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
    assert rc == P.OK, P.status_string(rc)
    return z, err


@pytest.mark.parametrize("d,dtype", [(2, torch.float64), (3, torch.float64), (8, torch.float64),
                                     (40, torch.float64), (4, torch.float32), (16, torch.float32)])
def test_noalloc_matches_workspace_scan(pint, d, dtype):
    P = pint
    code = P.F64 if dtype == torch.float64 else P.F32
    bar = 1e-12 if code == P.F64 else 1e-5
    # first a larger call (many tiles, ragged tail), then a smaller one on the same scratch
    for B, N, tile, seed in ((3, 5000 if d <= 8 else 700, 0, 1), (2, 333 if d <= 8 else 90, 16, 2)):
        print(f"[noalloc] d={d} {dtype} B={B} N={N} tile={tile}", flush=True)
        A, b, z0 = _inputs(N, d, B, seed + d, dtype)
        z_ref = _with_ws(P, d, B, N, code, A, b, z0, tile)
        z, err = _no_alloc(P, d, B, N, code, A, b, z0, tile)
        torch.cuda.synchronize()
        assert int(err[0]) == 0
        scale = z_ref.abs().amax(dim=(1, 2)).clamp_min(1.0)
        diff = (z - z_ref).abs().amax(dim=(1, 2))
        assert bool((diff <= bar * scale).all()), (diff / scale).max().item()
        assert bool(torch.isfinite(z).all())


def test_noalloc_refuses_sizes_beyond_its_scratch(pint):
    """Kuramoto-sized dense elements (d = 128, 8 x 4096) need more than the
    fixed scratch holds: refused on the host, nothing launched (the pointers
    are never dereferenced)."""
    P = pint
    need = P.pint_scan_workspace_bytes(128, 8, 4096, 0, P.F64)
    assert need > P.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(256)
    lib = P.load()
    assert lib.pint_affine_scan_noalloc(128, 8, 4096, P.F64, fake, fake, None, fake, 0, None,
                                        None) == P.ERR_WORKSPACE
    assert lib.pint_affine_scan_noalloc(3, 0, 16, P.F64, None, None, None, None, 0, None,
                                        None) == P.OK
    assert lib.pint_affine_scan_noalloc(9, 1, 16, P.F64, fake, fake, None, fake, 0, None,
                                        None) == P.ERR_UNSUPPORTED
