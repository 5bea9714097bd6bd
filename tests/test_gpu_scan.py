"""GPU parity of the decoupled-lookback affine scan (pint_affine_scan) against
the oracle's sequential recursion z_{n+1} = A_n z_n + b_n, element by
element.  Elements are orthogonal maps (products of Givens rotations) so long
prefixes stay bounded and exactly checkable; FP64 bar 1e-11 relative to the
largest |z|, FP32 bar 1e-4 relative."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# elements per tile of the small-d kernels: for d <= 3 a few chunks of 256
# threads x S elements (all but the last kept in registers between the two
# passes), for d >= 4 64 lanes x 64 elements; and per chunk for d <= 3
SMALL_TILE = {"f64": {1: 12288, 2: 2048, 3: 1024, 4: 4096, 5: 4096, 6: 4096, 7: 4096, 8: 4096},
              "f32": {1: 9216, 2: 8192, 3: 2048, 4: 4096, 5: 4096, 6: 4096, 7: 4096, 8: 4096}}
SMALL_CHUNK = {"f64": {1: 3072, 2: 1024, 3: 512}, "f32": {1: 3072, 2: 2048, 3: 512}}


def _ref(orc, A, b, z0):
    return np.stack([orc.affine_seq(A[s], b[s], None if z0 is None else z0[s]) for s in range(A.shape[0])])


def _check(pint, orc, d, N, B, dtype, with_z0, seed, tile=0):
    A = np.empty((B, N, d, d))
    b = np.empty((B, N, d))
    for s in range(B):
        A[s], b[s] = W.random_affine(N, d, seed=seed + s, kind="rotation")
    z0 = np.random.default_rng(seed).normal(size=(B, d)) if with_z0 else None
    tdt = torch.float64 if dtype == "f64" else torch.float32
    At, bt = torch.tensor(A, dtype=tdt, device=DEV), torch.tensor(b, dtype=tdt, device=DEV)
    z0t = None if z0 is None else torch.tensor(z0, dtype=tdt, device=DEV)
    z = pint.affine_scan(At, bt, z0t, tile=tile)
    torch.cuda.synchronize()
    if dtype == "f32":
        A, b = A.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        z0 = None if z0 is None else z0.astype(np.float32).astype(np.float64)
    ref = _ref(orc, A, b, z0)
    got = z.double().cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    err = np.abs(got - ref).max() / scale
    assert err <= (1e-11 if dtype == "f64" else 1e-4), (d, N, B, dtype, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_small_d_several_tiles_ragged(pint, orc, d, dtype):
    N = 3 * SMALL_TILE[dtype][d] + 17
    print(f"[scan] d={d} {dtype} N={N}", flush=True)
    _check(pint, orc, d, N, 3, dtype, True, seed=10 + d)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("extra", [1, 2])
def test_small_d_tail_chunks(pint, orc, d, dtype, extra):
    """A last tile that ends inside its second or third chunk: its earlier
    chunks are full, and the one it ends in is a chunk the second pass takes
    from registers (or, at the tile's chunk count, from LDS)."""
    N = 2 * SMALL_TILE[dtype][d] + extra * SMALL_CHUNK[dtype][d] + 29
    print(f"[scan] tail d={d} {dtype} N={N}", flush=True)
    _check(pint, orc, d, N, 2, dtype, True, seed=60 + d + 10 * extra)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d", [16, 32, 40, 64, 128])
def test_dense_d_several_tiles_ragged(pint, orc, d, dtype):
    N = 16 * 5 + 3
    print(f"[scan] d={d} {dtype} N={N}", flush=True)
    _check(pint, orc, d, N, 2, dtype, True, seed=20 + d)


# Explicit tile lengths, so that every tile folds several elements into its
# aggregate on MFMA (FP64 16x16x4: the running product held in the
# accumulators for even d, the augmented [[A, b], [0, 1]] product for
# d = 40; FP32 16x16x4: the product in LDS).  128 and 256 are the tiles the
# full-horizon dense scans run at (8 Kuramoto sequences of 4096 elements,
# one Lorenz-96 sequence of 65536); each case has at least three tiles per
# sequence and a ragged last tile.
DENSE_TILES = [(16, 8), (16, 32), (32, 8), (32, 32), (40, 16), (40, 128), (40, 256),
               (64, 8), (64, 32), (128, 16), (128, 128)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d,tile", DENSE_TILES)
def test_dense_fold_at_tile(pint, orc, d, tile, dtype):
    B = 8 if (d, tile) == (128, 128) else 3
    N = 3 * tile + 17
    print(f"[scan] dense d={d} tile={tile} {dtype} N={N} B={B}", flush=True)
    _check(pint, orc, d, N, B, dtype, True, seed=200 + d + tile, tile=tile)


@pytest.mark.parametrize("d", [40, 128])
def test_dense_fold_gauss_f32(pint, orc, d):
    """FP32 MFMA fold on elements that are not orthogonal (entries N(0, 1/d),
    products shrink or grow): relative 1e-4 against the FP64 recursion on the
    same FP32-rounded elements, over 48 elements (tiles of 16)."""
    B, N = 2, 48
    A = np.empty((B, N, d, d))
    b = np.empty((B, N, d))
    for s in range(B):
        A[s], b[s] = W.random_affine(N, d, seed=300 + d + s, kind="gauss")
    A32, b32 = A.astype(np.float32), b.astype(np.float32)
    z = pint.affine_scan(torch.tensor(A32, device=DEV), torch.tensor(b32, device=DEV), tile=16)
    torch.cuda.synchronize()
    ref = _ref(orc, A32.astype(np.float64), b32.astype(np.float64), None)
    got = z.double().cpu().numpy()
    for s in range(B):
        for n in range(N):
            scale = max(1e-30, np.abs(ref[s, n]).max())
            assert np.abs(got[s, n] - ref[s, n]).max() <= 1e-4 * scale, (d, s, n)


@pytest.mark.parametrize("d,N", [(3, 1), (3, 512), (40, 1), (40, 16), (40, 17), (2, 2)])
def test_edge_lengths(pint, orc, d, N):
    _check(pint, orc, d, N, 2, "f64", False, seed=5)


def test_dense_tile_sizes(pint, orc):
    for tile in (1, 3, 32):
        _check(pint, orc, 40, 70, 1, "f64", True, seed=7, tile=tile)


@pytest.mark.parametrize("d", [16, 40, 128])
def test_dense_one_tile_per_sequence(pint, orc, d):
    """tile = N: every tile starts from z0 and the fold is skipped."""
    _check(pint, orc, d, 150, 3, "f64", True, seed=90 + d, tile=150)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 8])
def test_many_tiles_mixed(pint, orc, d, dtype):
    """Several times more tiles than workgroups resident on the device, three
    sequences of odd length so that later sequences start misaligned for
    vector loads and end ragged."""
    N = 100 * SMALL_TILE[dtype][d] + 17
    print(f"[scan] many tiles d={d} {dtype} N={N} B=3", flush=True)
    _check(pint, orc, d, N, 3, dtype, True, seed=40 + d)


def test_long_sequence(pint, orc):
    """2^20 elements of d = 3: hundreds of tiles in flight at once."""
    _check(pint, orc, 3, 1 << 20, 1, "f64", True, seed=3)


def test_empty_and_errors(pint):
    A = torch.zeros((1, 0, 3, 3), dtype=torch.float64, device=DEV)
    b = torch.zeros((1, 0, 3), dtype=torch.float64, device=DEV)
    assert pint.affine_scan(A, b).shape == (1, 0, 3)
    A = torch.zeros((1, 4, 9, 9), dtype=torch.float64, device=DEV)   # d = 9 is not built
    b = torch.zeros((1, 4, 9), dtype=torch.float64, device=DEV)
    with pytest.raises(pint.PintError):
        pint.affine_scan(A, b)


# ------------------------------------------------------------ banded scan --

def _check_band(pint, orc, N, B, boff, dtype, with_z0, seed, tile=0):
    d, bw = 40, 13
    A = np.empty((B, N, d, d))
    band = np.empty((B, N, d, bw))
    b = np.empty((B, N, d))
    for s in range(B):
        A[s], band[s], b[s] = W.random_band_affine(N, d, bw, boff, seed=seed + s)
    z0 = np.random.default_rng(seed).normal(size=(B, d)) if with_z0 else None
    tdt = torch.float64 if dtype == "f64" else torch.float32
    bandt, bt = torch.tensor(band, dtype=tdt, device=DEV), torch.tensor(b, dtype=tdt, device=DEV)
    z0t = None if z0 is None else torch.tensor(z0, dtype=tdt, device=DEV)
    z = pint.affine_scan_band(bandt, bt, boff, z0t, tile=tile)
    torch.cuda.synchronize()
    if dtype == "f32":
        A, b = A.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        z0 = None if z0 is None else z0.astype(np.float32).astype(np.float64)
    ref = _ref(orc, A, b, z0)
    got = z.double().cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    err = np.abs(got - ref).max() / scale
    assert err <= (1e-11 if dtype == "f64" else 1e-4), (N, B, boff, dtype, tile, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("boff", [4, 8])
def test_band_several_tiles_ragged(pint, orc, boff, dtype):
    """Banded elements (d = 40, 13 diagonals) against the oracle's recursion on
    the same elements expanded to dense: several tiles, a ragged tail, a
    starting vector."""
    print(f"[scan-band] boff={boff} {dtype}", flush=True)
    _check_band(pint, orc, 5 * 64 + 13, 3, boff, dtype, True, seed=60 + boff, tile=64)


@pytest.mark.parametrize("N,tile", [(1, 0), (2, 0), (5, 1), (17, 16), (700, 0), (2048, 0)])
def test_band_lengths_and_tiles(pint, orc, N, tile):
    print(f"[scan-band] N={N} tile={tile}", flush=True)
    _check_band(pint, orc, N, 2, 4, "f64", N % 2 == 0, seed=70, tile=tile)


def test_band_one_tile_per_sequence(pint, orc):
    """tile = N: the output pass alone, from z0 (no fold launch)."""
    _check_band(pint, orc, 600, 3, 4, "f64", True, seed=85, tile=600)
    _check_band(pint, orc, 600, 2, 8, "f32", False, seed=86, tile=600)


def test_band_many_sequences(pint, orc):
    """More tiles than resident workgroups: 64 sequences of 1500 elements at
    the default tile length."""
    _check_band(pint, orc, 1500, 64, 4, "f64", True, seed=80)


def test_band_errors(pint):
    band = torch.zeros((1, 4, 40, 12), dtype=torch.float64, device=DEV)  # 12 diagonals: not built
    b = torch.zeros((1, 4, 40), dtype=torch.float64, device=DEV)
    with pytest.raises(pint.PintError):
        pint.affine_scan_band(band, b, 4)
    band = torch.zeros((1, 4, 40, 13), dtype=torch.float64, device=DEV)
    with pytest.raises(pint.PintError):
        pint.affine_scan_band(band, b, 5)  # offset 5: not built
    flat = torch.zeros(4 * 40 * 13 + 1, dtype=torch.float64, device=DEV)
    mis = flat[1:].view(1, 4, 40, 13)       # 8-byte aligned only
    z = torch.empty((1, 4, 40), dtype=torch.float64, device=DEV)
    ws = torch.empty(pint.pint_scan_band_workspace_bytes(40, 13, 4, 1, 4, 0, pint.F64),
                     dtype=torch.uint8, device=DEV)
    assert pint.pint_affine_scan_band(40, 13, 4, 1, 4, pint.F64, mis, b, None, z, 0, ws) == \
        pint.ERR_INVALID_ARG
    assert pint.affine_scan_band(band[:, :0].contiguous(), b[:, :0].contiguous(), 4).shape == (1, 0, 40)
