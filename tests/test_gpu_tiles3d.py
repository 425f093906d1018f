"""GPU parity of the default 3-D tile shapes against the oracle.

Where the column sweeps are available the plan takes (8, 16, 16) tiles.  The
padded-tile scheme (spread="tiled") cuts the oversampled grid into 8^3 tiles, or
into 8 x 16 x 16 tiles when the node set is sparse (fewer than one node per four
grid points): there the padded-tile scratch per node dominates spreading, and the
larger tile (whose fixed-point accumulators need most of the LDS) halves it.
Complex128 takes 8 x 16 x 16 tiles for dense node sets too: its interpolation
tile alone leaves no 8^3 tile within the 64 KiB the dense choice starts from, and
the whole LDS then holds the larger tile.
These tests check which shape the plan picks and that each, and requested
shapes (a tile shape of the sweeps, others of the padded tiles), reproduce the
oracle's NFFT (paper, Algorithms 1 and 2).
"""
import numpy as np
import pytest

import nfft_workloads as wl
from oracle import nfft_alg as na
from test_gpu_nfft import e2e_tol, rel2, run_pair

pytestmark = pytest.mark.gpu

N = (32, 32, 32)  # oversampled 64^3 = 262144 grid points at sigma = 2


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("M,spread,want", [
    (6000, "auto", {"c64": (8, 16, 16), "c128": (8, 16, 16)}),
    (6000, "tiled", {"c64": (8, 16, 16), "c128": (8, 16, 16)}),
    (70000, "tiled", {"c64": (8, 8, 8), "c128": (8, 16, 16)})])
def test_default_tile_and_parity(device, dt, M, spread, want):
    x = wl.uniform_nodes(M, 3, config=140, stream=0)
    f, fh = wl.cn01(N, config=140, stream=1), wl.cn01((M,), config=140, stream=2)
    m, sigma = 4, 2.0
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh, spread=spread)
    print("3d tiles", dt, M, spread, p.info(), flush=True)
    assert tuple(p.info()["tile"]) == want[dt]
    assert p.info()["spread"] == ("sweep" if spread == "auto" else "tiled")
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(fg, na.forward(xs, f, m, sigma)) < tol
    assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol


def test_requested_tile_shapes_agree(device):
    """8^3, 8 x 16 x 16 (column sweeps) and 16 x 8 x 16 tiles requested for the same sparse
    node set: each within the end-to-end tolerance of the oracle, hence of each other (the
    partial sums the merges add differ, so the results are not bit-identical)."""
    M, m, sigma, dt = 6000, 4, 2.0, "c64"
    x = wl.uniform_nodes(M, 3, config=141, stream=0)
    f, fh = wl.cn01(N, config=141, stream=1), wl.cn01((M,), config=141, stream=2)
    tol = e2e_tol(N, sigma, m, dt)
    for tile in [(8, 8, 8), (8, 16, 16), (16, 8, 16)]:
        p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh, tile=tile)
        assert tuple(p.info()["tile"]) == tile
        assert rel2(fg, na.forward(xs, f, m, sigma)) < tol
        assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol
