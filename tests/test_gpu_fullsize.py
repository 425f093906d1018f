"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

The direct NDFT oracle evaluates sampled outputs one by one (forward: a seeded
sample of nodes; adjoint: a seeded sample of coefficient indices); the FP64
oracle NFFT (Algorithms 1 and 2) is compared element by element where it runs
in seconds.  Tolerances as in test_gpu_nfft.py (derived from the arithmetic).
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import ndft
from oracle import nfft_alg as na
from test_gpu_nfft import (C64_VS_ORACLE, C128_VS_ORACLE, NDFT_GATE, TARGET, e2e_tol, make_plan,
                           rel2, to_dev)

pytestmark = pytest.mark.gpu


def sampled_ndft(xs, f, fh, N, nf, na_, seed):
    g = np.random.default_rng(seed)
    js = np.sort(g.choice(xs.shape[0], nf, replace=False))
    ks = np.sort(g.choice(int(np.prod(N)), na_, replace=False))
    return js, ndft.ndft_forward(xs[js], f), ks, ndft.ndft_adjoint(xs, fh, N, idx=ks)


CASES_2D = [("uniform", "c64", 4), ("uniform", "c128", 6), ("radial", "c64", 4),
            ("radial", "c128", 4), ("uniform", "c128", 8)]


@pytest.mark.parametrize("nodes,dt,m", CASES_2D)
def test_2d_512(device, nodes, dt, m):
    N, sigma = (512, 512), 2.0
    x = wl.workload_nodes("2d_n512_radial402x652" if nodes == "radial" else "2d_n512_m262144_uniform")
    M = x.shape[0]
    f = wl.cn01(N, config=1, stream=1)
    fh = wl.cn01((M,), config=1, stream=2)
    p, xs = make_plan(device, x, N, m, sigma, dt)
    fg = p.forward(to_dev(f, dt, device)).cpu().numpy()
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    print("case", nodes, dt, m, flush=True)
    tol = e2e_tol(N, sigma, m, dt)
    # element by element against the FP64 oracle NFFT
    fo = na.forward(xs, f, m, sigma)
    yo = na.adjoint(xs, fh, N, m, sigma)
    assert rel2(fg, fo) < tol and rel2(yg, yo) < tol, (rel2(fg, fo), rel2(yg, yo), tol)
    # sampled outputs against the direct NDFT
    js, fe, ks, ye = sampled_ndft(xs, f, fh, N, 2048, 256, seed=7)
    gate = NDFT_GATE[(m, sigma)] + tol
    ef, ea = rel2(fg[js], fe), rel2(yg.reshape(-1)[ks], ye)
    assert ef < gate and ea < gate, (ef, ea, gate)
    if (dt, m, sigma) in TARGET:
        assert max(ef, ea) <= TARGET[(dt, m, sigma)]


# Default tiles of the 3-D 128^3 workload (M = 2^21): the column sweeps' (8, 16, 16) for both
# sigma (oversampled 256^3 and 160^3) and both types, and the padded-tile scheme's
# (spread="tiled") for this sparse node set in complex128 at sigma = 2.
TILE_3D = {(2.0, "c64", "auto"): (8, 16, 16), (1.25, "c64", "auto"): (8, 16, 16),
           (2.0, "c128", "auto"): (8, 16, 16), (1.25, "c128", "auto"): (8, 16, 16),
           (2.0, "c128", "tiled"): (8, 16, 16)}
SIGMA_DT_3D = [(2.0, "c64", "auto"), (1.25, "c64", "auto"), (2.0, "c128", "auto"),
               (1.25, "c128", "auto"), (2.0, "c128", "tiled")]


@pytest.mark.parametrize("sigma,dt,spread", SIGMA_DT_3D)
def test_3d_128(device, sigma, dt, spread):
    N, m = (128, 128, 128), 4
    x = wl.workload_nodes("3d_n128_m2097152")
    M = x.shape[0]
    f = wl.cn01(N, config=2, stream=1)
    fh = wl.cn01((M,), config=2, stream=2)
    p, xs = make_plan(device, x, N, m, sigma, dt, spread=spread)
    print("case 3d", sigma, dt, p.info(), flush=True)
    assert p.info()["tile"] == TILE_3D[(sigma, dt, spread)]
    assert p.info()["spread"] == ("sweep" if spread == "auto" else spread)
    fg = p.forward(to_dev(f, dt, device)).cpu().numpy()
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    tol = e2e_tol(N, sigma, m, dt)
    # forward against the oracle NFFT on a node sample (its grid step is computed in full)
    g = np.random.default_rng(11)
    js = np.sort(g.choice(M, 4096, replace=False))
    fo = na.forward(xs[js], f, m, sigma)
    assert rel2(fg[js], fo) < tol, (rel2(fg[js], fo), tol)
    # sampled outputs against the direct NDFT
    js2, fe, ks, ye = sampled_ndft(xs, f, fh, N, 256, 48, seed=13)
    gate = NDFT_GATE[(m, sigma)] + tol
    ef, ea = rel2(fg[js2], fe), rel2(yg.reshape(-1)[ks], ye)
    assert ef < gate and ea < gate, (ef, ea, gate)


def _box_index(lo, shape, Nt):
    return np.ix_(*[(lo[d] + np.arange(shape[d])) % Nt[d] for d in range(len(Nt))])


def _nodes_reaching_box(xs, Nt, m, lo, shape):
    """Nodes whose stencil (2m points per axis from its origin, cyclic) meets the box."""
    origin, _ = na._stencil(xs, Nt, m)
    sel = np.ones(xs.shape[0], dtype=bool)
    for d in range(len(Nt)):
        r = np.mod(origin[:, d] - lo[d], Nt[d])
        sel &= (r < shape[d]) | (r > Nt[d] - 2 * m)
    return sel


@pytest.mark.parametrize("sigma,dt,spread", SIGMA_DT_3D)
def test_3d_128_spread_grid_on_boxes(device, sigma, dt, spread):
    """The full-size adjoint resampling (spreading + halo merge over all 2^21 nodes, in the
    default tiles bench.py times) element by element on boxes of grid points -- at the
    origin, across the cyclic end of every axis and at a seeded ragged position -- against
    the oracle's adjoint resampling of the nodes whose stencils reach each box."""
    N, m = (128, 128, 128), 4
    x = wl.workload_nodes("3d_n128_m2097152")
    M = x.shape[0]
    fh = wl.cn01((M,), config=2, stream=2)
    p, xs = make_plan(device, x, N, m, sigma, dt, spread=spread)
    Nt = p.Ntilde
    print("spread boxes 3d", sigma, dt, p.info(), flush=True)
    assert p.info()["tile"] == TILE_3D[(sigma, dt, spread)]
    grid = p.resample_adjoint(to_dev(fh, dt, device)).cpu().numpy() * p.window_scale
    g = np.random.default_rng(17)
    boxes = [((0, 0, 0), (16, 16, 16)), (tuple(n - 12 for n in Nt), (20, 20, 20)),
             (tuple(int(v) for v in g.integers(0, Nt[0], size=3)), (9, 17, 23))]
    tol = C128_VS_ORACLE if dt == "c128" else C64_VS_ORACLE
    for lo, shape in boxes:
        sel = _nodes_reaching_box(xs, Nt, m, lo, shape)
        ref = na.resample_adjoint(xs[sel], fh[sel], N, m, Nt)[_box_index(lo, shape, Nt)]
        got = grid[_box_index(lo, shape, Nt)]
        assert rel2(got, ref) < tol, (lo, shape, int(sel.sum()), rel2(got, ref), tol)


@pytest.mark.parametrize("sigma,dt,spread", SIGMA_DT_3D)
def test_3d_128_adjoint_elementwise_on_subset(device, sigma, dt, spread):
    """The whole 3-D adjoint (spreading, merge, pruned adjoint FFT passes, crop and
    correction) element by element against the oracle NFFT on a seeded 2^18-node subset of
    the 128^3 workload, in the tiles the full workload uses."""
    N, m = (128, 128, 128), 4
    x = wl.workload_nodes("3d_n128_m2097152")
    js = np.sort(np.random.default_rng(19).choice(x.shape[0], 1 << 18, replace=False))
    fh = wl.cn01((x.shape[0],), config=2, stream=2)[js]
    p, xs = make_plan(device, x[js], N, m, sigma, dt, tile=TILE_3D[(sigma, dt, spread)],
                      spread=spread)
    print("adjoint subset 3d", sigma, dt, p.info(), flush=True)
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    yo = na.adjoint(xs, fh, N, m, sigma)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(yg, yo) < tol, (rel2(yg, yo), tol)


def test_fp32_matches_fp64_on_gpu(device):
    """The metric's accuracy condition: FP32 results within rel-l2 1e-5 of FP64, same GPU."""
    N, m, sigma = (512, 512), 4, 2.0
    x = wl.workload_nodes("2d_n512_m262144_uniform")
    M = x.shape[0]
    f = wl.cn01(N, config=1, stream=1)
    fh = wl.cn01((M,), config=1, stream=2)
    p32, xs = make_plan(device, x, N, m, sigma, "c64")
    p64, _ = make_plan(device, xs, N, m, sigma, "c128")
    f32 = p32.forward(to_dev(f, "c64", device)).cpu().numpy()
    y32 = p32.adjoint(to_dev(fh, "c64", device)).cpu().numpy()
    f64 = p64.forward(to_dev(f, "c128", device)).cpu().numpy()
    y64 = p64.adjoint(to_dev(fh, "c128", device)).cpu().numpy()
    assert rel2(f32, f64) < 1e-5 and rel2(y32, y64) < 1e-5


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_adjoint_is_bitwise_reproducible(device, dt):
    """Spreading sums in fixed point, so repeated adjoints agree bit for bit."""
    N, m, sigma = (512, 512), 4, 2.0
    x = wl.workload_nodes("2d_n512_radial402x652")
    fh = wl.cn01((x.shape[0],), config=1, stream=2)
    p, _ = make_plan(device, x, N, m, sigma, dt)
    a = p.adjoint(to_dev(fh, dt, device)).clone()
    for _ in range(3):
        b = p.adjoint(to_dev(fh, dt, device))
        assert torch.equal(a, b)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_two_plans_of_the_same_nodes_agree_bitwise(device, dt):
    """The bin sort is stable, so two plans of one node set have the same work items --
    also where dense tiles are split (the radial centre) -- and give identical results."""
    N, m, sigma = (512, 512), 4, 2.0
    x = wl.workload_nodes("2d_n512_radial402x652")
    f = wl.cn01(N, config=1, stream=1)
    fh = wl.cn01((x.shape[0],), config=1, stream=2)
    p1, _ = make_plan(device, x, N, m, sigma, dt, max_block_nodes=100)  # many split tiles
    p2, _ = make_plan(device, x, N, m, sigma, dt, max_block_nodes=100)
    print("two plans", dt, flush=True)
    assert torch.equal(p1.adjoint(to_dev(fh, dt, device)), p2.adjoint(to_dev(fh, dt, device)))
    assert torch.equal(p1.forward(to_dev(f, dt, device)), p2.forward(to_dev(f, dt, device)))
