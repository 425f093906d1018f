"""GPU tests of the 3-D column-sweep spreading (adjoint resampling of Algorithm 2).

3-D plans whose oversampled axes 1 and 2 are multiples of 16 (>= 32) spread by
column sweeps: a workgroup sweeps a segment of a 16 x 16 column along axis 0 with
a ring of padded planes in LDS, and a merge adds the columns' axis-1/2 halos and
the segments' trailing planes.  Checked against the FP64 oracle NFFT (paper,
Algorithms 1 and 2) at the rounding gate of the type:

* several stencil widths (2m = 4 .. 10, which change the plane depth Q_0 and the
  segment length), both sigma, both types, several segments per column and the
  cyclic wrap of the last segment's halo into the first, and columns swept as one
  segment (the halo onto the segment's own first planes);
* a clustered node set whose dense tiles hold several staged chunks;
* the multi-channel call, bit for bit the single-channel one (the fixed-point
  sums are exact in both types), and repeated adjoints, bit for bit each other;
* the padded-tile scheme on the same nodes (spread="tiled") and the errors of a
  plan that asks for sweeps where they are not available;
* the order of the nodes: a plan of the permuted nodes gives the permuted forward
  values and the same adjoint, bit for bit (each node's value is summed by one group
  of lanes in a fixed order wherever the sort by LDS bank slot places it, and the
  spreading sums are exact).
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import nfft_alg as na
from test_gpu_nfft import e2e_tol, make_plan, rel2, run_pair, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,M,m,sigma", [((16, 16, 16), 3000, 4, 2.0), ((16, 16, 16), 4000, 2, 2.0),
                                         ((24, 16, 16), 3000, 3, 2.0), ((16, 16, 16), 2500, 5, 2.0),
                                         ((32, 32, 24), 9000, 4, 2.0), ((40, 64, 64), 20000, 4, 1.25),
                                         ((12, 32, 16), 1500, 1, 2.0)])
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_matches_oracle(device, N, M, m, sigma, dt):
    x = wl.uniform_nodes(M, 3, config=150, stream=0)
    f, fh = wl.cn01(N, config=150, stream=1), wl.cn01((M,), config=150, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    info = p.info()
    print("sweep", N, M, m, sigma, dt, info, flush=True)
    assert info["spread"] == "sweep" and info["tile"][1:] == (16, 16)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol, rel2(yg, na.adjoint(xs, fh, N, m, sigma))
    assert rel2(fg, na.forward(xs, f, m, sigma)) < tol


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_single_segment_columns(device, dt):
    """Oversampled 16 x 256 x 256: 256 columns of two tiles, which a device of 256 compute
    units sweeps as one segment per column (one round of workgroups), so that a column's
    last 2m - 1 planes wrap onto its own first ones."""
    N, M, m, sigma = (8, 128, 128), 20000, 4, 2.0
    x = wl.uniform_nodes(M, 3, config=156, stream=0)
    f, fh = wl.cn01(N, config=156, stream=1), wl.cn01((M,), config=156, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    print("sweep single segment", dt, p.info(), flush=True)
    assert p.info()["spread"] == "sweep"
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol
    assert rel2(fg, na.forward(xs, f, m, sigma)) < tol


def _clustered(M, config):
    """Half the nodes uniform, half in a ball of radius 0.03 (tiles of thousands of nodes)."""
    g = wl.rng(config, 0)
    x = g.random((M, 3)) - 0.5
    k = M // 2
    x[:k] = 0.1 + 0.03 * (g.random((k, 3)) - 0.5)
    return x


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_clustered_nodes(device, dt):
    N, M, m, sigma = (32, 32, 32), 40000, 4, 2.0
    x = _clustered(M, 151)
    f, fh = wl.cn01(N, config=151, stream=1), wl.cn01((M,), config=151, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    assert p.info()["spread"] == "sweep"
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol
    assert rel2(fg, na.forward(xs, f, m, sigma)) < tol


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_multichannel(device, dt):
    N, M, m, sigma, K = (32, 32, 32), 9000, 4, 2.0, 3
    x = wl.uniform_nodes(M, 3, config=152, stream=0)
    p, xs = make_plan(device, x, N, m, sigma, dt)
    assert p.info()["spread"] == "sweep"
    fh = to_dev(np.stack([wl.cn01((M,), config=152, stream=20 + k) for k in range(K)]), dt, device)
    many = p.adjoint_many(fh)
    for k in range(K):
        one = p.adjoint(fh[k].contiguous())
        assert torch.equal(many[k], one)
        assert torch.equal(p.adjoint(fh[k].contiguous()), one)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(many[1].cpu().numpy(), na.adjoint(xs, fh[1].cpu().numpy(), N, m, sigma)) < tol


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_against_tiled(device, dt):
    """The two spreading schemes on one node set: both within the rounding gate of the
    oracle, and of each other (their fixed-point scales and merges differ)."""
    N, M, m, sigma = (32, 48, 32), 12000, 4, 2.0
    x = wl.uniform_nodes(M, 3, config=153, stream=0)
    fh = wl.cn01((M,), config=153, stream=2)
    ps, xs = make_plan(device, x, N, m, sigma, dt)
    pt, _ = make_plan(device, x, N, m, sigma, dt, spread="tiled")
    assert ps.info()["spread"] == "sweep" and pt.info()["spread"] == "tiled"
    ys = ps.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    yt = pt.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    tol = e2e_tol(N, sigma, m, dt)
    yo = na.adjoint(xs, fh, N, m, sigma)
    assert rel2(ys, yo) < tol and rel2(yt, yo) < tol
    assert rel2(ys, yt) < tol


def test_sweep_not_available(device):
    from paper_2208_00049_amd import NfftError
    x = wl.uniform_nodes(100, 3, config=154, stream=0)
    # oversampled axis 1 of 20 points: not a multiple of 16
    with pytest.raises(NfftError) as e:
        make_plan(device, x, (16, 10, 16), 4, 2.0, "c64", spread="sweep")
    assert e.value.code == -2
    # the (2m + 2)-point stencil is not swept
    with pytest.raises(NfftError):
        make_plan(device, x, (16, 16, 16), 3, 2.0, "c64", spread="sweep", wide=True)
    # the automatic choice falls back to padded tiles for both
    p, _ = make_plan(device, x, (16, 10, 16), 4, 2.0, "c64")
    assert p.info()["spread"] == "tiled"
    p, _ = make_plan(device, x, (16, 16, 16), 3, 2.0, "c64", wide=True)
    assert p.info()["spread"] == "tiled"


@pytest.mark.parametrize("N,M,m", [((32, 32, 32), 9000, 4), ((24, 32, 16), 5000, 3)])
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_sweep_node_order(device, N, M, m, dt):
    x = wl.uniform_nodes(M, 3, config=155, stream=0)
    perm = wl.rng(155, 3).permutation(M)
    f, fh = wl.cn01(N, config=155, stream=1), wl.cn01((M,), config=155, stream=2)
    pa, _ = make_plan(device, x, N, m, 2.0, dt)
    pb, _ = make_plan(device, np.asarray(x)[perm], N, m, 2.0, dt)
    assert pa.info()["spread"] == "sweep" and pb.info()["spread"] == "sweep"
    fd = to_dev(f, dt, device)
    fa, fb = pa.forward(fd), pb.forward(fd)
    assert torch.equal(fb, fa[torch.as_tensor(perm, device=device)])
    fhd = to_dev(fh, dt, device)
    ya = pa.adjoint(fhd)
    yb = pb.adjoint(fhd[torch.as_tensor(perm, device=device)].contiguous())
    assert torch.equal(ya, yb)
