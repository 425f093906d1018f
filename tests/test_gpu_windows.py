"""GPU tests of the window-evaluation modes (the paper's precomputation options).

* TENSOR stores the polynomial-window weights per node: results are bit for bit
  those of POLYNOMIAL (same Horner evaluation, done at plan time).
* FULL stores the (2m)^D weight products per node (D <= 2): the oracle with the
  polynomial window, within the rounding tolerance; D = 3 is rejected.
* LINEAR looks the window up in a table of m 2^c + 2 samples with linear
  interpolation: the oracle with the same lookup, within the rounding tolerance,
  and the NDFT within the approximation gate.
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import ndft
from oracle import nfft_alg as na
from test_gpu_nfft import NDFT_GATE, direct_fp32_factor, e2e_tol, make_plan, rel2, to_dev

pytestmark = pytest.mark.gpu

CASES = [((256,), 512, 4, 2.0, "c128"), ((64, 64), 5000, 4, 2.0, "c64"),
         ((48, 64), 3000, 6, 2.0, "c128"), ((32, 32), 2000, 2, 2.0, "c64"),
         ((16, 16, 16), 3000, 4, 2.0, "c64"), ((16, 24, 16), 2000, 4, 1.25, "c128")]


def run(device, N, M, m, sigma, dt, window, config):
    x = wl.uniform_nodes(M, len(N), config=config, stream=0)
    f = wl.cn01(N, config=config, stream=1)
    fh = wl.cn01((M,), config=config, stream=2)
    p, xs = make_plan(device, x, N, m, sigma, dt, window=window)
    return p.forward(to_dev(f, dt, device)), p.adjoint(to_dev(fh, dt, device)), xs, f, fh


@pytest.mark.parametrize("N,M,m,sigma,dt", CASES)
def test_tensor_is_bitwise_poly(device, N, M, m, sigma, dt):
    ft, yt, *_ = run(device, N, M, m, sigma, dt, "tensor", 60)
    fp, yp, *_ = run(device, N, M, m, sigma, dt, "poly", 60)
    assert torch.equal(ft, fp) and torch.equal(yt, yp)


@pytest.mark.parametrize("N,M,m,sigma,dt", [c for c in CASES if len(c[0]) <= 2])
def test_full_matches_oracle(device, N, M, m, sigma, dt):
    fg, yg, xs, f, fh = run(device, N, M, m, sigma, dt, "full", 61)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(fg.cpu().numpy(), na.forward(xs, f, m, sigma)) < tol
    assert rel2(yg.cpu().numpy(), na.adjoint(xs, fh, N, m, sigma)) < tol


def test_full_rejects_3d(device):
    from paper_2208_00049_amd import NfftError
    with pytest.raises(NfftError):
        make_plan(device, np.zeros((10, 3)), (16, 16, 16), 4, 2.0, "c64", window="full")


@pytest.mark.parametrize("N,M,m,sigma,dt", CASES)
def test_linear_matches_oracle(device, N, M, m, sigma, dt):
    fg, yg, xs, f, fh = run(device, N, M, m, sigma, dt, "linear", 62)
    print("linear", N, m, sigma, dt, flush=True)
    # the table lookup's interpolation weight is computed from the FP32 fraction on the GPU
    # (FP64 in the oracle): same order as the rounding of the polynomial path
    tol = e2e_tol(N, sigma, m, dt)
    fo = na.forward(xs, f, m, sigma, window="linear")
    yo = na.adjoint(xs, fh, N, m, sigma, window="linear")
    assert rel2(fg.cpu().numpy(), fo) < tol and rel2(yg.cpu().numpy(), yo) < tol
    if (m, sigma) in NDFT_GATE:
        # linear interpolation in a table of spacing h = 1/(S-2) changes the window by at
        # most h^2/8 max|psi''| <= h^2 beta^2/8 relative to its peak (measured on the CPU for
        # these cases: the oracle's NDFT error moves by under 1e-10 relative)
        Nt = na.oversampled_size(N, sigma)
        beta = na.kb_beta(m, Nt[0] / N[0])
        h = 1.0 / (na.linear_table_size(m) - 2)
        gate = NDFT_GATE[(m, sigma)] + tol + len(N) * h * h * beta * beta / 8
        assert rel2(fg.cpu().numpy(), ndft.ndft_forward(xs, f)) < gate


# 3-D: the padded spreading tile (tile + 2m+1 halo, 16 B per cell in c64) must fit in LDS,
# which needs a tile edge of 10..12 at m = 4: Ntilde = 48 allows 12
WIDE = [((256,), 512, 4, 2.0, "c128"), ((64, 64), 5000, 4, 2.0, "c64"),
        ((48, 64), 3000, 3, 2.0, "c128"), ((24, 24, 24), 3000, 4, 2.0, "c64"),
        ((32, 32), 2000, 6, 2.0, "c128")]


@pytest.mark.parametrize("window", ["poly", "direct"])
@pytest.mark.parametrize("N,M,m,sigma,dt", WIDE)
def test_wide_stencil_matches_oracle(device, window, N, M, m, sigma, dt):
    x = wl.uniform_nodes(M, len(N), config=63, stream=0)
    f = wl.cn01(N, config=63, stream=1)
    fh = wl.cn01((M,), config=63, stream=2)
    p, xs = make_plan(device, x, N, m, sigma, dt, window=window, wide=True)
    fg = p.forward(to_dev(f, dt, device)).cpu().numpy()
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    tol = e2e_tol(N, sigma, m, dt) * direct_fp32_factor(N, m, sigma, window, dt)
    ef = rel2(fg, na.forward(xs, f, m, sigma, window=window, wide=True))
    ea = rel2(yg, na.adjoint(xs, fh, N, m, sigma, window=window, wide=True))
    print("wide", window, N, m, dt, "err/tol %.3f %.3f" % (ef / tol, ea / tol), flush=True)
    assert ef < tol and ea < tol


@pytest.mark.parametrize("m", [3, 4])
def test_wide_stencil_accuracy_ordering_on_gpu(device, m):
    """2m points < 2m+2 points (untruncated window) < 2(m+1) points, against the NDFT."""
    N, M = (48, 64), 3000
    x = wl.uniform_nodes(M, 2, config=64, stream=0)
    f = wl.cn01(N, config=64, stream=1)
    errs = []
    for mm, wide in [(m, False), (m, True), (m + 1, False)]:
        p, xs = make_plan(device, x, N, mm, 2.0, "c128", wide=wide)
        errs.append(rel2(p.forward(to_dev(f, "c128", device)).cpu().numpy(),
                         ndft.ndft_forward(xs, f)))
    print("ordering", m, errs, flush=True)
    assert errs[2] < errs[1] < errs[0]
