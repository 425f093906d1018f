"""GPU parity: libnfft (through the C ABI) against the CPU oracle.

* step parity: the oversampled FFT against numpy's FFT, the resampling steps
  against the oracle's Algorithm 1/2 resampling on the same grid;
* end to end: forward and adjoint against the oracle NFFT (same algorithm,
  FP64, rounding-level tolerance) and against the direct NDFT (approximation
  tolerance per (m, sigma, dtype));
* the exact adjointness of the GPU pair (A ~= B F D, A^H ~= D^T F^H B^T);
* edge cases: M = 0, one node, all nodes in one tile, grid-aligned nodes,
  x = -1/2, a hot spot of coincident nodes, nodes outside the torus.
* the order of the nodes (padded-tile plans of 2 and 3 axes): a plan of the
  permuted nodes gives the permuted forward values bit for bit and the adjoint
  within the rounding gate.

Tolerances (derived from the arithmetic, not fitted).  Rounding errors of
relative size u (2^-24 for c64, 2^-53 for c128) made on the oversampled grid
(window weights, (2m)^D-term sums, log2|I_Nt| FFT stages) reach the output
through the resampling correction, whose factors beta_d(n) grow towards the
edge of I_N; for flat random data this amplifies a white grid error by
kappa = prod_d sqrt(mean(beta_d^2) mean(beta_d^-2)) (about 1.5 at sigma = 2,
about 330 for 3-D sigma = 1.25).  Gates against the FP64 oracle:
  c64:  10 u kappa log2|I_Nt| / 8,   c128: 100 u kappa log2|I_Nt| / 8
(the c128 constant also covers the two independent least-squares fits of the
window polynomial).  Against the NDFT the gate is the oracle's own
approximation gate plus the above.  The stated targets are asserted
separately: c64 m=4 sigma=2 within 1e-5 and c128 m=6 sigma=2 within 1e-9 of
the NDFT (relative l2).
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import ndft
from oracle import nfft_alg as na

pytestmark = pytest.mark.gpu

C128_VS_ORACLE = 1e-11   # resampling steps alone (no resampling correction involved)
C64_VS_ORACLE = 5e-6
NDFT_GATE = {(4, 2.0): 1e-6, (6, 2.0): 1e-9, (8, 2.0): 1e-12, (4, 1.25): 2e-4, (3, 2.0): 3e-5}
TARGET = {("c64", 4, 2.0): 1e-5, ("c128", 6, 2.0): 1e-9}


def kappa(N, sigma, m):
    Nt = na.oversampled_size(N, sigma)
    k = 1.0
    for d in range(len(N)):
        b = na.deconv_factors(N[d], Nt[d], m)
        k *= np.sqrt(np.mean(b ** 2) * np.mean(b ** -2.0))
    return k


def e2e_tol(N, sigma, m, dt):
    Nt = na.oversampled_size(N, sigma)
    lg = np.log2(np.prod(Nt))
    return (10 * 2.0 ** -24 if dt == "c64" else 100 * 2.0 ** -53) * kappa(N, sigma, m) * lg / 8


def direct_fp32_factor(N, m, sigma, window, dt):
    """Gate multiplier for the window evaluated directly in FP32.  The rounded argument
    beta s of sinh carries a relative error of about u beta s, which sinh turns into a
    relative error of coth(beta s) beta s u <= (beta + 1) u; the square root, division and
    normalisation add a few u more.  Per axis the weight is off by about (beta + 6) u of the
    window's peak (the tails, where sqrt(1 - u^2) is small and the argument's relative error
    is larger, are below 1e-3 of the peak), against the few u of the polynomial's Horner
    evaluation that e2e_tol's constant 10 budgets for."""
    if window != "direct" or dt != "c64":
        return 1.0
    Nt = na.oversampled_size(N, sigma)
    beta = na.kb_beta(m, Nt[0] / N[0])
    return 1.0 + len(N) * (beta + 6.0) / 10.0


def rel2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_plan(device, x, N, m, sigma, dt, **kw):
    from paper_2208_00049_amd import Plan
    xdt = torch.float64 if dt == "c128" else torch.float32
    xt = torch.tensor(np.asarray(x).reshape(-1, len(N)), dtype=xdt, device=device)
    p = Plan(xt, N, m=m, sigma=sigma, **kw)
    return p, xt.double().cpu().numpy()


def to_dev(a, dt, device):
    return torch.tensor(np.asarray(a), dtype=torch.complex128 if dt == "c128" else torch.complex64,
                        device=device)


def run_pair(device, x, N, m, sigma, dt, f, fh, **kw):
    p, xs = make_plan(device, x, N, m, sigma, dt, **kw)
    fg = p.forward(to_dev(f, dt, device)).cpu().numpy()
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    return p, xs, fg, yg


# ---------------------------------------------------------------------------
# step parity

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,sigma", [((256,), 2.0), ((32, 48), 2.0), ((64, 64), 2.0),
                                     ((16, 16, 16), 2.0), ((16, 24, 16), 1.25), ((20,), 1.5)])
def test_fft_grid_matches_numpy(device, dt, N, sigma):
    p, _ = make_plan(device, np.zeros((1, len(N))), N, 2, sigma, dt)
    Nt = p.Ntilde
    g = wl.cn01(Nt, config=80, stream=1)
    tol = 1e-13 if dt == "c128" else 2e-6
    fw = p.fft_grid(to_dev(g, dt, device), -1).cpu().numpy()
    assert rel2(fw, np.fft.fftn(g)) < tol
    bw = p.fft_grid(to_dev(g, dt, device), +1).cpu().numpy()
    assert rel2(bw, np.fft.ifftn(g) * g.size) < tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M,m,sigma", [((256,), 512, 4, 2.0), ((64, 64), 5000, 4, 2.0),
                                         ((48, 64), 3000, 6, 2.0), ((16, 16, 16), 6000, 4, 2.0),
                                         ((32, 32, 16), 3000, 4, 1.25), ((16, 16, 16), 3000, 4, 1.25)])
def test_resampling_steps_match_oracle(device, dt, N, M, m, sigma):
    D = len(N)
    x = wl.uniform_nodes(M, D, config=81, stream=0)
    p, xs = make_plan(device, x, N, m, sigma, dt)
    Nt = p.Ntilde
    ghat = wl.cn01(Nt, config=81, stream=1)
    fh = wl.cn01((M,), config=81, stream=2)
    tol = C128_VS_ORACLE if dt == "c128" else C64_VS_ORACLE
    # the library's window is the paper's divided by C = prod_d sinh(beta_d)/pi
    C = p.window_scale
    got = p.resample_forward(to_dev(ghat, dt, device)).cpu().numpy() * C
    assert rel2(got, na.resample_forward(xs, ghat, N, m, Nt)) < tol
    spread = p.resample_adjoint(to_dev(fh, dt, device)).cpu().numpy() * C
    assert rel2(spread, na.resample_adjoint(xs, fh, N, m, Nt)) < tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_forward_grid_is_F_D_f(device, dt):
    N, M, m, sigma = (64, 48), 1000, 4, 2.0
    x = wl.uniform_nodes(M, 2, config=82, stream=0)
    f = wl.cn01(N, config=82, stream=1)
    p, xs = make_plan(device, x, N, m, sigma, dt)
    p.forward(to_dev(f, dt, device))
    g = p.grid().cpu().numpy() / p.window_scale
    _, st = na.forward(xs, f, m, sigma, return_steps=True)
    assert rel2(g, st["ghat"]) < (1e-13 if dt == "c128" else 2e-6)


# ---------------------------------------------------------------------------
# end to end

CASES = [((256,), 512, 4, 2.0), ((256,), 512, 6, 2.0), ((64, 64), 4096, 4, 2.0),
         ((64, 32), 3000, 6, 2.0), ((32, 32), 2048, 8, 2.0), ((64, 64), 4096, 4, 1.25),
         ((16, 16, 16), 4096, 4, 2.0), ((16, 16, 16), 4096, 4, 1.25), ((32, 32), 1500, 3, 2.0)]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M,m,sigma", CASES)
def test_end_to_end_against_oracle_and_ndft(device, dt, N, M, m, sigma):
    D = len(N)
    x = wl.uniform_nodes(M, D, config=83, stream=0)
    f = wl.cn01(N, config=83, stream=1)
    fh = wl.cn01((M,), config=83, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    fo = na.forward(xs, f, m, sigma)
    yo = na.adjoint(xs, fh, N, m, sigma)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(fg, fo) < tol and rel2(yg, yo) < tol, (rel2(fg, fo), rel2(yg, yo), tol)
    fe = ndft.ndft_forward(xs, f)
    ye = ndft.ndft_adjoint(xs, fh, N)
    gate = NDFT_GATE[(m, sigma)] + tol
    assert rel2(fg, fe) < gate and rel2(yg, ye) < gate, (rel2(fg, fe), rel2(yg, ye), gate)
    if (dt, m, sigma) in TARGET:
        assert max(rel2(fg, fe), rel2(yg, ye)) <= TARGET[(dt, m, sigma)]


# complex64 plans whose raw window peaks, multiplied over the axes, leave the float range
# (2-D m = 10: (sinh(beta)/pi)^2 ~ 5e39; 4-D m = 5, 6) or come close (3-D m = 5): the
# library stores the window divided by its peak per axis and the resampling correction
# multiplied by it, so the FP32 factors stay near 1.
@pytest.mark.parametrize("N,M,m", [((64, 64), 3000, 10), ((24, 24, 24), 2000, 5),
                                   ((10, 10, 10, 10), 1500, 5), ((12, 12, 12, 12), 400, 6)])
def test_c64_large_m_against_oracle(device, N, M, m):
    sigma, dt = 2.0, "c64"
    D = len(N)
    x = wl.uniform_nodes(M, D, config=88, stream=0)
    f = wl.cn01(N, config=88, stream=1)
    fh = wl.cn01((M,), config=88, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    print("c64 large m", N, m, p.info(), p.window_peaks(), flush=True)
    assert np.all(np.isfinite(fg)) and np.all(np.isfinite(yg))
    tol = e2e_tol(N, sigma, m, dt)
    fo = na.forward(xs, f, m, sigma)
    yo = na.adjoint(xs, fh, N, m, sigma)
    assert rel2(fg, fo) < tol and rel2(yg, yo) < tol, (rel2(fg, fo), rel2(yg, yo), tol)
    # the FP32 target against the NDFT
    assert rel2(fg, ndft.ndft_forward(xs, f)) < TARGET[("c64", 4, 2.0)]
    assert rel2(yg, ndft.ndft_adjoint(xs, fh, N)) < TARGET[("c64", 4, 2.0)]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M,m,sigma", [((128,), 300, 4, 2.0), ((64, 64), 4096, 6, 2.0),
                                         ((16, 16, 16), 3000, 4, 1.25)])
def test_gpu_pair_is_exactly_adjoint(device, dt, N, M, m, sigma):
    D = len(N)
    x = wl.uniform_nodes(M, D, config=84, stream=0)
    f = wl.cn01(N, config=84, stream=1)
    fh = wl.cn01((M,), config=84, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    lhs = np.vdot(fh, fg)
    rhs = np.vdot(yg, f)
    scale = np.linalg.norm(fh) * np.linalg.norm(fg)
    assert abs(lhs - rhs) < e2e_tol(N, sigma, m, dt) * scale


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_direct_window_mode(device, dt):
    N, M, m, sigma = (64, 64), 4096, 4, 2.0
    x = wl.uniform_nodes(M, 2, config=85, stream=0)
    f = wl.cn01(N, config=85, stream=1)
    fh = wl.cn01((M,), config=85, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh, window="direct")
    fo = na.forward(xs, f, m, sigma, window="direct")
    yo = na.adjoint(xs, fh, N, m, sigma, window="direct")
    tol = e2e_tol(N, sigma, m, dt) * direct_fp32_factor(N, m, sigma, "direct", dt)
    assert rel2(fg, fo) < tol and rel2(yg, yo) < tol, (rel2(fg, fo), rel2(yg, yo), tol)


# ---------------------------------------------------------------------------
# edge cases

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_empty_node_set(device, dt):
    from paper_2208_00049_amd import Plan
    xdt = torch.float64 if dt == "c128" else torch.float32
    p = Plan(torch.zeros((0, 2), dtype=xdt, device=device), (32, 32))
    y = p.adjoint(torch.zeros(0, dtype=p.cdtype, device=device),
                  out=torch.full((32, 32), 7.0, dtype=p.cdtype, device=device))
    assert torch.count_nonzero(y).item() == 0
    assert p.forward(torch.ones((32, 32), dtype=p.cdtype, device=device)).numel() == 0


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["one_tile", "grid_aligned", "hotspot", "outside", "single"])
def test_edge_node_sets(device, dt, kind):
    N, m, sigma = (64, 64), 4, 2.0
    Nt = na.oversampled_size(N, sigma)
    g = wl.rng(86, 0)
    if kind == "one_tile":
        x = 0.1 + g.random((3000, 2)) * (8.0 / Nt[0])
    elif kind == "grid_aligned":
        x = g.integers(-Nt[0] // 2, Nt[0] // 2, size=(2000, 2)) / Nt[0]
        x[:50] = -0.5
        x[50:100, 0] = 0.0
    elif kind == "hotspot":
        x = np.concatenate([np.zeros((700, 2)), wl.uniform_nodes(1000, 2, config=86, stream=0)])
    elif kind == "outside":
        x = wl.uniform_nodes(1500, 2, config=86, stream=0) * 7.0
    else:
        x = np.array([[0.25, -0.125]])
    M = x.shape[0]
    f = wl.cn01(N, config=86, stream=1)
    fh = wl.cn01((M,), config=86, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    fo = na.forward(xs, f, m, sigma)
    yo = na.adjoint(xs, fh, N, m, sigma)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(fg, fo) < tol and rel2(yg, yo) < tol, (rel2(fg, fo), rel2(yg, yo), tol)


@pytest.mark.parametrize("bad", ["nan", "inf"])
@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M", [((64,), 300), ((32, 32), 2000), ((16, 16, 16), 3000),
                                 ((8, 8, 8, 8), 1500)])
def test_non_finite_values(device, N, M, dt, bad):
    """One NaN or infinite part in fhat makes every value of the adjoint NaN (the
    fixed-point spreading would otherwise drop a NaN and saturate on an infinity); one in
    f makes every forward value non-finite.  The plan is left intact for finite inputs."""
    D = len(N)
    x = wl.uniform_nodes(M, D, config=89, stream=0)
    f = wl.cn01(N, config=89, stream=1)
    fh = wl.cn01((M,), config=89, stream=2)
    v = np.nan if bad == "nan" else np.inf
    fb, fhb = f.copy(), fh.copy()
    fb.flat[f.size // 3] = complex(0.25, v)
    fhb[M // 2] = complex(v, -0.5)
    p, xs, fg, yg = run_pair(device, x, N, 4, 2.0, dt, fb, fhb)
    print("non-finite", N, dt, bad, flush=True)
    assert np.isnan(yg).all()
    assert not np.isfinite(fg).any()
    tol = e2e_tol(N, 2.0, 4, dt)
    fg = p.forward(to_dev(f, dt, device)).cpu().numpy()
    yg = p.adjoint(to_dev(fh, dt, device)).cpu().numpy()
    assert rel2(fg, na.forward(xs, f, 4, 2.0)) < tol
    assert rel2(yg, na.adjoint(xs, fh, N, 4, 2.0)) < tol


def test_nan_node_is_rejected(device):
    from paper_2208_00049_amd import NfftError, Plan
    x = torch.zeros((10, 2), dtype=torch.float64, device=device)
    x[3, 1] = float("nan")
    with pytest.raises(NfftError) as e:
        Plan(x, (32, 32))
    assert e.value.code == -5


def test_explicit_tiles_and_small_blocks(device):
    """Other tilings and work-item caps give the same transform."""
    N, M, m, sigma = (64, 64), 5000, 4, 2.0
    x = wl.uniform_nodes(M, 2, config=87, stream=0)
    f = wl.cn01(N, config=87, stream=1)
    fh = wl.cn01((M,), config=87, stream=2)
    ref = None
    for kw in [dict(), dict(tile=(16, 64)), dict(tile=(64, 8)), dict(max_block_nodes=37)]:
        p, xs, fg, yg = run_pair(device, x, N, m, sigma, "c128", f, fh, **kw)
        if ref is None:
            ref = (fg, yg)
        else:
            assert rel2(fg, ref[0]) < 1e-13 and rel2(yg, ref[1]) < 1e-13, kw


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M", [((25,), 300), ((23, 31), 3000), ((9, 10, 11), 2000),
                                 ((33, 64), 4000)])
def test_odd_sizes(device, dt, N, M):
    """Odd N (n = -(N-1)/2 .. (N-1)/2): the zero-pad band and the crop follow floor(N/2)."""
    m, sigma = 4, 2.0
    x = wl.uniform_nodes(M, len(N), config=85, stream=0)
    f = wl.cn01(N, config=85, stream=1)
    fh = wl.cn01((M,), config=85, stream=2)
    p, xs, fg, yg = run_pair(device, x, N, m, sigma, dt, f, fh)
    print("odd", N, dt, p.info(), flush=True)
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(fg, na.forward(xs, f, m, sigma)) < tol
    assert rel2(yg, na.adjoint(xs, fh, N, m, sigma)) < tol
    gate = NDFT_GATE[(m, sigma)] + tol
    assert rel2(fg, ndft.ndft_forward(xs, f)) < gate


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("N,M,kw", [((64, 48), 5000, {}), ((32, 32), 20000, {}),
                                    ((32, 32, 32), 6000, {"spread": "tiled"}),
                                    ((32, 32, 32), 70000, {"spread": "tiled"})])
def test_node_order_tiled(device, dt, N, M, kw):
    # A plan of the permuted nodes gives the permuted forward values bit for bit: each
    # node's interpolated value is summed by one group of lanes in a fixed order
    # wherever the sort by LDS bank slot places the node.  The adjoint agrees within
    # the rounding gate: its fixed-point sums are exact, but a work item's scale comes
    # from the nodes it holds, and a dense tile's nodes split into work items by order.
    x = wl.uniform_nodes(M, len(N), config=158, stream=0)
    perm = wl.rng(158, 3).permutation(M)
    f, fh = wl.cn01(N, config=158, stream=1), wl.cn01((M,), config=158, stream=2)
    pa, _ = make_plan(device, x, N, 4, 2.0, dt, **kw)
    pb, _ = make_plan(device, np.asarray(x)[perm], N, 4, 2.0, dt, **kw)
    print("node order", dt, N, M, pa.info(), flush=True)
    assert pa.info()["spread"] == "tiled"
    pt = torch.as_tensor(perm, device=device)
    fd = to_dev(f, dt, device)
    assert torch.equal(pb.forward(fd), pa.forward(fd)[pt])
    fhd = to_dev(fh, dt, device)
    ya, yb = pa.adjoint(fhd).cpu().numpy(), pb.adjoint(fhd[pt].contiguous()).cpu().numpy()
    assert rel2(yb, ya) < e2e_tol(N, 2.0, 4, dt)
