"""Pins of the plain FP64 NFFT oracle (Algorithms 1 and 2) against the direct NDFT.

The NFFT approximates the NDFT (paper, subsections "Direct NFFT", "Adjoint NFFT");
its error decays exponentially in m (subsection "Algorithmic Complexity") and
saturates near machine precision at m = 8 for sigma = 2 (section "Results",
accuracy analysis).  The approximate pair is exactly adjoint, since
A ~= B F D and A^H ~= D^T F^H B^T (subsection "Matrix-Vector Notation").

Gates (relative l2 against the NDFT) come from the closed-form Kaiser-Bessel
error estimates -- aliasing 1/I0(2 pi m sqrt(1 - 1/sigma)), truncation
beta/sinh(beta) -- with margin for dimension and accumulation:
"""
import numpy as np
import pytest

from oracle import ndft
from oracle import nfft_alg as na
import nfft_workloads as wl

GATE = {(3, 2.0): 3e-5, (4, 2.0): 1e-6, (6, 2.0): 1e-9, (8, 2.0): 1e-12, (4, 1.25): 2e-4}

SHAPES = {1: ((256,), 512), 2: ((32, 32), 1024), 3: ((16, 16, 16), 4096)}


def _rel2(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


_cache = {}


def _case(D):
    if D not in _cache:
        N, M = SHAPES[D]
        x = wl.uniform_nodes(M, D, config=0, stream=0)
        f = wl.cn01(N, config=0, stream=1)
        fh = wl.cn01((M,), config=0, stream=2)
        _cache[D] = (N, x, f, fh, ndft.ndft_forward(x, f), ndft.ndft_adjoint(x, fh, N))
    return _cache[D]


def _errors(D, m, sigma, window="poly"):
    N, x, f, fh, ef, ea = _case(D)
    return (_rel2(na.forward(x, f, m, sigma, window=window), ef),
            _rel2(na.adjoint(x, fh, N, m, sigma, window=window), ea))


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("m,sigma", sorted(GATE))
def test_nfft_matches_ndft(D, m, sigma):
    ef, ea = _errors(D, m, sigma)
    assert ef < GATE[(m, sigma)] and ea < GATE[(m, sigma)], (ef, ea)


@pytest.mark.parametrize("D", [1, 2])
def test_direct_window_matches_ndft(D):
    for m, sigma in [(4, 2.0), (6, 2.0)]:
        ef, ea = _errors(D, m, sigma, window="direct")
        assert ef < GATE[(m, sigma)] and ea < GATE[(m, sigma)]


def test_error_decays_exponentially_in_m():
    e3 = max(_errors(2, 3, 2.0))
    e4 = max(_errors(2, 4, 2.0))
    e6 = max(_errors(2, 6, 2.0))
    assert e4 < e3 / 20 and e6 < e4 / 1000


@pytest.mark.parametrize("D,m,sigma", [(1, 4, 2.0), (2, 6, 2.0), (3, 4, 1.25)])
def test_approximate_pair_is_exactly_adjoint(D, m, sigma):
    N, x, f, fh, _, _ = _case(D)
    lhs = np.vdot(fh, na.forward(x, f, m, sigma))
    rhs = np.vdot(na.adjoint(x, fh, N, m, sigma), f)
    scale = np.linalg.norm(fh) * np.linalg.norm(na.forward(x, f, m, sigma))
    assert abs(lhs - rhs) < 1e-13 * scale


@pytest.mark.parametrize("N", [(32,), (16, 16)])
def test_grid_aligned_and_boundary_nodes(N):
    """Nodes with Nt*x integral (the tie case of the half-open support), at -1/2 and at 0."""
    D = len(N)
    Nt = na.oversampled_size(N, 2.0)
    g = wl.rng(96, 0)
    x = g.integers(-Nt[0] // 2, Nt[0] // 2, size=(60, D)) / np.asarray(Nt, float)
    x[0] = -0.5
    x[1] = 0.0
    f = wl.cn01(N, config=96, stream=1)
    fh = wl.cn01((60,), config=96, stream=2)
    assert _rel2(na.forward(x, f, 4, 2.0), ndft.ndft_forward(x, f)) < GATE[(4, 2.0)]
    assert _rel2(na.adjoint(x, fh, N, 4, 2.0), ndft.ndft_adjoint(x, fh, N)) < GATE[(4, 2.0)]


def test_nodes_outside_torus_are_wrapped():
    N = (16, 16)
    x = wl.uniform_nodes(40, 2, config=97, stream=0)
    f = wl.cn01(N, config=97, stream=1)
    a = na.forward(x, f, 4, 2.0)
    b = na.forward(x + np.array([1.0, -2.0]), f, 4, 2.0)
    assert _rel2(b, a) < 1e-13


def test_empty_node_set():
    N = (16,)
    x = np.zeros((0, 1))
    assert na.forward(x, np.ones(N, complex)).shape == (0,)
    assert np.array_equal(na.adjoint(x, np.zeros(0, complex), N), np.zeros(N, complex))


# --- planted mistakes: each plausible error in the oracle must fail a pin above ---

def _fails_pin(monkeypatch, target, replacement):
    monkeypatch.setattr(target[0], target[1], replacement)
    ef, ea = _errors(2, 4, 2.0)
    return ef > GATE[(4, 2.0)] or ea > GATE[(4, 2.0)]


def test_planted_fft_sign_is_caught(monkeypatch):
    G = 32 * 32 * 4
    assert _fails_pin(monkeypatch, (na.np.fft, "fftn"),
                      lambda a: np.fft.ifftn(a) * G)


def test_planted_stencil_offset_is_caught(monkeypatch):
    orig = na._stencil
    assert _fails_pin(monkeypatch, (na, "_stencil"),
                      lambda x, Nt, m, wide=False: (orig(x, Nt, m, wide)[0] - 1,
                                                    orig(x, Nt, m, wide)[1]))


def test_planted_deconv_scale_is_caught(monkeypatch):
    orig = na.deconv_factors
    assert _fails_pin(monkeypatch, (na, "deconv_factors"),
                      lambda N, Nt, m: orig(N, Nt, m) * m)


def test_planted_reversed_taps_are_caught(monkeypatch):
    orig = na.tap_weights
    assert _fails_pin(monkeypatch, (na, "tap_weights"),
                      lambda frac, m, beta, window="poly", wide=False:
                      orig(frac, m, beta, window, wide)[..., ::-1])


def test_planted_window_phi_frequency_is_caught(monkeypatch):
    import scipy.special
    def wrong(xi, beta):
        return scipy.special.i0(np.sqrt(beta * beta - (np.pi * np.asarray(xi)) ** 2))
    assert _fails_pin(monkeypatch, (na, "window_phi"), wrong)


def test_planted_axis_transpose_is_caught(monkeypatch):
    orig = na.forward
    N, x, f, fh, ef, _ = _case(2)
    bad = orig(x, f.T.copy(), 4, 2.0)
    assert _rel2(bad, ef) > GATE[(4, 2.0)]


@pytest.mark.parametrize("m,sigma,gate", [(2, 2.0, 3e-3), (4, 2.0, 2e-6)])
def test_linear_window_nfft_against_ndft(m, sigma, gate):
    """The LINEAR table sizes keep the window error below the NFFT error (2-D)."""
    N = (24, 32)
    x = wl.uniform_nodes(700, 2, config=70, stream=0)
    f = wl.cn01(N, config=70, stream=1)
    fh = wl.cn01((700,), config=70, stream=2)
    e_f = _rel2(na.forward(x, f, m, sigma, window="linear"), ndft.ndft_forward(x, f))
    e_a = _rel2(na.adjoint(x, fh, N, m, sigma, window="linear"), ndft.ndft_adjoint(x, fh, N))
    e_p = _rel2(na.forward(x, f, m, sigma, window="poly"), ndft.ndft_forward(x, f))
    assert e_f < gate and e_a < gate
    assert e_f < 2 * e_p + 1e-12


@pytest.mark.parametrize("m", [3, 4])
def test_wide_stencil_accuracy_ordering(m):
    """Window Size Considerations / Accuracy Analysis: 2m+2 taps with the untruncated window
    are more accurate than 2m taps at the same m, and less accurate than 2(m+1) taps
    (m increased by one)."""
    N = (24, 32)
    x = wl.uniform_nodes(600, 2, config=71, stream=0)
    f = wl.cn01(N, config=71, stream=1)
    fh = wl.cn01((600,), config=71, stream=2)
    ref_f, ref_a = ndft.ndft_forward(x, f), ndft.ndft_adjoint(x, fh, N)
    e = {}
    for key, mm, wide in [("2m", m, False), ("2m+2", m, True), ("2(m+1)", m + 1, False)]:
        e[key] = (_rel2(na.forward(x, f, mm, 2.0, wide=wide), ref_f),
                  _rel2(na.adjoint(x, fh, N, mm, 2.0, wide=wide), ref_a))
    for i in range(2):
        assert e["2(m+1)"][i] < e["2m+2"][i] < e["2m"][i], e


def test_wide_stencil_is_a_plain_sum_on_tiny_input():
    """Brute force: one node, the (2m+2)^D-term resampling sum written out by hand."""
    m, N, Nt = 2, (8,), (16,)
    x = np.array([[0.1234]])
    g = wl.cn01(Nt, config=72, stream=1)
    beta = na.kb_beta(m, 2.0)
    y = 16 * 0.1234
    c = np.floor(y)
    want = 0.0
    for l in range(int(c) - m, int(c) + m + 2):
        want += na.window_hat_full((y - l) / m, beta) * g[l % 16]
    got = na.resample_forward(x, g, N, m, Nt, window="direct", wide=True)[0]
    assert abs(got - want) < 1e-12 * abs(want)


@pytest.mark.parametrize("N", [(25,), (23, 31), (9, 10, 11)])
def test_odd_sizes_against_ndft(N):
    """Odd N (n = -(N-1)/2 .. (N-1)/2, subsection "NDFT"): the NFFT oracle meets the same gate."""
    D = len(N)
    x = wl.uniform_nodes(400, D, config=73, stream=0)
    f = wl.cn01(N, config=73, stream=1)
    fh = wl.cn01((400,), config=73, stream=2)
    assert _rel2(na.forward(x, f, 4, 2.0), ndft.ndft_forward(x, f)) < 1e-6
    assert _rel2(na.adjoint(x, fh, N, 4, 2.0), ndft.ndft_adjoint(x, fh, N)) < 1e-6


@pytest.mark.parametrize("N,m,gate", [((8, 8, 8, 8), 4, 1e-6), ((7, 6, 9, 8), 3, 3e-5)])
def test_four_dimensional_against_ndft(N, m, gate):
    """D = 4 (the method is dimension-agnostic, subsection "Direct NFFT"): the same gates,
    and the approximate pair stays exactly adjoint."""
    x = wl.uniform_nodes(300, 4, config=74, stream=0)
    f = wl.cn01(N, config=74, stream=1)
    fh = wl.cn01((300,), config=74, stream=2)
    y = na.forward(x, f, m, 2.0)
    a = na.adjoint(x, fh, N, m, 2.0)
    assert _rel2(y, ndft.ndft_forward(x, f)) < gate
    assert _rel2(a, ndft.ndft_adjoint(x, fh, N)) < gate
    assert abs(np.vdot(fh, y) - np.vdot(a, f)) < 1e-13 * np.linalg.norm(fh) * np.linalg.norm(y)


@pytest.mark.parametrize("N,m,gate", [((6, 6, 6, 6, 6), 3, 3e-5), ((5, 4, 6, 4, 3), 2, 3e-3),
                                      ((4, 4, 4, 4, 4, 4), 2, 3e-3)])
def test_five_and_six_dimensional_against_ndft(N, m, gate):
    """D = 5 and 6 (dimension-agnostic, subsection "Direct NFFT"): the NFFT oracle within the
    Kaiser-Bessel gates of its m against the NDFT, and the approximate pair exactly adjoint."""
    D = len(N)
    x = wl.uniform_nodes(200, D, config=75, stream=0)
    f = wl.cn01(N, config=75, stream=1)
    fh = wl.cn01((200,), config=75, stream=2)
    y = na.forward(x, f, m, 2.0)
    a = na.adjoint(x, fh, N, m, 2.0)
    assert _rel2(y, ndft.ndft_forward(x, f)) < gate
    assert _rel2(a, ndft.ndft_adjoint(x, fh, N)) < gate
    assert abs(np.vdot(fh, y) - np.vdot(a, f)) < 1e-13 * np.linalg.norm(fh) * np.linalg.norm(y)
