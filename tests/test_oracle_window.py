"""Pins of the oracle's Kaiser-Bessel window, deconvolution factors and polynomial fit.

Paper, subsection "Direct NFFT" (tensor-product window, phi as the inverse
Fourier transform of phi_hat, truncation to [-m/Nt, m/Nt)), subsection
"Resampling Correction" (beta_tensor factors) and the POLYNOMIAL item of the
"Window precomputation" subsection.
"""
import mpmath as mp
import numpy as np
import pytest
import scipy.special

from oracle import nfft_alg as na

mp.mp.dps = 30

CASES = [(4, 2.0), (6, 2.0), (8, 2.0), (4, 1.25)]


def _mp_window_hat(u, beta):
    s = mp.sqrt(1 - u * u)
    if s == 0:
        return beta / mp.pi
    return mp.sinh(beta * s) / (mp.pi * s)


@pytest.mark.parametrize("z", [0.0, 0.5, 3.0, 12.5, 25.1327, 37.6991, 47.0])
def test_i0_against_mpmath(z):
    assert abs(scipy.special.i0(z) / float(mp.besseli(0, z)) - 1) < 1e-14


@pytest.mark.parametrize("m,sigma", CASES)
def test_kb_fourier_pair(m, sigma):
    """psi_hat_Base on (-1, 1) is the Fourier transform of the compactly supported phi_Base.

    phi_Base(xi) = I0(sqrt(beta^2 - 4 pi^2 xi^2)) lives on |xi| <= beta/(2 pi); its
    transform is the sinh form inside |u| < 1 (a sin form outside, which the
    truncation to [-1, 1) drops).
    """
    beta = na.kb_beta(m, sigma)
    bmp = mp.mpf(beta)
    lim = bmp / (2 * mp.pi)
    for u in [0.0, 0.3, -0.55, 0.9, -0.999]:
        val = mp.quad(lambda xi: mp.besseli(0, mp.sqrt(max(bmp ** 2 - (2 * mp.pi * xi) ** 2, 0)))
                      * mp.cos(2 * mp.pi * u * xi), [-lim, 0, lim])
        got = na.window_hat(u, beta)
        assert abs(got / float(val) - 1) < 1e-13, (m, sigma, u)


# (m, sigma) -> relative accuracy the truncated quadrature reaches (aliasing and
# truncation estimates 1/I0(2 pi m sqrt(1 - 1/sigma)) and beta/sinh(beta), with margin)
QUAD_BOUND = {(4, 2.0): 2e-6, (6, 2.0): 5e-10, (8, 2.0): 2e-13, (4, 1.25): 2e-3}


@pytest.mark.parametrize("m,sigma,N", [(4, 2.0, 16), (6, 2.0, 12), (8, 2.0, 20), (4, 1.25, 16)])
def test_deconv_factor_quadrature(m, sigma, N):
    """Equation (expApprox) with the truncated window: for every n in I_N and node k,
    (1/(|I_Nt| phi(n))) sum_l psi_tilde(k - l/Nt) exp(-2 pi i n l/Nt) ~= exp(-2 pi i n k)."""
    Nt = na.oversampled_size((N,), sigma)[0]
    beta = na.kb_beta(m, Nt / N)
    fac = na.deconv_factors(N, Nt, m)
    n = np.arange(-(N // 2), N - N // 2)
    for k in [0.0, 0.1234, -0.5, 0.49, 3.0 / Nt]:
        l = np.arange(-Nt, 2 * Nt)  # enough periods to contain the support around k
        w = na.window_hat((Nt * k - l) / m, beta)
        approx = fac * (np.exp(-2j * np.pi * np.outer(n, l) / Nt) @ w)
        exact = np.exp(-2j * np.pi * n * k)
        err = np.max(np.abs(approx - exact))
        assert err < QUAD_BOUND[(m, sigma)], (k, err)


def test_window_half_open_support():
    beta = na.kb_beta(4, 2.0)
    v = na.window_hat(np.array([-1.0, -0.5, 0.0, 0.5, 1.0, 1.5, -1.5]), beta)
    assert v[0] == pytest.approx(beta / np.pi, rel=1e-15)
    assert v[4] == 0.0 and v[5] == 0.0 and v[6] == 0.0
    assert v[1] == pytest.approx(v[3], rel=1e-15)  # even inside the support
    assert v[2] == pytest.approx(np.sinh(beta) / np.pi, rel=1e-15)


@pytest.mark.parametrize("m,sigma,bound", [(4, 2.0, 3e-8), (6, 2.0, 1e-12), (8, 2.0, 3e-14),
                                           (4, 1.25, 1e-8)])
def test_polynomial_window_accuracy(m, sigma, bound):
    """Degree-2m polynomials reproduce the window well below the NFFT error (max-norm, relative)."""
    beta = na.kb_beta(m, sigma)
    frac = np.linspace(0.0, 1.0, 2001, endpoint=False)
    direct = na.tap_weights(frac, m, beta, "direct")
    poly = na.tap_weights(frac, m, beta, "poly")
    err = np.max(np.abs(direct - poly)) / np.max(np.abs(direct))
    assert err < bound, err


def test_tap_arguments_cover_the_support_once():
    """The 2m taps of a node sample the window at u_t = (frac + m - 1 - t)/m, all in [-1, 1)."""
    m = 4
    for frac in [0.0, 0.25, 0.999]:
        u = (frac + m - 1 - np.arange(2 * m)) / m
        assert np.all(u >= -1) and np.all(u < 1)
        assert np.allclose(np.diff(u), -1.0 / m)


@pytest.mark.parametrize("N,sigma,want", [((256,), 2.0, (512,)), ((128, 128, 128), 1.25, (160,) * 3),
                                          ((512, 512), 2.0, (1024, 1024)), ((100,), 1.5, (150,)),
                                          ((30,), 1.3, (40,))])
def test_oversampled_size_rule(N, sigma, want):
    assert na.oversampled_size(N, sigma) == want


# ---------------------------------------------------------------------------
# LINEAR precomputation (lookup table with linear interpolation)

def test_linear_table_size_matches_printed_example():
    """The paper prints S = 134217730 table entries for m = 8 (Kaiser-Bessel)."""
    assert na.linear_table_size(8) == 134217730
    assert [na.linear_table_size(m) for m in (1, 2, 4)] == [1 * 2 ** 3 + 2, 2 * 2 ** 7 + 2,
                                                            4 * 2 ** 14 + 2]


@pytest.mark.parametrize("m,sigma", [(2, 2.0), (4, 2.0), (4, 1.25)])
def test_linear_lookup_exact_at_samples_and_within_bound(m, sigma):
    beta = na.kb_beta(m, sigma)
    table = na.linear_table(m, beta)
    S = table.shape[0]
    # at the sample points the lookup is the window itself (alpha = 0)
    s = np.array([0, 1, 7, S // 3, S - 3])
    u = s / (S - 2.0)
    assert np.array_equal(na.linear_lookup(u, table), na.window_hat(u, beta))
    assert na.linear_lookup(np.array([-1.0]), table)[0] == beta / np.pi
    # between samples: |error| <= h^2/8 max|psi''| on the cell (h = 1/(S-2)); psi'' from
    # central differences of the exact window on a finer grid
    g = np.random.default_rng(3)
    uu = g.uniform(-0.999, 0.999, 4000)
    h = 1.0 / (S - 2)
    d = h / 4

    def psi2(v):
        return np.abs(na.window_hat(v + d, beta) - 2 * na.window_hat(v, beta)
                      + na.window_hat(v - d, beta)) / d ** 2
    # max |psi''| over the cell, sampled at the cell's ends and the point
    lo = np.floor(np.abs(uu) / h) * h
    second = np.maximum(np.maximum(psi2(lo), psi2(lo + h)), psi2(np.abs(uu)))
    err = np.abs(na.linear_lookup(uu, table) - na.window_hat(uu, beta))
    assert np.all(err <= 1.5 * h * h / 8 * second + 1e-14 * na.window_hat(0.0, beta))
    # symmetric in u
    assert np.array_equal(na.linear_lookup(uu, table), na.linear_lookup(-uu, table))


@pytest.mark.parametrize("m,sigma", [(4, 2.0), (3, 2.0)])
def test_kb_fourier_pair_beyond_the_support(m, sigma):
    """phi_hat_Base for |u| > 1 (sampled by the (2m+2)-tap stencil) is the same Fourier
    integral of phi_Base: the sin continuation of the sinh form."""
    beta = na.kb_beta(m, sigma)
    bmp = mp.mpf(beta)
    lim = bmp / (2 * mp.pi)
    peak = na.window_hat_full(0.0, beta)
    for u in [1.05, -1.2, 1.3, 0.5]:
        val = mp.quad(lambda xi: mp.besseli(0, mp.sqrt(max(bmp ** 2 - (2 * mp.pi * xi) ** 2, 0)))
                      * mp.cos(2 * mp.pi * u * xi), [-lim, 0, lim])
        got = na.window_hat_full(u, beta)
        # relative to the window's peak: the tail values are ~1/sinh(beta) of it
        assert abs(got - float(val)) <= 1e-13 * peak, (m, sigma, u)
    assert na.window_hat_full(1.0, beta) == beta / np.pi


@pytest.mark.parametrize("m", [3, 4])
def test_poly_fit_samples_the_sinh_limit_at_u_plus_one(m):
    """Reading of the POLYNOMIAL fit's samples.  Tap 0's last sample lies at zeta = +1/2,
    i.e. u = +1, just outside the half-open support, where the truncated window is 0.  The
    oracle samples the continuous sinh form there (its limit beta/pi), so that tap 0's
    polynomial stays close to the window on [-1/2, 1/2) up to the excluded endpoint.
    Pinned by the mathematics: the NFFT error against the direct NDFT is lower than with the
    literal truncated sample (planted here), at m = 3 and m = 4."""
    import nfft_workloads as wl
    from oracle import ndft
    sigma = 2.0
    N, M = (32, 32), 2000
    x = wl.uniform_nodes(M, 2, config=90, stream=0)
    f = wl.cn01(N, config=90, stream=1)
    exact = ndft.ndft_forward(x, f)
    beta = na.kb_beta(m, 2.0)
    mu = na.poly_coeffs(m, beta)
    # tap 0 at zeta = +1/2 reproduces the sinh limit to within the fit error
    p0 = np.polynomial.polynomial.polyval(0.5, mu[0])
    peak = np.sinh(beta) / np.pi
    assert abs(p0 - beta / np.pi) < 1e-6 * peak

    def err():
        fh = na.forward(x, f, m, sigma)
        return np.linalg.norm(fh - exact) / np.linalg.norm(exact)

    ours = err()
    Z = 2 * m + 1
    zeta = -0.5 + np.arange(2 * Z) / (2 * Z - 1.0)
    V = zeta[:, None] ** np.arange(Z)[None, :]

    def literal(mm, b, **kw):
        out = np.zeros((2 * mm, Z))
        for t in range(2 * mm):
            u = (zeta + mm - 0.5 - t) / mm
            out[t] = np.linalg.lstsq(V, na.window_hat(u, b), rcond=None)[0]
        return out

    orig = na.poly_coeffs
    try:
        na.poly_coeffs = literal
        planted = err()
    finally:
        na.poly_coeffs = orig
    assert ours < planted, (ours, planted)
