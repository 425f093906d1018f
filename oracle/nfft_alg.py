"""Plain FP64 NFFT following the paper's Algorithms 1 and 2 (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the GPU library.
It is pinned against the direct NDFT (``oracle.ndft``) and against closed forms
in ``tests/test_oracle_*.py``.

Notation (paper, section "Mathematical Description"):

* ``N``   equispaced size, ``Nt`` = oversampled size (Ntilde = sigma * N),
* ``m``   window half-width; the truncated window has support [-m/Nt, m/Nt),
* nodes ``x`` (the paper's k_j) in T^D = [-1/2, 1/2)^D, node-major (J, D),
* coefficients ``f`` on the centred index set I_N, stored row-major with
  storage index i_d = n_d + N_d/2.

Window (the paper names the Kaiser-Bessel pair without formulas; this is the
notation of its reference for the NFFT): Kaiser-Bessel with shape parameter
beta_d = pi * m * (2 - 1/sigma_d), sigma_d = Nt_d / N_d.

* convolution side, psi_hat_Base(u) = sinh(beta sqrt(1-u^2)) / (pi sqrt(1-u^2))
  on u in [-1, 1), zero outside (truncation, equation (approxTrunc));
* deconvolution side, phi_Base(xi) = I0(sqrt(beta^2 - 4 pi^2 xi^2)), the Fourier
  transform of the untruncated psi_hat_Base.

Resampling stencil (reading of the index set I_{Nt,m}(k)): for a node with
Nt*x = c + frac, c = floor(Nt*x), frac in [0, 1), the 2m taps are the grid
points l = c - m + 1 + t, t = 0..2m-1, with window argument
u_t = (Nt*x - l)/m = (frac + m - 1 - t)/m in [-1, 1); storage index l mod Nt
(DC-first FFT order, the fftshift of the resampling-correction subsection folded
into the index map).
"""
import numpy as np
import scipy.special

# ---------------------------------------------------------------------------
# sizes and window


def oversampled_size(N, sigma):
    """Ntilde_d: smallest even integer >= sigma*N_d whose prime factors lie in {2, 3, 5}.

    The paper sets Ntilde = sigma * N (subsection NFFT) without saying how a
    non-integer product is rounded; this rule keeps Ntilde an FFT-friendly even
    integer and is exact for every configuration used here.
    """
    out = []
    for n in np.atleast_1d(N):
        target = float(sigma) * int(n)
        cand = int(np.ceil(target - 1e-9 * target))
        cand += cand % 2
        while True:
            r = cand
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                break
            cand += 2
        out.append(cand)
    return tuple(out)


def kb_beta(m, sigma_d):
    """Kaiser-Bessel shape parameter beta = pi m (2 - 1/sigma)."""
    return np.pi * m * (2.0 - 1.0 / sigma_d)


def window_hat(u, beta):
    """psi_hat_Base(u): sinh form on [-1, 1), zero outside; limit beta/pi where sqrt(1-u^2)=0."""
    u = np.asarray(u, dtype=np.float64)
    s = np.sqrt(np.clip(1.0 - u * u, 0.0, None))
    with np.errstate(invalid="ignore", divide="ignore"):
        val = np.where(s > 0, np.sinh(beta * s) / (np.pi * np.where(s > 0, s, 1.0)), beta / np.pi)
    inside = (u >= -1.0) & (u < 1.0)
    return np.where(inside, val, 0.0)


def window_hat_full(u, beta):
    """phi_hat_Base(u): the Fourier transform of phi_Base on the whole line -- the sinh form
    for |u| < 1, beta/pi at |u| = 1, its continuation sin(beta sqrt(u^2-1)) / (pi sqrt(u^2-1))
    for |u| > 1.  The (2m+2)-tap stencil samples it beyond the truncation interval."""
    u = np.asarray(u, dtype=np.float64)
    q = 1.0 - u * u
    r = np.sqrt(np.abs(q))
    with np.errstate(invalid="ignore", divide="ignore"):
        inner = np.sinh(beta * r) / (np.pi * np.where(r > 0, r, 1.0))
        outer = np.sin(beta * r) / (np.pi * np.where(r > 0, r, 1.0))
    return np.where(r == 0, beta / np.pi, np.where(q > 0, inner, outer))


def window_phi(xi, beta):
    """phi_Base(xi) = I0(sqrt(beta^2 - 4 pi^2 xi^2)) for |2 pi xi| <= beta."""
    xi = np.asarray(xi, dtype=np.float64)
    arg = beta * beta - (2.0 * np.pi * xi) ** 2
    if np.any(arg < 0):
        raise ValueError("phi_Base evaluated outside [-beta/2pi, beta/2pi]")
    return scipy.special.i0(np.sqrt(arg))


def deconv_factors(N_d, Nt_d, m):
    """beta_tensor_d[n_d] = 1 / (m * phi_Base(m n_d / Nt_d)), n_d in I_{N_d}.

    Resampling-correction subsection: the product over d equals 1/(|I_Nt| phi(n)).
    """
    beta = kb_beta(m, Nt_d / N_d)
    n = np.arange(-(N_d // 2), N_d - N_d // 2, dtype=np.float64)
    return 1.0 / (m * window_phi(m * n / Nt_d, beta))


def poly_coeffs(m, beta, Z=None, Theta=None, wide=False):
    """Piecewise-polynomial window approximation (POLYNOMIAL precomputation).

    For each tap t = 0..2m-1 a polynomial P_t of degree Z-1 (default 2m) in
    zeta = frac - 1/2 in [-1/2, 1/2] is fitted by least squares to Theta = 2Z
    equispaced samples of psi_hat_Base((zeta + m - 1/2 - t)/m); returns
    mu[t, z] so that P_t(zeta) = sum_z mu[t, z] zeta^z.  The continuous sinh form
    is sampled (its value at |u| = 1 is the limit beta/pi).  wide: the 2m+2 taps
    t = 0..2m+1 of the (2m+2)-point stencil, samples of phi_hat_Base((zeta + m +
    1/2 - t)/m) (beyond |u| = 1 the sin continuation).
    """
    Z = 2 * m + 1 if Z is None else Z
    Theta = 2 * Z if Theta is None else Theta
    zeta = -0.5 + np.arange(Theta) / (Theta - 1.0)
    V = zeta[:, None] ** np.arange(Z)[None, :]
    taps, lo = (2 * m + 2, m) if wide else (2 * m, m - 1)
    mu = np.zeros((taps, Z))
    for t in range(taps):
        u = (zeta + lo + 0.5 - t) / m
        if wide:
            b = window_hat_full(u, beta)
        else:
            s = np.sqrt(np.clip(1.0 - u * u, 0.0, None))
            b = np.where(s > 0, np.sinh(beta * s) / (np.pi * np.where(s > 0, s, 1.0)), beta / np.pi)
        mu[t] = np.linalg.lstsq(V, b, rcond=None)[0]
    return mu


# Exponents of the linear-interpolation table sizes for the Kaiser-Bessel window, m = 1..8
# (LINEAR item of subsection "Window precomputation": S = m 2^{c_min(m,8)} + 2).
LINEAR_C = (3, 7, 9, 14, 17, 20, 23, 24)


def linear_table_size(m):
    """S = m 2^{c_min(m,8)} + 2 table entries."""
    return m * 2 ** LINEAR_C[min(m, 8) - 1] + 2


def linear_table(m, beta):
    """Lookup table psi_s = psi_hat_Base(s / (S - 2)), s = 0..S-1.  Entry S-2 (|u| = 1) is
    the sinh form's limit beta/pi, the value the half-open support gives at u = -1 (the only
    tap with |u| = 1); entry S-1 lies outside the support and is 0."""
    S = linear_table_size(m)
    u = np.arange(S) / (S - 2.0)
    s = np.sqrt(np.clip(1.0 - u * u, 0.0, None))
    with np.errstate(invalid="ignore", divide="ignore"):
        val = np.where(s > 0, np.sinh(beta * s) / (np.pi * np.where(s > 0, s, 1.0)), beta / np.pi)
    val[S - 1] = 0.0
    return val


def linear_lookup(u, table):
    """psi_hat_Base(u) by linear interpolation in the table: kappa = |u| (S - 2),
    s = floor(kappa), alpha = kappa - s, value psi_s + alpha (psi_{s+1} - psi_s)."""
    S = table.shape[0]
    kappa = np.abs(np.asarray(u, dtype=np.float64)) * (S - 2)
    s = np.floor(kappa).astype(np.int64)
    alpha = kappa - s
    return table[s] + alpha * (table[s + 1] - table[s])


def tap_weights(frac, m, beta, window="poly", wide=False):
    """Window weights for the 2m taps of nodes with fractional offset ``frac``; shape (..., 2m).

    window: "poly" (POLYNOMIAL), "direct" (no precomputation) or "linear" (LINEAR table
    lookup); the paper's TENSOR and FULL modes store "poly" weights and so compute the same.
    wide: the 2m+2 taps of the (2m+2)-point stencil, tap t at u = (frac + m - t)/m, with
    the untruncated window phi_hat_Base ("Window Size Considerations").
    """
    frac = np.asarray(frac, dtype=np.float64)
    taps, lo = (2 * m + 2, m) if wide else (2 * m, m - 1)
    t = np.arange(taps)
    u = (frac[..., None] + lo - t) / m
    if window == "direct":
        return window_hat_full(u, beta) if wide else window_hat(u, beta)
    if window == "poly":
        mu = poly_coeffs(m, beta, wide=wide)
        zeta = frac - 0.5
        powers = zeta[..., None] ** np.arange(mu.shape[1])
        return powers @ mu.T
    if window == "linear" and not wide:
        return linear_lookup(u, linear_table(m, beta))
    raise ValueError("window must be 'poly', 'direct' or 'linear' (not wide)")


# ---------------------------------------------------------------------------
# the two transforms


def _wrap(x):
    x = np.asarray(x, dtype=np.float64)
    return x - np.floor(x + 0.5)


def _stencil(x, Nt, m, wide=False):
    """Per node and axis: stencil origin c - m + 1 (wide: c - m; unwrapped) and frac."""
    y = _wrap(x) * np.asarray(Nt, dtype=np.float64)[None, :]
    c = np.floor(y)
    return (c - (m if wide else m - 1)).astype(np.int64), y - c


def _band_index(N_d, Nt_d):
    """Storage index (n mod Nt) on the oversampled grid of each n in I_{N_d}, in storage order."""
    n = np.arange(-(N_d // 2), N_d - N_d // 2)
    return np.mod(n, Nt_d)


def _weights_per_axis(x, N, Nt, m, window, wide=False):
    origin, frac = _stencil(x, Nt, m, wide)
    ws = []
    for d in range(len(N)):
        beta = kb_beta(m, Nt[d] / N[d])
        ws.append(tap_weights(frac[:, d], m, beta, window, wide))
    return origin, ws


def forward(x, f, m=4, sigma=2.0, Nt=None, window="poly", return_steps=False, wide=False):
    """Direct NFFT, Algorithm 1 (resampling correction, FFT, resampling); wide: the
    (2m+2)-point stencil."""
    f = np.asarray(f, dtype=np.complex128)
    N = f.shape
    D = len(N)
    Nt = oversampled_size(N, sigma) if Nt is None else tuple(Nt)
    x = np.asarray(x, dtype=np.float64).reshape(-1, D)

    # step 1: g_n = f_n / (|I_Nt| phi(n)) on I_N, zero elsewhere, stored at n mod Nt
    g = np.zeros(Nt, dtype=np.complex128)
    scale = np.ones(N)
    for d in range(D):
        shape = [1] * D
        shape[d] = N[d]
        scale = scale * deconv_factors(N[d], Nt[d], m).reshape(shape)
    g[np.ix_(*[_band_index(N[d], Nt[d]) for d in range(D)])] = f * scale

    # step 2: ghat_l = sum_n g_n exp(-2 pi i n.l/Nt)  (unnormalised)
    ghat = np.fft.fftn(g)

    # step 3: fhat_j = sum over the (2m)^D stencil of prod_d w_d * ghat[l mod Nt]
    fhat = resample_forward(x, ghat, N, m, Nt, window, wide)
    if return_steps:
        return fhat, {"g": g, "ghat": ghat, "Nt": Nt}
    return fhat


def adjoint(x, fhat, N, m=4, sigma=2.0, Nt=None, window="poly", return_steps=False, wide=False):
    """Adjoint NFFT, Algorithm 2 (adjoint resampling, adjoint FFT, resampling correction);
    wide: the (2m+2)-point stencil."""
    N = tuple(int(v) for v in N)
    D = len(N)
    Nt = oversampled_size(N, sigma) if Nt is None else tuple(Nt)
    x = np.asarray(x, dtype=np.float64).reshape(-1, D)
    fhat = np.asarray(fhat, dtype=np.complex128).reshape(-1)
    G = int(np.prod(Nt))

    # step 1: ghat_l = sum_j fhat_j psi_tilde(x_j - l/Nt)
    ghat = resample_adjoint(x, fhat, N, m, Nt, window, wide)

    # step 2: g_n = sum_l ghat_l exp(+2 pi i n.l/Nt)  (unnormalised)
    g = np.fft.ifftn(ghat) * G

    # step 3: y_n = g_n / (|I_Nt| phi(n)) for n in I_N
    y = g[np.ix_(*[_band_index(N[d], Nt[d]) for d in range(D)])]
    for d in range(D):
        shape = [1] * D
        shape[d] = N[d]
        y = y * deconv_factors(N[d], Nt[d], m).reshape(shape)
    if return_steps:
        return y, {"ghat": ghat, "g": g, "Nt": Nt}
    return y


def resample_forward(x, ghat, N, m, Nt, window="poly", wide=False):
    """Resampling of Algorithm 1 (step 3): fhat_j = sum_l ghat_l psi_tilde(x_j - l/Nt).

    ``ghat`` is the oversampled grid in storage order (index l mod Nt).
    """
    N = tuple(int(v) for v in N)
    D = len(N)
    Nt = tuple(int(v) for v in Nt)
    x = np.asarray(x, dtype=np.float64).reshape(-1, D)
    origin, ws = _weights_per_axis(x, N, Nt, m, window, wide)
    J = x.shape[0]
    flat_g = np.asarray(ghat, dtype=np.complex128).reshape(-1)
    fhat = np.zeros(J, dtype=np.complex128)
    for taps in np.ndindex(*([ws[0].shape[1]] * D)):
        w = np.ones(J)
        flat = np.zeros(J, dtype=np.int64)
        for d in range(D):
            w = w * ws[d][:, taps[d]]
            flat = flat * Nt[d] + np.mod(origin[:, d] + taps[d], Nt[d])
        fhat += w * flat_g[flat]
    return fhat


def resample_adjoint(x, fhat, N, m, Nt, window="poly", wide=False):
    """Adjoint resampling of Algorithm 2 (step 1): ghat_l = sum_j fhat_j psi_tilde(x_j - l/Nt).

    Every node adds fhat_j times the product of its per-axis tap weights to each grid point
    of its stencil.  The additions of a chunk of nodes (all their taps at once) are summed by
    one ``bincount`` over the grid -- the same sum as a loop over the nodes, accumulated in
    another order (which only moves rounding).
    """
    N = tuple(int(v) for v in N)
    D = len(N)
    Nt = tuple(int(v) for v in Nt)
    x = np.asarray(x, dtype=np.float64).reshape(-1, D)
    fhat = np.asarray(fhat, dtype=np.complex128).reshape(-1)
    origin, ws = _weights_per_axis(x, N, Nt, m, window, wide)
    J = x.shape[0]
    T = ws[0].shape[1] if D else 0
    G = int(np.prod(Nt))
    acc_re = np.zeros(G)
    acc_im = np.zeros(G)
    chunk = max(1, (1 << 24) // T ** D)
    for s in range(0, J, chunk):
        n = min(chunk, J - s)
        flat = np.zeros((n,) + (1,) * D, dtype=np.int64)
        w = np.ones((n,) + (1,) * D)
        for d in range(D):
            shape = [n] + [1] * D
            shape[1 + d] = T
            idx = np.mod(origin[s:s + n, d][:, None] + np.arange(T)[None, :], Nt[d])
            flat = flat * Nt[d] + idx.reshape(shape)
            w = w * ws[d][s:s + n].reshape(shape)
        v = (w * fhat[s:s + n].reshape((n,) + (1,) * D)).ravel()
        flat = np.broadcast_to(flat, (n,) + (T,) * D).ravel()
        acc_re += np.bincount(flat, weights=v.real, minlength=G)
        acc_im += np.bincount(flat, weights=v.imag, minlength=G)
    return (acc_re + 1j * acc_im).reshape(Nt)
