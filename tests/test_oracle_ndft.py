"""Pins of the direct NDFT oracle against facts the definition fixes.

Paper, section "Mathematical Description", subsection NDFT: equations (NDFT) and
(NDFTH), the centred index set I_N, and the remark that only equispaced nodes
with a normalisation make the adjoint an inverse.
"""
import os

import numpy as np
import pytest

from oracle import ndft
import nfft_workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ndft_hand.txt")


def _centred(N):
    return [np.arange(-(n // 2), n - n // 2) for n in N]


def _dense_matrix(x, N):
    """Explicit NDFT matrix A[j, flat n] built from an explicit list of multi-indices."""
    grids = np.meshgrid(*_centred(N), indexing="ij")
    nvec = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.float64)  # (|I_N|, D)
    return np.exp(-2j * np.pi * (x @ nvec.T))


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def test_golden_hand_values():
    recs = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    arrays = {}
    for r in recs:
        if r[0].endswith("_f") or r[0].endswith("_fhat"):
            v = np.array([float(t) for t in r[1:]])
            arrays[r[0]] = v[0::2] + 1j * v[1::2]
    fA = arrays["A_f"]
    fB = arrays["B_f"].reshape(2, 2)
    adj_nodes = []
    for r in recs:
        if r[0] == "F":
            case = r[1]
            f = fA if case == "A" else fB
            D = f.ndim
            k = np.array([float(t) for t in r[2:2 + D]])
            want = float(r[2 + D]) + 1j * float(r[3 + D])
            got = ndft.ndft_forward(k[None, :], f)[0]
            assert abs(got - want) < 1e-14, (r, got)
            if case == "A":
                adj_nodes.append(k[0])
    y = ndft.ndft_adjoint(np.array(adj_nodes)[:, None], arrays["A_fhat"], (4,))
    for r in recs:
        if r[0] == "A":
            want = float(r[3]) + 1j * float(r[4])
            assert abs(y[int(r[2])] - want) < 1e-14, (r, y[int(r[2])])


@pytest.mark.parametrize("N", [(6,), (8,), (4, 6), (2, 4, 4), (5,), (3, 4), (3, 5, 2), (2, 3, 2, 3),
                               (2, 3, 2, 2, 3), (2, 2, 3, 2, 2, 2)])
def test_bruteforce_dense_matrix(N):
    D = len(N)
    x = wl.uniform_nodes(17, D, config=90, stream=0)
    f = wl.cn01(N, config=90, stream=1)
    fh = wl.cn01((17,), config=90, stream=2)
    A = _dense_matrix(x, N)
    assert _rel(ndft.ndft_forward(x, f), A @ f.reshape(-1)) < 1e-13
    y = ndft.ndft_adjoint(x, fh, N)
    assert _rel(y.reshape(-1), A.conj().T @ fh) < 1e-13


@pytest.mark.parametrize("N", [(16,), (8, 12), (4, 6, 8), (15,), (7, 6), (3, 5, 4), (3, 4, 2, 5),
                               (2, 3, 4, 2, 3), (2, 2, 3, 2, 2, 3)])
def test_equispaced_nodes_give_the_dft(N):
    """Nodes on the grid I_N / N: the NDFT is the centred DFT, the adjoint the unnormalised inverse."""
    D = len(N)
    grids = np.meshgrid(*[c / n for c, n in zip(_centred(N), N)], indexing="ij")
    x = np.stack([g.reshape(-1) for g in grids], axis=1)
    f = wl.cn01(N, config=91, stream=1)
    want = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(f)))
    got = ndft.ndft_forward(x, f).reshape(N)
    assert _rel(got, want) < 1e-13
    fh = wl.cn01(N, config=91, stream=2)
    want_adj = np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(fh))) * np.prod(N)
    got_adj = ndft.ndft_adjoint(x, fh.reshape(-1), N)
    assert _rel(got_adj, want_adj) < 1e-13
    # A^H A = |I_N| * identity on equispaced nodes
    back = ndft.ndft_adjoint(x, got.reshape(-1), N)
    assert _rel(back, np.prod(N) * f) < 1e-13


@pytest.mark.parametrize("N", [(10,), (6, 8), (4, 4, 6), (2, 3, 4, 2)])
def test_single_node_at_zero(N):
    D = len(N)
    x = np.zeros((1, D))
    f = wl.cn01(N, config=92, stream=1)
    assert abs(ndft.ndft_forward(x, f)[0] - f.sum()) < 1e-12
    y = ndft.ndft_adjoint(x, np.array([1.0 + 0j]), N)
    assert np.array_equal(y, np.ones(N, dtype=np.complex128))


@pytest.mark.parametrize("N", [(32,), (12, 10), (6, 8, 4)])
def test_adjoint_identity(N):
    D = len(N)
    x = wl.uniform_nodes(50, D, config=93, stream=0)
    f = wl.cn01(N, config=93, stream=1)
    yh = wl.cn01((50,), config=93, stream=2)
    lhs = np.vdot(yh, ndft.ndft_forward(x, f))
    rhs = np.vdot(ndft.ndft_adjoint(x, yh, N), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("N,axis,a", [((16,), 0, 3), ((8, 10), 1, -2), ((4, 6, 8), 0, 1)])
def test_shift_theorem(N, axis, a):
    """Shifting every node by a/N_d along d equals modulating f by exp(-2 pi i n_d a / N_d)."""
    D = len(N)
    x = wl.uniform_nodes(40, D, config=94, stream=0) * 0.5
    f = wl.cn01(N, config=94, stream=1)
    xs = x.copy()
    xs[:, axis] += a / N[axis]
    shape = [1] * D
    shape[axis] = N[axis]
    mod = np.exp(-2j * np.pi * _centred(N)[axis] * a / N[axis]).reshape(shape)
    assert _rel(ndft.ndft_forward(xs, f), ndft.ndft_forward(x, f * mod)) < 1e-12


def test_linearity_and_subset():
    N = (8, 8)
    x = wl.uniform_nodes(30, 2, config=95, stream=0)
    f1 = wl.cn01(N, config=95, stream=1)
    f2 = wl.cn01(N, config=95, stream=2)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lhs = ndft.ndft_forward(x, a * f1 + b * f2)
    rhs = a * ndft.ndft_forward(x, f1) + b * ndft.ndft_forward(x, f2)
    assert _rel(lhs, rhs) < 1e-13
    fh = wl.cn01((30,), config=95, stream=3)
    full = ndft.ndft_adjoint(x, fh, N).reshape(-1)
    idx = np.array([0, 5, 17, 63])
    assert np.allclose(ndft.ndft_adjoint(x, fh, N, idx=idx), full[idx], rtol=0, atol=1e-13)


def test_empty_node_set():
    N = (8,)
    x = np.zeros((0, 1))
    assert ndft.ndft_forward(x, np.ones(N, complex)).shape == (0,)
    assert np.array_equal(ndft.ndft_adjoint(x, np.zeros(0, complex), N), np.zeros(N, complex))
