"""Direct NDFT oracle in FP64 (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the GPU library.

Definitions (paper, section "Mathematical Description", subsection NDFT):

* forward / type 2, equation (NDFT):  fhat_j = sum_{n in I_N} f_n e^{-2 pi i n.k_j}
* adjoint / type 1, equation (NDFTH): y_n = sum_j fhat_j e^{+2 pi i n.k_j}

I_N is the centred index set of the same subsection: n_d = -N_d/2 .. N_d/2-1 for
even N_d.  Arrays are C row-major with storage index i_d = n_d + N_d/2.
"""
import ctypes

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.ndft_forward.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, dp, dp]
        lib.ndft_forward.restype = ctypes.c_int
        lib.ndft_adjoint_subset.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, dp,
                                            ctypes.c_int64, i64p, dp]
        lib.ndft_adjoint_subset.restype = ctypes.c_int
        lib.ndft_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _prep(x, N):
    N = np.ascontiguousarray(np.asarray(N, dtype=np.int64).reshape(-1))
    D = N.size
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, D))
    return x, N, D


def ndft_forward(x, f):
    """fhat_j = sum_n f_n exp(-2 pi i n . x_j); f has shape N (centred, row-major)."""
    f = np.asarray(f)
    x, N, D = _prep(x, f.shape)
    J = x.shape[0]
    fc = np.ascontiguousarray(f, dtype=np.complex128)
    out = np.zeros(J, dtype=np.complex128)
    rc = _load().ndft_forward(D, _ptr(N, ctypes.c_int64), J, _ptr(x, ctypes.c_double),
                              _ptr(fc.view(np.float64), ctypes.c_double),
                              _ptr(out.view(np.float64), ctypes.c_double))
    if rc != 0:
        raise ValueError("ndft_forward: bad arguments")
    return out


def ndft_adjoint(x, fhat, N, idx=None):
    """y_n = sum_j fhat_j exp(+2 pi i n . x_j).

    With ``idx`` (flat storage indices) only those outputs are computed and a
    1-D array is returned; otherwise the full array of shape N.
    """
    x, Nv, D = _prep(x, N)
    J = x.shape[0]
    fh = np.ascontiguousarray(np.asarray(fhat, dtype=np.complex128).reshape(-1))
    if fh.size != J:
        raise ValueError("fhat must have one value per node")
    full = idx is None
    if full:
        idx = np.arange(int(np.prod(Nv)), dtype=np.int64)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1))
    out = np.zeros(idx.size, dtype=np.complex128)
    rc = _load().ndft_adjoint_subset(D, _ptr(Nv, ctypes.c_int64), J, _ptr(x, ctypes.c_double),
                                     _ptr(fh.view(np.float64), ctypes.c_double), idx.size,
                                     _ptr(idx, ctypes.c_int64),
                                     _ptr(out.view(np.float64), ctypes.c_double))
    if rc != 0:
        raise ValueError("ndft_adjoint: bad arguments")
    return out.reshape(tuple(int(v) for v in Nv)) if full else out


def threads():
    """OpenMP threads the oracle uses."""
    return int(_load().ndft_threads())
