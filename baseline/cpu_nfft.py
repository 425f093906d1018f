"""Plain CPU NFFT on all host cores: the C++/OpenMP steps of Algorithms 1 and 2 in
libcpu_nfft.so and the oversampled FFT by scipy.fft with one worker per core.

complex128 runs in FP64; complex64 in FP32 (grid, window values and FFT).  A timing
baseline for bench.py only.
"""
import ctypes
import os

import numpy as np
import scipy.fft

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.build())
        vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
        lib.cpu_nfft_plan.restype = vp
        lib.cpu_nfft_plan.argtypes = [ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64, vp,
                                      ctypes.c_int, ctypes.c_double]
        lib.cpu_nfft_free.argtypes = [ctypes.c_int, vp]
        lib.cpu_nfft_ntilde.argtypes = [ctypes.c_int, vp, i64p]
        for name in ("cpu_nfft_pad", "cpu_nfft_interp", "cpu_nfft_spread", "cpu_nfft_crop"):
            getattr(lib, name).argtypes = [ctypes.c_int, vp, vp, vp]
        lib.cpu_nfft_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads():
    """Threads the OpenMP steps use (the FFT uses as many workers)."""
    return int(_load().cpu_nfft_threads())


class CpuNfft:
    def __init__(self, x, N, m=4, sigma=2.0, dtype="c128"):
        self.lib = _load()
        self.dt = 1 if dtype == "c128" else 0
        self.cdt = np.complex128 if self.dt else np.complex64
        self.N = tuple(int(n) for n in N)
        self.D = len(self.N)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, self.D))
        self.M = x.shape[0]
        Narr = (ctypes.c_int64 * 3)(*(list(self.N) + [1] * (3 - self.D)))
        self.h = self.lib.cpu_nfft_plan(self.dt, self.D, Narr, self.M, x.ctypes.data, int(m),
                                        float(sigma))
        if not self.h:
            raise ValueError("cpu_nfft_plan: bad arguments")
        nt = (ctypes.c_int64 * 3)()
        self.lib.cpu_nfft_ntilde(self.dt, self.h, nt)
        self.Nt = tuple(int(v) for v in nt[:self.D])
        self.workers = threads()
        self.grid = np.empty(self.Nt, dtype=self.cdt)

    def forward(self, f):
        f = np.ascontiguousarray(f, dtype=self.cdt)
        out = np.empty(self.M, dtype=self.cdt)
        self.lib.cpu_nfft_pad(self.dt, self.h, f.ctypes.data, self.grid.ctypes.data)
        g = scipy.fft.fftn(self.grid, workers=self.workers, overwrite_x=True)
        self.lib.cpu_nfft_interp(self.dt, self.h, np.ascontiguousarray(g).ctypes.data, out.ctypes.data)
        return out

    def adjoint(self, fhat):
        fhat = np.ascontiguousarray(fhat, dtype=self.cdt)
        out = np.empty(self.N, dtype=self.cdt)
        self.lib.cpu_nfft_spread(self.dt, self.h, fhat.ctypes.data, self.grid.ctypes.data)
        # unnormalised inverse: ifftn scaled by |I_Nt|
        g = scipy.fft.ifftn(self.grid, workers=self.workers, norm="forward", overwrite_x=True)
        self.lib.cpu_nfft_crop(self.dt, self.h, np.ascontiguousarray(g).ctypes.data, out.ctypes.data)
        return out

    def close(self):
        if self.h:
            self.lib.cpu_nfft_free(self.dt, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
