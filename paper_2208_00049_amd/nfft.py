"""Thin PyTorch-facing binding of libnfft (argument marshalling only).

Torch supplies device memory and the stream; every step of the transform runs
in the library's HIP kernels.  Names follow the paper's API (section
"Implementation", example usage): a plan built from the nodes and the size N,
then ``forward`` (p * f) and ``adjoint`` (adjoint(p) * fhat), with optional
output buffers (mul!), and the one-shot helpers ``nfft`` and ``nfft_adjoint``.
"""
import ctypes

import torch

from . import _lib

_CDTYPE = {_lib.NFFT_C64: torch.complex64, _lib.NFFT_C128: torch.complex128}
_RDTYPE = {_lib.NFFT_C64: torch.float32, _lib.NFFT_C128: torch.float64}


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """NFFT plan for nodes ``x`` (device tensor (M, D), float32 or float64) and size ``N``.

    float32 nodes give a complex64 plan (FP32 arithmetic), float64 nodes a
    complex128 plan.  ``tile``: optional per-axis tile edges; ``window``: the window
    evaluation, "poly" (default), "direct", "tensor", "linear" or "full" (the paper's
    precomputation options); ``max_block_nodes``: cap on nodes per resampling
    work item; ``tune``: if > 0 (and no tile is given), the library's autotuner
    picks the tiles, timing each candidate ``tune`` times (``tuned_ms`` then
    holds the chosen plan's forward + adjoint milliseconds); ``wide``: the (2m+2)-point
    stencil with the untruncated window; ``spread``: the 3-D spreading scheme, "auto"
    (column sweeps where available), "tiled" (padded tiles, exact fixed-point sums in
    both types) or "sweep".
    """

    def __init__(self, x, N, m=4, sigma=2.0, tile=None, window="poly", max_block_nodes=0, tune=0,
                 wide=False, spread="auto"):
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError("x must be a CUDA (HIP) tensor")
        N = tuple(int(v) for v in N)
        if x.dim() == 1 and len(N) == 1:
            x = x.reshape(-1, 1)
        if x.dim() != 2 or x.shape[1] != len(N):
            raise ValueError("x must have shape (M, D) with D = len(N)")
        if x.dtype == torch.float32:
            self.dtype = _lib.NFFT_C64
        elif x.dtype == torch.float64:
            self.dtype = _lib.NFFT_C128
        else:
            raise TypeError("x must be float32 or float64")
        self._lib = _lib.load()
        self.N = N
        self.D = len(N)
        self.M = int(x.shape[0])
        self.m = int(m)
        self.sigma = float(sigma)
        self.device = x.device
        self.cdtype = _CDTYPE[self.dtype]
        x = x.contiguous()
        opts = _lib.Options()
        if tile is not None:
            for d, q in enumerate(tile):
                opts.tile[d] = int(q)
        opts.window = _lib.WINDOWS[window]
        opts.max_block_nodes = int(max_block_nodes)
        opts.wide = int(bool(wide))
        opts.spread = _lib.SPREAD[spread]
        Narr = (ctypes.c_int64 * self.D)(*N)
        handle = ctypes.c_void_p()
        self.tuned_ms = None
        with torch.cuda.device(self.device):
            if tune and tile is None:
                ms = ctypes.c_double()
                rc = self._lib.nfft_plan_create_tuned(
                    ctypes.byref(handle), self.D, Narr, self.M, ctypes.c_void_p(x.data_ptr()),
                    self.m, self.sigma, self.dtype, ctypes.byref(opts), int(tune),
                    _stream_handle(self.device), ctypes.byref(ms))
                if rc == _lib.NFFT_OK:
                    self.tuned_ms = ms.value
            else:
                rc = self._lib.nfft_plan_create_ex(ctypes.byref(handle), self.D, Narr, self.M,
                                                   ctypes.c_void_p(x.data_ptr()), self.m,
                                                   self.sigma, self.dtype, ctypes.byref(opts),
                                                   _stream_handle(self.device))
        _lib.check(rc, "nfft_plan_create")
        self._h = handle

    # -- introspection -------------------------------------------------------
    def info(self):
        nt = (ctypes.c_int64 * self.D)()
        se = ctypes.c_double()
        tl = (ctypes.c_int * self.D)()
        _lib.check(self._lib.nfft_plan_info(self._h, nt, ctypes.byref(se), tl), "nfft_plan_info")
        sp = ctypes.c_int()
        _lib.check(self._lib.nfft_plan_spread(self._h, ctypes.byref(sp)), "nfft_plan_spread")
        return {"Ntilde": tuple(nt), "sigma_eff": se.value, "tile": tuple(tl),
                "spread": {v: k for k, v in _lib.SPREAD.items()}[sp.value]}

    @property
    def Ntilde(self):
        return self.info()["Ntilde"]

    def window_peaks(self):
        """Per-axis window peak sinh(beta_d)/pi the stored window is divided by."""
        pk = (ctypes.c_double * self.D)()
        _lib.check(self._lib.nfft_plan_window_peak(self._h, pk), "nfft_plan_window_peak")
        return tuple(pk)

    @property
    def window_scale(self):
        """C = product of the window peaks: the single steps use the window divided by C
        (``resample_forward`` / ``resample_adjoint`` return the paper's step over C) and the
        grid after ``forward`` holds C F D f."""
        c = 1.0
        for v in self.window_peaks():
            c *= v
        return c

    def grid(self):
        """Copy of the plan's oversampled grid (holds C F D f after ``forward``, C =
        ``window_scale``)."""
        ptr = ctypes.c_void_p()
        _lib.check(self._lib.nfft_plan_grid(self._h, ctypes.byref(ptr)), "nfft_plan_grid")
        out = torch.empty(self.Ntilde, dtype=self.cdtype, device=self.device)
        _copy_device(out.data_ptr(), ptr.value, out.numel() * out.element_size(), self.device)
        return out

    def set_timing(self, enable=True):
        """Record HIP events around every kernel of forward/adjoint (see stage_times)."""
        _lib.check(self._lib.nfft_plan_set_timing(self._h, int(bool(enable))), "nfft_plan_set_timing")

    def stage_times(self):
        """Milliseconds of each stage of the latest forward and adjoint call (dict by stage name)."""
        ms = (ctypes.c_double * _lib.NFFT_NUM_STAGES)()
        _lib.check(self._lib.nfft_plan_timing(self._h, ms), "nfft_plan_timing")
        return {name: ms[i] for i, name in enumerate(_lib.STAGES)}

    def bench_stage(self, stage, reps, fhat=None):
        """Mean milliseconds per launch of a resampling stage run `reps` times back to back:
        "interp" (writes a scratch fhat) or "spread" (reads `fhat`)."""
        idx = _lib.STAGES.index(stage)
        if stage == "spread":
            self._check(fhat, (self.M,), "fhat")
            inp, out = ctypes.c_void_p(fhat.data_ptr()), None
        elif stage == "interp":
            buf = torch.empty(self.M, dtype=self.cdtype, device=self.device)
            inp, out = None, ctypes.c_void_p(buf.data_ptr())
        else:
            raise ValueError("stage must be 'interp' or 'spread'")
        ms = ctypes.c_double()
        _lib.check(self._lib.nfft_plan_bench_stage(self._h, idx, int(reps), inp, out,
                                                   _stream_handle(self.device), ctypes.byref(ms)),
                   "nfft_plan_bench_stage")
        return ms.value

    # -- transforms ----------------------------------------------------------
    def _check(self, t, shape, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise TypeError("%s must be a tensor on %s" % (name, self.device))
        if t.dtype != self.cdtype:
            raise TypeError("%s must be %s" % (name, self.cdtype))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    def forward(self, f, out=None):
        """fhat = A f (Algorithm 1); f has shape N."""
        self._check(f, self.N, "f")
        if out is None:
            out = torch.empty(self.M, dtype=self.cdtype, device=self.device)
        self._check(out, (self.M,), "out")
        rc = self._lib.nfft_forward(self._h, ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream_handle(self.device))
        _lib.check(rc, "nfft_forward")
        return out

    def adjoint(self, fhat, out=None):
        """y = A^H fhat (Algorithm 2); fhat has shape (M,)."""
        self._check(fhat, (self.M,), "fhat")
        if out is None:
            out = torch.empty(self.N, dtype=self.cdtype, device=self.device)
        self._check(out, self.N, "out")
        rc = self._lib.nfft_adjoint(self._h, ctypes.c_void_p(fhat.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream_handle(self.device))
        _lib.check(rc, "nfft_adjoint")
        return out

    # -- multi-channel ---------------------------------------------------------
    def forward_many(self, f, out=None, noalloc=False):
        """K channels at once: f has shape (K, *N), the result (K, M).  With noalloc, the
        library's no-allocation variant (its K grids in the library's static device
        scratch; ``out`` must then be given, since allocating it would defeat the point)."""
        K = int(f.shape[0]) if f.dim() == self.D + 1 else -1
        self._check(f, (K,) + self.N, "f")
        if out is None:
            if noalloc:
                raise ValueError("forward_many(noalloc=True) needs an output buffer")
            out = torch.empty((K, self.M), dtype=self.cdtype, device=self.device)
        self._check(out, (K, self.M), "out")
        fn = self._lib.nfft_forward_many_noalloc if noalloc else self._lib.nfft_forward_many
        rc = fn(self._h, K, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                _stream_handle(self.device))
        _lib.check(rc, "nfft_forward_many_noalloc" if noalloc else "nfft_forward_many")
        return out

    def adjoint_many(self, fhat, out=None):
        """K channels at once: fhat has shape (K, M), the result (K, *N)."""
        K = int(fhat.shape[0]) if fhat.dim() == 2 else -1
        self._check(fhat, (K, self.M), "fhat")
        if out is None:
            out = torch.empty((K,) + self.N, dtype=self.cdtype, device=self.device)
        self._check(out, (K,) + self.N, "out")
        rc = self._lib.nfft_adjoint_many(self._h, K, ctypes.c_void_p(fhat.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(self.device))
        _lib.check(rc, "nfft_adjoint_many")
        return out

    # -- derivatives with respect to the nodes -----------------------------------
    def forward_deriv(self, f, out=None):
        """(D, M): entry [d, j] ~= sum_n (-2 pi i n_d) f_n exp(-2 pi i n.x_j)."""
        self._check(f, self.N, "f")
        if out is None:
            out = torch.empty((self.D, self.M), dtype=self.cdtype, device=self.device)
        self._check(out, (self.D, self.M), "out")
        rc = self._lib.nfft_forward_deriv(self._h, ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(self.device))
        _lib.check(rc, "nfft_forward_deriv")
        return out

    def node_grad(self, a, dfhat, out=None):
        """(M, D) reals: Re(conj(a_j) dfhat[d, j])."""
        self._check(a, (self.M,), "a")
        self._check(dfhat, (self.D, self.M), "dfhat")
        if out is None:
            out = torch.empty((self.M, self.D), dtype=_RDTYPE[self.dtype], device=self.device)
        rc = self._lib.nfft_node_grad(self._h, ctypes.c_void_p(a.data_ptr()),
                                      ctypes.c_void_p(dfhat.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(self.device))
        _lib.check(rc, "nfft_node_grad")
        return out

    # -- single steps ----------------------------------------------------------
    def resample_forward(self, grid, out=None):
        self._check(grid, self.Ntilde, "grid")
        if out is None:
            out = torch.empty(self.M, dtype=self.cdtype, device=self.device)
        self._check(out, (self.M,), "out")
        rc = self._lib.nfft_resample_forward(self._h, ctypes.c_void_p(grid.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()),
                                             _stream_handle(self.device))
        _lib.check(rc, "nfft_resample_forward")
        return out

    def resample_adjoint(self, fhat, out=None):
        self._check(fhat, (self.M,), "fhat")
        if out is None:
            out = torch.empty(self.Ntilde, dtype=self.cdtype, device=self.device)
        self._check(out, self.Ntilde, "out")
        rc = self._lib.nfft_resample_adjoint(self._h, ctypes.c_void_p(fhat.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()),
                                             _stream_handle(self.device))
        _lib.check(rc, "nfft_resample_adjoint")
        return out

    def fft_grid(self, grid, direction=-1):
        """Unnormalised in-place FFT of an oversampled grid (direction -1 or +1)."""
        self._check(grid, self.Ntilde, "grid")
        rc = self._lib.nfft_fft_grid(self._h, ctypes.c_void_p(grid.data_ptr()), int(direction),
                                     _stream_handle(self.device))
        _lib.check(rc, "nfft_fft_grid")
        return grid

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.nfft_plan_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent transforms of several plans (see nfft_batch_create): one kernel launch per
    stage for all of them when the plans share type, D <= 3, stencil and window (``info()``
    reports the mode and the launches per call), else their kernel chains in one HIP graph.

    ``forward(fs, outs)`` / ``adjoint(fhats, outs)`` take lists of tensors, one per plan, in
    the plans' order; keep the same tensors from call to call (new pointers cost a stream
    synchronisation, or a graph capture).
    """

    def __init__(self, plans, nstreams=4):
        self.plans = list(plans)
        self._lib = _lib.load()
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        handle = ctypes.c_void_p()
        _lib.check(self._lib.nfft_batch_create(ctypes.byref(handle), len(self.plans), arr,
                                               int(nstreams)), "nfft_batch_create")
        self._h = handle
        self.device = self.plans[0].device

    def _run(self, fn, ins, outs, in_shape, out_shape, name):
        n = len(self.plans)
        if len(ins) != n or len(outs) != n:
            raise ValueError("need one input and one output per plan")
        for p, a, b in zip(self.plans, ins, outs):
            p._check(a, in_shape(p), name + " input")
            p._check(b, out_shape(p), name + " output")
        inp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ins])
        out = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
        _lib.check(fn(self._h, inp, out, _stream_handle(self.device)), name)
        return outs

    def info(self):
        """{"fused": bool, "launches_forward": int, "launches_adjoint": int}"""
        f, lf, la = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _lib.check(self._lib.nfft_batch_info(self._h, ctypes.byref(f), ctypes.byref(lf),
                                             ctypes.byref(la)), "nfft_batch_info")
        return {"fused": bool(f.value), "launches_forward": lf.value,
                "launches_adjoint": la.value}

    def forward(self, fs, outs):
        return self._run(self._lib.nfft_batch_forward, fs, outs, lambda p: p.N, lambda p: (p.M,),
                         "nfft_batch_forward")

    def adjoint(self, fhats, outs):
        return self._run(self._lib.nfft_batch_adjoint, fhats, outs, lambda p: (p.M,),
                         lambda p: p.N, "nfft_batch_adjoint")

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.nfft_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_device(dst_ptr, src_ptr, nbytes, device):
    """Device-to-device copy of a library-owned buffer into a torch tensor."""
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p]
    hip.hipMemcpyAsync.restype = ctypes.c_int
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr),
                            ctypes.c_size_t(nbytes), 3, _stream_handle(device))
    if rc != 0:
        raise RuntimeError("hipMemcpyAsync failed (%d)" % rc)


def nfft(x, f, m=4, sigma=2.0, **kw):
    """One-shot forward NFFT: fhat_j ~= sum_n f_n exp(-2 pi i n.x_j)."""
    return Plan(x, tuple(f.shape), m=m, sigma=sigma, **kw).forward(f)


def nfft_adjoint(x, N, fhat, m=4, sigma=2.0, **kw):
    """One-shot adjoint NFFT: y_n ~= sum_j fhat_j exp(+2 pi i n.x_j)."""
    return Plan(x, tuple(N), m=m, sigma=sigma, **kw).adjoint(fhat)


def calibrate_lds(op, pattern=0, reps=20, device=None):
    """Lane operations per second of one LDS operation on the current device
    (``op``: a key of ``_lib.LDS_OPS``; ``pattern``: 0 consecutive, 1 random,
    2 eight-lane rows at random starts), measured by the library's kernel."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    out = ctypes.c_double()
    _lib.check(_lib.load().nfft_calibrate_lds(_lib.LDS_OPS[op], int(pattern), int(reps),
                                              _stream_handle(device), ctypes.byref(out)),
               "nfft_calibrate_lds")
    return out.value

