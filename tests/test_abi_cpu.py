"""The C-ABI library loads, exports every declared symbol, and validates its
arguments before any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nfft.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2208_00049_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2208_00049_amd import build
        build.build()
    return _lib.load()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(nfft_\w+)\(", text, re.M)))


def test_header_declares_the_plan_api():
    names = _declared()
    for want in ["nfft_plan_create", "nfft_forward", "nfft_adjoint", "nfft_plan_destroy"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2208_00049_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def _create(lib, D=2, N=(64, 64), M=10, x=None, m=4, sigma=2.0, dtype=0, opts=None):
    h = ctypes.c_void_p()
    Narr = (ctypes.c_int64 * max(1, len(N)))(*N) if N is not None else None
    return lib.nfft_plan_create_ex(ctypes.byref(h), D, Narr, M, x, m, sigma, dtype, opts, None), h


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,code", [
    (dict(D=0), -1), (dict(D=7, N=(8,) * 7), -2), (dict(N=None), -1),
    (dict(M=-1), -1), (dict(M=5, x=None), -1), (dict(m=0, x=FAKE), -1), (dict(m=11, x=FAKE), -2),
    (dict(sigma=1.0, x=FAKE), -1), (dict(sigma=float("nan"), x=FAKE), -1),
    (dict(dtype=7, x=FAKE), -1), (dict(D=7, N=(8,) * 7, x=FAKE), -2), (dict(N=(1, 64), x=FAKE), -1),
    (dict(D=6, N=(8,) * 6, m=5, x=FAKE), -1),  # Ntilde = 16 < twice the stencil of m = 5
    (dict(D=4, N=(8, 8, 8, 1), x=FAKE), -1), (dict(D=4, N=(8, 8, 8, 4), m=4, x=FAKE), -1),
    (dict(N=(4, 64), m=4, x=FAKE), -1), (dict(N=(4096, 64), x=FAKE), -2),
])
def test_argument_errors_without_gpu(lib, kw, code):
    rc, h = _create(lib, **kw)
    assert rc == code
    assert not h.value


def test_option_errors(lib):
    from paper_2208_00049_amd import _lib
    o = _lib.Options()
    o.window = 5
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -1
    o = _lib.Options()
    o.reserved[0] = 1
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -1
    o = _lib.Options()
    o.tile[2] = 8  # axis beyond D
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -1
    o = _lib.Options()
    o.tile[3] = 8
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -1
    o = _lib.Options()
    o.tile[0] = 8  # the options' four tile edges do not reach D = 5: automatic tiles only
    assert _create(lib, D=5, N=(8,) * 5, M=0, opts=ctypes.byref(o))[0] == -2
    o = _lib.Options()
    o.wide = 1  # D >= 4: D * taps <= 128 (6 * 22 is not)
    assert _create(lib, D=6, N=(64,) * 6, M=0, m=10, opts=ctypes.byref(o))[0] == -2
    o = _lib.Options()
    o.window = _lib.NFFT_WINDOW_FULL  # (2m)^D products per node: D <= 2 only
    assert _create(lib, D=3, N=(16, 16, 16), M=0, opts=ctypes.byref(o))[0] == -2
    assert _create(lib, D=4, N=(8, 8, 8, 8), M=0, opts=ctypes.byref(o))[0] == -2
    o = _lib.Options()
    o.wide = 2
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -1
    o = _lib.Options()
    o.wide = 1
    o.window = _lib.NFFT_WINDOW_LINEAR  # the table does not reach beyond |u| = 1
    assert _create(lib, M=0, opts=ctypes.byref(o))[0] == -2


def test_null_plan_calls(lib):
    assert lib.nfft_forward(None, FAKE, FAKE, None) == -1
    assert lib.nfft_adjoint(None, FAKE, FAKE, None) == -1
    assert lib.nfft_plan_destroy(None) == 0
    assert lib.nfft_plan_info(None, None, None, None) == -1
    ms = ctypes.c_double()
    assert lib.nfft_plan_bench_stage(None, 3, 1, None, FAKE, None, ctypes.byref(ms)) == -1
    assert lib.nfft_forward_many(None, 2, FAKE, FAKE, None) == -1
    assert lib.nfft_adjoint_many(None, 2, FAKE, FAKE, None) == -1
    assert lib.nfft_batch_forward(None, None, None, None) == -1
    assert lib.nfft_batch_destroy(None) == 0


def test_batch_and_tuner_argument_errors(lib):
    """Rejected before any HIP call: empty batch, null plan, stream count, bad plan arguments."""
    out = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 2)(None, None)
    assert lib.nfft_batch_create(ctypes.byref(out), 0, plans, 1) == -1
    assert lib.nfft_batch_create(ctypes.byref(out), 2, plans, 1) == -1
    assert lib.nfft_batch_create(ctypes.byref(out), 2, plans, 0) == -1
    N = (ctypes.c_int64 * 2)(64, 64)
    ms = ctypes.c_double()
    # sigma <= 1, D > 4, reps < 1
    assert lib.nfft_plan_create_tuned(ctypes.byref(out), 2, N, 0, None, 4, ctypes.c_double(1.0), 0,
                                      None, 2, None, ctypes.byref(ms)) == -1
    N7 = (ctypes.c_int64 * 7)(8, 8, 8, 8, 8, 8, 8)
    assert lib.nfft_plan_create_tuned(ctypes.byref(out), 7, N7, 0, None, 4, ctypes.c_double(2.0),
                                      0, None, 2, None, ctypes.byref(ms)) == -2
    assert lib.nfft_plan_create_tuned(ctypes.byref(out), 2, N, 0, None, 4, ctypes.c_double(2.0), 0,
                                      None, 0, None, ctypes.byref(ms)) == -1
    assert lib.nfft_strerror(-5).decode() == "node coordinate is NaN or infinite"
    assert lib.nfft_strerror(12345).decode() == "unknown error"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="checks the behaviour without a GPU")
def test_valid_plan_without_device_is_a_hip_error(lib):
    """Valid arguments pass validation; the first HIP call then fails (no device) and the
    call returns NFFT_ERR_HIP with the handle untouched."""
    h = ctypes.c_void_p()
    N = (ctypes.c_int64 * 3)(32, 32, 32)
    rc = lib.nfft_plan_create(ctypes.byref(h), 3, N, 10, FAKE, 4, 2.0, 1, None)
    assert rc == -4 and h.value is None
