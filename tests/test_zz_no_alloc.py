"""GPU test of nfft_forward_many_noalloc, the multi-channel forward transform
whose K oversampled grids live in the library's static device scratch.

Called through the C ABI (ctypes, raw device pointers).  Two calls in a row,
the second on a smaller plan with fewer channels (so it reuses a prefix of the
scratch the first call filled), each compared bit for bit with
nfft_forward_many of the same plan and inputs, and one channel of each against
the FP64 oracle NFFT at the rounding gate.  A request larger than the scratch
is refused with NFFT_ERR_SCRATCH before any GPU work.
"""
import ctypes

import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import nfft_alg as na
from test_gpu_nfft import e2e_tol, rel2, to_dev

pytestmark = pytest.mark.gpu


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _case(device, lib, N, M, K, dt, config):
    from paper_2208_00049_amd import Plan
    x = wl.uniform_nodes(M, len(N), config=config, stream=0)
    xt = torch.tensor(x, dtype=torch.float64 if dt == "c128" else torch.float32, device=device)
    p = Plan(xt, N, m=4, sigma=2.0)
    f = np.stack([wl.cn01(N, config=config, stream=10 + k) for k in range(K)])
    fd = to_dev(f, dt, device)
    ref = torch.empty((K, M), dtype=fd.dtype, device=device)
    out = torch.full((K, M), float("nan"), dtype=fd.dtype, device=device)
    print("noalloc forward_many N=%s M=%d K=%d %s" % (N, M, K, dt), flush=True)
    rc = lib.nfft_forward_many(p._h, K, ctypes.c_void_p(fd.data_ptr()),
                               ctypes.c_void_p(ref.data_ptr()), _stream(device))
    assert rc == 0
    rc = lib.nfft_forward_many_noalloc(p._h, K, ctypes.c_void_p(fd.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream(device))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    xs = xt.double().cpu().numpy()
    k = K - 1
    assert rel2(out[k].cpu().numpy(), na.forward(xs, f[k], 4, 2.0)) < e2e_tol(N, 2.0, 4, dt)
    return p


def test_noalloc_forward_many_two_calls(device):
    from paper_2208_00049_amd import _lib
    lib = _lib.load()
    p1 = _case(device, lib, (64, 96), 7000, 4, "c64", config=95)
    p2 = _case(device, lib, (32, 32), 1500, 2, "c128", config=96)
    p1.close()
    p2.close()


def test_noalloc_rejects_more_than_the_scratch(device):
    from paper_2208_00049_amd import Plan, _lib
    lib = _lib.load()
    N, M = (512, 512), 1000  # grid 1024^2 complex64 = 8 MiB per channel
    xt = torch.tensor(wl.uniform_nodes(M, 2, config=97, stream=0), dtype=torch.float32,
                      device=device)
    p = Plan(xt, N)
    kmax = _lib.NOALLOC_SCRATCH_BYTES // (1024 * 1024 * 8)
    f = torch.zeros((kmax + 1,) + N, dtype=torch.complex64, device=device)
    out = torch.zeros((kmax + 1, M), dtype=torch.complex64, device=device)
    rc = lib.nfft_forward_many_noalloc(p._h, kmax + 1, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream(device))
    assert rc == _lib.NFFT_ERR_SCRATCH
    assert _lib.strerror(rc).startswith("request exceeds")
    # the largest K that fits is accepted and matches the allocating call
    f = to_dev(np.stack([wl.cn01(N, config=97, stream=10 + k) for k in range(kmax)]), "c64",
               device)
    a = p.forward_many(f, out=torch.empty((kmax, M), dtype=torch.complex64, device=device),
                       noalloc=True)
    b = p.forward_many(f)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    p.close()
