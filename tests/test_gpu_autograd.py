"""GPU tests of the differentiable NFFT (gradients with respect to the
coefficients and to the nodes), against the FP64 direct NDFT.

The reference gradients are written out from the NDFT's definition: for the
loss L = ||A(x) f - y||^2 with r = A(x) f - y,
  dL/d conj(f) = A^H r           (PyTorch's gradient of f is 2 A^H r),
  dL/dx[j, d]  = 2 Re(conj(r_j) sum_n (-2 pi i n_d) f_n e^{-2 pi i n.x_j}),
and for L = ||A(x)^H fhat - z||^2 with s = A^H fhat - z,
  PyTorch's gradient of fhat = 2 A s,
  dL/dx[j, d]  = 2 Re(conj(fhat_j) sum_n (-2 pi i n_d) s_n e^{-2 pi i n.x_j}).
They are also checked against FP64 central differences of the NDFT loss.
Workload (scaled down for the oracle): jittered radial nodes, y = A(x') f with
x' = x + U(-0.25/N, 0.25/N) per coordinate (stream 3).
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import ndft
from test_gpu_nfft import rel2

pytestmark = pytest.mark.gpu

# relative-l2 gates of the gradients against the NDFT: the NFFT's own accuracy
# (m = 4: 1e-6 in FP64, FP32 rounding on top; m = 8: 1e-12) with a margin of 10
GATE = {("c64", 4): 2e-5, ("c128", 4): 1e-5, ("c128", 8): 1e-10}


def centred(N):
    return np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")


def ndft_deriv(x, f, N):
    """(D, M): sum_n (-2 pi i n_d) f_n e^{-2 pi i n.x_j} from the NDFT oracle."""
    idx = centred(N)
    return np.stack([ndft.ndft_forward(x, (-2j * np.pi) * idx[d] * f) for d in range(len(N))])


def problem(N, spokes, samples, dt, device):
    Nt = 2 * N[0]
    x = wl.jittered_radial_nodes(spokes, samples, Nt, config=4, stream=0)
    g = wl.rng(4, 3)
    xp = x + g.uniform(-0.25 / N[0], 0.25 / N[0], size=x.shape)
    xp = xp - np.floor(xp + 0.5)
    rdt = torch.float64 if dt == "c128" else torch.float32
    cdt = torch.complex128 if dt == "c128" else torch.complex64
    xt = torch.tensor(x, dtype=rdt, device=device)
    xs = xt.double().cpu().numpy()   # the nodes the GPU sees, in FP64
    f = wl.cn01(N, config=4, stream=1)
    ft = torch.tensor(f, dtype=cdt, device=device)
    f = ft.cpu().numpy().astype(np.complex128)
    y = ndft.ndft_forward(xp, f)
    return xt, xs, ft, f, torch.tensor(y, dtype=cdt, device=device), y


@pytest.mark.parametrize("dt,m", [("c64", 4), ("c128", 4), ("c128", 8)])
def test_forward_gradients_match_ndft(device, dt, m):
    from paper_2208_00049_amd import Plan
    from paper_2208_00049_amd.autograd import nfft
    N = (32, 32)
    xt, xs, ft, f, yt, y = problem(N, 32, 32, dt, device)
    plan = Plan(xt, N, m=m, sigma=2.0)
    x_req = xt.clone().requires_grad_(True)
    f_req = ft.clone().requires_grad_(True)
    loss = (nfft(x_req, f_req, plan=plan) - yt).abs().pow(2).sum()
    loss.backward()
    r = ndft.ndft_forward(xs, f) - y
    gf_ref = 2 * ndft.ndft_adjoint(xs, r, N)
    gx_ref = 2 * np.real(np.conj(r)[None, :] * ndft_deriv(xs, f, N)).T
    print("forward grads", dt, m, rel2(f_req.grad.cpu().numpy(), gf_ref),
          rel2(x_req.grad.cpu().numpy(), gx_ref), flush=True)
    assert rel2(f_req.grad.cpu().numpy(), gf_ref) < GATE[(dt, m)]
    assert rel2(x_req.grad.cpu().numpy(), gx_ref) < GATE[(dt, m)]


@pytest.mark.parametrize("dt,m", [("c64", 4), ("c128", 8)])
def test_adjoint_gradients_match_ndft(device, dt, m):
    from paper_2208_00049_amd import Plan
    from paper_2208_00049_amd.autograd import nfft_adjoint
    N = (32, 32)
    xt, xs, ft, f, yt, y = problem(N, 32, 32, dt, device)
    M = xs.shape[0]
    cdt = ft.dtype
    fh = wl.cn01((M,), config=4, stream=2)
    fht = torch.tensor(fh, dtype=cdt, device=device)
    fh = fht.cpu().numpy().astype(np.complex128)
    z = wl.cn01(N, config=4, stream=5)
    zt = torch.tensor(z, dtype=cdt, device=device)
    z = zt.cpu().numpy().astype(np.complex128)
    plan = Plan(xt, N, m=m, sigma=2.0)
    x_req = xt.clone().requires_grad_(True)
    fh_req = fht.clone().requires_grad_(True)
    loss = (nfft_adjoint(x_req, N, fh_req, plan=plan) - zt).abs().pow(2).sum()
    loss.backward()
    s = ndft.ndft_adjoint(xs, fh, N) - z
    gfh_ref = 2 * ndft.ndft_forward(xs, s)
    gx_ref = 2 * np.real(np.conj(fh)[None, :] * ndft_deriv(xs, s, N)).T
    assert rel2(fh_req.grad.cpu().numpy(), gfh_ref) < GATE[(dt, m)]
    assert rel2(x_req.grad.cpu().numpy(), gx_ref) < GATE[(dt, m)]


def test_node_gradient_matches_central_differences(device):
    """FP64 central differences of the NDFT loss at a few node coordinates."""
    from paper_2208_00049_amd import Plan
    from paper_2208_00049_amd.autograd import nfft
    N = (16, 16)
    xt, xs, ft, f, yt, y = problem(N, 16, 16, "c128", device)
    plan = Plan(xt, N, m=8, sigma=2.0)
    x_req = xt.clone().requires_grad_(True)
    loss = (nfft(x_req, ft, plan=plan) - yt).abs().pow(2).sum()
    loss.backward()
    gx = x_req.grad.cpu().numpy()

    def L(xv):
        return float(np.sum(np.abs(ndft.ndft_forward(xv, f) - y) ** 2))
    h = 1e-6
    g = np.random.default_rng(7)
    for j, d in zip(g.choice(xs.shape[0], 6, replace=False), g.integers(0, 2, 6)):
        xp, xm = xs.copy(), xs.copy()
        xp[j, d] += h
        xm[j, d] -= h
        fd = (L(xp) - L(xm)) / (2 * h)
        assert abs(fd - gx[j, d]) <= 1e-6 * max(1.0, abs(fd)), (j, d, fd, gx[j, d])


def test_gradcheck_small(device):
    """torch.autograd.gradcheck of the forward in FP64 with m = 8 (NFFT ~ NDFT to 1e-13)."""
    from paper_2208_00049_amd import Plan
    from paper_2208_00049_amd.autograd import nfft
    N = (16, 16)
    x = torch.tensor(wl.uniform_nodes(20, 2, config=4, stream=6), dtype=torch.float64, device=device)
    f = torch.tensor(wl.cn01(N, config=4, stream=7), dtype=torch.complex128, device=device)
    plan = Plan(x, N, m=8, sigma=2.0)
    f.requires_grad_(True)
    # gradcheck perturbs its inputs without re-planning, so it checks the
    # f-gradient; the node gradient is checked against the NDFT above
    assert torch.autograd.gradcheck(lambda ff: nfft(x, ff, plan=plan), (f,), eps=1e-6, atol=1e-7,
                                    rtol=1e-6)


@pytest.mark.parametrize("N,dt,m,gate", [((256,), "c128", 4, 1e-5), ((32, 48), "c64", 4, 2e-5),
                                         ((32, 48), "c128", 6, 1e-8), ((16, 12, 20), "c128", 4, 1e-5),
                                         ((16, 12, 20), "c64", 3, 3e-4)])
def test_forward_deriv_both_methods_match_ndft(device, N, dt, m, gate):
    """nfft_forward_deriv with the polynomial window interpolates with the window's
    derivative (the exact gradient of the NFFT); with DIRECT it runs D NFFTs of
    -2 pi i n_d f.  Both approximate the NDFT derivative within (about) the NFFT's
    own accuracy, relative-l2 over the D x M outputs."""
    from paper_2208_00049_amd import Plan
    M = 3000
    x = wl.uniform_nodes(M, len(N), config=4, stream=8)
    rdt = torch.float64 if dt == "c128" else torch.float32
    cdt = torch.complex128 if dt == "c128" else torch.complex64
    xt = torch.tensor(x, dtype=rdt, device=device)
    xs = xt.double().cpu().numpy()
    ft = torch.tensor(wl.cn01(N, config=4, stream=9), dtype=cdt, device=device)
    f = ft.cpu().numpy().astype(np.complex128)
    ref = ndft_deriv(xs, f, N)
    got_poly = Plan(xt, N, m=m, sigma=2.0).forward_deriv(ft).cpu().numpy()
    got_direct = Plan(xt, N, m=m, sigma=2.0, window="direct").forward_deriv(ft).cpu().numpy()
    print("deriv", N, dt, m, rel2(got_poly, ref), rel2(got_direct, ref), flush=True)
    assert rel2(got_poly, ref) < gate
    assert rel2(got_direct, ref) < gate


def test_gradcheck_nodes(device):
    """With the polynomial window the node gradient is the exact derivative of the computed
    NFFT (derivative-of-window interpolation), so torch.autograd.gradcheck passes for the
    nodes too (FP64, m = 8: the truncated window's jump at the support edge, beta/sinh(beta)
    of its peak, is far below the finite-difference tolerance)."""
    from paper_2208_00049_amd.autograd import nfft, nfft_adjoint
    N = (16, 16)
    x = torch.tensor(wl.uniform_nodes(12, 2, config=4, stream=10), dtype=torch.float64,
                     device=device, requires_grad=True)
    f = torch.tensor(wl.cn01(N, config=4, stream=11), dtype=torch.complex128, device=device)
    fh = torch.tensor(wl.cn01((12,), config=4, stream=12), dtype=torch.complex128, device=device)
    # a plan is built per call from the perturbed nodes (plan=None)
    assert torch.autograd.gradcheck(lambda xx: nfft(xx, f, m=8), (x,), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)
    assert torch.autograd.gradcheck(lambda xx: nfft_adjoint(xx, N, fh, m=8), (x,), eps=1e-6,
                                    atol=1e-6, rtol=1e-5)
