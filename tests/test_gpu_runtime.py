"""GPU tests of the runtime around the plans: multi-channel transforms, batches
run as one HIP graph, and the tile autotuner.

* Multi-channel: each channel of forward_many / adjoint_many is bit for bit
  what forward / adjoint give for that channel alone (same kernels, same
  summation order), and one channel is checked against the FP64 oracle NFFT.
* Batch: graph replays give bit for bit the eager results of every plan; the
  graph is replayed several times with eager work of the same plans and
  synchronisations in between, every replay is checked, and a changed output
  tensor makes the batch capture a new graph.
* Fused batch (plans of one type, D, stencil and window): one launch per stage
  (the count is asserted), results bit for bit those of the plans' own calls
  over repeated calls, with a plan without nodes, odd and mixed sizes, and new
  tensors between calls; one transform is checked against the FP64 oracle.
* Tuner: the chosen tiles are among the candidates and the tuned plan agrees
  with a default plan within the rounding tolerance of the type.
"""
import numpy as np
import pytest
import torch

import nfft_workloads as wl
from oracle import nfft_alg as na
from test_gpu_nfft import e2e_tol, rel2, to_dev

pytestmark = pytest.mark.gpu

CASES = [((256,), 512, 4, 2.0, "c128"), ((64, 64), 5000, 4, 2.0, "c64"),
         ((48, 64), 3000, 6, 2.0, "c128"), ((16, 16, 16), 6000, 4, 2.0, "c64"),
         ((16, 16, 16), 3000, 4, 1.25, "c128")]


def plan_for(device, N, M, m, sigma, dt, config, **kw):
    from paper_2208_00049_amd import Plan
    x = wl.uniform_nodes(M, len(N), config=config, stream=0)
    xt = torch.tensor(x, dtype=torch.float64 if dt == "c128" else torch.float32, device=device)
    return Plan(xt, N, m=m, sigma=sigma, **kw), xt.double().cpu().numpy()


@pytest.mark.parametrize("N,M,m,sigma,dt", CASES)
def test_multichannel_equals_single_channel(device, N, M, m, sigma, dt):
    K = 3
    p, xs = plan_for(device, N, M, m, sigma, dt, config=90)
    f = np.stack([wl.cn01(N, config=90, stream=10 + k) for k in range(K)])
    fh = np.stack([wl.cn01((M,), config=90, stream=20 + k) for k in range(K)])
    fd, fhd = to_dev(f, dt, device), to_dev(fh, dt, device)
    many_f = p.forward_many(fd)
    many_a = p.adjoint_many(fhd)
    print("multichannel", N, M, m, sigma, dt, flush=True)
    for k in range(K):
        assert torch.equal(many_f[k], p.forward(fd[k].contiguous()))
        assert torch.equal(many_a[k], p.adjoint(fhd[k].contiguous()))
    tol = e2e_tol(N, sigma, m, dt)
    assert rel2(many_f[1].cpu().numpy(), na.forward(xs, f[1], m, sigma)) < tol
    assert rel2(many_a[2].cpu().numpy(), na.adjoint(xs, fh[2], N, m, sigma)) < tol


def test_multichannel_empty_and_growing(device):
    """M = 0 gives zeros; a larger K after a smaller one reallocates and stays exact."""
    from paper_2208_00049_amd import Plan
    p0 = Plan(torch.zeros((0, 2), dtype=torch.float32, device=device), (32, 32))
    y = p0.adjoint_many(torch.zeros((4, 0), dtype=torch.complex64, device=device))
    assert y.shape == (4, 32, 32) and not torch.any(y)
    p, _ = plan_for(device, (64, 64), 4000, 4, 2.0, "c64", config=91)
    for K in (1, 2, 5):
        fh = to_dev(np.stack([wl.cn01((4000,), config=91, stream=30 + k) for k in range(K)]), "c64",
                    device)
        a = p.adjoint_many(fh)
        for k in range(K):
            assert torch.equal(a[k], p.adjoint(fh[k].contiguous()))


def test_batch_graph_replays(device):
    from paper_2208_00049_amd import Batch
    specs = [((256,), 512, 4, 2.0, "c128"), ((64, 64), 5000, 4, 2.0, "c64"),
             ((32, 48), 2000, 6, 2.0, "c128"), ((16, 16, 16), 3000, 4, 2.0, "c64"),
             ((128, 128), 20000, 4, 2.0, "c64")]
    plans = [plan_for(device, N, M, m, s, dt, config=92 + i)[0] for i, (N, M, m, s, dt) in enumerate(specs)]
    fs = [to_dev(wl.cn01(N, config=92, stream=i), dt, device) for i, (N, M, m, s, dt) in enumerate(specs)]
    fhs = [to_dev(wl.cn01((M,), config=93, stream=i), dt, device)
           for i, (N, M, m, s, dt) in enumerate(specs)]
    ref_f = [p.forward(f).clone() for p, f in zip(plans, fs)]
    ref_a = [p.adjoint(fh).clone() for p, fh in zip(plans, fhs)]
    outs_f = [torch.empty_like(r) for r in ref_f]
    outs_a = [torch.empty_like(r) for r in ref_a]
    b = Batch(plans, nstreams=3)
    for rep in range(4):
        for o in outs_f + outs_a:
            o.fill_(float("nan"))
        b.forward(fs, outs_f)
        b.adjoint(fhs, outs_a)
        torch.cuda.synchronize()
        print("batch replay", rep, flush=True)
        for r, o in zip(ref_f + ref_a, outs_f + outs_a):
            assert torch.equal(r, o)
        # eager work of the same plans between replays
        plans[rep % len(plans)].forward(fs[rep % len(plans)])
        torch.cuda.synchronize()
    # a different output tensor: the batch captures a new graph
    outs_f[0] = torch.empty_like(ref_f[0])
    b.forward(fs, outs_f)
    torch.cuda.synchronize()
    for r, o in zip(ref_f, outs_f):
        assert torch.equal(r, o)
    b.close()


FUSED_CASES = [
    # (specs [(N, M)], m, dtype, tiled 3-D, launches forward, launches adjoint)
    ([((512, 512), 262144), ((64, 64), 10000), ((128, 128), 0), ((256, 256), 50000),
      ((128, 128), 130000), ((64, 64), 500)], 4, "c64", False, 3, 3),
    ([((48, 64), 4000), ((33, 20), 900), ((64, 64), 7000)], 6, "c128", False, 3, 3),
    ([((256,), 512), ((1000,), 3000), ((96,), 0), ((64,), 200)], 4, "c128", False, 2, 3),
    ([((16, 16, 16), 6000), ((32, 32, 32), 30000), ((16, 24, 16), 2000)], 4, "c64", True, 4, 5),
]


@pytest.mark.parametrize("specs,m,dt,tiled,lf,la", FUSED_CASES)
def test_batch_fused_equals_plans(device, specs, m, dt, tiled, lf, la):
    from paper_2208_00049_amd import Batch
    kw = {"spread": "tiled"} if tiled else {}
    plans, xs = [], []
    for i, (N, M) in enumerate(specs):
        p, x = plan_for(device, N, M, m, 2.0, dt, config=96 + i, **kw)
        plans.append(p)
        xs.append(x)
    fs = [to_dev(wl.cn01(N, config=96, stream=i), dt, device) for i, (N, M) in enumerate(specs)]
    fhs = [to_dev(wl.cn01((M,), config=97, stream=i), dt, device) for i, (N, M) in enumerate(specs)]
    ref_f = [p.forward(f).clone() for p, f in zip(plans, fs)]
    ref_a = [p.adjoint(fh).clone() for p, fh in zip(plans, fhs)]
    b = Batch(plans)
    info = b.info()
    print("fused batch", [s for s in specs], dt, info, flush=True)
    assert info == {"fused": True, "launches_forward": lf, "launches_adjoint": la}
    outs_f = [torch.empty_like(r) for r in ref_f]
    outs_a = [torch.empty_like(r) for r in ref_a]
    for rep in range(3):
        for o in outs_f + outs_a:
            o.fill_(float("nan"))
        b.forward(fs, outs_f)
        b.adjoint(fhs, outs_a)
        torch.cuda.synchronize()
        for r, o in zip(ref_f + ref_a, outs_f + outs_a):
            assert torch.equal(r, o)
        plans[rep % len(plans)].adjoint(fhs[rep % len(plans)])  # eager work in between
        torch.cuda.synchronize()
    # new tensors: the pointer table is rewritten
    outs_a = [torch.full_like(r, float("nan")) for r in ref_a]
    fs2 = [f.clone() for f in fs]
    b.adjoint(fhs, outs_a)
    b.forward(fs2, outs_f)
    torch.cuda.synchronize()
    for r, o in zip(ref_f + ref_a, outs_f + outs_a):
        assert torch.equal(r, o)
    k = max(range(len(specs)), key=lambda i: specs[i][1])
    N, M = specs[k]
    tol = e2e_tol(N, 2.0, m, dt)
    assert rel2(outs_f[k].cpu().numpy(), na.forward(xs[k], fs[k].cpu().numpy(), m, 2.0)) < tol
    assert rel2(outs_a[k].cpu().numpy(), na.adjoint(xs[k], fhs[k].cpu().numpy(), N, m, 2.0)) < tol
    b.close()


def test_batch_mixed_plans_use_a_graph(device):
    from paper_2208_00049_amd import Batch
    p1, _ = plan_for(device, (64, 64), 1000, 4, 2.0, "c64", config=98)
    p2, _ = plan_for(device, (64, 64), 1000, 4, 2.0, "c128", config=98)
    assert Batch([p1, p2]).info()["fused"] is False


def test_batch_rejects_duplicate_plans(device):
    from paper_2208_00049_amd import Batch, NfftError
    p, _ = plan_for(device, (64, 64), 100, 4, 2.0, "c64", config=94)
    with pytest.raises(NfftError):
        Batch([p, p])


@pytest.mark.parametrize("N,M,dt", [((128, 128), 20000, "c64"), ((16, 16, 16), 3000, "c128")])
def test_tuned_plan(device, N, M, dt):
    from paper_2208_00049_amd import Plan
    x = wl.uniform_nodes(M, len(N), config=95, stream=0)
    xt = torch.tensor(x, dtype=torch.float64 if dt == "c128" else torch.float32, device=device)
    pt = Plan(xt, N, m=4, sigma=2.0, tune=2)
    pd = Plan(xt, N, m=4, sigma=2.0)
    cands = {2: [(16, 16), (16, 32), (32, 32), (32, 64), (64, 64)],
             3: [(8, 8, 8), (8, 8, 16), (8, 16, 16), (16, 16, 16)]}[len(N)]
    tile = pt.info()["tile"]
    print("tuned", N, dt, tile, pt.tuned_ms, flush=True)
    assert tile in cands and pt.tuned_ms > 0
    f = to_dev(wl.cn01(N, config=95, stream=1), dt, device)
    fh = to_dev(wl.cn01((M,), config=95, stream=2), dt, device)
    tol = 2 * e2e_tol(N, 2.0, 4, dt)
    assert rel2(pt.forward(f).cpu().numpy(), pd.forward(f).cpu().numpy()) < tol
    assert rel2(pt.adjoint(fh).cpu().numpy(), pd.adjoint(fh).cpu().numpy()) < tol
