"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-number recipes and workload shapes only -- none of the
transform's arithmetic.  Both the GPU path and the CPU oracle are fed from here.

Recipes (the paper's experiments use uniformly random nodes with J = |I_N|,
section "Materials and Methods"; no public dataset is involved):

* seed = 220800049 + 1000 * config + stream; stream 0 = nodes, 1 = f,
  2 = fhat (adjoint input), 3 = node perturbation;
* coefficient vectors ~ CN(0, 1): real and imaginary parts iid N(0, 1/2);
* uniform nodes: ``rng.random((M, D)) - 0.5`` in FP64 (rounded to FP32 for the
  single-precision path by the caller);
* radial nodes: S spokes x T samples, theta_s = pi s / S, r_t = (t - T/2) / T,
  x = (r cos theta, r sin theta), which lies in [-1/2, 1/2)^2;
* batched transforms (config 3): transform b draws its size N_b uniformly from
  {64^2, 128^2, 256^2, 512^2} and M_b uniformly from the integers in
  [10^4, 5 10^5] (stream 0), then its nodes from stream 100 + b, its f from
  stream 300 + b and its fhat from stream 500 + b;
* multi-channel (config 3): K coefficient vectors through one node set,
  channel k from stream 700 + k (f) and 900 + k (fhat).
"""
import numpy as np

SEED_BASE = 220800049


def seed(config: int, stream: int) -> int:
    return SEED_BASE + 1000 * int(config) + int(stream)


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(seed(config, stream))


def uniform_nodes(M: int, D: int, config: int = 0, stream: int = 0) -> np.ndarray:
    """(M, D) FP64 nodes, iid uniform in [-1/2, 1/2)^D."""
    return rng(config, stream).random((int(M), int(D))) - 0.5


def radial_nodes(spokes: int, samples: int) -> np.ndarray:
    """(spokes*samples, 2) FP64 radial trajectory; sample t = samples/2 of every spoke is at 0."""
    s = np.arange(spokes, dtype=np.float64)
    t = np.arange(samples, dtype=np.float64)
    theta = np.pi * s / spokes
    r = (t - samples / 2.0) / samples
    x = np.empty((spokes, samples, 2))
    x[:, :, 0] = r[None, :] * np.cos(theta)[:, None]
    x[:, :, 1] = r[None, :] * np.sin(theta)[:, None]
    x = x.reshape(-1, 2)
    # cos/sin rounding can land a coordinate a hair outside the half-open torus
    return np.where(x >= 0.5, x - 1.0, x)


def jittered_radial_nodes(spokes: int, samples: int, Nt: int, config: int = 4,
                          stream: int = 0) -> np.ndarray:
    """Radial nodes with a radial jitter U(-0.5/Nt, 0.5/Nt) on each sample."""
    s = np.arange(spokes, dtype=np.float64)
    t = np.arange(samples, dtype=np.float64)
    theta = np.pi * s / spokes
    r = (t[None, :] - samples / 2.0) / samples
    r = r + rng(config, stream).uniform(-0.5 / Nt, 0.5 / Nt, size=(spokes, samples))
    x = np.empty((spokes, samples, 2))
    x[:, :, 0] = r * np.cos(theta)[:, None]
    x[:, :, 1] = r * np.sin(theta)[:, None]
    x = x.reshape(-1, 2)
    return x - np.floor(x + 0.5)


def cn01(shape, config: int = 0, stream: int = 1) -> np.ndarray:
    """Complex normal CN(0, 1) array (complex128)."""
    g = rng(config, stream)
    shape = tuple(np.atleast_1d(shape).tolist()) if not isinstance(shape, tuple) else shape
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def batched_specs(count: int = 64, config: int = 3):
    """Sizes of a batch of independent 2-D transforms: a list of (N, M) pairs."""
    g = rng(config, 0)
    edges = np.array([64, 128, 256, 512])
    ns = g.choice(edges, size=count)
    ms = g.integers(10_000, 500_000, size=count, endpoint=True)
    return [((int(n), int(n)), int(mm)) for n, mm in zip(ns, ms)]


# Workload shapes of the hot path (plain NFFT, forward + adjoint).
WORKLOADS = {
    "1d_n256_m512": dict(config=0, D=1, N=(256,), M=512, nodes="uniform"),
    "2d_n512_m262144_uniform": dict(config=1, D=2, N=(512, 512), M=262144, nodes="uniform"),
    "2d_n512_radial402x652": dict(config=1, D=2, N=(512, 512), M=402 * 652, nodes="radial",
                                  spokes=402, samples=652),
    "3d_n128_m2097152": dict(config=2, D=3, N=(128, 128, 128), M=2097152, nodes="uniform"),
    "4d_n16_m65536": dict(config=5, D=4, N=(16, 16, 16, 16), M=65536, nodes="uniform"),
    # batched / multi-channel (the runtime around the plans)
    "2d_n256_radial256x256_k32": dict(config=3, D=2, N=(256, 256), M=256 * 256, nodes="radial",
                                      spokes=256, samples=256, K=32),
    "2d_batch64": dict(config=3, D=2, count=64, nodes="uniform"),
}


def workload_nodes(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w["nodes"] == "radial":
        return radial_nodes(w["spokes"], w["samples"])
    return uniform_nodes(w["M"], w["D"], config=w["config"], stream=0)
