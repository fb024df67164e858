"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the solver: it only draws numbers.  The
generator is SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter-based generator: draw i of
stream `seed` is mix(seed + (i+1)*0x9E3779B97F4A7C15), and a uniform in [0,1)
is the top 53 bits of that word times 2^-53.

Initial state (the paper's experiment, Sec. 4, asks for u0 = m + p with a
perturbation p of zero integral): p_i = amp*(2U_i - 1) per node, then its
integral -- that of the multilinear interpolant, i.e. the trapezoid rule -- is
subtracted so that int p = 0; w0 = 0.
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Words offset .. offset+count-1 of the SplitMix64 stream `seed` (uint64)."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0,1) with 53 random bits each."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def nodes_count(dim: int, n: int) -> int:
    return (n + 1) ** dim


def dofs(dim: int, n: int) -> int:
    """u and w at every node."""
    return 2 * (n + 1) ** dim


def _trapezoid_1d(n: int) -> np.ndarray:
    w = np.full(n + 1, 1.0 / n)
    w[0] = w[-1] = 0.5 / n
    return w


def noise_state(dim: int, n: int, m: float, seed: int, amp: float = 0.05,
                zero_mean: bool = True):
    """(u0, w0) as float64 numpy arrays of (n+1)^dim nodes, x fastest."""
    nn = n + 1
    p = amp * (2.0 * uniform01(seed, nn ** dim) - 1.0)
    if zero_mean:
        t = _trapezoid_1d(n)
        grid = p.reshape((nn,) * dim)
        mean = grid
        for _ in range(dim):
            mean = mean @ t          # integrate out the fastest remaining axis
        p = p - float(mean)
    u0 = m + p
    w0 = np.zeros_like(u0)
    return u0, w0


def cosine_state(dim: int, n: int, m: float, amp: float = 1.0 / 50.0):
    """(u0, w0) of the paper's experiment (Sec. 4): u0 = m + amp * prod_d
    cos(2 pi x_d) at the nodes, w0 = 0.  The perturbation is a DCT-I mode of
    index 2 per direction, orthogonal to the constant in the trapezoid (and
    the Q1 mass) inner product, so its discrete integral is zero."""
    x = np.arange(n + 1, dtype=np.float64) / n
    c = np.cos(2.0 * np.pi * x)
    p = c
    for _ in range(dim - 1):
        p = np.multiply.outer(c, p)
    u0 = m + amp * p.reshape(-1)
    return u0, np.zeros_like(u0)


# Robustness experiments (Sec. 4, Tables 1-2): parameters of the paper's run
# with theta = 1/2 and dt = eps^2.
def table2_cases():
    """eps sweep with h = eps/2 (N = 2/eps) and dt = eps^2, 2D."""
    return [dict(dim=2, n=int(round(2.0 / e)), eps=e, sigma=100.0, m=0.4, theta=0.5, dt=e * e)
            for e in (0.02, 0.01, 0.005)]


def table1_cases(dim: int = 3, sizes=(16, 32, 64, 128)):
    """mesh refinement at fixed parameters eps = 0.02, sigma = 100, m = 0.4."""
    return [dict(dim=dim, n=n, eps=0.02, sigma=100.0, m=0.4, theta=0.5, dt=4e-4) for n in sizes]


# --------------------------------------------------------------------------- #
# Workload recipes (the benchmark's configurations and the sweep/serving mixes) #
# --------------------------------------------------------------------------- #

CONFIGS = {
    # 2D 64^2, FP64, one timestep.
    "2d64": dict(dim=2, n=64, eps=0.02, sigma=100.0, m=0.0, theta=1.0, dt=1e-4, seed=1, steps=1,
                 precision="fp64"),
    # 3D 128^3, FP64, 5 timesteps, 5-level multigrid.
    "3d128": dict(dim=3, n=128, eps=0.01, sigma=1000.0, m=0.1, theta=1.0, dt=2e-5, seed=2,
                  steps=5, precision="fp64"),
    # 3D 256^3, same parameters, FP64 and mixed precision.
    "3d256": dict(dim=3, n=256, eps=0.01, sigma=1000.0, m=0.1, theta=1.0, dt=2e-5, seed=2,
                  steps=5, precision="mixed"),
}


def sweep_instance(i: int, base_seed: int = 4000, sizes=(128, 256, 512, 1024)):
    """Parameters of instance i of the batched 2D sweep: eps ~ U[0.01,0.05],
    sigma ~ logU[10,1000], m ~ U[-0.4,0.4], dt = eps^2/2, N uniform over sizes."""
    seed = base_seed + i
    r = uniform01(seed + (1 << 40), 4)
    eps = 0.01 + 0.04 * r[0]
    sigma = 10.0 ** (1.0 + 2.0 * r[1])
    m = -0.4 + 0.8 * r[2]
    n = int(sizes[min(int(r[3] * len(sizes)), len(sizes) - 1)])
    return dict(dim=2, n=n, eps=float(eps), sigma=float(sigma), m=float(m), theta=1.0,
                dt=float(0.5 * eps * eps), seed=seed)


def serving_simulation(s: int, base_seed: int = 5000):
    """Simulation s of the serving mix: 70% 2D with N in {256,...,2048},
    30% 3D with N in {64,128}; physical parameters drawn as in the sweep."""
    seed = base_seed + s
    r = uniform01(seed + (1 << 40), 6)
    eps = 0.01 + 0.04 * r[0]
    sigma = 10.0 ** (1.0 + 2.0 * r[1])
    m = -0.4 + 0.8 * r[2]
    if r[3] < 0.7:
        sizes = (256, 512, 1024, 2048)
        dim = 2
    else:
        sizes = (64, 128)
        dim = 3
    n = int(sizes[min(int(r[4] * len(sizes)), len(sizes) - 1)])
    return dict(dim=dim, n=n, eps=float(eps), sigma=float(sigma), m=float(m), theta=1.0,
                dt=float(0.5 * eps * eps), seed=seed)


def poisson_arrivals(rate: float, count: int, nsims: int, seed: int = 5999):
    """Arrival times (s) of `count` requests of one Poisson stream of the given
    rate, each assigned to a uniformly drawn simulation."""
    u = uniform01(seed, 2 * count)
    gaps = -np.log1p(-u[:count]) / rate
    t = np.cumsum(gaps)
    sim = np.minimum((u[count:] * nsims).astype(np.int64), nsims - 1)
    return t, sim


def sample_nodes(nodes: int, count: int, seed: int = 77):
    """A sorted set of distinct node indices (for sampled checks at full size)."""
    count = min(count, nodes)
    z = splitmix64(seed, 4 * count)
    idx = np.unique((z % np.uint64(nodes)).astype(np.int64))[:count]
    return np.sort(idx)


def log2_int(n: int) -> int:
    return int(math.log2(n))
