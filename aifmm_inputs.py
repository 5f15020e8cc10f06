"""Seeded synthetic workloads shaped like the paper's experiments (Sec. 4: targets = sources,
i.i.d. uniform in a hypercube, random right-hand side).

This module only draws random numbers; it holds none of the method's arithmetic, so both the
HIP path and the CPU oracle may use it.  Generator: numpy PCG64 ``default_rng(seed)``; the
points are drawn first, then b from the same stream.
"""
import math

import numpy as np

# kernel = (kind, scale, shift):  exp -> exp(-r/scale),  invmq -> 1/sqrt(r^2 + scale^2)
CONFIGS = {
    # plain FP64, one system: exp(-r) + 0.1 delta, N=4096 in [-1,1]^2, 64/leaf (depth 3), tol 1e-10, 1 RHS
    "c1": dict(n=4096, d=2, kernel=("exp", 1.0, 0.1), tol=1e-10, leaf=64, depth=3, nrhs=1, seed=1001),
    # plain FP64, batched per-level: 1/sqrt(r^2+1e-4) + delta, N=262144 in [-1,1]^2, depth 6, tol 1e-8, 16 RHS
    "c2": dict(n=262144, d=2, kernel=("invmq", 1e-2, 1.0), tol=1e-8, leaf=64, depth=6, nrhs=16, seed=2001),
    # precision form: 1/sqrt(r^2+h^2) + delta, h = N^(-1/3), N=262144 in [-1,1]^3, 64/leaf, tol 1e-5, 8 RHS
    "c3": dict(n=262144, d=3, kernel=("invmq", 262144 ** (-1.0 / 3.0), 1.0), tol=1e-5, leaf=64, depth=4,
               nrhs=8, seed=3001),
    "c3_reduced": dict(n=32768, d=3, kernel=("invmq", 32768 ** (-1.0 / 3.0), 1.0), tol=1e-5, leaf=64, depth=3,
                       nrhs=8, seed=3002),
}


def points_and_rhs(n, d, nrhs, seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1.0, 1.0, (n, d))
    b = rng.standard_normal((n, nrhs))
    return np.ascontiguousarray(pts), np.asfortranarray(b)


def config(name):
    c = dict(CONFIGS[name])
    pts, b = points_and_rhs(c["n"], c["d"], c["nrhs"], c["seed"])
    c["pts"], c["b"] = pts, b
    return c


def small_case(n, d=2, kernel=("exp", 1.0, 0.1), tol=1e-10, leaf=64, depth=0, nrhs=1, seed=7):
    pts, b = points_and_rhs(n, d, nrhs, seed)
    return dict(n=n, d=d, kernel=kernel, tol=tol, leaf=leaf, depth=depth, nrhs=nrhs, seed=seed, pts=pts, b=b)


def batch_sizes(count=256, seed=4999, lo=2048, hi=32768):
    """System sizes of the many-systems workload: N log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(count)]
