"""Seeded synthetic problem data shared by the HIP path's tests, the benchmark
and the oracle's tests.

This module holds none of the method's arithmetic: it only lays out the
problem data of the synthetic workloads (grids, the target y_d, the source f,
controls u, random test directions and the workload table).  The random draws
the method itself makes (the KL variables xi) are not here: both the HIP path
and the oracle implement Philox4x64-10 from its published definition.

Arrays are float64 in the ``[n][n][n]`` vertex layout, z fastest, vertex
``(ix, iy, iz)`` at ``(ix h, iy h, iz h)`` with ``h = 1/(n-1)``.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def coords(n):
    """Vertex coordinates of an n^3 grid on the unit cube as (X, Y, Z)."""
    t = np.linspace(0.0, 1.0, n)
    return np.meshgrid(t, t, t, indexing="ij")


def target_sin(n, freq=1):
    """y_d = sin(f pi x) sin(f pi y) sin(f pi z) at the vertices."""
    X, Y, Z = coords(n)
    return np.sin(freq * np.pi * X) * np.sin(freq * np.pi * Y) * np.sin(freq * np.pi * Z)


def control_xyz(n, scale=0.1):
    """u = scale * x y z at the vertices."""
    X, Y, Z = coords(n)
    return scale * X * Y * Z


def constant(n, value):
    return np.full((n, n, n), float(value))


def random_field(n, seed, scale=1.0):
    """Seeded N(0, scale^2) field on all vertices (boundary entries included;
    the method ignores them)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((n, n, n))


def random_directions(n, count, seed):
    """Seeded unit-variance directions for finite-difference checks."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, n, n)) for _ in range(count)]


def random_smooth_directions(n, count, seed, kmax=3):
    """Seeded smooth directions: random combinations of the sine modes
    prod_d sin(k_d pi x_d), k_d <= kmax (zero on the boundary)."""
    rng = np.random.default_rng(seed)
    X, Y, Z = coords(n)
    modes = []
    for a in range(1, kmax + 1):
        for b in range(1, kmax + 1):
            for c in range(1, kmax + 1):
                modes.append(np.sin(a * np.pi * X) * np.sin(b * np.pi * Y) * np.sin(c * np.pi * Z))
    out = []
    for _ in range(count):
        w = rng.standard_normal(len(modes))
        out.append(sum(wi * m for wi, m in zip(w, modes)))
    return out


ODD_SIZES = (33, 41, 49, 57, 65)
# the batch of independent solves on grids of random size that accompanies
# the 257^3 MLMC workload: 300 state solves, f = 1, u = 0, draws keyed by
# level 6 (beyond the MLMC levels), seed 0
ODD_SOLVES = {"count": 300, "level": 6, "first": 0, "f_value": 1.0, "seed": 0}


def odd_sizes(count, seed=0, level=6, first=0):
    """Grid sizes of the independent-solve batch: problem j takes
    ODD_SIZES[floor(5 (w >> 11) / 2^53)], w the first word of the
    Philox4x64-10 block with key (seed, 0) and counter (0, first + j, level, 1).
    numpy's Philox advances its counter before each block, so it is started
    one below the wanted counter."""
    out = []
    for j in range(count):
        v = ((first + j) << 64) | (level << 128) | (1 << 192)
        v -= 1
        ctr = np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
        bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64), counter=ctr)
        w = int(bg.random_raw(1)[0])
        idx = ((w >> 11) * len(ODD_SIZES)) >> 53
        out.append(ODD_SIZES[idx])
    return out


def grids(first_n, levels):
    """Nested vertex counts n_i = 2 (n_{i-1} - 1) + 1 starting at first_n."""
    out = [first_n]
    for _ in range(levels - 1):
        out.append(2 * (out[-1] - 1) + 1)
    return out


@dataclass
class Workload:
    """One synthetic workload shaped like the paper's experiments."""
    name: str
    grid_n: List[int]
    M: List[int]
    K: int = 4
    sigma2: float = 1.0
    theta: float = 1.0
    alpha: float = 1e-3
    seed: int = 0
    solver: str = "mgpcg"          # "cg" | "mgpcg"
    precision: str = "fp64"        # "fp64" | "mixed" | "mixed_bf16"
    rtol: float = 1e-12
    f_value: float = 0.0
    u_kind: str = "xyz"            # "zero" | "xyz"
    steps: int = 1
    tau: Optional[float] = None
    law: int = 0                   # 0 algebraic (N(0,1), (1+|k|^2)^-5/2); 1 exponential (Sec. 5)
    rho: float = 0.15              # correlation length of the exponential law
    target_freq: int = 1           # y_d = prod sin(freq pi x_d)
    extra: dict = field(default_factory=dict)

    def u0(self):
        n = self.grid_n[-1]
        return control_xyz(n) if self.u_kind == "xyz" else constant(n, 0.0)

    def f(self):
        return constant(self.grid_n[-1], self.f_value)

    def y_d(self):
        return target_sin(self.grid_n[-1], freq=self.target_freq)


# The five synthetic workloads (sizes of the paper's 3-D experiments: nested
# cubes, KL coefficient, sin target, MLMC level hierarchy).
WORKLOADS = {
    "single_level_17": Workload(
        name="single-level risk-averse gradient, 17^3, 64 samples, CG",
        grid_n=[17], M=[64], solver="cg", u_kind="zero", steps=5, tau=10.0),
    "mlmc_129": Workload(
        name="MLMC gradient, levels 9^3..129^3, M=4096/1024/256/64/16, FP64 MG-PCG",
        grid_n=grids(9, 5), M=[4096, 1024, 256, 64, 16]),
    "mlmc_129_mixed": Workload(
        name="MLMC gradient, levels 9^3..129^3, sigma^2=2, theta=10, FP32 V-cycles in FP64 refinement",
        grid_n=grids(9, 5), M=[4096, 1024, 256, 64, 16], sigma2=2.0, theta=10.0,
        precision="mixed"),
    "mlmc_129_bf16": Workload(
        name="MLMC gradient, levels 9^3..129^3, sigma^2=2, theta=10, FP32 V-cycles with bfloat16 "
             "smoother coefficients in FP64 refinement",
        grid_n=grids(9, 5), M=[4096, 1024, 256, 64, 16], sigma2=2.0, theta=10.0,
        precision="mixed_bf16"),
    "mlmc_257_batched": Workload(
        name="MLMC gradient, levels 9^3..257^3, M=8192/2048/512/128/32/8",
        grid_n=grids(9, 6), M=[8192, 2048, 512, 128, 32, 8], precision="mixed", rtol=1e-10),
    # the paper's own law (Sec. 5): xi ~ U(-4, 4), lam = exp(-pi (j+k+l) 0.15),
    # permuted axes, 125 terms, target prod sin(2 pi x_d), strong risk
    # aversion theta = 72, initial batch 128/16/2 on 17^3/33^3/65^3, u_0 = 0
    "paper_law_65": Workload(
        name="MLMC gradient, Sec. 5 law (U(-4,4), exp(-pi(j+k+l)0.15), K=5), levels "
             "17^3..65^3, M=128/16/2, theta=72",
        grid_n=grids(17, 3), M=[128, 16, 2], K=5, theta=72.0, law=1, rho=0.15,
        target_freq=2, u_kind="zero"),
    "adaptive_257": Workload(
        name="adaptive MLSGD, levels 9^3..257^3, K=5, alpha=1e-4, f=1",
        grid_n=grids(9, 6), M=[8192, 2048, 512, 128, 32, 8], K=5, alpha=1e-4,
        f_value=1.0, u_kind="zero", precision="mixed", steps=50, rtol=1e-10),
}
