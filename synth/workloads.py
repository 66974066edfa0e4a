"""Named synthetic workloads with their seeds and sizes.

* ``lap2d_64``           : 2D 5-point Laplacian, 64 x 64 (n=4096), CG, tol 1e-10.
* ``spmv_set``           : 48 SpMV matrices, 4 families x 12 sizes (n 1e4..2e6).
* ``training_set``       : disjoint-seed matrices from the same families, plus
                           Chung-Lu graph Laplacians (hub rows *and* hub
                           columns, which no set family has).
* ``poisson3d_128``      : 3D 7-point Poisson 128^3, CG, tol 1e-10.
* ``graph_laplacian_1m`` : Chung-Lu graph Laplacian + 1e-2 I, n = 2^20.
* ``convdiff_1024``      : 2D convection-diffusion 1024^2, Pe 10, GMRES(30).
* ``serving_pool``       : 64 solvable matrices, n log-uniform in [1e3, 1e6].
"""
from __future__ import annotations

import math

import numpy as np

from . import matrices as M

FAMILIES = ("banded", "powerlaw", "blockdiag", "uniform")
TRAIN_FAMILIES = FAMILIES + ("graph",)
GRAPH_MAX_N = 600_000        # keeps a training graph's generation to seconds
BANDED_R = (5, 7, 9, 13, 19, 27, 5, 7, 9, 13, 19, 27)


def set_sizes(count: int = 12, lo: float = 1e4, hi: float = 2e6):
    """Log-spaced sizes n_k = round(10^(log10(lo) + k log10(hi/lo)/(count-1)))."""
    return [int(round(10 ** (math.log10(lo) + k * math.log10(hi / lo) / (count - 1))))
            for k in range(count)]


def zipf_exponent(k: int) -> float:
    """Exponent spread over [1.5, 2.5] so both tails appear at large n."""
    return 1.5 + ((5 * k) % 12) / 11.0


def family_matrix(family: str, k: int, n: int, seed: int) -> M.CSR:
    if family == "banded":
        return M.banded_stencil(n, BANDED_R[k % 12], seed)
    if family == "powerlaw":
        return M.power_law_rows(n, zipf_exponent(k), seed)
    if family == "blockdiag":
        return M.block_diagonal(n, seed)
    if family == "uniform":
        return M.uniform_random(n, seed)
    if family == "graph":
        return M.graph_laplacian_chung_lu(n, seed, mean_degree=(4, 8, 16, 32)[k % 4],
                                          zipf_s=(1.8, 2.0, 2.2)[k % 3],
                                          wmax=min(10_000, max(n // 4, 16)))
    raise ValueError(family)


def spmv_set_specs(max_n: int | None = None):
    """(name, family, k, n, seed) for the 48 held-out SpMV matrices."""
    out = []
    for f, fam in enumerate(FAMILIES):
        for k, n in enumerate(set_sizes()):
            if max_n is not None and n > max_n:
                continue
            seed = 2000 + k + 12 * f
            out.append((f"{fam}_k{k}_n{n}", fam, k, n, seed))
    return out


def spmv_set_matrix(spec) -> M.CSR:
    name, fam, k, n, seed = spec
    A = family_matrix(fam, k, n, seed)
    A.name = name
    return A


def training_specs(count: int = 600, seed: int = 9000, lo: float = 1e4, hi: float = 2e6):
    """Disjoint-seed training matrices: the families cycle, n log-uniform in
    [lo, hi] (graphs at most GRAPH_MAX_N rows)."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        fam = TRAIN_FAMILIES[t % len(TRAIN_FAMILIES)]
        n = int(round(10 ** rng.uniform(math.log10(lo), math.log10(hi))))
        if fam == "graph":
            n = min(n, GRAPH_MAX_N)
        k = int(rng.integers(0, 12))
        out.append((f"train{t}_{fam}_n{n}", fam, k, n, seed + 1 + t))
    return out


def lap2d_64():
    A = M.laplacian_2d(64)
    return A, M.vector(A.n, 1)


def poisson3d_128(N: int = 128):
    A = M.laplacian_3d(N)
    return A, M.vector(A.n, 3001)


def graph_laplacian_1m(n: int = 1 << 20):
    A = M.graph_laplacian_chung_lu(n, 3002)
    return A, M.vector(A.n, 3002 + 7)


def convdiff_1024(N: int = 1024):
    A = M.convection_diffusion_2d(N, 10.0)
    return A, M.vector(A.n, 4001)


def serving_pool(count: int = 64, seed: int = 5002, lo: float = 1e3, hi: float = 1e6):
    """Solvable matrices for the request loop.

    SPD members (2D/3D Laplacians, graph Laplacian + 1e-2 I) are solved with
    CG; the nonsymmetric members (convection-diffusion, power-law and
    uniform-random patterns made strictly diagonally dominant) with GMRES(30).
    Returns a list of (CSR, symmetric: bool).
    """
    rng = np.random.default_rng(seed)
    pool = []
    for t in range(count):
        n = int(round(10 ** rng.uniform(math.log10(lo), math.log10(hi))))
        kind = t % 6
        if kind == 0:
            N = max(2, int(round(math.sqrt(n))))
            pool.append((M.laplacian_2d(N), True))
        elif kind == 1:
            N = max(2, int(round(n ** (1 / 3))))
            pool.append((M.laplacian_3d(N), True))
        elif kind == 2:
            pool.append((M.graph_laplacian_chung_lu(max(n, 64), seed + 100 + t,
                                                    wmax=min(10_000, max(n, 64) // 4)), True))
        elif kind == 3:
            N = max(2, int(round(math.sqrt(n))))
            pool.append((M.convection_diffusion_2d(N, 10.0), False))
        elif kind == 4:
            A = M.power_law_rows(n, 2.0, seed + 100 + t, rmax=min(10_000, n // 4))
            pool.append((M.diagonally_dominant(A), False))
        else:
            A = M.uniform_random(n, seed + 100 + t, 4, 32)
            pool.append((M.diagonally_dominant(A), False))
        pool[-1][0].name = f"pool{t}_" + pool[-1][0].name
    return pool
