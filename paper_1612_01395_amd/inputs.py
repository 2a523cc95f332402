"""Seeded synthetic inputs shared by the GPU path, the tests and the CPU oracle.

This module holds only random draws and the workload descriptions (grid
sizes, convection vectors, tolerances).  It does no part of the solver's
arithmetic: no matrix assembly, no products, no sums.  Both the HIP library
and the oracle receive these arrays as plain inputs.

Workloads (all operators are h^2-scaled finite-difference convection-diffusion
operators on the interior nodes of a uniform grid with homogeneous Dirichlet
boundaries, rows ordered x fastest):

* ``c1``   2-D 5-point, 64 x 64, beta = (20, 10), no preconditioner.
* ``c2``   3-D 7-point, 128^3, beta = (50, 30, 10), Jacobi.
* ``c3``   3-D 27-point variable coefficient, 256^3, beta = (100, 0, 50),
           log-normal (sigma = 1) cell diffusion, shift +0.1, Jacobi, RR k = 50.
* ``c4``   3-D 7-point, 256^3, beta = (50, 30, 10), Jacobi, tol 1e-10, RR k = 20
           (precision form).
* ``c5``   512 independent 2-D 5-point systems, side n_k log-uniform in
           [32, 512], beta_k ~ U[0, 200]^2 (batched form).
* ``ptp1`` / ``ptp2``  the paper's two parallel test problems (Section 5),
           1000 x 1000 five-point stencils with exact solution all ones.
* ``c1s`` / ``c2s`` / ``c3s``  the same grids without convection (beta = 0):
           symmetric positive definite operators for the CG family
           (Algorithms 2, 4 and 6), which needs symmetry.

The right-hand side of every system is b = A x_true with x_true drawn here.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_XTRUE = 1
SEED_KAPPA = 2
SEED_BATCH = 3
SEED_LOSS_W = 4


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int            # 2 or 3
    n: int              # interior nodes per axis
    npts: int           # 5, 7 or 27
    beta: tuple         # convection vector, one entry per axis
    shift: float = 0.0  # diagonal shift (27-point operator only)
    kappa_sigma: float = 0.0  # log-normal sigma of the cell diffusion (27-point)
    precond: str = "none"     # "none" or "jacobi"
    tol: float = 1e-8
    maxit: int = 2000
    rr_period: int = 50
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.dim


WORKLOADS = {
    "c1": Workload("c1", 2, 64, 5, (20.0, 10.0), precond="none"),
    "c2": Workload("c2", 3, 128, 7, (50.0, 30.0, 10.0), precond="jacobi"),
    "c3": Workload("c3", 3, 256, 27, (100.0, 0.0, 50.0), shift=0.1,
                   kappa_sigma=1.0, precond="jacobi"),
    "c4": Workload("c4", 3, 256, 7, (50.0, 30.0, 10.0), precond="jacobi",
                   tol=1e-10, maxit=5000, rr_period=20),
    # symmetric positive definite counterparts (beta = 0) for the CG family
    "c1s": Workload("c1s", 2, 64, 5, (0.0, 0.0), precond="none"),
    "c2s": Workload("c2s", 3, 128, 7, (0.0, 0.0, 0.0), precond="jacobi"),
    "c3s": Workload("c3s", 3, 256, 27, (0.0, 0.0, 0.0), shift=0.1,
                    kappa_sigma=1.0, precond="jacobi"),
}


def workload(name: str, n: int | None = None) -> Workload:
    """The named workload, optionally at a different grid side ``n``."""
    w = WORKLOADS[name]
    if n is None:
        return w
    return Workload(w.name, w.dim, n, w.npts, w.beta, w.shift, w.kappa_sigma,
                    w.precond, w.tol, w.maxit, w.rr_period, dict(w.extra))


def x_true(N: int, seed=SEED_XTRUE) -> np.ndarray:
    """Exact solution x_true ~ U[0, 1), float64, length N."""
    return np.random.default_rng(seed).random(N)


def kappa_cells(n: int, sigma: float = 1.0, seed=SEED_KAPPA) -> np.ndarray:
    """Cell diffusion coefficients kappa_c = exp(sigma g_c), g_c ~ N(0, 1).

    One value per cell of the (n+1)^3 cells of a 3-D grid with n interior
    nodes per axis; flat index ci + (n+1) (cj + (n+1) ck).
    """
    g = np.random.default_rng(seed).standard_normal((n + 1) ** 3)
    return np.exp(sigma * g)


@dataclass(frozen=True)
class BatchSystem:
    k: int
    n: int
    beta: tuple


def batch_systems(count: int = 512, lo: int = 32, hi: int = 512,
                  seed=SEED_BATCH) -> list[BatchSystem]:
    """The batched workload: ``count`` 2-D 5-point systems of uneven size.

    Grid sides are log-uniform in [lo, hi] (rounded to an integer) and the
    convection vectors are uniform in [0, 200]^2.
    """
    g = np.random.default_rng(seed)
    sides = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), count))).astype(int)
    betas = g.uniform(0.0, 200.0, (count, 2))
    return [BatchSystem(k, int(sides[k]), (float(betas[k, 0]), float(betas[k, 1])))
            for k in range(count)]


def batch_x_true(k: int, N: int) -> np.ndarray:
    return np.random.default_rng([SEED_XTRUE, k]).random(N)


def batch_loss_weights(k: int, N: int) -> np.ndarray:
    """Weights w_k ~ N(0, 1) of the loss L = sum_k (w_k, x_k)."""
    return np.random.default_rng([SEED_LOSS_W, k]).standard_normal(N)


def random_vector(N: int, seed: int) -> np.ndarray:
    """A generic U[-1, 1) test vector (initial guesses, parity states)."""
    return np.random.default_rng([99, seed]).uniform(-1.0, 1.0, N)
