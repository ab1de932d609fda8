"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds problem *data* only: mesh descriptions, the potential
functions V(x), random multivectors X and right-hand sides.  It contains none of
the finite-element method's arithmetic (no quadrature rules, no basis
functions, no Jacobians): each side computes its own quadrature points and
evaluates V there through the callables defined here.

The paper benchmarks a Helmholtz-type operator on uniform hexahedral meshes with
FEOrder 6-8 and 8...1024 random vectors (Sec. 4), and its eigenvalue workload
uses a precomputed potential that is not available here.  The configurations
below stand in for those workloads with synthetic, seeded data of the same
shape: polynomial degree, dofs per GPU partition, number of vectors.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np

BC_NONE = 0
BC_DIRICHLET0 = 1
BC_PERIODIC = 2


@dataclasses.dataclass
class BoxMesh:
    """Structured hexahedral mesh of the box [lo, hi] with n[d] cells per direction.

    ``lin`` is an optional 3x3 linear map applied to box coordinates (physical
    x = lin @ y); None means the identity.  Cells are then parallelepipeds and
    the cell Jacobian is a full (non-diagonal) 3x3 matrix.
    """
    n: Sequence[int]
    lo: Sequence[float] = (0.0, 0.0, 0.0)
    hi: Sequence[float] = (1.0, 1.0, 1.0)
    bc: int = BC_NONE
    lin: Optional[np.ndarray] = None

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def lin_matrix(self) -> np.ndarray:
        return np.eye(3) if self.lin is None else np.asarray(self.lin, dtype=np.float64)

    def volume(self) -> float:
        box = float(np.prod(np.asarray(self.hi, float) - np.asarray(self.lo, float)))
        return box * abs(float(np.linalg.det(self.lin_matrix())))


def _min_image(d: np.ndarray, period: np.ndarray) -> np.ndarray:
    return d - period * np.round(d / period)


def single_well(center=(0.5, 0.5, 0.5), width2: float = 0.05,
                period: Optional[Sequence[float]] = None) -> Callable[[np.ndarray], np.ndarray]:
    """V(x) = -exp(-|x - c|^2 / width2); minimum-image distance if ``period`` is given."""
    c = np.asarray(center, dtype=np.float64)
    per = None if period is None else np.asarray(period, dtype=np.float64)

    def V(x: np.ndarray) -> np.ndarray:
        d = np.asarray(x, dtype=np.float64) - c
        if per is not None:
            d = _min_image(d, per)
        return -np.exp(-np.sum(d * d, axis=-1) / width2)
    return V


def gaussian_wells(seed, L: float = 10.0, k: int = 8, width: float = 0.5,
                   depth=(-5.0, -1.0)) -> Callable[[np.ndarray], np.ndarray]:
    """Sum of ``k`` seeded Gaussian wells on the periodic cube [0, L)^3.

    V(x) = sum_k d_k exp(-|x - c_k|_T^2 / width^2), d_k ~ U[depth], c_k ~ U[0, L)^3,
    with |.|_T the minimum-image distance on the L-torus.
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, L, size=(k, 3))
    depths = rng.uniform(depth[0], depth[1], size=k)
    per = np.full(3, L)

    def V(x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1])
        for c, dk in zip(centers, depths):
            d = _min_image(x - c, per)
            out += dk * np.exp(-np.sum(d * d, axis=-1) / (width * width))
        return out
    V.centers = centers  # type: ignore[attr-defined]
    V.depths = depths    # type: ignore[attr-defined]
    return V


def random_multivector(seed, nrows: int, nvec: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Dof-major multivector (nrows x nvec, vectors contiguous per dof), U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nrows, nvec))


def n_nodes(mesh: BoxMesh, p: int) -> int:
    """Node count of the full numbering (constrained nodes included)."""
    per = mesh.bc == BC_PERIODIC
    m = 1
    for d in range(3):
        m *= int(mesh.n[d]) * p + (0 if per else 1)
    return m


@dataclasses.dataclass
class Workload:
    name: str
    mesh: BoxMesh
    p: int
    q: int
    mu: float
    V: Callable[[np.ndarray], np.ndarray]
    sigma: float
    nvec: int
    x_seed: tuple

    def ndofs(self) -> int:
        return n_nodes(self.mesh, self.p)

    def X(self, nvec: Optional[int] = None) -> np.ndarray:
        return random_multivector(self.x_seed, self.ndofs(), nvec or self.nvec)


def config1() -> Workload:
    """Unit cube, 4^3 cells, p=2, q=3, zero Dirichlet, single well, nvec=8."""
    m = BoxMesh(n=(4, 4, 4), lo=(0, 0, 0), hi=(1, 1, 1), bc=BC_DIRICHLET0)
    return Workload("unit-cube-4^3-p2q3-dirichlet", m, 2, 3, 0.5, single_well(),
                    0.0, 8, (1001, 99))


def config2() -> Workload:
    """Periodic [0,10]^3, 16^3 cells, p=6, q=7 (884,736 dofs), 8 Gaussian wells, nvec=64."""
    m = BoxMesh(n=(16, 16, 16), lo=(0, 0, 0), hi=(10, 10, 10), bc=BC_PERIODIC)
    return Workload("periodic-box10-16^3-p6q7", m, 6, 7, 0.5, gaussian_wells((1002, 0)),
                    0.0, 64, (1002, 99))


def config3(nvec: int = 64) -> Workload:
    """Periodic unit cube, 12^3 cells, p=8, q=9 (884,736 dofs), single well (minimum image)."""
    m = BoxMesh(n=(12, 12, 12), lo=(0, 0, 0), hi=(1, 1, 1), bc=BC_PERIODIC)
    return Workload("periodic-unit-12^3-p8q9", m, 8, 9, 0.5,
                    single_well(period=(1.0, 1.0, 1.0)), 0.0, nvec, (1003, 99))


def config4_meshes(count: int = 32) -> List[Workload]:
    """Batch of uneven periodic [0,10]^3 meshes: n ~ U{6..16}, p ~ U{4,6,8}, q = p+1, nvec ~ U{16,32,64,128}."""
    rng = np.random.default_rng(1004)
    out = []
    for i in range(count):
        n = int(rng.integers(6, 17))
        p = int(rng.choice([4, 6, 8]))
        nvec = int(rng.choice([16, 32, 64, 128]))
        m = BoxMesh(n=(n, n, n), lo=(0, 0, 0), hi=(10, 10, 10), bc=BC_PERIODIC)
        out.append(Workload(f"batch{i}-{n}^3-p{p}", m, p, p + 1, 0.5,
                            gaussian_wells((1004, i)), 0.0, nvec, (1004, 1000 + i)))
    return out


def small_meshes(count: int = 64) -> List[Workload]:
    """Batch of small uneven periodic [0,10]^3 meshes (the regime where one launch per
    operator leaves the GPU mostly idle): n ~ U{2..6}, p ~ U{4,6,8}, q = p+1,
    nvec ~ U{4,8,16}."""
    rng = np.random.default_rng(1014)
    out = []
    for i in range(count):
        n = int(rng.integers(2, 7))
        p = int(rng.choice([4, 6, 8]))
        nvec = int(rng.choice([4, 8, 16]))
        m = BoxMesh(n=(n, n, n), lo=(0, 0, 0), hi=(10, 10, 10), bc=BC_PERIODIC)
        out.append(Workload(f"small{i}-{n}^3-p{p}", m, p, p + 1, 0.5,
                            gaussian_wells((1014, i)), 0.0, nvec, (1014, 1000 + i)))
    return out


def config5() -> Workload:
    """Periodic [0,10]^3, 20^3 cells, p=6, q=7 (1,728,000 dofs), sigma=0.5, 128 right-hand sides."""
    m = BoxMesh(n=(20, 20, 20), lo=(0, 0, 0), hi=(10, 10, 10), bc=BC_PERIODIC)
    return Workload("periodic-box10-20^3-p6q7-shift0.5", m, 6, 7, 0.5, gaussian_wells((1005, 0)),
                    0.5, 128, (1005, 99))


@dataclasses.dataclass
class RefinedMesh:
    """A coarse box mesh (n, lo, hi, bc, lin as in BoxMesh) whose cells in the index box
    [rlo, rhi) are each split into 2 x 2 x 2 children (hanging nodes on the interface)."""
    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    rlo: Sequence[int]
    rhi: Sequence[int]
    bc: int = BC_DIRICHLET0
    lin: Optional[np.ndarray] = None


@dataclasses.dataclass
class RefinedWorkload:
    name: str
    mesh: RefinedMesh
    p: int
    q: int
    mu: float
    V: Callable[[np.ndarray], np.ndarray]
    sigma: float
    nvec: int
    x_seed: tuple

    def X(self, ndofs: int, nvec: Optional[int] = None) -> np.ndarray:
        return random_multivector(self.x_seed, ndofs, nvec or self.nvec)


def refined_config(nvec: int = 64) -> RefinedWorkload:
    """Adaptively refined stand-in for the paper's refined-mesh runs: zero-Dirichlet [0,10]^3,
    12^3 coarse cells with the central 6^3 block refined once (1,512 coarse + 1,728 fine
    cells, 735,159 nodes), p=6, q=7, 8 Gaussian wells, nvec=64."""
    m = RefinedMesh(n=(12, 12, 12), lo=(0, 0, 0), hi=(10, 10, 10), rlo=(3, 3, 3), rhi=(9, 9, 9),
                    bc=BC_DIRICHLET0)
    return RefinedWorkload("refined-box10-12^3-core6^3-p6q7-dirichlet", m, 6, 7, 0.5,
                           gaussian_wells((1006, 0)), 0.0, nvec, (1006, 99))

