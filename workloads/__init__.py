"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generators only: mesh/domain parameters of the named
workloads, the coefficient fields kappa(x) evaluated at caller-given points, and
seeded cotangents / vectors.  It contains none of the method's arithmetic (no
basis functions, no quadrature rules, no classification, no assembly).

Workloads (all on the unit cube, open uniform knots, identity geometry map as in
Section 2 of the paper; the paper's own experiment uses [-1,1]^3 with a plane cut,
Section 3.1 / Fig. 4):

  uncut8_p2    8^3 elements, p=2, no cut, kappa = 1, mass + stiffness
  ball16_p3    16^3 elements, p=3, ball r=0.4 at the cube centre,
               kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)
  plane48_p4   48^3 elements, p=4, domain {x+y+z < 1.6},
               kappa = exp(g), g a seeded Fourier random field (seed 3)
  torus32_p3   32^3 elements, p=3, torus R=0.3, r=0.12 (axis z through the centre),
               kappa = exp(g) (seed 4), u, v ~ N(0,1) (seed 4, u drawn first)
  ball64_p6    64^3 elements, p=6, ball r=0.45, kappa = exp(g) (seed 5)

Random field: g(x) = sigma/sqrt(512) * sum_{k in {0..7}^3} [a_k cos(2 pi k.x) +
b_k sin(2 pi k.x)], sigma = 0.5, with a then b drawn as
numpy.random.default_rng(seed).standard_normal(512), k lexicographic (k1 slowest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

LS_NONE, LS_PLANE, LS_BALL, LS_TORUS = 0, 1, 2, 3
MASS, STIFF = 1, 2


@dataclass(frozen=True)
class LevelSet:
    """Domain Omega = {phi < 0}.

    kind 0: no cut (the whole box).
    kind 1: plane, phi = (n.x - r0)/|n|.
    kind 2: ball, phi = |x - c| - r0.
    kind 3: torus around the axis through c parallel to z, major radius r0,
            minor radius r1: phi = sqrt((rho - r0)^2 + (z - c_z)^2) - r1,
            rho = distance of (x, y) from (c_x, c_y).
    """
    kind: int = LS_NONE
    c: tuple = (0.0, 0.0, 0.0)
    n: tuple = (0.0, 0.0, 0.0)
    r0: float = 0.0
    r1: float = 0.0


@dataclass(frozen=True)
class Workload:
    name: str
    nel: tuple
    degree: int
    levelset: LevelSet
    kappa: str                 # "one" | "sin3" | "rf"
    seed: int = 0
    which: int = MASS | STIFF
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    octree_levels: int = 3
    cut_rule: str = "octree"   # "octree" | "fit": cut elements by the octree or by its fitted rule
    notes: str = field(default="", compare=False)


WORKLOADS = {
    "uncut8_p2": Workload("uncut8_p2", (8, 8, 8), 2, LevelSet(), "one"),
    "ball16_p3": Workload("ball16_p3", (16, 16, 16), 3,
                          LevelSet(LS_BALL, c=(0.5, 0.5, 0.5), r0=0.4), "sin3"),
    "plane48_p4": Workload("plane48_p4", (48, 48, 48), 4,
                           LevelSet(LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6), "rf", seed=3),
    "torus32_p3": Workload("torus32_p3", (32, 32, 32), 3,
                           LevelSet(LS_TORUS, c=(0.5, 0.5, 0.5), r0=0.3, r1=0.12), "rf", seed=4),
    "ball64_p6": Workload("ball64_p6", (64, 64, 64), 6,
                          LevelSet(LS_BALL, c=(0.5, 0.5, 0.5), r0=0.45), "rf", seed=5),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def custom(nel, degree, levelset=LevelSet(), kappa="one", seed=0, octree_levels=3,
           lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), cut_rule="octree") -> Workload:
    if isinstance(nel, int):
        nel = (nel, nel, nel)
    return Workload(f"custom{nel}_p{degree}", tuple(nel), degree, levelset, kappa, seed,
                    octree_levels=octree_levels, lo=tuple(lo), hi=tuple(hi), cut_rule=cut_rule)


def with_cut_rule(w: Workload, cut_rule: str) -> Workload:
    """The same workload with the cut elements integrated by the octree or its fitted rule."""
    import dataclasses
    return dataclasses.replace(w, name=f"{w.name}_{cut_rule}", cut_rule=cut_rule)


# ----------------------------------------------------------------------------------------
# coefficient fields
# ----------------------------------------------------------------------------------------
_RF_SIGMA = 0.5
_RF_MODES = 8


def _rf_coeffs(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(_RF_MODES ** 3)
    b = rng.standard_normal(_RF_MODES ** 3)
    # a cos(t) + b sin(t) = Re[(a - i b) e^{i t}]
    return (a - 1j * b).reshape(_RF_MODES, _RF_MODES, _RF_MODES)


def _rf_log(xyz: torch.Tensor, seed: int) -> torch.Tensor:
    c = torch.as_tensor(_rf_coeffs(seed), dtype=torch.complex128, device=xyz.device)
    k = torch.arange(_RF_MODES, dtype=torch.float64, device=xyz.device)
    e = [torch.polar(torch.ones_like(xyz[:, d:d + 1] * k),
                     2.0 * math.pi * xyz[:, d:d + 1] * k) for d in range(3)]  # (N, 8) each
    # sum_{k1,k2,k3} c[k1,k2,k3] e1[k1] e2[k2] e3[k3]
    t = e[2] @ c.reshape(-1, _RF_MODES).transpose(0, 1)          # (N, 64): [k1,k2]
    t = (t.reshape(-1, _RF_MODES, _RF_MODES) * e[1][:, None, :]).sum(-1)   # (N, 8): [k1]
    t = (t * e[0]).sum(-1)
    return (_RF_SIGMA / math.sqrt(_RF_MODES ** 3)) * t.real


def kappa_at(w: Workload, xyz, chunk: int = 1 << 20) -> torch.Tensor:
    """kappa at points xyz ((N,3) float64 tensor or array, any device) -> (N,) float64."""
    xyz = torch.as_tensor(xyz, dtype=torch.float64)
    n = xyz.shape[0]
    out = torch.empty(n, dtype=torch.float64, device=xyz.device)
    for s in range(0, n, chunk):
        x = xyz[s:s + chunk]
        if w.kappa == "one":
            out[s:s + chunk] = 1.0
        elif w.kappa == "sin3":
            out[s:s + chunk] = 1.0 + 0.5 * torch.prod(torch.sin(2.0 * math.pi * x), dim=1)
        elif w.kappa == "rf":
            out[s:s + chunk] = torch.exp(_rf_log(x, w.seed))
        else:
            raise ValueError(f"unknown kappa field {w.kappa!r}")
    return out


def kappa_separable(factors):
    """kappa(x) = f1(x) f2(y) f3(z) for three callables on float64 arrays (test input)."""
    def f(xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        return factors[0](xyz[:, 0]) * factors[1](xyz[:, 1]) * factors[2](xyz[:, 2])
    return f


# ----------------------------------------------------------------------------------------
# cotangents and vectors
# ----------------------------------------------------------------------------------------
def uv_vectors(seed: int, n: int):
    """u then v, each N(0,1) of length n, from one generator."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(n)
    v = rng.standard_normal(n)
    return u, v


def random_values(seed: int, n: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


def sample_indices(seed: int, n: int, k: int) -> np.ndarray:
    """k distinct sorted indices out of range(n)."""
    k = min(k, n)
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


# ----------------------------------------------------------------------------------------
# the paper's accuracy experiment (Section 3.1, Fig. 4)
# ----------------------------------------------------------------------------------------
PAPER_PLANE_POINT = (0.1, 0.2, 0.3)
PAPER_PLANE_NORMAL = (0.5, -0.2, 0.9)


def paper_plane(h: int, degree: int, octree_levels: int = 3) -> Workload:
    """Background [-1,1]^3 with h elements per direction; Omega is the part of it below the
    plane through PAPER_PLANE_POINT with normal PAPER_PLANE_NORMAL; mass matrix only
    (kappa = 1)."""
    r0 = sum(a * b for a, b in zip(PAPER_PLANE_NORMAL, PAPER_PLANE_POINT))
    return Workload(f"paper_plane{h}_p{degree}", (h, h, h), degree,
                    LevelSet(LS_PLANE, n=PAPER_PLANE_NORMAL, r0=r0), "one", which=MASS,
                    lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), octree_levels=octree_levels)


def target_f(xyz):
    """The projected function f = sin(2xz) cos(3yz) at points xyz ((N,3) array or tensor)."""
    if isinstance(xyz, torch.Tensor):
        x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
        return torch.sin(2.0 * x * z) * torch.cos(3.0 * y * z)
    xyz = np.asarray(xyz, dtype=np.float64)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.sin(2.0 * x * z) * np.cos(3.0 * y * z)


def poly2_f(xyz):
    """A polynomial of degree at most 2 in each variable (test input): it lies in every
    spline space of degree p >= 2."""
    if not isinstance(xyz, torch.Tensor):
        xyz = np.asarray(xyz, dtype=np.float64)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 0.5 + x * x * y - 3.0 * z * y * y + 0.25 * x * z


FUNCTIONS = {"target_f": target_f, "poly2_f": poly2_f}


# ----------------------------------------------------------------------------------------
# full coefficient tensors (stiffness under a geometry map)
# ----------------------------------------------------------------------------------------
# Component order of a symmetric 3x3 tensor field at the slots: C11, C22, C33, C12, C13, C23.
TENSOR_COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
MAP_EPS = 0.05


def _lib_of(xyz):
    return torch if isinstance(xyz, torch.Tensor) else np


def map_jacobian(xyz):
    """DF of the map F_i(x) = x_i + eps sin(pi x_{i+1}) sin(pi x_{i+2}) (indices mod 3,
    eps = 0.05), a smooth bijection of the unit cube onto itself (the boundary terms vanish):
    (P, 3, 3) array, DF[:, i, j] = dF_i / dx_j."""
    L = _lib_of(xyz)
    pi = math.pi
    s = L.sin(pi * xyz)
    c = L.cos(pi * xyz)
    P = xyz.shape[0]
    J = L.zeros((P, 3, 3), dtype=xyz.dtype) if L is np else torch.zeros((P, 3, 3), dtype=xyz.dtype, device=xyz.device)
    for i in range(3):
        a, b = (i + 1) % 3, (i + 2) % 3
        J[:, i, i] = 1.0
        J[:, i, a] = MAP_EPS * pi * c[:, a] * s[:, b]
        J[:, i, b] = MAP_EPS * pi * s[:, a] * c[:, b]
    return J


def map_tensor(xyz):
    """Coefficient tensor of the Laplacian pulled back through the map: C = |det DF|
    DF^{-1} DF^{-T} at the points, (P, 3, 3)."""
    L = _lib_of(xyz)
    J = map_jacobian(xyz)
    Ji = L.linalg.inv(J)
    det = L.linalg.det(J)
    return L.abs(det)[:, None, None] * (Ji @ Ji.transpose(0, 2, 1) if L is np else Ji @ Ji.transpose(1, 2))


def constant_tensor(seed: int):
    """A seeded symmetric positive definite constant tensor: C = A A^T / 3 + I / 2, A with
    N(0,1) entries (numpy.random.default_rng(seed), row-major)."""
    A = np.random.default_rng(seed).standard_normal((3, 3))
    return A @ A.T / 3.0 + 0.5 * np.eye(3)


def tensor_components(C):
    """(P, 3, 3) tensors -> (6, P) components in TENSOR_COMPONENTS order (the layout the
    library takes at the slots)."""
    L = _lib_of(C)
    return L.stack([C[:, d, e] for d, e in TENSOR_COMPONENTS])


TENSOR_FIELDS = {
    "map": map_tensor,
}
