"""Seeded synthetic inputs: structured triangle/tetrahedron meshes, node
perturbations and per-element coefficients.

This module holds no finite-element arithmetic. It only lays out node
coordinates and element-to-node lists, and draws random numbers. Both the CPU
oracle and the GPU library's tests and benchmarks take their inputs from here.

Mesh conventions (0-based ids):

* 2D unit square ``nx x ny``: node ``(i, j)`` has id ``i + (nx+1) j``; cells are
  ordered with ``i`` fastest and each cell is split along its ``x1 = x2``
  diagonal into ``(v00, v10, v11)`` and ``(v00, v11, v01)``. Both triangles are
  positively oriented. The diagonal split is the one the paper's eddy-current
  example needs (its exact solution jumps across ``x1 = x2``, Section 4.2).
* 3D Kuhn box ``nx x ny x nz``: node ``(i, j, k)`` has id
  ``i + (nx+1)(j + (ny+1) k)``; cubes are ordered with ``i`` fastest and each
  cube is split into the 6 tetrahedra of the Kuhn (Freudenthal) subdivision,
  one per permutation ``p`` of the axes in lexicographic order, with local nodes
  along the monotone path ``v0 -> v0+e_p0 -> v0+e_p0+e_p1 -> v0+(1,1,1)``.
  The orientation of such a tetrahedron is the sign of ``p``, so half of the
  elements have a negative Jacobian determinant (the paper allows both
  orientations, Section 2.3).
* 2D L-shape ``(0,1)^2 \\ (1/2,1)^2`` with ``m`` cells per half side (the domain
  of the paper's 2D timing table, Section 3.3): the nodes of the ``2m x 2m`` grid
  with ``i > m and j > m`` are removed and the rest renumbered in grid order.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order: node
perturbation first, then the coefficient ``a``, then ``b``, then any vector
``u``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def unit_square(nx: int, ny: Optional[int] = None, lx: float = 1.0, ly: float = 1.0):
    """Uniform triangle mesh of ``(0,lx) x (0,ly)``: returns (nodes [V,2] f64, elems [T,3] i32)."""
    ny = nx if ny is None else ny
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # shape (ny+1, nx+1), i fastest
    nodes = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00 = i + (nx + 1) * j
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    elems = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return nodes, elems


def unit_square_torch(n: int, device):
    """The mesh of ``unit_square(n)`` (n cells per side), laid out with torch on
    ``device`` (the same node coordinates, from the same ``numpy.linspace``
    values, and the same element lists): float64 nodes [V, 2] and int32 elems
    [T, 3] tensors."""
    import torch
    xs = torch.tensor(np.linspace(0.0, 1.0, n + 1), dtype=torch.float64, device=device)
    g = torch.arange(n + 1, device=device)
    j, i = torch.meshgrid(g, g, indexing="ij")  # i fastest
    nodes = torch.stack([xs[i.reshape(-1)], xs[j.reshape(-1)]], dim=1)
    del i, j
    c = torch.arange(n, device=device, dtype=torch.int32)
    j, i = torch.meshgrid(c, c, indexing="ij")
    v00 = (i + (n + 1) * j).reshape(-1)
    del i, j
    v11 = v00 + (n + 2)
    elems = torch.stack([v00, v00 + 1, v11, v00, v11, v00 + (n + 1)], dim=1).reshape(-1, 3)
    return nodes, elems


def kuhn_box(nx: int, ny: Optional[int] = None, nz: Optional[int] = None,
             lx: float = 1.0, ly: float = 1.0, lz: float = 1.0):
    """Kuhn (6 tets per cube) mesh of a box: returns (nodes [V,3] f64, elems [T,4] i32)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")  # i fastest
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    k, j, i = np.meshgrid(np.arange(nz, dtype=np.int64), np.arange(ny, dtype=np.int64),
                          np.arange(nx, dtype=np.int64), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    k = k.ravel()
    stride = np.array([1, nx + 1, (nx + 1) * (ny + 1)], dtype=np.int64)
    v0 = i + stride[1] * j + stride[2] * k
    tets = []
    for p in KUHN_PERMS:
        n1 = v0 + stride[p[0]]
        n2 = n1 + stride[p[1]]
        n3 = n2 + stride[p[2]]
        tets.append(np.stack([v0, n1, n2, n3], axis=1))
    elems = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return nodes, elems


def kuhn_box_torch(n: int, device):
    """The mesh of ``kuhn_box(n)`` (unit cube, n cubes per side), laid out with
    torch on ``device`` (the same node coordinates, taken from the same
    ``numpy.linspace`` values, and the same element lists), for sizes whose
    host-side layout would be slow: float64 nodes [V, 3] and int32 elems
    [T, 4] tensors."""
    import torch
    xs = torch.tensor(np.linspace(0.0, 1.0, n + 1), dtype=torch.float64, device=device)
    g = torch.arange(n + 1, device=device)
    k, j, i = torch.meshgrid(g, g, g, indexing="ij")  # i fastest
    nodes = torch.stack([xs[i.reshape(-1)], xs[j.reshape(-1)], xs[k.reshape(-1)]], dim=1)
    del i, j, k
    c = torch.arange(n, device=device, dtype=torch.int32)
    k, j, i = torch.meshgrid(c, c, c, indexing="ij")
    stride = (1, n + 1, (n + 1) * (n + 1))
    v0 = (i + stride[1] * j + stride[2] * k).reshape(-1)
    del i, j, k
    tets = []
    for p in KUHN_PERMS:
        n1 = v0 + stride[p[0]]
        n2 = n1 + stride[p[1]]
        tets.append(torch.stack([v0, n1, n2, n2 + stride[p[2]]], dim=1))
        del n1, n2
    elems = torch.stack(tets, dim=1).reshape(-1, 4)
    return nodes, elems


def l_shape(m: int):
    """Triangle mesh of (0,1)^2 minus [1/2,1)^2 with ``m`` cells per half side."""
    n = 2 * m
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    keep = ~((i > m) & (j > m))
    new_id = -np.ones((n + 1) * (n + 1), dtype=np.int64)
    new_id[keep.ravel()] = np.arange(int(keep.sum()))
    h = 1.0 / n
    nodes = np.stack([i.ravel()[keep.ravel()] * h, j.ravel()[keep.ravel()] * h], axis=1)
    cj, ci = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    cell_keep = ~((ci >= m) & (cj >= m))
    ci = ci[cell_keep]
    cj = cj[cell_keep]
    g00 = ci + (n + 1) * cj
    v00 = new_id[g00]
    v10 = new_id[g00 + 1]
    v01 = new_id[g00 + n + 1]
    v11 = new_id[g00 + n + 2]
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    elems = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return nodes.astype(np.float64), elems


def l_shape_torch(m: int, device):
    """The mesh of ``l_shape(m)``, laid out with torch on ``device`` (the same
    node order and element lists), for sizes whose host-side layout would be
    slow: float64 nodes [V, 2] and int32 elems [T, 3] tensors."""
    import torch
    n = 2 * m
    g = torch.arange(n + 1, device=device)
    j, i = torch.meshgrid(g, g, indexing="ij")  # node (i, j) at grid index i + (n+1) j
    keep = (~((i > m) & (j > m))).reshape(-1)
    new_id = torch.cumsum(keep.to(torch.int64), 0) - 1
    h = 1.0 / n
    nodes = torch.stack([i.reshape(-1)[keep], j.reshape(-1)[keep]], dim=1).to(torch.float64) * h
    del i, j
    c = torch.arange(n, device=device)
    cj, ci = torch.meshgrid(c, c, indexing="ij")
    cell_keep = (~((ci >= m) & (cj >= m))).reshape(-1)
    g00 = (ci.reshape(-1) + (n + 1) * cj.reshape(-1))[cell_keep]
    del ci, cj, cell_keep
    v00, v10, v01, v11 = (new_id[g00 + d].to(torch.int32) for d in (0, 1, n + 1, n + 2))
    elems = torch.stack([v00, v10, v11, v00, v11, v01], dim=1).reshape(-1, 3)
    return nodes, elems


def boundary_mask(nodes: np.ndarray, lo=None, hi=None, tol: float = 1e-12) -> np.ndarray:
    """True for nodes on the boundary of the bounding box of ``nodes``."""
    lo = nodes.min(axis=0) if lo is None else np.asarray(lo)
    hi = nodes.max(axis=0) if hi is None else np.asarray(hi)
    return np.any((np.abs(nodes - lo) < tol) | (np.abs(nodes - hi) < tol), axis=1)


def perturb_interior(nodes: np.ndarray, h: float, delta: float, rng) -> np.ndarray:
    """Move every interior node by independent U(-delta h, delta h) per coordinate.

    Boundary nodes stay put so the domain is exactly the box. One uniform draw of
    shape ``nodes.shape`` is made (boundary rows are drawn and discarded) so the
    stream position does not depend on the boundary layout.
    """
    d = rng.uniform(-delta * h, delta * h, size=nodes.shape)
    interior = ~boundary_mask(nodes)
    out = nodes.copy()
    out[interior] += d[interior]
    return out


def lognormal_coeffs(rng, T: int, sigma: float = 0.5) -> np.ndarray:
    return rng.lognormal(mean=0.0, sigma=sigma, size=T)


def uniform_coeffs(rng, T: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=T)


def kuhn_counts(n: int):
    """Closed-form vertex/element/edge/face counts of the Kuhn n^3 unit cube mesh."""
    V = (n + 1) ** 3
    T = 6 * n ** 3
    E = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    F = 1 - V + E + T
    return V, T, E, F


@dataclass
class Problem:
    """One assembly problem: mesh, kind ('ned' or 'rt') and coefficients."""
    name: str
    kind: str
    nodes: np.ndarray
    elems: np.ndarray
    a: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.nodes.shape[1]

    @property
    def T(self) -> int:
        return self.elems.shape[0]


def kuhn_problem(name: str, n: int, kind: str, seed: int, delta: float, coeff: str,
                 with_u: bool = False, n_dofs: Optional[int] = None) -> Problem:
    """Perturbed Kuhn n^3 cube with per-element coefficients (seeded)."""
    rng = np.random.default_rng(seed)
    nodes, elems = kuhn_box(n)
    nodes = perturb_interior(nodes, 1.0 / n, delta, rng)
    T = elems.shape[0]
    if coeff == "lognormal":
        a = lognormal_coeffs(rng, T)
        b = lognormal_coeffs(rng, T)
    elif coeff == "uniform":
        a = uniform_coeffs(rng, T)
        b = uniform_coeffs(rng, T)
    else:
        raise ValueError(coeff)
    u = None
    if with_u:
        if n_dofs is None:
            _, _, E, F = kuhn_counts(n)
            n_dofs = E if kind == "ned" else F
        u = rng.standard_normal(n_dofs)
    return Problem(name, kind, nodes, elems, a, b, u, {"n": n, "seed": seed, "delta": delta})


def square_ned32() -> Problem:
    """2D Nedelec, unit square 32x32 cells x 2 triangles, unit coefficients."""
    nodes, elems = unit_square(32)
    return Problem("square32_ned2d", "ned", nodes, elems, None, None, None, {"n": 32})


def kuhn64_ned() -> Problem:
    """3D Nedelec, Kuhn 64^3, interior nodes +-0.2h, a, b ~ lognormal(0, 0.5), seed 2."""
    return kuhn_problem("kuhn64_ned3d", 64, "ned", 2, 0.2, "lognormal")


def kuhn128_rt() -> Problem:
    """3D Raviart-Thomas, Kuhn 128^3, interior nodes +-0.15h, a, b ~ U[0.5, 2], seed 3."""
    return kuhn_problem("kuhn128_rt3d", 128, "rt", 3, 0.15, "uniform")


def kuhn128_ned() -> Problem:
    """3D Nedelec, Kuhn 128^3, interior nodes +-0.15h, a, b ~ lognormal(0, 0.5), seed 1."""
    return kuhn_problem("kuhn128_ned3d", 128, "ned", 1, 0.15, "lognormal")


def kuhn96_ned_grad() -> Problem:
    """3D Nedelec, Kuhn 96^3, +-0.2h, lognormal a, b and u ~ N(0,1) per edge, seed 5."""
    return kuhn_problem("kuhn96_ned3d_grad", 96, "ned", 5, 0.2, "lognormal", with_u=True)


def batch_sizes(seed: int = 4, count: int = 256, lo: int = 2000, hi: int = 400000):
    """Element-count targets of the batched workload: lognormal, clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    mu = 0.5 * (math.log(lo) + math.log(hi))
    sigma = 0.25 * (math.log(hi) - math.log(lo))
    z = rng.normal(mu, sigma, size=count)
    N = np.clip(np.round(np.exp(z)), lo, hi).astype(np.int64)
    return rng, N


def batch_problems(seed: int = 4, count: int = 256, scale: float = 1.0) -> List[Problem]:
    """Many uneven meshes: the first half 2D unit squares, the second half 3D Kuhn
    boxes; kinds alternate Nedelec / Raviart-Thomas by index parity; perturbation
    +-0.15h of the smallest cell width; a, b ~ U[0.5, 2]. ``scale`` shrinks the
    element-count targets (for quick tests) without changing the recipe.
    """
    rng, N = batch_sizes(seed, count)
    probs = []
    for m in range(count):
        target = max(1, int(round(N[m] * scale)))
        kind = "ned" if m % 2 == 0 else "rt"
        if m < count // 2:
            n = max(1, int(round(math.sqrt(target / 2.0))))
            nodes, elems = unit_square(n, n)
            h = 1.0 / n
        else:
            nxy = max(1, int(round((target / 6.0) ** (1.0 / 3.0))))
            nz = max(1, int(round(target / (6.0 * nxy * nxy))))
            nodes, elems = kuhn_box(nxy, nxy, nz)
            h = min(1.0 / nxy, 1.0 / nz)
        nodes = perturb_interior(nodes, h, 0.15, rng)
        T = elems.shape[0]
        a = uniform_coeffs(rng, T)
        b = uniform_coeffs(rng, T)
        probs.append(Problem(f"batch{m:03d}", kind, nodes, elems, a, b, None, {"target": int(target)}))
    return probs
