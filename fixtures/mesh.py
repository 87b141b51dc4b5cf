"""Structured Q1 meshes and element matrices for the multifrontal workloads.

The paper states the problem as element matrices plus mesh connectivity: the fronts at the leaves
of the elimination tree are the element matrices, and they are joined according to the mesh
(Sec. 2.4).  Its model problem is the L2 projection M u = b (Sec. 2.1, eqs. L2_proj and
Linear_system); the workloads here add a diffusion term (reaction-diffusion) or diffusion plus
advection.  With the diffusion coefficient set to zero the system is exactly the paper's mass
matrix system.

Conventions (fixed here, used by every consumer):
  * element (i, j[, k]) of an nx x ny[ x nz] grid has id  i + nx*(j + ny*k);
  * node (i, j[, k]) has id  i + (nx+1)*(j + (ny+1)*k);
  * local node a of an element is the tensor-product corner a = c_x + 2*c_y [+ 4*c_z];
  * element matrices are row-major [a][b] with rows indexed by the test function phi_a:
      K_e[a, b] = k_e * int grad phi_a . grad phi_b + int phi_a phi_b + int phi_a (v . grad phi_b).
All integrals use 2-point Gauss-Legendre per axis, exact for these (bi/tri)linear integrands.

Seeds: every configuration draws from ``numpy.random.default_rng(config_number)`` in the order
sides (batched config only), per-mesh coefficients (diffusion, then velocity), then the RHS.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


@dataclass
class Mesh:
    dim: int
    shape: tuple            # elements per axis
    conn: np.ndarray        # (E, 2**dim) int32 global node ids in tensor-product local order
    ijk: np.ndarray         # (E, dim) int32 element index coordinates
    h: tuple                # element edge length per axis

    @property
    def npe(self) -> int:
        return 1 << self.dim

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(np.prod([s + 1 for s in self.shape]))


@dataclass
class Problem:
    name: str
    meshes: list            # list[Mesh]; a batch when len > 1
    K: np.ndarray           # (sum E, npe, npe) float64 element matrices
    b: np.ndarray           # (sum n, nrhs) float64 right-hand sides, row-major
    coef: np.ndarray        # (sum E,) diffusion coefficient per element
    S: list                 # per mesh: reference stiffness (npe, npe)
    M: list                 # per mesh: reference mass (npe, npe)
    vel: Optional[np.ndarray] = None     # (sum E, dim) advection velocity per element
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(sum(m.n_nodes for m in self.meshes))

    @property
    def nrhs(self) -> int:
        return int(self.b.shape[1])

    @property
    def node_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([m.n_nodes for m in self.meshes])]).astype(np.int64)

    @property
    def elem_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([m.n_elem for m in self.meshes])]).astype(np.int64)


def structured_q1(shape: Sequence[int], lengths: Optional[Sequence[float]] = None) -> Mesh:
    """Uniform Q1 mesh of ``shape`` elements on the box with side ``lengths`` (unit box default)."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3) or min(shape) < 1:
        raise ValueError(f"bad mesh shape {shape}")
    lengths = tuple(1.0 for _ in shape) if lengths is None else tuple(float(x) for x in lengths)
    h = tuple(L / s for L, s in zip(lengths, shape))
    grids = np.meshgrid(*[np.arange(s, dtype=np.int64) for s in shape], indexing="ij")
    # element id i + nx*(j + ny*k): axis 0 fastest, so flatten in Fortran order
    ijk = np.stack([g.ravel(order="F") for g in grids], axis=1)
    nstride = np.cumprod([1] + [s + 1 for s in shape[:-1]]).astype(np.int64)
    npe = 1 << dim
    conn = np.empty((ijk.shape[0], npe), dtype=np.int64)
    for a in range(npe):
        c = np.array([(a >> d) & 1 for d in range(dim)], dtype=np.int64)
        conn[:, a] = ((ijk + c) * nstride).sum(axis=1)
    return Mesh(dim, shape, conn.astype(np.int32), ijk.astype(np.int32), h)


def q1_reference_matrices(h: Sequence[float]):
    """Stiffness S, mass M and advection parts C[d] (C[d][a,b] = int phi_a d(phi_b)/dx_d)
    of one Q1 element with edge lengths ``h``, by 2-point Gauss-Legendre per axis."""
    h = tuple(float(x) for x in h)
    dim = len(h)
    npe = 1 << dim
    g = 1.0 / np.sqrt(3.0)
    pts = np.array([(1.0 - g) / 2.0, (1.0 + g) / 2.0])    # on [0, 1]
    wts = np.array([0.5, 0.5])
    S = np.zeros((npe, npe))
    M = np.zeros((npe, npe))
    C = [np.zeros((npe, npe)) for _ in range(dim)]
    vol = float(np.prod(h))
    for q in np.ndindex(*([2] * dim)):
        t = [pts[q[d]] for d in range(dim)]
        w = vol * float(np.prod([wts[q[d]] for d in range(dim)]))
        phi = np.empty(npe)
        grad = np.empty((npe, dim))
        for a in range(npe):
            c = [(a >> d) & 1 for d in range(dim)]
            f = [t[d] if c[d] else 1.0 - t[d] for d in range(dim)]
            df = [(1.0 if c[d] else -1.0) / h[d] for d in range(dim)]
            phi[a] = np.prod(f)
            for d in range(dim):
                grad[a, d] = df[d] * np.prod([f[e] for e in range(dim) if e != d])
        S += w * grad @ grad.T
        M += w * np.outer(phi, phi)
        for d in range(dim):
            C[d] += w * np.outer(phi, grad[:, d])
    return S, M, C


def element_matrices(mesh: Mesh, coef: np.ndarray, vel: Optional[np.ndarray] = None) -> np.ndarray:
    """K_e = coef_e * S + M (+ sum_d vel_e[d] * C[d]) for every element, shape (E, npe, npe)."""
    S, M, C = q1_reference_matrices(mesh.h)
    K = coef[:, None, None] * S[None] + M[None]
    if vel is not None:
        for d in range(mesh.dim):
            K = K + vel[:, d, None, None] * C[d][None]
    return np.ascontiguousarray(K)


def _lognormal(rng, sigma: float, size: int) -> np.ndarray:
    return np.exp(rng.normal(0.0, sigma, size=size))


def reaction_diffusion(name: str, shape, rng, coef_kind: str, sigma: float, nrhs: int,
                       lengths=None) -> Problem:
    mesh = structured_q1(shape, lengths)
    if coef_kind == "uniform":
        coef = rng.uniform(0.5, 2.0, size=mesh.n_elem)
    elif coef_kind == "lognormal":
        coef = _lognormal(rng, sigma, mesh.n_elem)
    elif coef_kind == "zero":
        coef = np.zeros(mesh.n_elem)
    else:
        raise ValueError(coef_kind)
    K = element_matrices(mesh, coef)
    b = rng.normal(0.0, 1.0, size=(mesh.n_nodes, nrhs))
    S, M, _ = q1_reference_matrices(mesh.h)
    return Problem(name, [mesh], K, b, coef, [S], [M])


def advection_diffusion(name: str, sides: np.ndarray, rng, sigma: float, nrhs: int) -> Problem:
    """Batch of 2D unit-square meshes with per-element diffusion D_e ~ lognormal(sigma) and
    velocity u_e ~ U[-1,1]^2 scaled so that the element Peclet number |v| h / (2 D) <= 0.9,
    h = max(hx, hy).  A unit reaction (mass) term keeps each system nonsingular."""
    meshes, Ks, coefs, vels, Ss, Ms = [], [], [], [], [], []
    for nx, ny in sides:
        mesh = structured_q1((int(nx), int(ny)))
        D = _lognormal(rng, sigma, mesh.n_elem)
        u = rng.uniform(-1.0, 1.0, size=(mesh.n_elem, 2))
        hmax = max(mesh.h)
        speed = np.linalg.norm(u, axis=1)
        scale = np.minimum(1.0, 0.9 * 2.0 * D / (hmax * np.maximum(speed, 1e-300)))
        v = u * scale[:, None]
        meshes.append(mesh)
        Ks.append(element_matrices(mesh, D, v))
        coefs.append(D)
        vels.append(v)
        S, M, _ = q1_reference_matrices(mesh.h)
        Ss.append(S)
        Ms.append(M)
    n = sum(m.n_nodes for m in meshes)
    b = rng.normal(0.0, 1.0, size=(n, nrhs))
    return Problem(name, meshes, np.concatenate(Ks), b, np.concatenate(coefs), Ss, Ms,
                   vel=np.concatenate(vels))


CONFIGS = {
    1: "2D Q1 16x16 reaction-diffusion, k ~ U[0.5,2], 1 RHS, FP64",
    2: "2D Q1 256x256 reaction-diffusion, k ~ lognormal(0,1), 8 RHS, FP64",
    3: "3D Q1 32x32x32 reaction-diffusion, k ~ lognormal(0,1), 1 RHS, mixed precision",
    4: "256 2D Q1 meshes, sides U{32..128}, advection-diffusion, 1 RHS, batched",
    5: "2D Q1 128x128 reaction-diffusion, k ~ lognormal(0,0.5), 64 RHS, adjoint",
}


def config_problem(cfg: int, shape=None, n_mesh: Optional[int] = None,
                   side_range=(32, 128), nrhs: Optional[int] = None) -> Problem:
    """The seeded workload of configuration ``cfg`` (1..5).  ``shape``/``n_mesh``/``side_range``
    /``nrhs`` shrink it for tests while keeping the recipe (distributions, seed, draw order)."""
    rng = np.random.default_rng(cfg)
    if cfg == 1:
        return reaction_diffusion("cfg1", shape or (16, 16), rng, "uniform", 0.0, nrhs or 1)
    if cfg == 2:
        return reaction_diffusion("cfg2", shape or (256, 256), rng, "lognormal", 1.0, nrhs or 8)
    if cfg == 3:
        return reaction_diffusion("cfg3", shape or (32, 32, 32), rng, "lognormal", 1.0, nrhs or 1)
    if cfg == 4:
        nm = 256 if n_mesh is None else int(n_mesh)
        lo, hi = side_range
        sides = rng.integers(lo, hi + 1, size=(nm, 2))
        return advection_diffusion("cfg4", sides, rng, 1.0, nrhs or 1)
    if cfg == 5:
        p = reaction_diffusion("cfg5", shape or (128, 128), rng, "lognormal", 0.5, nrhs or 64)
        rt = np.random.default_rng(50)
        p.extra["k_target"] = _lognormal(rt, 0.5, p.meshes[0].n_elem)
        return p
    raise ValueError(f"unknown configuration {cfg}")
