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
    conn: np.ndarray        # (E, (p+1)**dim) int32 global node ids in tensor-product local order
    ijk: np.ndarray         # (E, dim) int32 element index coordinates
    h: tuple                # element edge length per axis
    p: int = 1              # polynomial degree per axis (Q_p Lagrange elements)

    @property
    def npe(self) -> int:
        return (self.p + 1) ** self.dim

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(np.prod([self.p * s + 1 for s in self.shape]))


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


def structured_qp(shape: Sequence[int], p: int, lengths: Optional[Sequence[float]] = None) -> Mesh:
    """Uniform mesh of Q_p Lagrange elements (equispaced nodes, p = 1..3).  Nodes form the
    (p*nx+1) x (p*ny+1)[ x (p*nz+1)] lattice, lattice point (I, J[, K]) has id
    I + (p*nx+1)*(J + (p*ny+1)*K); local node a = c_x + (p+1)*c_y [+ (p+1)^2*c_z] with
    c in {0..p} sits at lattice point p*(i, j[, k]) + c.  p = 1 is ``structured_q1``."""
    p = int(p)
    if p < 1 or p > 3:
        raise ValueError(f"polynomial degree {p} not in 1..3")
    q1 = structured_q1(shape, lengths)
    dim, ijk = q1.dim, q1.ijk.astype(np.int64)
    if p == 1:
        return q1
    nstride = np.cumprod([1] + [p * s + 1 for s in q1.shape[:-1]]).astype(np.int64)
    npe = (p + 1) ** dim
    conn = np.empty((ijk.shape[0], npe), dtype=np.int64)
    for a in range(npe):
        c = np.array([(a // (p + 1) ** d) % (p + 1) for d in range(dim)], dtype=np.int64)
        conn[:, a] = ((p * ijk + c) * nstride).sum(axis=1)
    return Mesh(dim, q1.shape, conn.astype(np.int32), q1.ijk, q1.h, p)


def lagrange_1d(p: int, t: np.ndarray):
    """Values and derivatives (d/dt) of the p+1 Lagrange polynomials on the nodes i/p of [0, 1]
    at the points t: two arrays (len(t), p+1)."""
    nodes = np.arange(p + 1) / p
    t = np.asarray(t, dtype=np.float64)
    val = np.ones((t.size, p + 1))
    der = np.zeros((t.size, p + 1))
    for i in range(p + 1):
        others = [j for j in range(p + 1) if j != i]
        den = np.prod([nodes[i] - nodes[j] for j in others])
        fac = [(t - nodes[j]) for j in others]
        val[:, i] = np.prod(fac, axis=0) / den
        for s_ in range(len(others)):
            der[:, i] += np.prod([fac[r] for r in range(len(others)) if r != s_], axis=0) / den
    return val, der


def _tensor_basis(h: Sequence[float], p: int):
    """phi (Q, npe), grad (Q, npe, dim), weights (Q,) at the (p+1)^dim Gauss-Legendre points of
    an element with edge lengths h (exact for the mass and stiffness integrands of Q_p)."""
    dim = len(h)
    x, w = np.polynomial.legendre.leggauss(p + 1)
    t, wt = (x + 1.0) / 2.0, w / 2.0
    B, D = lagrange_1d(p, t)
    npe = (p + 1) ** dim
    pts = list(np.ndindex(*([p + 1] * dim)))
    phi = np.ones((len(pts), npe))
    grad = np.ones((len(pts), npe, dim))
    wq = np.empty(len(pts))
    for qi, q in enumerate(pts):
        wq[qi] = float(np.prod([wt[q[d]] * h[d] for d in range(dim)]))
        for a in range(npe):
            c = [(a // (p + 1) ** d) % (p + 1) for d in range(dim)]
            for d in range(dim):
                phi[qi, a] *= B[q[d], c[d]]
                for e in range(dim):
                    grad[qi, a, e] *= (D[q[d], c[d]] / h[d]) if d == e else B[q[d], c[d]]
    return phi, grad, wq, pts, t


def qp_reference_matrices(h: Sequence[float], p: int):
    """Stiffness S, mass M and advection parts C[d] of one Q_p element with edge lengths h, by
    (p+1)-point Gauss-Legendre per axis on tensor-product Lagrange bases."""
    h = tuple(float(x) for x in h)
    phi, grad, wq, _, _ = _tensor_basis(h, p)
    S = np.einsum("q,qad,qbd->ab", wq, grad, grad)
    M = np.einsum("q,qa,qb->ab", wq, phi, phi)
    C = [np.einsum("q,qa,qb->ab", wq, phi, grad[:, :, d]) for d in range(len(h))]
    return S, M, C


def load_vector(mesh: Mesh, f) -> np.ndarray:
    """b_i = int f phi_i over the mesh, by (p+1)-point Gauss-Legendre per axis on each element;
    f maps an (N, dim) array of points to N values."""
    phi, _, wq, pts, t = _tensor_basis(mesh.h, mesh.p)
    dim = mesh.dim
    off = np.asarray(mesh.ijk, dtype=np.float64) * np.asarray(mesh.h)[None, :]   # (E, dim)
    loc = np.array([[t[q[d]] * mesh.h[d] for d in range(dim)] for q in pts])  # (Q, dim)
    fx = f((off[:, None, :] + loc[None, :, :]).reshape(-1, dim)).reshape(mesh.n_elem, len(pts))
    be = (fx * wq[None, :]) @ phi                                               # (E, npe)
    b = np.zeros(mesh.n_nodes)
    np.add.at(b, mesh.conn.reshape(-1), be.reshape(-1))
    return b


def node_coords(mesh: Mesh) -> np.ndarray:
    """(n_nodes, dim) coordinates of the lattice nodes."""
    ax = [np.arange(mesh.p * s + 1) * (hd / mesh.p) for s, hd in zip(mesh.shape, mesh.h)]
    g = np.meshgrid(*ax, indexing="ij")
    return np.stack([x.ravel(order="F") for x in g], axis=1)


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


def reference_matrices(mesh: Mesh):
    """(S, M, C) of the mesh's element: the Q1 closed construction for p = 1, else Q_p."""
    return q1_reference_matrices(mesh.h) if mesh.p == 1 else qp_reference_matrices(mesh.h, mesh.p)


def element_matrices(mesh: Mesh, coef: np.ndarray, vel: Optional[np.ndarray] = None) -> np.ndarray:
    """K_e = coef_e * S + M (+ sum_d vel_e[d] * C[d]) for every element, shape (E, npe, npe)."""
    S, M, C = reference_matrices(mesh)
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


def l2_projection(name: str, shape, p: int, rng, nrhs: int, f=None) -> Problem:
    """The paper's model problem (Sec. 2.1, eqs. L2_proj and Linear_system): the Q_p mass-matrix
    system M u = b with b_i = (f, phi_i).  Without ``f`` the right-hand sides are the load
    vectors of f_r(x) = cos(w_r . x + c_r), w_r ~ N(0, 4^2)^dim, c_r ~ U[0, 2 pi), drawn in the
    order w, c per column; with ``f`` every column is f's load vector."""
    mesh = structured_qp(shape, p)
    S, M, _ = reference_matrices(mesh)
    K = np.ascontiguousarray(np.broadcast_to(M, (mesh.n_elem,) + M.shape))
    cols = []
    for _ in range(nrhs):
        if f is not None:
            cols.append(load_vector(mesh, f))
            continue
        w = rng.normal(0.0, 4.0, size=mesh.dim)
        c = rng.uniform(0.0, 2.0 * np.pi)
        cols.append(load_vector(mesh, lambda x, w=w, c=c: np.cos(x @ w + c)))
    b = np.ascontiguousarray(np.stack(cols, axis=1))
    return Problem(name, [mesh], K, b, np.zeros(mesh.n_elem), [S], [M], extra={"p": p})


# The paper's benchmark axis (Sec. 5): L2 projection with linear, quadratic and cubic bases up
# to 3e5 unknowns.  All three use the same 547 x 547 node lattice (299,209 unknowns).
L2_SHAPES = {1: (546, 546), 2: (273, 273), 3: (182, 182)}


def l2_workload(p: int, shape=None, nrhs: int = 1) -> Problem:
    """Seeded L2-projection workload of degree p (seed 100 + p)."""
    return l2_projection(f"l2p{p}", shape or L2_SHAPES[p], p, np.random.default_rng(100 + p), nrhs)


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
