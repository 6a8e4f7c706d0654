"""Seeded synthetic inputs for the Sparse Gauss-Newton workloads.

This module is shared by the FP64 oracle (``oracle/``) and by the GPU path's
harness (tests, ``bench.py``).  It holds only problem *data*: meshes, boundary
conditions, lumped dead loads, parameter layouts and seeded random fields.  It
holds none of the method's arithmetic (no energies, derivatives, equilibria or
solves).  Quantities that need a forward simulation (targets that are
equilibrium positions, the length scale ``ell``) are left to the side that uses
the problem; the random numbers they need (stiffness fields, target noise) are
drawn here and passed in.

The physical setting follows the paper's inverse elastic design example
(Sec. 5.1): linear simplices, a neo-Hookean material with E = 1e6 Pa, one end
clamped.  Mesh conventions:

* 2D: an ``n x n`` node grid on the unit square, node id ``j*n + i``; square
  (i, j) with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) is split into
  triangles (a,b,c), (a,c,d), squares in row-major order.  Bottom row fixed,
  gravity rho*g = 9810 N/m^3 along -y lumped 1/3 of each triangle's area to
  its nodes (plane strain, unit thickness).
* 3D: an ``nx x ny x nz`` hex grid of spacing h, node id
  ``(k*(ny+1) + j)*(nx+1) + i``.  Each hex is split into 5 tets: a central tet
  on the four corners whose global index parity (i+di+j+dj+k+dk) is odd, and
  four corner tets (each remaining corner with its three edge neighbours), so
  face diagonals match between neighbouring hexes.  Tet order per hex: central
  first, then corner tets by ascending local corner index di + 2 dj + 4 dk.
  Every tet is oriented to positive volume.  The x = 0 face is clamped; a
  traction of 800 N/m^2 along a seeded unit direction acts on the x = L face,
  lumped h^2/4 per face quad to its corners.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

P_LOGE = 0        # one log-Young's-modulus parameter per element: E_e = E0 exp(p_e)
P_REST_POS = 1    # rest positions of the free nodes (n_free * dim parameters)
P_NODAL_FORCE = 2  # test-only: one additive nodal force per free DOF, c = grad E - f_ext - p


@dataclasses.dataclass
class Problem:
    """An equilibrium-constrained inverse problem  min_p f(x(p), p)  s.t.  c(x, p) = 0.

    All arrays are host numpy arrays.  ``x`` and the constraint vector are laid
    out over free DOFs only: free nodes in ascending node id, ``dim``
    components each.
    """
    name: str
    dim: int
    rest_pos: np.ndarray          # [n_nodes, dim] float64
    elems: np.ndarray             # [n_elems, dim+1] int32, positively oriented
    fixed: np.ndarray             # [n_nodes] uint8, 1 = Dirichlet on all components
    f_ext: np.ndarray             # [n_nodes, dim] float64 dead nodal loads
    E0: float
    nu: float
    param_kind: int
    target_dof: np.ndarray        # [n_t] int32 indices into the free-DOF vector
    target_val: Optional[np.ndarray] = None  # [n_t] float64 (set once known)
    target_w: float = 1.0
    length_scale: Optional[float] = None      # ell, frozen at setup
    reg_mu: float = 1e-4
    p_ref: Optional[np.ndarray] = None        # [n_p]
    # seeded random fields consumed by whoever builds targets
    p_star: Optional[np.ndarray] = None       # stiffness field that generates targets (log-E)
    target_noise: Optional[np.ndarray] = None  # [n_t] additive noise on x(p0)
    seed: int = 0
    grid: tuple = ()
    # a batch of independent problems: node ranges of the components and their own grid coordinates
    components: Optional[np.ndarray] = None
    node_grid_override: Optional[np.ndarray] = None

    @property
    def n_nodes(self) -> int:
        return int(self.rest_pos.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def free_nodes(self) -> np.ndarray:
        return np.flatnonzero(self.fixed == 0).astype(np.int32)

    @property
    def n_x(self) -> int:
        return int(self.free_nodes.size * self.dim)

    @property
    def n_p(self) -> int:
        if self.param_kind == P_LOGE:
            return self.n_elems
        return self.n_x

    def free_dof_of_node(self) -> np.ndarray:
        """[n_nodes] -> first free-DOF index of the node, -1 when fixed."""
        m = np.full(self.n_nodes, -1, dtype=np.int64)
        fn = self.free_nodes
        m[fn] = np.arange(fn.size, dtype=np.int64) * self.dim
        return m

    def node_grid(self) -> np.ndarray:
        """[n_nodes, dim] integer grid coordinates of every node (axis 0 fastest in the node id)."""
        if self.node_grid_override is not None:
            return self.node_grid_override
        ids = np.arange(self.n_nodes)
        if self.dim == 2:
            n = self.grid[0]
            return np.stack([ids % n, ids // n], axis=1).astype(np.int32)
        nx, ny, _ = self.grid
        Nx, Ny = nx + 1, ny + 1
        return np.stack([ids % Nx, (ids // Nx) % Ny, ids // (Nx * Ny)], axis=1).astype(np.int32)

    def x_rest(self) -> np.ndarray:
        """Free-DOF vector of the rest positions (the natural initial guess)."""
        return self.rest_pos[self.free_nodes].reshape(-1).astype(np.float64).copy()

    def p_init(self) -> np.ndarray:
        if self.param_kind == P_REST_POS:
            return self.x_rest()
        return np.zeros(self.n_p)

    def copy(self) -> "Problem":
        return dataclasses.replace(self)


# ----------------------------------------------------------------------------- meshes

def grid2d(n: int):
    """Node positions, triangles and the bottom-row Dirichlet mask of an n x n unit-square grid."""
    h = 1.0 / (n - 1)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pos = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            b = a + 1
            c = a + n + 1
            d = a + n
            tris.append((a, b, c))
            tris.append((a, c, d))
    elems = np.asarray(tris, dtype=np.int32)
    fixed = np.zeros(n * n, dtype=np.uint8)
    fixed[:n] = 1
    return pos, elems, fixed


def _orient(pos: np.ndarray, elems: np.ndarray) -> np.ndarray:
    """Swap the last two vertices of negatively oriented simplices (mesh hygiene)."""
    P = pos[elems]
    D = P[:, 1:, :] - P[:, :1, :]
    s = np.linalg.det(D)
    e = elems.copy()
    neg = s < 0
    e[neg, -1], e[neg, -2] = elems[neg, -2], elems[neg, -1]
    return e


def hexgrid3d(nx: int, ny: int, nz: int, h: float):
    """Node positions, 5-tet-per-hex tets and the x = 0 clamp of an nx x ny x nz hex grid."""
    Nx, Ny, Nz = nx + 1, ny + 1, nz + 1
    kk, jj, ii = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    pos = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)

    corner_bits = [(c & 1, (c >> 1) & 1, (c >> 2) & 1) for c in range(8)]
    tets = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                q = (i + j + k) & 1
                node = [((k + b[2]) * Ny + (j + b[1])) * Nx + (i + b[0]) for b in corner_bits]
                central = [c for c in range(8) if ((sum(corner_bits[c]) + q) & 1) == 1]
                corners = [c for c in range(8) if c not in central]
                tets.append([node[c] for c in central])
                for c in corners:  # ascending local corner index
                    tets.append([node[c], node[c ^ 1], node[c ^ 2], node[c ^ 4]])
    elems = _orient(pos, np.asarray(tets, dtype=np.int32))
    fixed = (ii.ravel() == 0).astype(np.uint8)
    return pos, elems, fixed


# ----------------------------------------------------------------------------- loads

def gravity2d(pos: np.ndarray, elems: np.ndarray, rho_g: float = 9810.0) -> np.ndarray:
    """Gravity along -y lumped a third of each triangle's area to each of its nodes."""
    P = pos[elems]
    d1 = P[:, 1] - P[:, 0]
    d2 = P[:, 2] - P[:, 0]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    f = np.zeros_like(pos)
    for a in range(3):
        np.add.at(f[:, 1], elems[:, a], -rho_g * area / 3.0)
    return f


def tip_traction3d(nx: int, ny: int, nz: int, h: float, direction: np.ndarray,
                   magnitude: float = 800.0) -> np.ndarray:
    """Traction on the x = L face lumped h^2/4 per face quad to its four corners."""
    Nx, Ny, Nz = nx + 1, ny + 1, nz + 1
    f = np.zeros((Nx * Ny * Nz, 3))
    w = np.zeros(Nx * Ny * Nz)
    i = nx
    for k in range(nz):
        for j in range(ny):
            for dk in (0, 1):
                for dj in (0, 1):
                    w[((k + dk) * Ny + (j + dj)) * Nx + i] += h * h / 4.0
    f += magnitude * w[:, None] * direction[None, :]
    return f


# ----------------------------------------------------------------------------- problems

def problem_2d(n: int = 21, seed: int = 0, param_kind: int = P_LOGE, nu: float = 0.3,
               reg_mu: float = 1e-4, name: Optional[str] = None) -> Problem:
    """The 2D membrane family: n x n nodes, bottom row fixed, gravity, top-row targets.

    Targets are the top-row node positions (both components) of the forward
    solve under the seeded stiffness field p* = 0.3 z, z ~ N(0, 1) per
    triangle; ``p_star`` carries that field.
    """
    pos, elems, fixed = grid2d(n)
    rng = np.random.default_rng(seed)
    p_star = 0.3 * rng.standard_normal(elems.shape[0])
    prob = Problem(name=name or f"grid2d_{n}x{n}_s{seed}", dim=2, rest_pos=pos, elems=elems,
                   fixed=fixed, f_ext=gravity2d(pos, elems), E0=1e6, nu=nu,
                   param_kind=param_kind, target_dof=np.zeros(0, np.int32), reg_mu=reg_mu,
                   seed=seed, grid=(n, n))
    fdof = prob.free_dof_of_node()
    top = np.arange(n * (n - 1), n * n)
    prob.target_dof = np.concatenate([[fdof[v], fdof[v] + 1] for v in top]).astype(np.int32)
    prob.p_star = p_star if param_kind == P_LOGE else None
    prob.p_ref = prob.p_init()
    return prob


def surface_nodes3d(nx: int, ny: int, nz: int) -> np.ndarray:
    Nx, Ny, Nz = nx + 1, ny + 1, nz + 1
    kk, jj, ii = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    on = (ii == 0) | (ii == nx) | (jj == 0) | (jj == ny) | (kk == 0) | (kk == nz)
    return np.flatnonzero(on & (ii != 0)).astype(np.int32)


def problem_3d(nx: int = 40, ny: int = 10, nz: int = 10, h: float = 0.1, seed: int = 0,
               param_kind: int = P_LOGE, nu: float = 0.45, reg_mu: float = 1e-4,
               target_sigma_frac: float = 0.01, name: Optional[str] = None) -> Problem:
    """The 3D cantilever family: x = 0 clamped, seeded tip traction, surface targets.

    Targets are x(p0) + noise on every free boundary-surface node, the noise
    drawn here as N(0, (target_sigma_frac * L)^2) per coordinate, L = nx*h.
    """
    pos, elems, fixed = hexgrid3d(nx, ny, nz, h)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    f_ext = tip_traction3d(nx, ny, nz, h, d)
    prob = Problem(name=name or f"cantilever_{nx}x{ny}x{nz}_s{seed}", dim=3, rest_pos=pos,
                   elems=elems, fixed=fixed, f_ext=f_ext, E0=1e6, nu=nu, param_kind=param_kind,
                   target_dof=np.zeros(0, np.int32), reg_mu=reg_mu, seed=seed, grid=(nx, ny, nz))
    fdof = prob.free_dof_of_node()
    surf = surface_nodes3d(nx, ny, nz)
    prob.target_dof = (fdof[surf][:, None] + np.arange(3)[None, :]).ravel().astype(np.int32)
    L = nx * h
    prob.target_noise = target_sigma_frac * L * rng.standard_normal(prob.target_dof.size)
    if param_kind == P_LOGE:
        prob.p_star = 0.3 * rng.standard_normal(elems.shape[0])
    prob.p_ref = prob.p_init()
    return prob


# Workload presets -------------------------------------------------------------------------

def config_tiny(seed: int = 0) -> Problem:
    """4 x 4-node 2D grid (18 triangles): the dense-GN equivalence case."""
    return problem_2d(4, seed=seed, name=f"grid2d_4x4_s{seed}")


def config_2d(seed: int = 0) -> Problem:
    """21 x 21-node 2D grid, 800 triangles, log-E per triangle."""
    return problem_2d(21, seed=seed)


def config_cantilever_small(seed: int = 0) -> Problem:
    """40 x 10 x 10 hex cantilever (20,000 tets), rest-position parameters."""
    return problem_3d(40, 10, 10, 0.1, seed=seed, param_kind=P_REST_POS)


def config_cantilever_200k(seed: int = 0) -> Problem:
    """100 x 25 x 25 hex cantilever (312,500 tets, 202,800 free DOF), log-E per tet."""
    return problem_3d(100, 25, 25, 0.04, seed=seed, param_kind=P_LOGE)


def learned_pc_problem(seed: int) -> Problem:
    """Cantilever (even seed) or plate (odd seed) with s ~ U{5..20}: 4s x s x s or 4s x s x max(2, ceil(s/4))."""
    rng = np.random.default_rng(50_000 + seed)
    s = int(rng.integers(5, 21))
    nz = s if seed % 2 == 0 else max(2, -(-s // 4))
    return problem_3d(4 * s, s, nz, 1.0 / s, seed=seed, param_kind=P_LOGE,
                      name=f"{'cantilever' if seed % 2 == 0 else 'plate'}_{4*s}x{s}x{nz}_s{seed}")


def union_problem(problems, name: str = "batch") -> Problem:
    """The disjoint union of independent problems of one family as a single problem: nodes, elements,
    free DOFs, parameters, targets and fields concatenated in order; ``components`` marks each
    problem's node range and ``node_grid_override`` keeps each problem's own grid coordinates.
    Problems must share dim, parameter kind, material constants, target weight, ell and mu."""
    first = problems[0]
    for q in problems[1:]:
        assert (q.dim, q.param_kind, q.E0, q.nu, q.target_w, q.reg_mu) == \
            (first.dim, first.param_kind, first.E0, first.nu, first.target_w, first.reg_mu)
    node_off = np.concatenate([[0], np.cumsum([q.n_nodes for q in problems])])
    x_off = np.concatenate([[0], np.cumsum([q.n_x for q in problems])])

    def cat(field):
        vals = [getattr(q, field) for q in problems]
        return None if any(v is None for v in vals) else np.concatenate(vals)
    u = Problem(
        name=name, dim=first.dim,
        rest_pos=np.concatenate([q.rest_pos for q in problems]),
        elems=np.concatenate([q.elems + node_off[i] for i, q in enumerate(problems)]).astype(np.int32),
        fixed=np.concatenate([q.fixed for q in problems]),
        f_ext=np.concatenate([q.f_ext for q in problems]),
        E0=first.E0, nu=first.nu, param_kind=first.param_kind,
        target_dof=np.concatenate([q.target_dof + x_off[i] for i, q in enumerate(problems)]).astype(np.int32),
        target_val=cat("target_val"), target_w=first.target_w, length_scale=first.length_scale,
        reg_mu=first.reg_mu, p_ref=cat("p_ref"), p_star=cat("p_star"), target_noise=cat("target_noise"),
        seed=first.seed, grid=(),
        components=node_off.astype(np.int32),
        node_grid_override=np.concatenate([q.node_grid() for q in problems]).astype(np.int32))
    return u


def batch_problems(count: int = 256, base_seed: int = 10000, lo: int = 8, hi: int = 48):
    """Independent 2D membrane problems with n ~ U{lo..hi} nodes per side."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.integers(lo, hi + 1))
        out.append(problem_2d(n, seed=base_seed + i))
    return out
