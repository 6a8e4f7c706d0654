"""Symbolic structure of the SGN saddle-point matrix (test infrastructure).

The matrix of eq. sparseSystemGN, K = [[A, B^T, Kx^T], [B, C, Kp^T],
[Kx, Kp, 0]], over the unknowns [dx; dp; dlam] (n_x + n_p + n_x of them).  The
paper delegates ordering and symbolic analysis to its sparse direct solver, so
everything here is a reading (listed in the design notes):

* Pattern.  A is diagonal (nonzero on target DOFs), C = mu I, B = 0; every
  diagonal of x, p and lambda is kept structurally, even when zero.  The
  Kx block holds every (lambda_i, x_j) pair of free DOFs whose nodes share an
  element.  Kp holds (lambda_i, p_e) for each free DOF i of element e
  (log-modulus parameters), the node-pair blocks (lambda_i, X_j) for
  rest-position parameters, and (lambda_i, p_i) for nodal forces.
* Node order: geometric nested dissection on the node grid.  rec(box) over
  free nodes: if the box has <= 8 grid points or its largest extent is <= 2,
  emit its free nodes lexicographically (axis 0 fastest); otherwise split the
  largest axis (ties to the lowest axis) at mid = lo + ext // 2, recurse into
  [lo, mid), then [mid+1, hi), then emit the plane coord = mid.
* Variable order: walk the node order; for node v emit its owned parameters
  (log-E: elements whose earliest-ordered free node is v, ascending element
  id; rest position / nodal force: v's d components), then x_v's d
  components, then lambda_v's d components.
* CSR: lower triangle of P K P^T, rows ascending, columns ascending.
* Elimination tree of that lower pattern: parent(j) = min{i > j : L_ij != 0}.

Three independent etree routines are provided (Liu's ancestor algorithm, the
column-structure definition, and brute-force dense boolean elimination) so
that each can be checked against the others.
"""
from __future__ import annotations

import numpy as np

from sgn_inputs import P_LOGE, P_NODAL_FORCE, P_REST_POS, Problem


def grid_coords(prob: Problem) -> np.ndarray:
    """Integer grid coordinates of every node, [n_nodes, dim]."""
    if prob.dim == 2:
        n = prob.grid[0]
        ids = np.arange(prob.n_nodes)
        return np.stack([ids % n, ids // n], axis=1)
    nx, ny, nz = prob.grid
    Nx, Ny = nx + 1, ny + 1
    ids = np.arange(prob.n_nodes)
    return np.stack([ids % Nx, (ids // Nx) % Ny, ids // (Nx * Ny)], axis=1)


def grid_shape(prob: Problem):
    if prob.dim == 2:
        return (prob.grid[0], prob.grid[0])
    nx, ny, nz = prob.grid
    return (nx + 1, ny + 1, nz + 1)


def nd_node_order(prob: Problem) -> np.ndarray:
    """Free nodes in nested-dissection order (the rule in the module docstring)."""
    shape = grid_shape(prob)
    d = len(shape)
    fixed = prob.fixed.reshape(shape[::-1])  # index [k][j][i] or [j][i]
    out = []

    def node_id(c):
        if d == 2:
            return c[1] * shape[0] + c[0]
        return (c[2] * shape[1] + c[1]) * shape[0] + c[0]

    def emit_box(lo, hi):
        # lexicographic with axis 0 fastest: iterate the highest axis outermost
        if d == 2:
            for j in range(lo[1], hi[1]):
                for i in range(lo[0], hi[0]):
                    v = node_id((i, j))
                    if not prob.fixed[v]:
                        out.append(v)
        else:
            for k in range(lo[2], hi[2]):
                for j in range(lo[1], hi[1]):
                    for i in range(lo[0], hi[0]):
                        v = node_id((i, j, k))
                        if not prob.fixed[v]:
                            out.append(v)

    def rec(lo, hi):
        ext = [hi[a] - lo[a] for a in range(d)]
        if min(ext) <= 0:
            return
        if int(np.prod(ext)) <= 8 or max(ext) <= 2:
            emit_box(lo, hi)
            return
        ax = int(np.argmax(ext))  # first maximum = lowest axis on ties
        mid = lo[ax] + ext[ax] // 2
        hi1 = list(hi)
        hi1[ax] = mid
        lo2 = list(lo)
        lo2[ax] = mid + 1
        rec(lo, hi1)
        rec(lo2, hi)
        los = list(lo)
        his = list(hi)
        los[ax] = mid
        his[ax] = mid + 1
        emit_box(los, his)

    rec([0] * d, list(shape))
    return np.asarray(out, dtype=np.int64)


def variable_order(prob: Problem) -> np.ndarray:
    """perm[new] = old over [x; p; lambda]."""
    d = prob.dim
    nx = prob.n_x
    npar = prob.n_p
    fdof = prob.free_dof_of_node()
    order = nd_node_order(prob)
    rank = np.full(prob.n_nodes, np.iinfo(np.int64).max)
    rank[order] = np.arange(order.size)
    owned = [[] for _ in range(prob.n_nodes)]
    orphan = []
    if prob.param_kind == P_LOGE:
        for e in range(prob.n_elems):
            best = None
            for v in prob.elems[e]:
                if not prob.fixed[v] and (best is None or rank[v] < rank[best]):
                    best = v
            if best is None:
                orphan.append(e)
            else:
                owned[best].append(e)
    perm = [nx + e for e in orphan]
    for v in order:
        base = fdof[v]
        if prob.param_kind == P_LOGE:
            perm.extend(nx + e for e in owned[v])  # appended in ascending element id
        else:
            perm.extend(nx + base + c for c in range(d))
        perm.extend(base + c for c in range(d))
        perm.extend(nx + npar + base + c for c in range(d))
    perm = np.asarray(perm, dtype=np.int64)
    assert perm.size == 2 * nx + npar
    return perm


def pattern_pairs(prob: Problem, newton: bool = False):
    """Unique (row, col) pairs, row >= col, of the lower pattern in the original numbering.  newton:
    the pattern of the Newton form (Appendix A; log-modulus parameters), whose x-x block couples the
    DOFs of one element (the second derivatives of lam^T c) and whose x-p block has the Kp pattern."""
    d = prob.dim
    nx, npar = prob.n_x, prob.n_p
    lam0 = nx + npar
    fdof = prob.free_dof_of_node()
    base = fdof[prob.elems]  # [ne, d+1]
    ne, nv = base.shape
    dofs = (base[:, :, None] + np.arange(d)[None, None, :]).reshape(ne, nv * d)
    freem = np.repeat(base >= 0, d, axis=1)
    keys = []
    N = 2 * nx + npar

    def add(r, c):
        r = np.asarray(r, dtype=np.int64).ravel()
        c = np.asarray(c, dtype=np.int64).ravel()
        hi = np.maximum(r, c)
        lo = np.minimum(r, c)
        keys.append(hi * N + lo)

    # Kx block: (lambda_i, x_j) for free i, j in one element
    R = np.broadcast_to(dofs[:, :, None], (ne, nv * d, nv * d))
    C = np.broadcast_to(dofs[:, None, :], (ne, nv * d, nv * d))
    m = np.broadcast_to(freem[:, :, None], R.shape) & np.broadcast_to(freem[:, None, :], R.shape)
    add(lam0 + R[m], C[m])
    # Kp block
    if prob.param_kind == P_LOGE:
        E = np.broadcast_to(np.arange(ne)[:, None], dofs.shape)
        add(lam0 + dofs[freem], nx + E[freem])
    elif prob.param_kind == P_REST_POS:
        add(lam0 + R[m], nx + C[m])
    else:
        add(lam0 + np.arange(nx), nx + np.arange(nx))
    if newton:
        if prob.param_kind != P_LOGE:
            raise ValueError("the Newton form is built for log-modulus parameters")
        add(R[m], C[m])
        add(dofs[freem], nx + E[freem])
    # all diagonals
    add(np.arange(N), np.arange(N))
    k = np.unique(np.concatenate(keys))
    return k // N, k % N


def permuted_lower_csr(prob: Problem, perm: np.ndarray = None, newton: bool = False):
    """(rowptr int64, colind int32) of the lower triangle of P K P^T."""
    if perm is None:
        perm = variable_order(prob)
    N = perm.size
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    r, c = pattern_pairs(prob, newton)
    nr, nc = inv[r], inv[c]
    hi = np.maximum(nr, nc)
    lo = np.minimum(nr, nc)
    key = np.sort(hi * N + lo)
    rows = key // N
    cols = (key % N).astype(np.int32)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols


def etree_liu(rowptr: np.ndarray, colind: np.ndarray) -> np.ndarray:
    """Elimination tree by Liu's ancestor algorithm with path compression (-1 = root)."""
    N = rowptr.size - 1
    parent = [-1] * N
    anc = [-1] * N
    rp = rowptr.tolist()
    ci = colind.tolist()
    for i in range(N):
        for t in range(rp[i], rp[i + 1]):
            j = ci[t]
            while j != -1 and j < i:
                nxt = anc[j]
                anc[j] = i
                if nxt == -1:
                    parent[j] = i
                j = nxt
    return np.asarray(parent, dtype=np.int64)


def etree_by_columns(rowptr: np.ndarray, colind: np.ndarray) -> np.ndarray:
    """Elimination tree from the definition: struct(L_j) = struct(A_j) U children's structs minus j."""
    N = rowptr.size - 1
    cols = [set() for _ in range(N)]
    for i in range(N):
        for t in range(rowptr[i], rowptr[i + 1]):
            j = int(colind[t])
            if j < i:
                cols[j].add(i)
    parent = np.full(N, -1, dtype=np.int64)
    children = [[] for _ in range(N)]
    for j in range(N):
        s = cols[j]
        for c in children[j]:
            s |= cols[c]
        s.discard(j)
        cols[j] = s
        if s:
            parent[j] = min(s)
            children[parent[j]].append(j)
        for c in children[j]:
            cols[c] = None
    return parent


def etree_dense(rowptr: np.ndarray, colind: np.ndarray) -> np.ndarray:
    """Elimination tree by explicit boolean Gaussian elimination (tiny matrices only)."""
    N = rowptr.size - 1
    M = np.zeros((N, N), dtype=bool)
    for i in range(N):
        for t in range(rowptr[i], rowptr[i + 1]):
            M[i, colind[t]] = True
            M[colind[t], i] = True
    parent = np.full(N, -1, dtype=np.int64)
    for j in range(N):
        below = np.flatnonzero(M[j + 1:, j]) + j + 1
        if below.size:
            parent[j] = below[0]
            M[np.ix_(below, below)] = True
    return parent
