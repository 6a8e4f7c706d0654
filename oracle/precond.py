"""Node-block preconditioner of the SGN saddle-point matrix, written out densely.

Test infrastructure only (see the package header): a plain FP64 statement of the
operator the library applies in its MINRES path.  The paper does not define a
preconditioner; it names preconditioning of the saddle-point system and iterative
saddle-point solvers as future work (Sec. 6.1) after standard preconditioned Krylov
methods did poorly on its problems (Sec. 5).  The construction is the library's:

  * variables in elimination order (nested-dissection node order, per node its
    owned parameters, x_v, lambda_v), symmetric equilibration
    S = diag(1 / sqrt(max_j |K_ij|));
  * LDL^T of S K S with Bunch-Kaufman pivoting (alpha = (1 + sqrt 17) / 8)
    restricted to each node's variable group: candidate rows and the column /
    row maxima that decide the pivot are taken inside the group only;
  * M = S^-1 P^T L B L^T P S^-1 with B = blockdiag_i(R_i C_i C_i^T R_i^T),
    R_i R_i^T = |D_i| (eigen-absolute value of the 1x1 / 2x2 pivots), and
    C_i built from raw corrections r: exp(r) on owned-parameter positions, and
    on the trailing 2d positions a lower-triangular block with diagonal
    exp(r_tt) and off-diagonal r_ij.

Parity pins (tests/test_oracle_precond.py): the factor reproduces P S K S P^T;
its inertia is (n_x + n_p, n_x, 0) (Sylvester); with zero corrections the
eigenvalues of M^-1 K are +-1 with that inertia; M is symmetric positive definite for random corrections; uniform
corrections scale M by exp(2c); the 2x2 eigen-convention gives eigenvectors with
the larger eigenvalue first; complex-step gradients agree with central
differences.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from sgn_inputs import P_LOGE, Problem

from . import dense as D
from .symbolic import nd_node_order, variable_order

ALPHA_BK = (1.0 + np.sqrt(17.0)) / 8.0


def node_groups(prob: Problem):
    """(starts [n_free+1], nodes [n_free]) of the node variable groups in elimination order."""
    d = prob.dim
    order = nd_node_order(prob)
    rank = np.full(prob.n_nodes, -1)
    rank[order] = np.arange(order.size)
    n_own = np.zeros(prob.n_nodes, dtype=np.int64)
    if prob.param_kind == P_LOGE:
        for e in range(prob.n_elems):
            free = [v for v in prob.elems[e] if not prob.fixed[v]]
            n_own[min(free, key=lambda v: rank[v])] += 1
    else:
        n_own[:] = d
    sizes = np.array([n_own[v] + 2 * d for v in order], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    return starts, np.asarray(order, dtype=np.int64)


def equilibration(K: np.ndarray) -> np.ndarray:
    """S_i = 1 / sqrt(max_j |K_ij|) (1 for an empty row)."""
    m = np.max(np.abs(K), axis=1)
    return np.where(m > 0, 1.0 / np.sqrt(np.where(m > 0, m, 1.0)), 1.0)


def group_bk_ldlt(A: np.ndarray, starts: np.ndarray):
    """P A P^T = L D L^T with Bunch-Kaufman pivots restricted to the groups [starts[i], starts[i+1]).

    Returns (piv, L, dmat, kinds): piv[k] = row of A at pivot position k, L unit lower
    triangular, dmat the block-diagonal D, kinds[k] = 0 (1x1), 1 / 2 (first / second of 2x2).
    Dense, right-looking, with explicit symmetric interchanges.
    """
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    gend = np.zeros(n, dtype=np.int64)
    for g in range(len(starts) - 1):
        gend[starts[g]:starts[g + 1]] = starts[g + 1]
    piv = np.arange(n)
    L = np.eye(n)
    dmat = np.zeros((n, n))
    kinds = np.zeros(n, dtype=np.int64)

    def swap(i, j):
        if i == j:
            return
        A[[i, j], :] = A[[j, i], :]
        A[:, [i, j]] = A[:, [j, i]]
        L[[i, j], :k] = L[[j, i], :k]
        piv[[i, j]] = piv[[j, i]]

    k = 0
    while k < n:
        ge = gend[k]
        col = np.abs(A[k + 1:ge, k])
        if col.size and col.max() > 0:
            imax = k + 1 + int(np.argmax(col))
            colmax = col.max()
        else:
            imax, colmax = k, 0.0
        akk = abs(A[k, k])
        if max(akk, colmax) == 0.0:
            raise ZeroDivisionError(f"zero pivot column at {k}")
        size = 1
        if akk < ALPHA_BK * colmax:
            row = np.abs(A[imax, k:ge])
            row[imax - k] = 0.0
            rowmax = row.max()
            if akk * rowmax >= ALPHA_BK * colmax * colmax:
                pass
            elif abs(A[imax, imax]) >= ALPHA_BK * rowmax:
                swap(k, imax)
            else:
                swap(k + 1, imax)
                size = 2
        if size == 1:
            dmat[k, k] = A[k, k]
            l = A[k + 1:, k] / A[k, k]
            L[k + 1:, k] = l
            A[k + 1:, k + 1:] -= np.outer(l, A[k, k + 1:])
            kinds[k] = 0
        else:
            E = A[k:k + 2, k:k + 2].copy()
            dmat[k:k + 2, k:k + 2] = E
            l = np.linalg.solve(E, A[k:k + 2, k + 2:]).T  # rows below: U E^-1
            L[k + 2:, k:k + 2] = l
            A[k + 2:, k + 2:] -= l @ A[k:k + 2, k + 2:]
            kinds[k], kinds[k + 1] = 1, 2
        k += size
    return piv, L, dmat, kinds


def eig2(a: float, b: float, e: float):
    """Eigen-pairs of [[a, b], [b, e]] in the preconditioner's convention.

    Angle t = atan2(b, (a - e)/2) / 2; the first position takes q1 = (cos t, sin t), the second
    q2 = (-sin t, cos t); eigenvalues as Rayleigh quotients.  Returns (Q, lam) with Q's columns q1, q2.
    """
    t = 0.5 * np.arctan2(b, 0.5 * (a - e))
    Q = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    A = np.array([[a, b], [b, e]])
    lam = np.array([Q[:, 0] @ A @ Q[:, 0], Q[:, 1] @ A @ Q[:, 1]])
    return Q, lam


def whitening(dmat: np.ndarray, kinds: np.ndarray) -> np.ndarray:
    """R with R R^T = |D| (block diagonal, per pivot block: sqrt|d| or Q |Lambda|^1/2)."""
    n = dmat.shape[0]
    R = np.zeros((n, n))
    k = 0
    while k < n:
        if kinds[k] == 0:
            R[k, k] = np.sqrt(abs(dmat[k, k]))
            k += 1
        else:
            Q, lam = eig2(dmat[k, k], dmat[k, k + 1], dmat[k + 1, k + 1])
            R[k:k + 2, k:k + 2] = Q @ np.diag(np.sqrt(np.abs(lam)))
            k += 2
    return R


def correction_matrix(prob: Problem, perm: np.ndarray, starts, nodes, corr_node, corr_par, dtype=np.float64):
    """Block-diagonal C (pivot positions) from raw corrections (None = zero)."""
    d = prob.dim
    nb = 2 * d
    tri = nb * (nb + 1) // 2
    n = int(starts[-1])
    C = np.zeros((n, n), dtype=dtype)
    for g in range(len(nodes)):
        g0, g1 = int(starts[g]), int(starts[g + 1])
        nown = g1 - g0 - nb
        for k in range(nown):
            r = corr_par[perm[g0 + k] - prob.n_x] if corr_par is not None else 0.0
            C[g0 + k, g0 + k] = np.exp(r)
        base = g0 + nown
        for i in range(nb):
            for j in range(i + 1):
                r = corr_node[nodes[g] * tri + i * (i + 1) // 2 + j] if corr_node is not None else 0.0
                C[base + i, base + j] = np.exp(r) if i == j else r
    return C


class Preconditioner:
    """The reference factor of K (dense, user order) and the preconditioner it defines."""

    def __init__(self, prob: Problem, K: np.ndarray):
        self.prob = prob
        self.perm = variable_order(prob)
        self.starts, self.nodes = node_groups(prob)
        Kn = K[np.ix_(self.perm, self.perm)]
        self.S = equilibration(Kn)
        self.piv, self.L, self.D, self.kinds = group_bk_ldlt(self.S[:, None] * Kn * self.S[None, :], self.starts)
        self.R = whitening(self.D, self.kinds)

    def inertia(self):
        ev = np.linalg.eigvalsh(self.D)
        return int(np.sum(ev > 0)), int(np.sum(ev < 0)), int(np.sum(ev == 0))

    def forward(self, v: np.ndarray) -> np.ndarray:
        """y = L^-1 P S v_new (pivot order); v may be [N] or [N, k]."""
        vn = v[self.perm] * (self.S if v.ndim == 1 else self.S[:, None])
        return sla.solve_triangular(self.L, vn[self.piv], lower=True, unit_diagonal=True)

    def matrix(self, corr_node=None, corr_par=None) -> np.ndarray:
        """M in user order (dense)."""
        C = correction_matrix(self.prob, self.perm, self.starts, self.nodes, corr_node, corr_par)
        B = self.R @ C @ C.T @ self.R.T
        Mp = self.L @ B @ self.L.T                      # pivot order, scaled
        n = Mp.shape[0]
        Mn = np.zeros((n, n))
        Mn[np.ix_(self.piv, self.piv)] = Mp             # new order, scaled
        Mn = Mn / self.S[:, None] / self.S[None, :]     # new order
        M = np.zeros((n, n))
        M[np.ix_(self.perm, self.perm)] = Mn
        return M

    def apply(self, v: np.ndarray, corr_node=None, corr_par=None) -> np.ndarray:
        """M^-1 v = S P^T L^-T B^-1 L^-1 P S v (user order), by triangular and block solves: restricted
        pivoting leaves L badly conditioned, so the dense M is not inverted directly.  v may be [N] or [N, k];
        complex corrections or v propagate (complex step)."""
        cplx = np.iscomplexobj(corr_node) or np.iscomplexobj(corr_par)
        C = correction_matrix(self.prob, self.perm, self.starts, self.nodes, corr_node, corr_par,
                              dtype=np.complex128 if cplx else np.float64)
        B = self.R @ C @ C.T @ self.R.T
        vv = v.reshape(v.shape[0], -1)
        y = self.forward(vv)
        w = np.linalg.solve(B, y)
        zp = sla.solve_triangular(self.L.T, w, lower=False, unit_diagonal=True)
        zn = np.zeros_like(zp)
        zn[self.piv] = zp
        zn = self.S[:, None] * zn
        z = np.zeros_like(zn)
        z[self.perm] = zn
        return z.reshape(v.shape)

    def bilinear(self, ya, yb, corr_node, corr_par):
        """ya^T B(r)^-1 yb for forward results ya, yb (complex-safe in the corrections)."""
        cplx = np.iscomplexobj(corr_node) or np.iscomplexobj(corr_par)
        C = correction_matrix(self.prob, self.perm, self.starts, self.nodes, corr_node, corr_par,
                              dtype=np.complex128 if cplx else np.float64)
        B = self.R @ C @ C.T @ self.R.T
        return ya @ np.linalg.solve(B, yb)

    def bilinear_grad(self, ya, yb, corr_node, corr_par, h=1e-30):
        """Complex-step gradient of ya^T B^-1 yb with respect to every raw correction."""
        gn = np.zeros_like(np.asarray(corr_node, dtype=np.float64))
        gp = np.zeros_like(np.asarray(corr_par, dtype=np.float64))
        cn = np.asarray(corr_node, dtype=np.complex128)
        cp = np.asarray(corr_par, dtype=np.complex128)
        used_nodes = set(int(v) for v in self.nodes)
        nb = 2 * self.prob.dim
        tri = nb * (nb + 1) // 2
        for v in used_nodes:
            for t in range(tri):
                i = v * tri + t
                cn[i] += 1j * h
                gn[i] = self.bilinear(ya, yb, cn, cp).imag / h
                cn[i] -= 1j * h
        for i in range(cp.size):
            cp[i] += 1j * h
            gp[i] = self.bilinear(ya, yb, cn, cp).imag / h
            cp[i] -= 1j * h
        return gn, gp


class BlockDiagonalPreconditioner:
    """The ablation without a reference factor: M = S^-1 blockdiag_i(|B_i|) S^-1 with S the symmetric
    equilibration of the current matrix and B_i its diagonal block (of S K S) over node group i;
    |B_i| = V |Lambda| V^T from the symmetric eigendecomposition B_i = V Lambda V^T.  SPD whenever no
    B_i is singular.  Apply: M^-1 v = S blockdiag(|B_i|^-1) S v (user order)."""

    def __init__(self, prob: Problem, K: np.ndarray):
        self.prob = prob
        self.perm = variable_order(prob)
        self.starts, self.nodes = node_groups(prob)
        Kn = K[np.ix_(self.perm, self.perm)]
        self.S = equilibration(Kn)
        Ks = self.S[:, None] * Kn * self.S[None, :]
        self.blocks = []
        for g in range(len(self.starts) - 1):
            a, b = int(self.starts[g]), int(self.starts[g + 1])
            lam, V = np.linalg.eigh(Ks[a:b, a:b])
            self.blocks.append((a, b, V, lam))

    def abs_block(self, g: int) -> np.ndarray:
        a, b, V, lam = self.blocks[g]
        return V @ np.diag(np.abs(lam)) @ V.T

    def matrix(self) -> np.ndarray:
        """M in user order (dense)."""
        n = self.S.size
        Mn = np.zeros((n, n))
        for g in range(len(self.blocks)):
            a, b = self.blocks[g][:2]
            Mn[a:b, a:b] = self.abs_block(g)
        Mn = Mn / self.S[:, None] / self.S[None, :]
        M = np.zeros((n, n))
        M[np.ix_(self.perm, self.perm)] = Mn
        return M

    def apply(self, v: np.ndarray) -> np.ndarray:
        vn = self.S * v[self.perm]
        zn = np.zeros_like(vn)
        for a, b, V, lam in self.blocks:
            zn[a:b] = V @ ((V.T @ vn[a:b]) / np.abs(lam))
        zn = self.S * zn
        z = np.zeros_like(zn)
        z[self.perm] = zn
        return z


def sgn_matrix(prob: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """The assembled K_SGN at (x, p) in user (block) order, from the dense oracle."""
    return D.sgn_matrix_dense(prob, x, p)
