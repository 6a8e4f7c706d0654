"""Element model of the oracle (test infrastructure; see ``oracle/__init__``).

Linear simplices with a compressible neo-Hookean energy density, the
material of the paper's inverse elastic design example (Sec. 5.1, which names
a neo-Hookean material with E = 1e6 Pa on linear tetrahedra without fixing
its form).  The form used here (a reading, listed in the design notes):

    Psi(F) = mu/2 (tr F^T F - d) - mu ln J + lam/2 (ln J)^2,   J = det F,
    mu = E / (2 (1 + nu)),  lam = E nu / ((1 + nu)(1 - 2 nu)),

plane strain with unit thickness in 2D.  Element e has energy
E_e = V0_e Psi(F_e), F_e = Ds Dm^-1 with Ds / Dm the edge matrices of the
deformed / rest simplex and V0_e = det(Dm) / d!.

The first Piola stress is written in closed form, P = mu (F - F^-T) +
lam ln J F^-T, and every function is complex-analytic (no abs, conj or
branch other than the principal log near J > 0), so the Hessians the method
needs -- d2E/dx2 (the constraint Jacobian dc/dx of Sec. 3.1) and d2E/dx dp
(dc/dp) -- are taken by complex-step differentiation of the gradient,
dg/dq_k = Im g(q + i h e_k) / h with h = 1e-30, which is exact to rounding.
This makes the oracle's Hessians independent of any hand-derived tangent.
"""
from __future__ import annotations

import numpy as np

CS_H = 1e-30


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def _fact(d: int) -> float:
    return 2.0 if d == 2 else 6.0


def edge_matrix(P: np.ndarray) -> np.ndarray:
    """P: [ne, d+1, d] vertex positions -> [ne, d, d] with column k = P[k+1] - P[0]."""
    return np.swapaxes(P[:, 1:, :] - P[:, :1, :], 1, 2)


def _inv(M: np.ndarray) -> np.ndarray:
    return np.linalg.inv(M)


def _det(M: np.ndarray) -> np.ndarray:
    d = M.shape[-1]
    if d == 2:
        return M[..., 0, 0] * M[..., 1, 1] - M[..., 0, 1] * M[..., 1, 0]
    return (M[..., 0, 0] * (M[..., 1, 1] * M[..., 2, 2] - M[..., 1, 2] * M[..., 2, 1])
            - M[..., 0, 1] * (M[..., 1, 0] * M[..., 2, 2] - M[..., 1, 2] * M[..., 2, 0])
            + M[..., 0, 2] * (M[..., 1, 0] * M[..., 2, 1] - M[..., 1, 1] * M[..., 2, 0]))


def rest_data(Xe: np.ndarray):
    """Dm^-1 and signed rest volume V0 of every element (Xe: [ne, d+1, d])."""
    d = Xe.shape[-1]
    Dm = edge_matrix(Xe)
    return _inv(Dm), _det(Dm) / _fact(d)


def energy_density(F, mu, lam):
    d = F.shape[-1]
    J = _det(F)
    lnJ = np.log(J)
    trC = np.sum(F * F, axis=(-2, -1))
    return 0.5 * mu * (trC - d) - mu * lnJ + 0.5 * lam * lnJ * lnJ


def piola(F, mu, lam):
    J = _det(F)
    lnJ = np.log(J)
    FinvT = np.swapaxes(_inv(F), -1, -2)
    return mu[..., None, None] * (F - FinvT) + (lam * lnJ)[..., None, None] * FinvT


def element_energy(xe, Xe, mu, lam):
    """E_e for every element; +inf where the deformed simplex is inverted (real inputs only)."""
    Dminv, V0 = rest_data(Xe)
    F = edge_matrix(xe) @ Dminv
    J = _det(F)
    out = np.full(xe.shape[0], np.inf)
    ok = np.real(J) > 0
    if np.any(ok):
        out[ok] = np.real(V0[ok] * energy_density(F[ok], mu[ok], lam[ok]))
    return out


def element_gradient(xe, Xe, mu, lam):
    """dE_e/dx for every element, [ne, d+1, d]: node k>0 gets column k-1 of V0 P Dm^-T."""
    Dminv, V0 = rest_data(Xe)
    F = edge_matrix(xe) @ Dminv
    G = V0[:, None, None] * (piola(F, mu, lam) @ np.swapaxes(Dminv, -1, -2))  # [ne, d, d]
    Gt = np.swapaxes(G, 1, 2)  # row k = force on node k+1
    g0 = -np.sum(Gt, axis=1, keepdims=True)
    return np.concatenate([g0, Gt], axis=1)


def element_hessian(xe, Xe, mu, lam):
    """d2E_e/dx2 by complex step, [ne, (d+1)d, (d+1)d] (row/col = node*d + comp)."""
    ne, nv, d = xe.shape
    n = nv * d
    H = np.empty((ne, n, n))
    for k in range(n):
        xc = xe.astype(np.complex128)
        xc[:, k // d, k % d] += 1j * CS_H
        H[:, :, k] = np.imag(element_gradient(xc, Xe, mu, lam)).reshape(ne, n) / CS_H
    return H


def element_dgrad_dlogE(xe, Xe, mu, lam):
    """d(dE_e/dx)/dp_e for E_e = E0 exp(p_e), by complex step on p_e, [ne, (d+1)d]."""
    ne, nv, d = xe.shape
    z = np.full(ne, 1j * CS_H)
    s = np.exp(z)  # scaling of both Lame parameters
    g = element_gradient(xe.astype(np.complex128), Xe, mu * s, lam * s)
    return np.imag(g).reshape(ne, nv * d) / CS_H


def element_dgrad_drest(xe, Xe, mu, lam):
    """d(dE_e/dx)/dX_e (mixed derivative w.r.t. rest positions) by complex step, [ne, n, n]."""
    ne, nv, d = xe.shape
    n = nv * d
    M = np.empty((ne, n, n))
    for k in range(n):
        Xc = Xe.astype(np.complex128)
        Xc[:, k // d, k % d] += 1j * CS_H
        M[:, :, k] = np.imag(element_gradient(xe.astype(np.complex128), Xc, mu, lam)).reshape(ne, n) / CS_H
    return M
