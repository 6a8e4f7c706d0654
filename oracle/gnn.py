"""Mesh graph network of the learned preconditioner, written out in numpy (FP64).

Test infrastructure only (see the package header).  The paper has no learned
component; this is the plain statement of the network the library evaluates in
FP32 (its inputs, layers and weight layout are the library's interface and are
stated in its public header):

  graph:     mesh nodes, a directed edge each way between nodes sharing an element;
  node in:   (x - x_a)/ell, (x - X)/ell (0 on fixed nodes), fixed flag, and for
             log-modulus parameters the means over the node's elements of
             (p - p_a) and p, for per-node parameters |p_v - p_a,v|/ell, |p_v|/ell;
  edge in:   (X_s - X_d)/hbar, ((x_s - x_d) - (X_s - X_d))/ell, hbar = mean rest edge length;
  encoders:  tanh(W f + b) to width 64;
  3 layers:  e += tanh(W [h_dst, h_src, e] + b);  h += tanh(W [h, mean of e into the node] + b);
  decoders:  per node W h + b -> (2d)(2d+1)/2 block entries (+ d parameter entries for
             per-node parameters); per element (log modulus) W mean(h over its nodes) + b.

Weights: dense layers in the order enc_node, enc_edge, (edge_l, node_l) for l = 0, 1, 2,
dec_node, dec_elem; each W (K x N, row-major) followed by b (N).  Everything is
written so that complex weights propagate (complex-step gradients).

Pins (tests/test_oracle_gnn.py): zero decoders give zero outputs; outputs are
invariant under a rigid translation of the mesh and states; relabelling the
nodes permutes the outputs; complex-step gradients agree with central
differences.  symmetric_operator: symmetric, T^2 = I at the reference matrix with
zero corrections, spectrum equal to that of M^-1 K with M built densely from the
reference factor.  train_loss: zero for uniform corrections at the reference
matrix (T^2 = e^{-4c} I, absorbed by the best scale), unchanged when K is scaled,
complex-step derivative equal to central differences.
"""
from __future__ import annotations

import numpy as np

from sgn_inputs import P_LOGE, Problem

H = 64
LAYERS = 3


def layer_shapes(prob: Problem):
    d = prob.dim
    tri = (2 * d) * (2 * d + 1) // 2
    nout = tri + (0 if prob.param_kind == P_LOGE else d)
    shapes = [("enc_node", 2 * d + 3, H), ("enc_edge", 2 * d, H)]
    for l in range(LAYERS):
        shapes += [(f"edge{l}", 3 * H, H), (f"node{l}", 2 * H, H)]
    shapes += [("dec_node", H, nout), ("dec_elem", H, 1 if prob.param_kind == P_LOGE else 0)]
    return shapes


def unpack(prob: Problem, w: np.ndarray):
    """name -> (W [K, N], b [N]) views of the flat weight vector."""
    out, off = {}, 0
    for name, k, n in layer_shapes(prob):
        W = w[off:off + k * n].reshape(k, n)
        b = w[off + k * n:off + (k + 1) * n]
        out[name] = (W, b)
        off += (k + 1) * n
    assert off == w.size, (off, w.size)
    return out


def num_weights(prob: Problem) -> int:
    return sum((k + 1) * n for _, k, n in layer_shapes(prob))


def edges(prob: Problem):
    """(src, dst) of the directed edges (every ordered pair of distinct nodes sharing an element)."""
    pairs = set()
    for el in prob.elems:
        for a in el:
            for b in el:
                if a != b:
                    pairs.add((int(a), int(b)))
    e = np.array(sorted(pairs), dtype=np.int64)
    return e[:, 0], e[:, 1]


def features(prob: Problem, x_ref, p_ref, x, p, ell):
    d = prob.dim
    fdof = prob.free_dof_of_node()
    X = prob.rest_pos
    xn = X.copy()
    xa = X.copy()
    free = fdof >= 0
    for c in range(d):
        xn[free, c] = x[fdof[free] + c]
        xa[free, c] = x_ref[fdof[free] + c]
    nf = np.zeros((prob.n_nodes, 2 * d + 3))
    nf[:, 0:d] = (xn - xa) / ell
    nf[:, d:2 * d] = (xn - X) / ell
    nf[:, 2 * d] = (~free).astype(float)
    if prob.param_kind == P_LOGE:
        s0 = np.zeros(prob.n_nodes)
        s1 = np.zeros(prob.n_nodes)
        cnt = np.zeros(prob.n_nodes)
        for e, el in enumerate(prob.elems):
            for v in el:
                s0[v] += p[e] - p_ref[e]
                s1[v] += p[e]
                cnt[v] += 1
        nz = cnt > 0
        nf[nz, 2 * d + 1] = s0[nz] / cnt[nz]
        nf[nz, 2 * d + 2] = s1[nz] / cnt[nz]
    else:
        for v in np.nonzero(free)[0]:
            sl = slice(fdof[v], fdof[v] + d)
            nf[v, 2 * d + 1] = np.linalg.norm(p[sl] - p_ref[sl]) / ell
            nf[v, 2 * d + 2] = np.linalg.norm(p[sl]) / ell
    src, dst = edges(prob)
    hbar = np.mean(np.linalg.norm(X[src] - X[dst], axis=1))
    ef = np.concatenate([(X[src] - X[dst]) / hbar, ((xn[src] - xn[dst]) - (X[src] - X[dst])) / ell], axis=1)
    return nf, ef, src, dst


def forward(prob: Problem, w, x_ref, p_ref, x, p, ell):
    """(corr_node [n_nodes * tri], corr_par [n_p]); w may be complex."""
    d = prob.dim
    tri = (2 * d) * (2 * d + 1) // 2
    L = unpack(prob, w)
    nf, ef, src, dst = features(prob, x_ref, p_ref, x, p, ell)

    def dense(name, xin, act):
        W, b = L[name]
        z = xin @ W + b
        return np.tanh(z) if act else z

    h = dense("enc_node", nf, True)
    e = dense("enc_edge", ef, True)
    deg = np.bincount(dst, minlength=prob.n_nodes).astype(float)
    for l in range(LAYERS):
        e = e + dense(f"edge{l}", np.concatenate([h[dst], h[src], e], axis=1), True)
        agg = np.zeros((prob.n_nodes, H), dtype=e.dtype)
        np.add.at(agg, dst, e)
        agg = agg / np.maximum(deg, 1)[:, None]
        h = h + dense(f"node{l}", np.concatenate([h, agg], axis=1), True)
    out = dense("dec_node", h, False)
    corr_node = out[:, :tri].reshape(-1)
    dtype = np.result_type(out.dtype, np.float64)
    corr_par = np.zeros(prob.n_p, dtype=dtype)
    if prob.param_kind == P_LOGE:
        emb = h[prob.elems].mean(axis=1)
        corr_par[:] = dense("dec_elem", emb, False)[:, 0]
    else:
        fdof = prob.free_dof_of_node()
        for v in np.nonzero(fdof >= 0)[0]:
            corr_par[fdof[v]:fdof[v] + d] = out[v, tri:tri + d]
    return corr_node, corr_par


def loss_dot(prob, w, gn, gp, *state):
    """sum(gn * corr_node) + sum(gp * corr_par): the scalar whose weight gradient the library's
    backward pass returns for cotangents (gn, gp)."""
    cn, cp = forward(prob, w, *state)
    return np.sum(gn * cn) + np.sum(gp * cp)


def grad_complex_step(prob, w, gn, gp, state, idx, h=1e-30):
    """d loss_dot / d w[i] for i in idx, by the complex step."""
    out = np.zeros(len(idx))
    wc = w.astype(np.complex128)
    for k, i in enumerate(idx):
        wc[i] += 1j * h
        out[k] = loss_dot(prob, wc, gn, gp, *state).imag / h
        wc[i] -= 1j * h
    return out


def directional_complex_step(prob, w, gn, gp, state, u, h=1e-30):
    """d/de loss_dot(w + e u) at e = 0."""
    return loss_dot(prob, w.astype(np.complex128) + 1j * h * u, gn, gp, *state).imag / h


def symmetric_operator(prob: Problem, P, K, corr_node, corr_par):
    """T = (R C)^-1 L^-1 Q K Q^T L^-T (R C)^-T, Q the map from block order to the equilibrated pivot
    order (Q v = (S v_new)[piv]); dense, complex-safe in the corrections."""
    from .precond import correction_matrix
    cplx = np.iscomplexobj(corr_node) or np.iscomplexobj(corr_par)
    C = correction_matrix(prob, P.perm, P.starts, P.nodes, corr_node, corr_par,
                          dtype=np.complex128 if cplx else np.float64)
    n = K.shape[0]
    Q = np.zeros((n, n))
    Q[np.arange(n), P.perm[P.piv]] = P.S[P.piv]
    F = P.L @ P.R @ C  # M = Q^T F F^T Q in the equilibrated pivot order
    Kp = Q @ K @ Q.T
    return np.linalg.solve(F, np.linalg.solve(F, Kp.T).T)


def train_loss(prob: Problem, P, K, w, state, probes):
    """Mean over probes u (whitened pivot coordinates) of min_gamma |gamma T^2 u - u|^2 / |u|^2 with T
    the symmetric form of the preconditioned matrix (symmetric_operator) and the network's
    corrections for `state` (x_ref, p_ref, x, p, ell).  The minimising gamma = u^T b / b^T b
    (b = T^2 u) is substituted.  Plain products (no conjugation) keep it holomorphic in the weights,
    for the complex step."""
    cn, cp = forward(prob, w, *state)
    T = symmetric_operator(prob, P, K, cn, cp)
    total = 0.0
    for u in probes:
        b = T @ (T @ u)
        gam = np.sum(u * b) / np.sum(b * b)
        e = gam * b - u
        total = total + np.sum(e * e) / np.sum(u * u)
    return total / len(probes)
