"""Training and evaluation of the learned node-block preconditioner.

Python here only orders the work; every numerical step runs in libsgn's kernels:
the SGN iterations that log the training states (sgn_step), the reference
factorisations (sgn_factor), the loss |T^2 u - u|^2 / |u|^2 of the symmetric
preconditioned matrix with its weight gradient (sgn_pc_train_loss, which runs
the network's forward and backward passes), and Adam (sgn_adam).

Data: SGN runs on seeded cantilevers of the log-modulus family (linear tets,
neo-Hookean, clamped end).  A sample pairs the reference factor at iterate k
with the matrix at a point along the step to iterate k + 1: parameters
p_k + t (p_k+1 - p_k) for t in FRACTIONS, x at their equilibrium.  t = 1 is
the reuse of the previous iteration's factor for the next step; smaller t are
the shorter moves of late iterations and line-search trials.  Evaluation counts
MINRES iterations to the 1e-10 equilibrated residual on held-out seeds, with
and without the network, per fraction.

  python -m paper_2107_03285_amd.learned_pc --out paper_2107_03285_amd/weights/pc_3d_loge
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import sgn_inputs as si  # noqa: E402

from . import sgn  # noqa: E402

TRAIN_MESHES = [(12, 3, 3, 1 / 3), (16, 4, 4, 0.25), (20, 5, 5, 0.2)]
# fractions t of an SGN step p_k -> p_k+1 at which the matrix is taken (x at equilibrium of p_k + t dp)
FRACTIONS = (0.05, 0.1, 0.25, 0.5, 1.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _t(a, dev, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device=dev)


def run_sgn(prob, n_iter, dev="cuda:0"):
    """Set targets from the initial equilibrium (ell = max displacement, targets = x0[T] + noise) and
    log the SGN iterates; returns the list of (x, p) host arrays, iterate 0 first."""
    ctx = sgn.Context(prob, sgn.default_options()).allocate(dev)
    p = _t(prob.p_init(), dev)
    x = _t(prob.x_rest(), dev)
    ctx.equilibrium(p, x)
    xh = x.cpu().numpy()
    ell = float(np.max(np.abs(xh - prob.x_rest())))
    prob.length_scale = ell
    prob.target_val = xh[prob.target_dof] + prob.target_noise
    ctx.set_targets(prob.target_val, ell)
    ctx.equilibrium(p, x)
    states = [(x.cpu().numpy().copy(), p.cpu().numpy().copy())]
    for _ in range(n_iter):
        try:
            ctx.step(p, x)
        except sgn.SgnError as e:
            log(f"[learned_pc] {prob.name}: SGN stopped ({e})")
            break
        states.append((x.cpu().numpy().copy(), p.cpu().numpy().copy()))
    del ctx
    return states


class Trainer:
    def __init__(self, template_prob, seed=0, lr=1e-3, dev="cuda:0"):
        import torch
        self.dev = dev
        self.ctxs = {}
        ctx = self.context(template_prob)
        n = ctx.gnn_num_weights()
        self.w = torch.zeros(n, dtype=torch.float32, device=dev)
        ctx.gnn_init(self.w, seed)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.t = 0
        self.lr = lr
        self.rng = np.random.default_rng(seed)

    def context(self, prob):
        if prob.name not in self.ctxs:
            o = sgn.default_options(solver=sgn.SGN_MINRES_LEARNED, max_minres=300)
            ctx = sgn.Context(prob, o).allocate(self.dev)
            ctx.set_targets(prob.target_val, prob.length_scale)
            self.ctxs[prob.name] = ctx
        return self.ctxs[prob.name]

    def prepare(self, prob, a, b):
        """Reference factor at state a, matrix at state b."""
        ctx = self.context(prob)
        ctx.assemble(_t(a[0], self.dev), _t(a[1], self.dev))
        ctx.factor()
        ctx.assemble(_t(b[0], self.dev), _t(b[1], self.dev))
        return ctx

    def loss(self, prob, a, b, nprobe=2, accumulate=True, rng=None, log_form=True):
        import torch
        ctx = self.prepare(prob, a, b)
        N = 2 * prob.n_x + prob.n_p
        probes = _t((rng or self.rng).standard_normal((nprobe, N)), self.dev)
        g = self.g if accumulate else torch.zeros_like(self.w)
        return ctx.pc_train_loss(self.w, probes, g, log_form=log_form)

    def step(self):
        self.t += 1
        sgn.adam(self.w, self.g, self.m, self.v, self.lr, self.t)
        self.g.zero_()

    def minres_iterations(self, prob, a, b, use_net, seed=0):
        """MINRES iterations (and fallback flag) for a seeded right-hand side."""
        ctx = self.prepare(prob, a, b)
        if use_net:
            ctx.set_pc_weights(self.w)
        else:
            ctx.set_pc_correction(None, None)
        N = 2 * prob.n_x + prob.n_p
        rhs = _t(np.random.default_rng(seed).standard_normal(N), self.dev)
        import torch
        sol = torch.zeros(N, dtype=torch.float64, device=self.dev)
        info = ctx.solve_minres(rhs, sol)
        ctx.set_pc_correction(None, None)
        return info.sweeps, info.fallback, info.rel_res


def family_problems(seeds, max_side=20):
    """The learned-preconditioner family (cantilevers 4s x s x s for even seeds, plates 4s x s x
    max(2, ceil(s/4)) for odd ones, s ~ U{5..20} per seed, log-modulus parameters); seeds whose s
    exceeds max_side are skipped (a training budget, stated in the report)."""
    out = []
    for sd in seeds:
        q = si.learned_pc_problem(sd)
        if q.grid[1] <= max_side:
            out.append(q)
    return out


def build_pairs(meshes, seeds, n_iter, dev, fractions=FRACTIONS, problems=None):
    """(prob, state_a, state_b, t) samples: reference at iterate k, matrix a fraction t along the step.
    The problems are the cantilevers `meshes` x `seeds`, or `problems` when given."""
    pairs = []
    if problems is None:
        problems = [si.problem_3d(nx, ny, nz, h, seed=s) for (nx, ny, nz, h) in meshes for s in seeds]
    for prob in problems:
        states = run_sgn(prob, n_iter, dev)
        ctx = sgn.Context(prob, sgn.default_options()).allocate(dev)
        ctx.set_targets(prob.target_val, prob.length_scale)
        for k in range(len(states) - 1):
            (xa, pa), (xb, pb) = states[k], states[k + 1]
            for t in fractions:
                if t == 1.0:
                    pairs.append((prob, states[k], states[k + 1], t))
                    continue
                p = _t(pa + t * (pb - pa), dev)
                x = _t(xa, dev)
                try:
                    ctx.equilibrium(p, x)
                except sgn.SgnError:  # no equilibrium there; an error is sticky, so start a fresh context
                    ctx = sgn.Context(prob, sgn.default_options()).allocate(dev)
                    ctx.set_targets(prob.target_val, prob.length_scale)
                    continue
                pairs.append((prob, states[k], (x.cpu().numpy().copy(), p.cpu().numpy().copy()), t))
        del ctx
        log(f"[learned_pc] logged {prob.name}: {len(states) - 1} iterations")
    return pairs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="output path prefix (writes .f32 weights and .json report)")
    ap.add_argument("--train-seeds", type=int, default=6)
    ap.add_argument("--iters", type=int, default=6, help="SGN iterations logged per run")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--nprobe", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--family", action="store_true",
                    help="train and evaluate on the cantilever/plate family with s ~ U{5..20} (seeds 0.. for "
                         "training, 1000.. held out) instead of the three fixed small cantilevers")
    ap.add_argument("--held-seeds", type=int, default=3)
    ap.add_argument("--max-side", type=int, default=20, help="skip training seeds of the family with a larger s")
    ap.add_argument("--held-max-side", type=int, default=20, help="skip held-out seeds with a larger s")
    args = ap.parse_args()
    dev = "cuda:0"
    t0 = time.time()
    if args.family:
        train = build_pairs(None, None, args.iters, dev,
                            problems=family_problems(range(args.train_seeds), args.max_side))
        held = build_pairs(None, None, args.iters, dev,
                           problems=family_problems(range(1000, 1000 + args.held_seeds), args.held_max_side))
    else:
        train = build_pairs(TRAIN_MESHES, range(args.train_seeds), args.iters, dev)
        held = build_pairs([TRAIN_MESHES[-1]], range(1000, 1000 + args.held_seeds), args.iters, dev)
    log(f"[learned_pc] {len(train)} training pairs, {len(held)} held-out pairs ({time.time() - t0:.1f} s)")
    tr = Trainer(train[0][0], seed=args.seed, lr=args.lr, dev=dev)

    def held_loss():
        r = np.random.default_rng(12345)
        return float(np.exp(np.mean([np.log(tr.loss(p, a, b, nprobe=4, accumulate=False, rng=r))
                                     for p, a, b, _ in held])))

    report = {"n_weights": int(tr.w.numel()), "train_pairs": len(train), "held_pairs": len(held),
              "meshes": sorted({p.name for p, *_ in train}), "held_meshes": sorted({p.name for p, *_ in held}),
              "family": bool(args.family), "max_side": args.max_side, "held_max_side": args.held_max_side,
              "sgn_iterations_logged": args.iters,
              "epochs": args.epochs, "lr": args.lr, "history": []}
    base_iters = [tr.minres_iterations(p, a, b, False) for p, a, b, _ in held]
    report["held_loss_untrained"] = held_loss()
    log(f"[learned_pc] held-out loss before training {report['held_loss_untrained']:.4e}")
    order = np.arange(len(train))
    rng = np.random.default_rng(args.seed)
    for ep in range(args.epochs):
        rng.shuffle(order)
        tl = []
        for i in order:
            p, a, b, _ = train[i]
            tl.append(np.log(tr.loss(p, a, b, nprobe=args.nprobe)))
            tr.step()
        hl = held_loss()
        report["history"].append({"epoch": ep, "train_loss_geomean": float(np.exp(np.mean(tl))), "held_loss_geomean": hl})
        log(f"[learned_pc] epoch {ep}: train {np.exp(np.mean(tl)):.4e} held-out {hl:.4e} (geometric means; "
            f"{time.time() - t0:.1f} s)")
    net_iters = [tr.minres_iterations(p, a, b, True) for p, a, b, _ in held]
    report["minres_held"] = [{"pair": f"{p.name}:{k}", "t": t, "without": list(map(float, bi)),
                              "with": list(map(float, ni))}
                             for k, ((p, a, b, t), bi, ni) in enumerate(zip(held, base_iters, net_iters))]
    summary = {}
    for t in FRACTIONS:
        rows = [r for r in report["minres_held"] if r["t"] == t]
        if rows:
            summary[str(t)] = {"pairs": len(rows),
                               "mean_iters_without": float(np.mean([r["without"][0] for r in rows])),
                               "mean_iters_with": float(np.mean([r["with"][0] for r in rows])),
                               "fallbacks_without": int(sum(r["without"][1] for r in rows)),
                               "fallbacks_with": int(sum(r["with"][1] for r in rows))}
    report["minres_by_fraction"] = summary
    report["seconds"] = time.time() - t0
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    tr.w.cpu().numpy().astype(np.float32).tofile(args.out + ".f32")
    with open(args.out + ".json", "w") as fh:
        json.dump(report, fh, indent=1)
    for t, r in summary.items():
        log(f"[learned_pc] t = {t}: {r}")


if __name__ == "__main__":
    main()
