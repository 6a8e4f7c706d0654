"""Benchmark: SGN search directions per second on one MI355X.

One "step" is the paper's timed unit, the computation of one search
direction at a fixed equilibrium (x, p): assembly of the saddle-point matrix
from per-element blocks with its right-hand side, supernodal LDL^T, and the
solve with FP64 refinement to an equilibrated relative residual of 1e-10.  The
right-hand side is the KKT form [-df/dx; -df/dp; 0], which gives the same dp
as [0; -g; 0] without the adjoint solve that forms g (Appendix A, Theorem 2);
the adjoint form is timed too (path fp32ir_adjoint).  The headline path factorises in FP32 on the
matrix cores and refines in FP64; the plain FP64 factorisation is timed beside
it on identical inputs and its step is the reference the FP32 step is
compared with.

Workload: the 100 x 25 x 25-hex cantilever (312,500 tets, 202,800 free DOF,
312,500 log-modulus parameters, N = 718,100), seeded synthetic inputs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import sgn_inputs as si  # noqa: E402

WORKLOADS = {
    "cantilever_100x25x25": lambda: si.config_cantilever_200k(seed=0),
    "cantilever_40x10x10_loge": lambda: si.problem_3d(40, 10, 10, 0.1, seed=0),
    "cantilever_20x5x5": lambda: si.problem_3d(20, 5, 5, 0.2, seed=0),
    "grid2d_21x21": lambda: si.config_2d(seed=0),
}
PEAK = {"fp64": 78.6, "fp32": 157.3}  # dense matrix-core TFLOP/s of one MI355X
HBM_PEAK = 8000.0  # GB/s
# HBM traffic of the update kernel, from two hardware-counter runs of this script (FETCH_SIZE, then
# WRITE_SIZE, scaled by what the counters read for a plain copy of known size).  The record holds a
# hash of the kernel's source; a record taken from another version of the kernel is not used.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_update_cantilever_100x25x25_traffic.json")
UPDATE_SOURCES = [os.path.join(ROOT, "paper_2107_03285_amd", "csrc", f) for f in ("k_factor.hip", "kernels.h")]
COPY_ELEMS = 1 << 28  # float32 elements of the calibration copy: 1 GiB read + 1 GiB written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(budget_s: float = 20.0, budget_1t_s: float = 8.0):
    """The FP64 oracle's dense Gauss-Newton step, timed on the host cores, on the smallest
    cantilever of the same family (20 x 5 x 5 hexes): the dense method cannot hold the
    200k-DOF problem (its sensitivity matrix alone would be ~500 GB).  Timed with the BLAS
    threads the host gives and again with one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import dense as D
    prob = D.setup_targets(si.problem_3d(20, 5, 5, 0.2, seed=0))
    p = prob.p_init()
    x, _ = D.equilibrium(prob, p)

    def timed(budget, cap):
        n = 0
        t0 = time.perf_counter()
        while True:
            D.dense_gn_step(prob, x, p)
            n += 1
            if time.perf_counter() - t0 > budget or n >= cap:
                break
        return n, time.perf_counter() - t0

    n, dt = timed(budget_s, 50)
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        n1, dt1 = timed(budget_1t_s, 20)
    return {"value": n / dt, "unit": "SGN steps/s", "cores": int(threads), "kind": "oracle",
            "value_1thread": n1 / dt1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"dense GN step (S = -Kx^-1 Kp, H = S^T A S + C, Cholesky) of the oracle on the "
                      f"20x5x5-hex cantilever of the same family (n_x={prob.n_x}, n_p={prob.n_p}), "
                      f"{n} steps in {dt:.1f} s with {threads} BLAS threads, {n1} steps in {dt1:.1f} s "
                      f"with one"}


def update_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in UPDATE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload):
    """Bytes per update launch from the counter record, or None if there is none for this workload or the
    kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("source_sha256") != update_source_hash():
        return None
    return rec


def copy_calibration():
    """A plain elementwise copy (negation) of 1 GiB float32, three times: its counter readings give the
    scale from FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    a = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 x torch.neg over {COPY_ELEMS * 4} bytes read and written")
    del a, b
    torch.cuda.empty_cache()


TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2107_03285_amd", "tuning")


def tuned_options(sgn, workload: str, **kw):
    """FP32 options for a workload with the blocking of its autotuner record, if one exists; returns
    (options, where the blocking came from)."""
    o = sgn.default_options(**kw)
    path = os.path.join(TUNING_DIR, f"{workload}.json")
    if os.path.exists(path):
        return sgn.apply_tuning(o, sgn.load_tuning(path)), os.path.relpath(path, os.path.dirname(TUNING_DIR))
    return o, "library defaults"


def run_autotune(sgn, prob, x, p, dev):
    """Tunes the FP32 schedule blocking of prob at (x, p) and stores the record beside the package."""
    os.makedirs(TUNING_DIR, exist_ok=True)
    base = sgn.default_options(precision=sgn.SGN_FP32_IR, rhs_kind=sgn.SGN_RHS_KKT)
    t0 = time.perf_counter()
    rec = sgn.autotune(prob, x, p, base, reps=2, path=os.path.join(TUNING_DIR, f"{prob.name}.json"))
    log(f"[bench] autotune {prob.name}: {sgn.tuning_of(sgn.apply_tuning(base, rec))} in "
        f"{time.perf_counter() - t0:.0f} s; candidates ms {['%.1f' % v for v in rec['candidate_ms']]}")
    return rec


def batch_leg(steps: int, warmup: int, dev: str = "cuda:0", autotune: bool = False):
    """256 independent 2D membranes (8..48 nodes per side, seeds 10000..10255) as one disjoint union:
    the captured-graph step (level-batched FP32 factorisation, refinement sweeps as many as an eager solve
    of the same union needs, checked on the device at every replay) against solving
    the same problems one at a time with their own FP64 contexts (assemble, factor, solve)."""
    import torch

    from paper_2107_03285_amd import sgn
    probs = si.batch_problems(256, base_seed=10000, lo=8, hi=48)
    u = si.union_problem(probs, name="membranes_2d_256")
    N = 2 * u.n_x + u.n_p
    # set-up (untimed): ell from x(p0) of the union, targets x(p*) on each top row
    ref = sgn.Context(u, sgn.default_options()).allocate(dev)
    p0 = torch.tensor(u.p_init(), dtype=torch.float64, device=dev)
    x0 = torch.tensor(u.x_rest(), dtype=torch.float64, device=dev)
    ref.equilibrium(p0, x0)
    ell = float((x0.cpu() - torch.tensor(u.x_rest())).abs().max())
    xs = x0.clone()
    ref.equilibrium(torch.tensor(u.p_star, dtype=torch.float64, device=dev), xs)
    u.length_scale = ell
    u.target_val = xs.cpu().numpy()[u.target_dof]
    del ref
    torch.cuda.empty_cache()
    if autotune:
        run_autotune(sgn, u, x0, p0, dev)
    o, blocking_src = tuned_options(sgn, u.name, precision=sgn.SGN_FP32_IR, rhs_kind=sgn.SGN_RHS_KKT)
    ctx = sgn.Context(u, o).allocate(dev)
    rhs = torch.zeros(N, dtype=torch.float64, device=dev)
    sol = torch.zeros(N, dtype=torch.float64, device=dev)
    # the refinement sweeps the replayed step runs: those an eager solve of the union needs
    ctx.assemble(x0, p0, rhs)
    ctx.factor()
    n_ir = int(ctx.solve(rhs, sol).sweeps)
    for _ in range(warmup):
        ctx.graph_step(x0, p0, rhs, sol, n_ir)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rel = 0.0
    for _ in range(steps):
        rel = max(rel, ctx.graph_step(x0, p0, rhs, sol, n_ir))
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    dp_batch = sol.cpu().numpy()[u.n_x:u.n_x + u.n_p]
    del ctx
    torch.cuda.empty_cache()
    # one at a time, FP64, each problem in its own context at the union's state and targets
    xh = x0.cpu().numpy()
    x_off = np.concatenate([[0], np.cumsum([q.n_x for q in probs])])
    p_off = np.concatenate([[0], np.cumsum([q.n_p for q in probs])])
    t_off = np.concatenate([[0], np.cumsum([len(q.target_dof) for q in probs])])
    singles = []
    for i, q in enumerate(probs):
        q.length_scale = ell
        q.target_val = u.target_val[t_off[i]:t_off[i + 1]]
        c = sgn.Context(q, sgn.default_options(rhs_kind=sgn.SGN_RHS_KKT)).allocate(dev)
        n = 2 * q.n_x + q.n_p
        singles.append((c, torch.tensor(xh[x_off[i]:x_off[i + 1]], device=dev),
                        torch.tensor(q.p_init(), dtype=torch.float64, device=dev),
                        torch.zeros(n, dtype=torch.float64, device=dev), torch.zeros(n, dtype=torch.float64, device=dev)))
    for c, x, p, r, z in singles:  # warm-up
        c.assemble(x, p, r)
        c.factor()
        c.solve(r, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, x, p, r, z in singles:
        c.assemble(x, p, r)
        c.factor()
        c.solve(r, z)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    err = max(float(np.linalg.norm(z.cpu().numpy()[q.n_x:q.n_x + q.n_p] - dp_batch[p_off[i]:p_off[i + 1]]) /
                    max(1e-300, np.linalg.norm(z.cpu().numpy()[q.n_x:q.n_x + q.n_p])))
              for i, (q, (c, x, p, r, z)) in enumerate(zip(probs, singles)))
    return {"problems": len(probs), "N_union": N, "graph_step_ms": 1e3 * t_graph,
            "problem_steps_per_s_batched": len(probs) / t_graph, "one_at_a_time_fp64_ms": 1e3 * t_single,
            "problem_steps_per_s_one_at_a_time": len(probs) / t_single, "speedup": t_single / t_graph,
            "max_rel_residual": rel, "max_dp_rel_diff_vs_single_fp64": err, "refine_sweeps": n_ir,
            "blocking": dict(sgn.tuning_of(o), source=blocking_src),
            "graph": f"assemble + KKT rhs + FP32 LDL^T + solve + {n_ir} FP64 refinement sweeps (those of an eager "
                     f"solve), replayed; the residual checked on the device at every replay"}


WEIGHTS_DIR = os.path.join(ROOT, "paper_2107_03285_amd", "weights")


def learned_pc_leg(sgn, prob, x, p, dp, dev, steps, fractions=(1.0, 0.05)):
    """The learned-preconditioner form at the workload's size: the reference factor (FP32 fronts) is
    the exact LDL^T at the current iterate (x, p); the next system is the one a fraction t along the
    FP64 Gauss-Newton step dp (t = 1: the next iterate; t = 0.05: a short move, like a late iteration
    or a line-search trial), at its equilibrium.  One timed step = assembly of the next system + MINRES
    with the reference factor's node-block preconditioner to the 1e-10 equilibrated residual, with
    the exact LDL^T + refinement as its fallback.  Timed with the trained network's corrections (weights
    file of the 3D log-modulus family, when present) and with none; the reference is re-established
    (untimed) before every step."""
    import torch
    wpath = os.path.join(WEIGHTS_DIR, "pc_3d_loge.f32")
    o = sgn.default_options(precision=sgn.SGN_FP32_IR, solver=sgn.SGN_MINRES_LEARNED, rhs_kind=sgn.SGN_RHS_KKT,
                            max_minres=300)
    ctx = sgn.Context(prob, o).allocate(dev)
    ctx.set_targets(prob.target_val, prob.length_scale)
    w = None
    if os.path.exists(wpath):
        wh = np.fromfile(wpath, dtype=np.float32)
        if wh.size == ctx.gnn_num_weights():
            w = torch.tensor(wh, device=dev)
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device=dev)
    sol = torch.zeros(N, dtype=torch.float64, device=dev)
    out = {"weights": os.path.relpath(wpath, ROOT) if w is not None else None, "fractions": {}}
    for t0_ in fractions:
        t = t0_
        while True:  # the next system must have an equilibrium (the outer line search halves the same way)
            p1 = p + t * dp
            x1 = x.clone()
            try:
                ctx.equilibrium(p1, x1)
                break
            except sgn.SgnError:
                ctx = sgn.Context(prob, o).allocate(dev)  # an error is sticky: start a fresh context
                ctx.set_targets(prob.target_val, prob.length_scale)
                t *= 0.5
                if t < 1e-3:
                    raise
        row = {"t": t}
        for label, use in (("with_network", True), ("without_network", False)):
            if use and w is None:
                row[label] = None
                continue
            times, iters, fb, res = [], [], [], []
            for k in range(steps):
                ctx.assemble(x, p)  # reference factor at the current iterate (untimed)
                ctx.factor()
                if use:
                    ctx.set_pc_weights(w)
                else:
                    ctx.set_pc_correction(None, None)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.assemble(x1, p1, rhs)
                info = ctx.solve_minres(rhs, sol)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                iters.append(int(info.sweeps))
                fb.append(int(info.fallback))
                res.append(info.rel_res)
            row[label] = {"steps_per_s": len(times) / sum(times), "ms_per_step": 1e3 * sum(times) / len(times),
                          "minres_iterations": iters[-1], "fallback_rate": float(np.mean(fb)),
                          "rel_res_max": max(res)}
        # the ablation without a reference factor: MINRES preconditioned by blockdiag(|B_i|^-1) of the
        # next system's own node-group blocks (its set-up is inside the timed solve)
        ob = sgn.default_options(precision=sgn.SGN_FP32_IR, solver=sgn.SGN_MINRES_LEARNED,
                                 rhs_kind=sgn.SGN_RHS_KKT, max_minres=300, pc_kind=sgn.SGN_PC_BLOCK)
        bctx = sgn.Context(prob, ob).allocate(dev)
        bctx.set_targets(prob.target_val, prob.length_scale)
        times, iters, fb, res = [], [], [], []
        for k in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bctx.assemble(x1, p1, rhs)
            info = bctx.solve_minres(rhs, sol)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(int(info.sweeps))
            fb.append(int(info.fallback))
            res.append(info.rel_res)
        row["block_diagonal_no_reference"] = {
            "steps_per_s": len(times) / sum(times), "ms_per_step": 1e3 * sum(times) / len(times),
            "minres_iterations": iters[-1], "fallback_rate": float(np.mean(fb)), "rel_res_max": max(res)}
        del bctx
        torch.cuda.empty_cache()
        out["fractions"][str(t0_)] = row
        log(f"[bench] learned-PC t = {t}: {row}")
    del ctx
    torch.cuda.empty_cache()
    return out


def variants_leg(sgn, dev, steps):
    """The Sec. 4/5 variants, each timed for one search direction beside the plain direction on the same
    system: the block solve on a rest-position bar (every free DOF a target, no regulariser: the
    conditions of the block solve) against the full SGN solve of the same system in FP64; and BiCGSTAB
    preconditioned by the LDL^T of the stabilised matrix (eps = 1e-6, Sec. 5) at the workload's size."""
    import torch
    out = {}
    prob = si.problem_3d(40, 10, 10, 0.1, seed=0, param_kind=si.P_REST_POS)
    prob.reg_mu = 0.0
    x = torch.tensor(prob.x_rest(), dtype=torch.float64, device=dev)
    p = torch.tensor(prob.p_init(), dtype=torch.float64, device=dev)
    setup = sgn.Context(prob, sgn.default_options()).allocate(dev)
    setup.equilibrium(p, x)
    xh = x.cpu().numpy()
    prob.target_dof = np.arange(prob.n_x, dtype=np.int32)
    prob.target_val = xh + 1e-3 * np.sin(np.arange(prob.n_x))
    prob.length_scale = float(np.max(np.abs(xh - prob.x_rest())))
    del setup
    N = 2 * prob.n_x + prob.n_p
    sols = {}
    for label, solver in (("block_gn", sgn.SGN_BLOCK_GN), ("sgn_ldlt_fp64", sgn.SGN_LDLT)):
        ctx = sgn.Context(prob, sgn.default_options(solver=solver, rhs_kind=sgn.SGN_RHS_KKT)).allocate(dev)
        xe = x.clone()
        ctx.equilibrium(p, xe)
        rhs = torch.zeros(N, dtype=torch.float64, device=dev)
        sol = torch.zeros(N, dtype=torch.float64, device=dev)

        def one():
            if solver == sgn.SGN_BLOCK_GN:
                return ctx.block_step(xe, p, sol)
            ctx.assemble(xe, p, rhs)
            ctx.factor()
            return ctx.solve(rhs, sol)
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = one()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        sols[label] = sol.cpu().numpy()
        out[label] = {"ms_per_direction": 1e3 * dt, "iterations": int(info.sweeps), "rel_res": info.rel_res}
        del ctx
        torch.cuda.empty_cache()
    nx, npar = prob.n_x, prob.n_p
    a, b = sols["block_gn"][nx:nx + npar], sols["sgn_ldlt_fp64"][nx:nx + npar]
    out["block_vs_sgn"] = {"workload": f"{prob.name}, every free DOF a target, reg_mu = 0 (n_x = {nx})",
                           "speedup": out["sgn_ldlt_fp64"]["ms_per_direction"] / out["block_gn"]["ms_per_direction"],
                           "dp_rel_diff": float(np.linalg.norm(a - b) / np.linalg.norm(b))}
    torch.cuda.empty_cache()
    return out


def newton_leg(sgn, prob, x, p, dev):
    """One Sparse Newton iteration with inertia control (Sec. 4 eq. totalHessian, Appendix A, Sec. 5;
    FP32 factors + FP64 refinement) beside one Gauss-Newton iteration, both from the workload's
    equilibrium: the direction's stages (for Newton: the multipliers, the Newton-form assembly, every
    factorisation the inertia test took, the refined solve) and the whole iteration with its line
    search."""
    import torch
    out = {}
    for label, hess in (("gauss_newton", sgn.SGN_HESSIAN_GN), ("newton", sgn.SGN_HESSIAN_NEWTON)):
        ctx = sgn.Context(prob, sgn.default_options(precision=sgn.SGN_FP32_IR, hessian=hess)).allocate(dev)
        ctx.set_targets(prob.target_val, prob.length_scale)
        xe, pe = x.clone(), p.clone()
        ctx.equilibrium(pe, xe)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.newton_step(pe, xe, restart=True) if hess == sgn.SGN_HESSIAN_NEWTON else ctx.step(pe, xe)
        torch.cuda.synchronize()
        out[label] = {"ms_iteration": 1e3 * (time.perf_counter() - t0),
                      "ms_direction": info.ms_assemble + info.ms_factor + info.ms_solve,
                      "ms_assemble": info.ms_assemble, "ms_factor": info.ms_factor, "ms_solve": info.ms_solve,
                      "alpha": info.alpha, "f0": info.f0, "f1": info.f1, "grad_norm": info.grad_norm,
                      "rel_res": info.solve.rel_res}
        if hess == sgn.SGN_HESSIAN_NEWTON:
            out[label].update(inertia_trials=info.inertia_trials, delta=info.delta)
        del ctx
        torch.cuda.empty_cache()
    return out


def bicgstab_leg(sgn, prob, x, p, dev, steps, dp_ref):
    """BiCGSTAB on K preconditioned by the FP32 LDL^T of the stabilised matrix (eps_x = eps_lambda =
    1e-6, Sec. 5) at the workload's size: one direction (assembly + factorisation + BiCGSTAB)."""
    import torch
    o = sgn.default_options(precision=sgn.SGN_FP32_IR, solver=sgn.SGN_BICGSTAB, rhs_kind=sgn.SGN_RHS_KKT,
                            eps_x=1e-6, eps_lambda=1e-6)
    ctx = sgn.Context(prob, o).allocate(dev)
    ctx.set_targets(prob.target_val, prob.length_scale)
    N = 2 * prob.n_x + prob.n_p
    rhs = torch.zeros(N, dtype=torch.float64, device=dev)
    sol = torch.zeros(N, dtype=torch.float64, device=dev)

    def one():
        ctx.assemble(x, p, rhs)
        ctx.factor()
        return ctx.solve(rhs, sol)
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    nx, npar = prob.n_x, prob.n_p
    dp = sol.cpu().numpy()[nx:nx + npar]
    del ctx
    torch.cuda.empty_cache()
    return {"steps_per_s": 1.0 / dt, "ms_per_step": 1e3 * dt, "bicgstab_iterations": int(info.sweeps),
            "rel_res": info.rel_res, "raw_rel_res": info.raw_rel_res,
            "dp_rel_diff_vs_fp64": float(np.linalg.norm(dp - dp_ref) / np.linalg.norm(dp_ref))
            if dp_ref is not None else None}


def speedups(results):
    """FP32 + refinement over FP64, like for like: replayed graph against replayed graph, eager against
    eager."""
    out = {}
    for label, a, b in (("graph_vs_graph", "fp32ir_graph", "fp64_graph"), ("eager_vs_eager", "fp32ir", "fp64")):
        if a in results and b in results:
            out[label] = results[a]["steps_per_s"] / results[b]["steps_per_s"]
    return out or None


def stage_rooflines(results):
    """Assembly (HBM bound: algorithmic bytes of inputs and CSR values over the measured assembly time) and
    factorisation (matrix cores: dense front flops over the measured factorisation time) of the eager
    paths as fractions of the chip's peaks; the graph replays time the whole step only."""
    out = {}
    for path, peak in (("fp32ir", PEAK["fp32"]), ("fp64", PEAK["fp64"])):
        r = results.get(path)
        if not r or r.get("assemble_gbs") is None:
            continue
        out[path] = {
            "assembly": {"bound": "hbm", "achieved": round(r["assemble_gbs"], 2), "peak": HBM_PEAK, "unit": "GB/s",
                         "frac": round(r["assemble_gbs"] / HBM_PEAK, 4), "ms": r["assemble_ms"]},
            "factorization": {"bound": "mfma", "achieved": round(r["factor_tflops"], 2), "peak": peak,
                              "unit": "TFLOP/s", "frac": round(r["factor_tflops"] / peak, 4), "ms": r["factor_ms"]},
        }
    return out or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cantilever_100x25x25", choices=sorted(WORKLOADS))
    ap.add_argument("--paths", default="fp32ir_graph,fp32ir,fp64,fp64_graph,fp32ir_adjoint",
                    help="fp32ir / fp64: KKT right-hand side, eager launches; fp32ir_graph / fp64_graph: the same "
                         "step captured once into a HIP graph and replayed; fp32ir_adjoint: adjoint right-hand "
                         "side (one Kx solve)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no per-launch events on the update kernel")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-problem leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the learned-preconditioner, BiCGSTAB and block-solve legs")
    ap.add_argument("--autotune", action="store_true",
                    help="run the blocking autotuner on the workload and the batched union first and store its "
                         "records (paper_2107_03285_amd/tuning/); later runs use them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB copy first (for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sharded factorisation "
              f"over several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2107_03285_amd import sgn

    dev = "cuda:0"
    if args.copy_calibration:
        copy_calibration()
    prob = WORKLOADS[args.workload]()
    log(f"[bench] workload {prob.name}: n_x={prob.n_x} n_p={prob.n_p} N={2 * prob.n_x + prob.n_p}")
    paths = [s.strip() for s in args.paths.split(",") if s.strip()]

    blocking = {}

    def make_ctx(precision, rhs_kind=None):
        t0 = time.perf_counter()
        kw = dict(precision=precision, profile=0 if args.no_profile else 1,
                  rhs_kind=sgn.SGN_RHS_KKT if rhs_kind is None else rhs_kind)
        if precision == sgn.SGN_FP32_IR:  # the tuning records are taken for the FP32 path
            o, src = tuned_options(sgn, prob.name, **kw)
        else:
            o, src = sgn.default_options(**kw), "library defaults"
        blocking[precision] = dict(sgn.tuning_of(o), source=src)
        ctx = sgn.Context(prob, o).allocate(dev)
        log(f"[bench] context precision={precision} ready in {time.perf_counter() - t0:.1f} s "
            f"(workspace {ctx.workspace_size() / 1e9:.1f} GB)")
        return ctx

    # ---- set-up (untimed): x(p0), ell, targets = x(p0) + seeded noise
    f64 = sgn.SGN_FP64
    ref_ctx = make_ctx(f64)
    p = torch.tensor(prob.p_init(), dtype=torch.float64, device=dev)
    x = torch.tensor(prob.x_rest(), dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    eq = ref_ctx.equilibrium(p, x)
    log(f"[bench] equilibrium: {eq.iters} Newton iterations, |c|/|f| = {eq.res_norm / eq.f_ext_norm:.2e}, "
        f"{time.perf_counter() - t0:.2f} s")
    xh = x.cpu().numpy()
    ell = float(np.max(np.abs(xh - prob.x_rest())))
    prob.length_scale = ell
    prob.target_val = xh[prob.target_dof] + prob.target_noise
    ref_ctx.set_targets(prob.target_val, ell)
    ref_ctx.equilibrium(p, x)  # re-establishes the Kx factor for the adjoint right-hand side
    N = 2 * prob.n_x + prob.n_p
    if args.autotune:
        run_autotune(sgn, prob, x, p, dev)

    def run_step(ctx, rhs, sol):
        ctx.assemble(x, p, rhs)
        fi = ctx.factor()
        si_ = ctx.solve(rhs, sol)
        return fi, si_

    class GraphInfo:  # what the graph step reports in place of the eager factor / solve infos
        def __init__(self, rel, n_ir):
            self.rel_res, self.sweeps, self.ms = rel, n_ir, 0.0
            self.raw_rel_res = None
            self.n_pos = self.n_neg = self.n_zero = self.n_perturbed = -1

    results = {}
    sols = {}
    for path in paths:
        prec = {"fp32ir": sgn.SGN_FP32_IR, "fp64": sgn.SGN_FP64, "fp32ir_adjoint": sgn.SGN_FP32_IR,
                "fp32ir_graph": sgn.SGN_FP32_IR, "fp64_graph": sgn.SGN_FP64}[path]
        adj = path.endswith("_adjoint")
        graph = path.endswith("_graph")
        ctx = ref_ctx if (prec == f64 and not adj) else make_ctx(prec, sgn.SGN_RHS_ADJOINT if adj else None)
        if ctx is not ref_ctx:
            ctx.set_targets(prob.target_val, ell)
            xe = x.clone()
            ctx.equilibrium(p, xe)
        rhs = torch.zeros(N, dtype=torch.float64, device=dev)
        sol = torch.zeros(N, dtype=torch.float64, device=dev)
        step_fn = run_step
        if graph:
            # the eager step tells how many refinement sweeps reach 1e-10; the graph replays exactly that
            # many and checks the residual on the device at every replay (an error if it is not met)
            _, si0 = run_step(ctx, rhs, sol)
            n_ir = int(si0.sweeps)

            def step_fn(ctx, rhs, sol, n_ir=n_ir):
                rel = ctx.graph_step(x, p, rhs, sol, n_ir)
                return GraphInfo(rel, n_ir), GraphInfo(rel, n_ir)
        for w in range(args.warmup):
            fi, si_ = step_fn(ctx, rhs, sol)
            log(f"[bench] {path} warmup {w}: factor {fi.ms:.1f} ms, solve {si_.ms:.1f} ms "
                f"({si_.sweeps} refinement sweeps, res {si_.rel_res:.1e})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        upd_ms = upd_fl = 0.0
        upd_n = 0
        asm_ms = fac_ms = sol_ms = 0.0
        res = []
        raw = []
        sweeps = []
        step_ms = []
        for k in range(args.steps):
            ts = time.perf_counter()
            fi, si_ = step_fn(ctx, rhs, sol)
            torch.cuda.synchronize()
            step_ms.append(1e3 * (time.perf_counter() - ts))
            st = ctx.stats()
            upd_ms += st.update_ms
            upd_fl += st.update_flops
            upd_n += st.update_launches
            asm_ms += st.assemble_ms
            fac_ms += st.factor_ms
            sol_ms += st.solve_ms
            res.append(si_.rel_res)
            raw.append(si_.raw_rel_res)
            sweeps.append(si_.sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.stats()
        K = args.steps
        results[path] = dict(
            steps_per_s=K / dt, ms_per_step=1e3 * dt / K, median_ms=float(np.median(step_ms)),
            iqr_ms=float(np.percentile(step_ms, 75) - np.percentile(step_ms, 25)), factor_ms=fac_ms / K, solve_ms=sol_ms / K,
            assemble_ms=asm_ms / K, assemble_gbs=st.assemble_bytes / (asm_ms / K * 1e-3) / 1e9,
            factor_tflops=st.factor_flops / (fac_ms / K * 1e-3) / 1e12, rel_res_max=max(res),
            raw_rel_res_max=max(raw) if all(v is not None for v in raw) else None,
            refine_sweeps=max(sweeps), inertia=[fi.n_pos, fi.n_neg, fi.n_zero], perturbed=fi.n_perturbed,
            update_ms=upd_ms / K, update_tflops=(upd_fl / (upd_ms * 1e-3) / 1e12) if upd_ms > 0 else None,
            update_launches=upd_n // K, update_avg_us=(1e3 * upd_ms / upd_n) if upd_n else None,
            update_flops_per_launch=(upd_fl / upd_n) if upd_n else None)
        if graph:  # one replay covers every stage: per-stage host timings do not exist
            for key in ("factor_ms", "solve_ms", "assemble_ms", "assemble_gbs", "factor_tflops", "inertia",
                        "perturbed"):
                results[path][key] = None
            results[path]["graph_refine_sweeps"] = n_ir
        sols[path] = sol.cpu().numpy()
        log(f"[bench] {path}: {results[path]}")
        if ctx is not ref_ctx:
            del ctx
            torch.cuda.empty_cache()

    # ---- FP32 step against the FP64 step (per block)
    err = None
    if "fp32ir" in sols and "fp64" in sols:
        nx, npar = prob.n_x, prob.n_p
        a, b = sols["fp32ir"], sols["fp64"]
        err = {blk: float(np.linalg.norm(a[s] - b[s]) / np.linalg.norm(b[s]))
               for blk, s in (("dx", slice(0, nx)), ("dp", slice(nx, nx + npar)), ("dlambda", slice(nx + npar, N)))}
        if "fp32ir_graph" in sols:
            g = sols["fp32ir_graph"]
            err["dp_graph_vs_fp64"] = float(np.linalg.norm(g[nx:nx + npar] - b[nx:nx + npar]) /
                                            np.linalg.norm(b[nx:nx + npar]))
        if "fp32ir_adjoint" in sols:  # same dx and dp from the two right-hand sides (Appendix A)
            c = sols["fp32ir_adjoint"]
            err["dp_adjoint_vs_kkt"] = float(np.linalg.norm(c[nx:nx + npar] - b[nx:nx + npar]) /
                                             np.linalg.norm(b[nx:nx + npar]))
        log(f"[bench] FP32+IR step vs FP64 step: {err}")

    head = next((h for h in ("fp32ir_graph", "fp32ir") if h in results), paths[0])
    r = results[head]
    peak = PEAK["fp32" if head.startswith("fp32") else "fp64"]
    roof = None
    if r["update_tflops"] is not None:
        rec = recorded_traffic(prob.name) if head.startswith("fp32") else None
        roof = {"bound": "mfma", "achieved": round(r["update_tflops"], 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(r["update_tflops"] / peak, 4),
                "traffic": rec["bytes_per_launch"] if rec else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "k_update (MFMA trailing update of the fronts)",
                "avg_launch_us": r["update_avg_us"], "flops_per_launch": r["update_flops_per_launch"]}
    if roof is not None:
        roof["stages"] = stage_rooflines(results)
    learned = bicg = variants = newton = None
    if not args.no_variants:
        nx, npar = prob.n_x, prob.n_p
        dp_ref = sols["fp64"][nx:nx + npar] if "fp64" in sols else None
        if dp_ref is not None:
            log("[bench] learned-preconditioner leg")
            learned = learned_pc_leg(sgn, prob, x, p, torch.tensor(dp_ref, device=dev), dev, max(2, args.steps // 4))
        log("[bench] BiCGSTAB leg")
        bicg = bicgstab_leg(sgn, prob, x, p, dev, max(2, args.steps // 4), dp_ref)
        log(f"[bench] BiCGSTAB: {bicg}")
        log("[bench] Sparse Newton leg")
        newton = newton_leg(sgn, prob, x, p, dev)
        log(f"[bench] Newton vs Gauss-Newton: {newton}")
        log("[bench] block-solve leg")
        variants = variants_leg(sgn, dev, max(3, args.steps // 2))
        log(f"[bench] variants: {variants}")
    batch = None
    if not args.no_batch:
        log("[bench] batched leg: 256 2D problems, captured-graph step vs one at a time")
        batch = batch_leg(max(3, args.steps // 2), 1, dev, autotune=args.autotune)
        log(f"[bench] batched: {batch}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle sample")
        cpu = cpu_baseline()
    out = {
        "metric": "SGN steps/s at 200k DOF: FP32-MFMA+IR & learned-PC vs FP64 LDLᵀ @1e-10 res",
        "value": round(r["steps_per_s"], 4),
        "unit": "SGN steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 factor + f64 refinement" if head.startswith("fp32") else "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "n_x": prob.n_x, "n_p": prob.n_p, "N": N,
                   "path": head, "rhs": "KKT form [-df/dx; -df/dp; 0] (Appendix A, Theorem 2: same dp as [0; -g; 0])",
                   "solve_rtol": 1e-10},
        "paths": results,
        "blocking": {("fp32" if k == sgn.SGN_FP32_IR else "fp64"): v for k, v in blocking.items()},
        "fp32_vs_fp64_step": err,
        "speedup_vs_fp64": speedups(results),
        "roofline": roof,
        "learned_pc": learned,
        "bicgstab_stabilised": bicg,
        "block_solve": variants,
        "newton_vs_gauss_newton": newton,
        "batched_2d_256": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
