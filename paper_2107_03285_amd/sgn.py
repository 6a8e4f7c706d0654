"""ctypes binding of libsgn (the C ABI in include/sgn.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch provides device memory (the workspace and the caller's
vectors) and the stream.  Loading fails loudly when libsgn.so has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgn.so")

SGN_OK, SGN_E_ARG, SGN_E_STATE, SGN_E_NOMEM, SGN_E_HIP = 0, 1, 2, 3, 4
SGN_E_NEWTON, SGN_E_INVERTED, SGN_E_PIVOT, SGN_E_REFINE, SGN_E_LINESEARCH = 5, 6, 7, 8, 9
STATUS_NAMES = {0: "SGN_OK", 1: "SGN_E_ARG", 2: "SGN_E_STATE", 3: "SGN_E_NOMEM", 4: "SGN_E_HIP",
                5: "SGN_E_NEWTON", 6: "SGN_E_INVERTED", 7: "SGN_E_PIVOT", 8: "SGN_E_REFINE",
                9: "SGN_E_LINESEARCH"}
SGN_P_LOGE, SGN_P_REST_POS, SGN_P_NODAL_FORCE = 0, 1, 2
SGN_FP64, SGN_FP32_IR = 0, 1
SGN_LDLT, SGN_MINRES_LEARNED, SGN_BICGSTAB, SGN_BLOCK_GN = 0, 1, 2, 3
SGN_RHS_ADJOINT, SGN_RHS_KKT = 0, 1
SGN_HESSIAN_GN, SGN_HESSIAN_NEWTON = 0, 1
SGN_PC_FACTOR, SGN_PC_BLOCK = 0, 1
SGN_SYS_SGN, SGN_SYS_KX = 0, 1

EXPORTS = ["sgn_create", "sgn_default_options", "sgn_workspace_size", "sgn_set_workspace", "sgn_set_targets",
           "sgn_equilibrium", "sgn_assemble", "sgn_factor", "sgn_solve", "sgn_step", "sgn_get_sizes",
           "sgn_get_symbolic", "sgn_get_values", "sgn_get_stats", "sgn_selftest_mfma", "sgn_last_error",
           "sgn_destroy", "sgn_set_pc_correction", "sgn_spmv", "sgn_pc_apply", "sgn_pc_forward", "sgn_pc_grad",
           "sgn_solve_minres", "sgn_gnn_num_weights", "sgn_gnn_init", "sgn_gnn_forward", "sgn_gnn_backward",
           "sgn_adam", "sgn_set_pc_weights", "sgn_pc_train_loss", "sgn_graph_step", "sgn_autotune",
           "sgn_block_step", "sgn_lbfgs_step", "sgn_batch_create", "sgn_batch_step", "sgn_solve_static",
           "sgn_newton_step"]


class sgn_problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_nodes", C.c_int), ("n_elems", C.c_int),
                ("rest_pos", C.POINTER(C.c_double)), ("elems", C.POINTER(C.c_int32)),
                ("node_grid", C.POINTER(C.c_int32)), ("fixed", C.POINTER(C.c_uint8)),
                ("f_ext", C.POINTER(C.c_double)), ("E0", C.c_double), ("nu", C.c_double),
                ("param_kind", C.c_int), ("n_targets", C.c_int), ("target_dof", C.POINTER(C.c_int32)),
                ("target_val", C.POINTER(C.c_double)), ("target_w", C.c_double),
                ("length_scale", C.c_double), ("reg_mu", C.c_double), ("p_ref", C.POINTER(C.c_double)),
                ("n_components", C.c_int), ("component_ptr", C.POINTER(C.c_int32))]


class sgn_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("solver", C.c_int), ("rhs_kind", C.c_int),
                ("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("solve_rtol", C.c_double),
                ("eps_x", C.c_double), ("eps_lambda", C.c_double), ("max_newton", C.c_int),
                ("max_ir", C.c_int), ("max_minres", C.c_int), ("max_halvings", C.c_int),
                ("profile", C.c_int), ("max_gmres", C.c_int), ("outer_panels", C.c_int * 3),
                ("seq_panels", C.c_int), ("max_bicgstab", C.c_int), ("lbfgs_m", C.c_int),
                ("hessian", C.c_int), ("pc_kind", C.c_int), ("panel_waves", C.c_int)]


class sgn_stats(C.Structure):
    _fields_ = [("assemble_ms", C.c_double), ("assemble_bytes", C.c_double), ("factor_ms", C.c_double),
                ("factor_flops", C.c_double), ("update_ms", C.c_double), ("update_flops", C.c_double),
                ("update_launches", C.c_int64), ("solve_ms", C.c_double)]


class sgn_eq_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("halvings", C.c_int), ("res_norm", C.c_double),
                ("f_ext_norm", C.c_double), ("converged", C.c_int)]


class sgn_factor_info(C.Structure):
    _fields_ = [("n_pos", C.c_int64), ("n_neg", C.c_int64), ("n_zero", C.c_int64),
                ("n_perturbed", C.c_int64), ("min_abs_pivot", C.c_double), ("flops", C.c_double),
                ("ms", C.c_double)]


class sgn_solve_info(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("fallback", C.c_int), ("rel_res", C.c_double),
                ("raw_rel_res", C.c_double), ("ms", C.c_double), ("gmres_iters", C.c_int)]


class sgn_step_info(C.Structure):
    _fields_ = [("alpha", C.c_double), ("f0", C.c_double), ("f1", C.c_double), ("grad_norm", C.c_double),
                ("gtdp", C.c_double), ("halvings", C.c_int), ("newton_iters", C.c_int),
                ("ms_rhs", C.c_double), ("ms_assemble", C.c_double), ("ms_factor", C.c_double),
                ("ms_solve", C.c_double), ("ms_linesearch", C.c_double), ("solve", sgn_solve_info),
                ("delta", C.c_double), ("inertia_trials", C.c_int)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libsgn.so; raises if it is missing (build it with paper_2107_03285_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libsgn.so not found at {path}: build it first (python -m paper_2107_03285_amd.build)")
    # torch ships its own HIP runtime; load it first so that libsgn binds to the same
    # runtime instance that owns the device memory and streams it is handed
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i64p, i32p, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    sig = {
        "sgn_create": (C.c_int, [C.POINTER(sgn_problem), C.POINTER(sgn_options), vp, C.POINTER(vp)]),
        "sgn_default_options": (None, [C.POINTER(sgn_options)]),
        "sgn_workspace_size": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "sgn_set_workspace": (C.c_int, [vp, vp, C.c_size_t]),
        "sgn_set_targets": (C.c_int, [vp, dp, C.c_double]),
        "sgn_equilibrium": (C.c_int, [vp, vp, vp, C.POINTER(sgn_eq_info)]),
        "sgn_assemble": (C.c_int, [vp, vp, vp, vp, vp, dp]),
        "sgn_factor": (C.c_int, [vp, C.POINTER(sgn_factor_info)]),
        "sgn_solve": (C.c_int, [vp, vp, vp, C.POINTER(sgn_solve_info)]),
        "sgn_solve_static": (C.c_int, [vp, vp, vp, C.POINTER(sgn_solve_info)]),
        "sgn_block_step": (C.c_int, [vp, vp, vp, vp, C.POINTER(sgn_solve_info)]),
        "sgn_lbfgs_step": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(sgn_step_info)]),
        "sgn_newton_step": (C.c_int, [vp, vp, vp, C.c_int, C.POINTER(sgn_step_info)]),
        "sgn_batch_create": (C.c_int, [C.c_int, C.POINTER(C.POINTER(sgn_problem)), C.POINTER(sgn_options), vp,
                                       C.POINTER(vp)]),
        "sgn_batch_step": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(sgn_step_info)]),
        "sgn_step": (C.c_int, [vp, vp, vp, C.POINTER(sgn_step_info)]),
        "sgn_get_sizes": (C.c_int, [vp, C.c_int, i64p, i64p, i64p, i64p, dp]),
        "sgn_get_symbolic": (C.c_int, [vp, C.c_int, i32p, i32p, i64p, i32p]),
        "sgn_get_values": (C.c_int, [vp, C.c_int, dp]),
        "sgn_selftest_mfma": (C.c_int, [C.c_int, vp, vp, vp, vp]),
        "sgn_get_stats": (C.c_int, [vp, C.POINTER(sgn_stats)]),
        "sgn_last_error": (C.c_char_p, [vp]),
        "sgn_destroy": (None, [vp]),
        "sgn_set_pc_correction": (C.c_int, [vp, vp, vp]),
        "sgn_spmv": (C.c_int, [vp, vp, vp]),
        "sgn_pc_apply": (C.c_int, [vp, vp, vp, vp]),
        "sgn_pc_forward": (C.c_int, [vp, vp, vp]),
        "sgn_pc_grad": (C.c_int, [vp, vp, vp, C.c_double, vp, vp]),
        "sgn_solve_minres": (C.c_int, [vp, vp, vp, C.POINTER(sgn_solve_info)]),
        "sgn_gnn_num_weights": (C.c_int, [vp, i64p]),
        "sgn_gnn_init": (C.c_int, [vp, vp, C.c_uint64]),
        "sgn_gnn_forward": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "sgn_gnn_backward": (C.c_int, [vp, vp, vp, vp, vp]),
        "sgn_set_pc_weights": (C.c_int, [vp, vp]),
        "sgn_graph_step": (C.c_int, [vp, vp, vp, vp, vp, C.c_int, dp]),
        "sgn_pc_train_loss": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, vp, dp]),
        "sgn_adam": (C.c_int, [C.c_int64, vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int,
                               vp]),
        "sgn_autotune": (C.c_int, [C.POINTER(sgn_problem), C.POINTER(sgn_options), vp, vp, C.c_int, vp,
                                   C.POINTER(sgn_options), dp, C.POINTER(C.c_int)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SgnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def default_options(**kw) -> sgn_options:
    o = sgn_options()
    load_library().sgn_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _dev_ptr(t):
    return C.c_void_p(int(t.data_ptr())) if t is not None else None


def _problem_struct(prob):
    """The sgn_problem view of a Problem, with the arrays it points into (kept alive by the caller)."""
    d = prob.dim
    keep = dict(
        rest=np.ascontiguousarray(prob.rest_pos, dtype=np.float64),
        elems=np.ascontiguousarray(prob.elems, dtype=np.int32),
        grid=np.ascontiguousarray(prob.node_grid(), dtype=np.int32),
        fixed=np.ascontiguousarray(prob.fixed, dtype=np.uint8),
        fext=np.ascontiguousarray(prob.f_ext, dtype=np.float64),
        tdof=np.ascontiguousarray(prob.target_dof, dtype=np.int32),
        tval=np.ascontiguousarray(prob.target_val if prob.target_val is not None
                                  else np.zeros(len(prob.target_dof)), dtype=np.float64),
        pref=np.ascontiguousarray(prob.p_ref if prob.p_ref is not None else np.zeros(prob.n_p),
                                  dtype=np.float64),
        comp=np.ascontiguousarray(getattr(prob, "components", None) if getattr(prob, "components", None)
                                  is not None else [0, prob.n_nodes], dtype=np.int32),
    )
    k = keep
    P = sgn_problem(dim=d, n_nodes=prob.n_nodes, n_elems=prob.n_elems,
                    rest_pos=_ptr(k["rest"], C.c_double), elems=_ptr(k["elems"], C.c_int32),
                    node_grid=_ptr(k["grid"], C.c_int32), fixed=_ptr(k["fixed"], C.c_uint8),
                    f_ext=_ptr(k["fext"], C.c_double), E0=prob.E0, nu=prob.nu,
                    param_kind=prob.param_kind, n_targets=len(k["tdof"]),
                    target_dof=_ptr(k["tdof"], C.c_int32), target_val=_ptr(k["tval"], C.c_double),
                    target_w=prob.target_w,
                    length_scale=prob.length_scale if prob.length_scale else 1.0,
                    reg_mu=prob.reg_mu, p_ref=_ptr(k["pref"], C.c_double),
                    n_components=len(k["comp"]) - 1, component_ptr=_ptr(k["comp"], C.c_int32))
    return P, keep


def tuning_of(o: sgn_options) -> dict:
    """The schedule-blocking fields of an options struct."""
    return {"outer_panels": [int(v) for v in o.outer_panels], "seq_panels": int(o.seq_panels),
            "panel_waves": int(o.panel_waves)}


def apply_tuning(o: sgn_options, tuning: dict) -> sgn_options:
    """Sets the schedule-blocking fields of o from a tuning record (as written by autotune)."""
    for b, v in enumerate(tuning["outer_panels"]):
        o.outer_panels[b] = int(v)
    o.seq_panels = int(tuning["seq_panels"])
    o.panel_waves = int(tuning.get("panel_waves", 0))  # records from before this field: by launch
    return o


def autotune(prob, x, p, options: sgn_options = None, reps: int = 3, stream=None, path: str = None) -> dict:
    """Runs sgn_autotune for prob at the device state (x, p); returns the tuning record (and writes it
    as JSON to path if given): the chosen blocking, the candidates' milliseconds per round."""
    import json
    lib = load_library()
    P, keep = _problem_struct(prob)
    base = options if options is not None else default_options()
    best = sgn_options()
    ms = (C.c_double * 24)()
    n = C.c_int(0)
    sp = C.c_void_p(int(stream.cuda_stream)) if stream is not None else None
    st = lib.sgn_autotune(C.byref(P), C.byref(base), _dev_ptr(x), _dev_ptr(p), int(reps), sp, C.byref(best), ms,
                          C.byref(n))
    if st != SGN_OK:
        raise SgnError(st, "autotune: a candidate context failed")
    rec = dict(tuning_of(best), base=tuning_of(base), candidate_ms=[float(v) for v in ms[:min(n.value, 24)]],
               reps=int(reps), problem=getattr(prob, "name", ""))
    if path:
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
    return rec


def load_tuning(path: str) -> dict:
    import json
    with open(path) as f:
        return json.load(f)


class Context:
    """One libsgn context: host symbolic analysis at construction, a caller-owned
    device workspace (a torch uint8 tensor) once ``allocate()`` is called."""

    def __init__(self, prob, options: sgn_options = None, stream=None):
        lib = load_library()
        self.lib = lib
        self.prob = prob
        self.options = options if options is not None else default_options()
        P, self._keep = _problem_struct(prob)
        self._stream = stream
        h = C.c_void_p()
        st = lib.sgn_create(C.byref(P), C.byref(self.options), self._stream_ptr(), C.byref(h))
        self.h = h
        if st != SGN_OK:
            msg = lib.sgn_last_error(h).decode() if h.value else "invalid problem"
            raise SgnError(st, msg)
        self.workspace = None

    @classmethod
    def from_batch(cls, problems, options: sgn_options = None, stream=None):
        """A context over a batch of independent problems built by sgn_batch_create (the union is the
        problems in order; ``prob`` of the returned context is None)."""
        lib = load_library()
        self = cls.__new__(cls)
        self.lib = lib
        self.prob = None
        self.options = options if options is not None else default_options()
        structs, keeps = zip(*[_problem_struct(q) for q in problems])
        for P in structs:
            P.n_components = 0
        arr = (C.POINTER(sgn_problem) * len(structs))(*[C.pointer(P) for P in structs])
        self._keep = {"structs": structs, "arrays": keeps, "ptrs": arr}
        self._stream = stream
        h = C.c_void_p()
        st = lib.sgn_batch_create(len(structs), arr, C.byref(self.options), self._stream_ptr(), C.byref(h))
        self.h = h
        self.workspace = None
        if st != SGN_OK:
            msg = lib.sgn_last_error(h).decode() if h.value else "invalid batch"
            raise SgnError(st, msg)
        return self

    def batch_step(self, ps, xs):
        """One outer iteration of every problem of a batch (device tensors per problem, updated in
        place); returns the per-problem step infos."""
        n = len(ps)
        infos = (sgn_step_info * n)()
        pp = (C.c_void_p * n)(*[int(t.data_ptr()) for t in ps])
        xx = (C.c_void_p * n)(*[int(t.data_ptr()) for t in xs])
        self._check(self.lib.sgn_batch_step(self.h, pp, xx, infos))
        return list(infos)

    def _stream_ptr(self):
        if self._stream is None:
            return None
        return C.c_void_p(int(self._stream.cuda_stream))

    def _check(self, st):
        if st != SGN_OK:
            raise SgnError(st, self.lib.sgn_last_error(self.h).decode())
        return st

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and self.h.value:
                self.lib.sgn_destroy(self.h)
                self.h = C.c_void_p()
        except Exception:
            pass

    # ------------------------------------------------------------ sizes / symbolic (host only)
    def sizes(self, which=SGN_SYS_SGN):
        n, nnz, nsn, fe = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        fl = C.c_double()
        self._check(self.lib.sgn_get_sizes(self.h, which, C.byref(n), C.byref(nnz), C.byref(nsn), C.byref(fe),
                                           C.byref(fl)))
        return dict(n=n.value, nnz=nnz.value, n_supernodes=nsn.value, factor_entries=fe.value, flops=fl.value)

    def symbolic(self, which=SGN_SYS_SGN):
        s = self.sizes(which)
        n, nnz = s["n"], s["nnz"]
        perm = np.empty(n, np.int32)
        etree = np.empty(n, np.int32)
        rowptr = np.empty(n + 1, np.int64)
        colind = np.empty(nnz, np.int32)
        self._check(self.lib.sgn_get_symbolic(self.h, which, _ptr(perm, C.c_int32), _ptr(etree, C.c_int32),
                                              _ptr(rowptr, C.c_int64), _ptr(colind, C.c_int32)))
        return perm, etree, rowptr, colind

    def workspace_size(self) -> int:
        b = C.c_size_t()
        self._check(self.lib.sgn_workspace_size(self.h, C.byref(b)))
        return b.value

    # ------------------------------------------------------------ device
    def allocate(self, device="cuda"):
        import torch
        nbytes = self.workspace_size()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = int(self.workspace.data_ptr())
        aligned = (base + 255) & ~255
        self._check(self.lib.sgn_set_workspace(self.h, C.c_void_p(aligned), C.c_size_t(nbytes)))
        return self

    def set_targets(self, target_val, length_scale):
        tv = np.ascontiguousarray(target_val, dtype=np.float64)
        self._keep["tval"] = tv
        self._check(self.lib.sgn_set_targets(self.h, _ptr(tv, C.c_double), float(length_scale)))

    def equilibrium(self, p, x):
        info = sgn_eq_info()
        self._check(self.lib.sgn_equilibrium(self.h, _dev_ptr(p), _dev_ptr(x), C.byref(info)))
        return info

    def assemble(self, x, p, rhs=None, grad=None, want_obj=False):
        obj = C.c_double()
        self._check(self.lib.sgn_assemble(self.h, _dev_ptr(x), _dev_ptr(p), _dev_ptr(rhs), _dev_ptr(grad),
                                          C.byref(obj) if want_obj else None))
        return obj.value

    def factor(self):
        info = sgn_factor_info()
        self._check(self.lib.sgn_factor(self.h, C.byref(info)))
        return info

    def factor_status(self):
        """sgn_factor returning (status, info) instead of raising."""
        info = sgn_factor_info()
        st = self.lib.sgn_factor(self.h, C.byref(info))
        return st, info

    def solve(self, rhs, sol):
        info = sgn_solve_info()
        self._check(self.lib.sgn_solve(self.h, _dev_ptr(rhs), _dev_ptr(sol), C.byref(info)))
        return info

    def solve_static(self, rhs, sol):
        """sgn_solve with its working memory in the library's static device array (no allocation)."""
        info = sgn_solve_info()
        self._check(self.lib.sgn_solve_static(self.h, _dev_ptr(rhs), _dev_ptr(sol), C.byref(info)))
        return info

    def block_step(self, x, p, sol):
        """Block Gauss-Newton direction [dx; dp; dlam] at the equilibrium (x, p) (solver SGN_BLOCK_GN)."""
        info = sgn_solve_info()
        self._check(self.lib.sgn_block_step(self.h, _dev_ptr(x), _dev_ptr(p), _dev_ptr(sol), C.byref(info)))
        return info

    def solve_minres(self, rhs, sol):
        info = sgn_solve_info()
        self._check(self.lib.sgn_solve_minres(self.h, _dev_ptr(rhs), _dev_ptr(sol), C.byref(info)))
        return info

    def set_pc_correction(self, corr_node=None, corr_par=None):
        """Raw FP32 corrections (device tensors [n_nodes * (2d)(2d+1)/2], [n_p]) or None."""
        self._keep["corr"] = (corr_node, corr_par)
        self._check(self.lib.sgn_set_pc_correction(self.h, _dev_ptr(corr_node), _dev_ptr(corr_par)))

    def spmv(self, x, y):
        self._check(self.lib.sgn_spmv(self.h, _dev_ptr(x), _dev_ptr(y)))

    def pc_apply(self, v, out, fwd=None):
        self._check(self.lib.sgn_pc_apply(self.h, _dev_ptr(v), _dev_ptr(out), _dev_ptr(fwd)))

    def pc_forward(self, v, fwd):
        self._check(self.lib.sgn_pc_forward(self.h, _dev_ptr(v), _dev_ptr(fwd)))

    def pc_grad(self, fwd_a, fwd_b, weight, grad_node=None, grad_par=None):
        self._check(self.lib.sgn_pc_grad(self.h, _dev_ptr(fwd_a), _dev_ptr(fwd_b), float(weight),
                                         _dev_ptr(grad_node), _dev_ptr(grad_par)))

    def gnn_num_weights(self) -> int:
        n = C.c_int64()
        self._check(self.lib.sgn_gnn_num_weights(self.h, C.byref(n)))
        return n.value

    def gnn_init(self, w, seed=0):
        self._check(self.lib.sgn_gnn_init(self.h, _dev_ptr(w), C.c_uint64(seed)))

    def gnn_forward(self, w, x_ref, p_ref, x, p, corr_node, corr_par):
        self._check(self.lib.sgn_gnn_forward(self.h, _dev_ptr(w), _dev_ptr(x_ref), _dev_ptr(p_ref), _dev_ptr(x),
                                             _dev_ptr(p), _dev_ptr(corr_node), _dev_ptr(corr_par)))

    def gnn_backward(self, w, gcorr_node, gcorr_par, gw):
        self._check(self.lib.sgn_gnn_backward(self.h, _dev_ptr(w), _dev_ptr(gcorr_node), _dev_ptr(gcorr_par),
                                              _dev_ptr(gw)))

    def set_pc_weights(self, w):
        self._keep["pc_weights"] = w
        self._check(self.lib.sgn_set_pc_weights(self.h, _dev_ptr(w)))

    def pc_train_loss(self, w, probes, gw, log_form=False) -> float:
        """probes: device float64 tensor [k, N]; gw += gradient (of log(loss) with log_form); returns the mean loss."""
        loss = C.c_double()
        self._check(self.lib.sgn_pc_train_loss(self.h, _dev_ptr(w), _dev_ptr(probes), int(probes.shape[0]),
                                               int(bool(log_form)), _dev_ptr(gw), C.byref(loss)))
        return loss.value

    def graph_step(self, x, p, rhs, sol, n_ir=2):
        """Captured-graph step (KKT right-hand side, n_ir refinement sweeps); returns the final residual."""
        rel = C.c_double()
        self._check(self.lib.sgn_graph_step(self.h, _dev_ptr(x), _dev_ptr(p), _dev_ptr(rhs), _dev_ptr(sol),
                                            int(n_ir), C.byref(rel)))
        return rel.value

    def step(self, p, x):
        info = sgn_step_info()
        self._check(self.lib.sgn_step(self.h, _dev_ptr(p), _dev_ptr(x), C.byref(info)))
        return info

    def lbfgs_step(self, p, x, restart=False):
        """One SGN-initialised L-BFGS iteration (updates p and x in place)."""
        info = sgn_step_info()
        self._check(self.lib.sgn_lbfgs_step(self.h, _dev_ptr(p), _dev_ptr(x), int(bool(restart)), C.byref(info)))
        return info

    def newton_step(self, p, x, restart=False):
        """One Sparse Newton iteration with inertia control (updates p and x in place)."""
        info = sgn_step_info()
        self._check(self.lib.sgn_newton_step(self.h, _dev_ptr(p), _dev_ptr(x), int(bool(restart)), C.byref(info)))
        return info

    def values(self, which=SGN_SYS_SGN):
        out = np.empty(self.sizes(which)["nnz"], np.float64)
        self._check(self.lib.sgn_get_values(self.h, which, _ptr(out, C.c_double)))
        return out

    def stats(self) -> sgn_stats:
        out = sgn_stats()
        self._check(self.lib.sgn_get_stats(self.h, C.byref(out)))
        return out

    def last_error(self) -> str:
        return self.lib.sgn_last_error(self.h).decode()


def adam(w, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step on FP32 device tensors (w updated in place)."""
    lib = load_library()
    st = lib.sgn_adam(w.numel(), _dev_ptr(w), _dev_ptr(g), _dev_ptr(m), _dev_ptr(v), float(lr), float(beta1),
                      float(beta2), float(eps), int(step),
                      C.c_void_p(int(stream.cuda_stream)) if stream is not None else None)
    if st != SGN_OK:
        raise SgnError(st, "adam")


def selftest_mfma(prec, a, b, out, stream=None):
    """One 16x16x4 matrix-core product (device tensors a [16,4], b [4,16], out [16,16], float64)."""
    lib = load_library()
    st = lib.sgn_selftest_mfma(prec, _dev_ptr(a), _dev_ptr(b), _dev_ptr(out),
                               C.c_void_p(int(stream.cuda_stream)) if stream is not None else None)
    if st != SGN_OK:
        raise SgnError(st, "mfma self test")
