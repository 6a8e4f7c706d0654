// C ABI of libsgn (declared in include/sgn.h): context, workspace layout and
// the host drivers of the hot path -- Newton equilibrium (Sec. 5), SGN
// assembly and right-hand side (Sec. 4, eq. sparseSystemGN; adjoint gradient
// of eq. totalGradient), supernodal LDL^T, refined solves, and the outer
// iteration with backtracking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/sgn.h"
#include "gnn.h"
#include "kernels.h"

static_assert(sgn::kTile == sgn::kUpdTile, "the schedule counts the update kernel's tiles");
#include "symbolic.h"

using namespace sgn;

namespace {

struct DevSys {
  int64_t* rowptr = nullptr;
  int32_t* colind = nullptr;
  int32_t* slot_row = nullptr;
  int64_t* csr_front_pos = nullptr;
  int64_t* slot_ptr = nullptr;
  int32_t* slot_src = nullptr;
  int32_t* diag_kind = nullptr;
  int64_t* frowptr = nullptr;
  int32_t* fcol = nullptr;
  int32_t* fslot = nullptr;
  int32_t* perm = nullptr;
  int32_t* sn_begin = nullptr;
  int32_t* sn_m = nullptr;
  int64_t* sn_front_off = nullptr;
  int64_t* sn_vec_off = nullptr;
  int64_t* sn_rows_ptr = nullptr;
  int32_t* sn_rows = nullptr;
  int64_t* relmap_off = nullptr;
  int32_t* relmap = nullptr;
  int32_t* child_ptr = nullptr;
  int32_t* child_list = nullptr;
  int32_t* var_group_end = nullptr;
  int32_t* solve_sn = nullptr;
  int32_t* panel_ptr = nullptr;
  int32_t* panel_col = nullptr;
  int64_t* panel_tasks = nullptr;
  int64_t* upd_tasks = nullptr;
  int32_t* upd_tile_task = nullptr;
  int64_t* ea_cols = nullptr;
  int64_t* ea_kids = nullptr;
  int32_t* fill_tasks = nullptr;
  int64_t* vec_ptr = nullptr;
  int32_t* vec_src = nullptr;
  int32_t* solve_fwd_tasks = nullptr;
  int32_t* solve_bwd_tasks = nullptr;
  int64_t* sn_part_off = nullptr;
  double* part = nullptr;      // split-k partial sums of the forward solve
  int* solve_ctr = nullptr;    // [2 * nsn] per-front ticket counters of the forward / backward pipelined solves
  int64_t* const_slots = nullptr;
  int64_t n_const = 0;
  double* vals = nullptr;
  double* scale = nullptr;
  double* dpiv = nullptr;
  double* epiv = nullptr;
  int32_t* pivtype = nullptr;
  int32_t* lperm = nullptr;
  void* front = nullptr;
  double* tv = nullptr;
  double* tp = nullptr;
  double* b = nullptr;     // caller-facing work vectors of the drivers
  double* z = nullptr;
  double* r = nullptr;
  double* t = nullptr;
  double* sv = nullptr;    // internal to solve_once: scaled right-hand side
  double* ir_r = nullptr;  // internal to refined_solve: residual
  double* ir_d = nullptr;  // internal to refined_solve: correction
  double* ir_s = nullptr;  // internal to refined_solve: scaled residual
  double* gm_V = nullptr;  // FGMRES escalation: Arnoldi basis [(kGmresM + 1) x N]
  double* gm_Z = nullptr;  // preconditioned basis [kGmresM x N]
  double* gm_t = nullptr;  // correction [N]
  // node-block preconditioner (SGN system only)
  int32_t* grp_ptr = nullptr;
  int32_t* grp_node = nullptr;
  int64_t* grp_vec = nullptr;
  int64_t ngroups = 0;
  double* pc_w = nullptr;      // [N] block-solved forward result (pivot order)
  double* cur_scale = nullptr; // [N] row scaling of the currently assembled matrix (residual weights)
  double* mr[10] = {};         // MINRES work vectors
  int64_t* bp_off = nullptr;   // block-diagonal preconditioner (pc_kind = SGN_PC_BLOCK): offsets of the
  double* bp_minv = nullptr;   // dense |B_i|^-1 blocks, one per node group
  bool bp_ready = false;       // the blocks are of the currently assembled matrix
  int prec = 0;  // 0: FP64 fronts, 1: FP32 fronts
  int row_lanes = 16;  // lanes per row of the SpMV-shaped kernels
  bool factored = false;  // a factorisation is held (the MINRES reference)
  bool current = false;   // ... and it is of the currently assembled matrix
  int64_t inertia[3] = {0, 0, 0};
};

struct Layout {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

bool verbose() {
  static const bool v = std::getenv("SGN_VERBOSE") != nullptr;
  return v;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

constexpr int kGmresM = 30;  // FGMRES restart length of the refinement escalation

struct sgn_ctx_s {
  Analysis A;
  sgn_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  bool sticky = false;
  bool has_ws = false;
  std::vector<int32_t> target_dof;
  std::vector<double> target_val, p_ref, fext_free;
  std::vector<int32_t> efdof;
  double target_w = 1, ell = 1, mu_in = 0, mu_reg = 0, mu0 = 0, lam0 = 0, fext_norm = 0;
  DevSys sys[2];
  int32_t* d_elems = nullptr;
  int32_t* d_efdof = nullptr;
  double* d_rest = nullptr;
  double* d_fext = nullptr;
  int32_t* d_tdof = nullptr;
  double* d_tval = nullptr;
  double* d_pref = nullptr;
  double* d_ebuf = nullptr;
  double* d_x = nullptr;
  double* d_xt = nullptr;
  double* d_p = nullptr;
  double* d_pt = nullptr;
  double* d_c = nullptr;
  double* d_dx = nullptr;
  double* d_fx = nullptr;
  double* d_fp = nullptr;
  double* d_lam = nullptr;
  double* d_g = nullptr;
  double* d_old = nullptr;
  double* d_old2 = nullptr;
  double* d_rt = nullptr;
  double* d_srhs = nullptr;  // [N] step right-hand side (boundary order)
  double* d_ssol = nullptr;  // [N] step solution (boundary order)
  double* d_part = nullptr;
  double* d_scal = nullptr;
  double* d_gm = nullptr;             // FGMRES coefficients: two Gram-Schmidt passes, |w|^2, solution
  std::vector<double> gm_host;        // host copy of the FGMRES solution coefficients
  int* d_cnt = nullptr;
  unsigned long long* d_ull = nullptr;
  // preconditioner network: graph tables and activations (FP32)
  GnnGraph G;
  struct {
    int32_t *src, *dst, *in_ptr, *out_ptr, *out_list, *inc_ptr, *inc_list, *nfdof;
    float *nf, *ef, *h[kGnnLayers + 1], *yn[kGnnLayers], *agg[kGnnLayers], *e[kGnnLayers + 1], *ye[kGnnLayers];
    float *dec, *emb, *dh[2], *de[2], *dz, *dx, *dagg, *ddec, *demb, *part;
  } g{};
  bool gnn_fwd_done = false;
  bool capturing = false;             // enqueueing into a graph: no host syncs
  hipStream_t gstream = nullptr;      // stream of the captured step graph
  hipStream_t side = nullptr;         // the factorisation's second stream (updates beyond the next block)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_key[4] = {};      // (x, p, rhs, sol) the graph was captured for
  int graph_nir = -1;
  bool graph_prof = false;            // the graph holds event records around the update launches
  size_t prof_nev = 0;                // event pairs of the last (or captured) factorisation
  double prof_flops = 0.0;
  const float* pc_weights = nullptr;  // caller-owned network weights (null: corrections as set)
  bool use_own = false;               // the preconditioner reads own_cn / own_cp
  float* own_cn = nullptr;            // corrections computed by the network
  float* own_cp = nullptr;
  float* g_cn = nullptr;              // their gradients (training loss)
  float* g_cp = nullptr;
  double* d_x_asm = nullptr;          // state of the last SGN assembly
  double* d_p_asm = nullptr;
  double* d_x_fac = nullptr;          // state of the reference factor
  double* d_p_fac = nullptr;
  const float* corr_node = nullptr;  // caller-owned raw preconditioner corrections (null: none)
  const float* corr_par = nullptr;
  bool kx_valid = false;
  bool sgn_assembled = false;
  double newton_delta_last = 0.0;     // regularisation of the last sgn_newton_step that needed one
  std::vector<int64_t> bp_off;        // block-diagonal preconditioner: offsets of the groups' blocks
  // L-BFGS memory (sgn_lbfgs_step): newest pair at lb_head - 1 (circular), curvature 1 / s^T y
  double* lb_s = nullptr;             // [lbfgs_m x n_p]
  double* lb_y = nullptr;             // [lbfgs_m x n_p]
  double* lb_pprev = nullptr;         // [n_p] parameters and gradient of the previous iterate
  double* lb_gprev = nullptr;
  double* lb_q = nullptr;             // [n_p] two-loop vectors
  double* lb_r = nullptr;
  std::vector<double> lb_rho;
  int lb_count = 0, lb_head = 0;
  bool lb_have_prev = false;
  // batches (n_components problems): contiguous ranges of each problem's free DOFs and parameters
  // (sgn_batch_step needs the parameters stored problem by problem: batch_ok)
  int ncomp = 1;
  bool batch_ok = false;
  std::vector<int64_t> seg_x, seg_p;
  int64_t* d_seg_x = nullptr;
  int64_t* d_seg_p = nullptr;
  double* d_seg_val = nullptr;        // [4 x ncomp] per-problem reductions
  double* d_seg_alpha = nullptr;      // [ncomp] per-problem step lengths
  int32_t* d_seg_mask = nullptr;      // [ncomp]
  size_t ws_need = 0;  // workspace bytes, fixed at create (layout() with a null base resets pointers)
  sgn_stats stats{};
  std::vector<hipEvent_t> ev_pool;  // per-launch timing events (profile = 1)
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  ~sgn_ctx_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
  }
};

namespace {

sgn_status fail(sgn_ctx c, sgn_status s, const std::string& msg) {
  if (c && s != SGN_OK) {
    c->err = msg;
    c->sticky = true;
  }
  return s;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(c, SGN_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                    \
  do {                               \
    sgn_status s_ = (expr);          \
    if (s_ != SGN_OK) return s_;     \
  } while (0)

template <typename T>
size_t bytes_of(const std::vector<T>& v) {
  return v.size() * sizeof(T);
}

// The factorisation's second stream (default priority, ordered against the context's stream by
// events only) and its fork / join events.
hipError_t ensure_side(sgn_ctx c) {
  hipError_t e = hipSuccess;
  if (!c->side) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess && !c->ev_fork) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess && !c->ev_join) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  return e;
}

hipError_t ensure_events(sgn_ctx c, size_t n) {
  if (!c->ev_a) {
    hipError_t e = hipEventCreate(&c->ev_a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&c->ev_b);
    if (e != hipSuccess) return e;
  }
  while (c->ev_pool.size() < n) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    c->ev_pool.push_back(ev);
  }
  return hipSuccess;
}

size_t layout(sgn_ctx c, char* base) {
  Layout L{base};
  const Analysis& A = c->A;
  const int64_t nx = A.mesh.n_x, np = A.mesh.n_p, ne = A.mesh.n_elems, nv = A.mesh.dim + 1;
  const size_t nt = c->target_dof.size();
  for (int si = 0; si < 2; ++si) {
    const System& S = si == 0 ? A.sgn : A.kx;
    DevSys& D = c->sys[si];
    D.rowptr = L.take<int64_t>(S.rowptr.size());
    D.colind = L.take<int32_t>(S.colind.size());
    D.slot_row = L.take<int32_t>(S.slot_row.size());
    D.csr_front_pos = L.take<int64_t>(S.csr_front_pos.size());
    D.slot_ptr = L.take<int64_t>(S.slot_ptr.size());
    D.slot_src = L.take<int32_t>(S.slot_src.size());
    D.diag_kind = L.take<int32_t>(S.diag_kind.size());
    D.frowptr = L.take<int64_t>(S.frowptr.size());
    D.row_lanes = row_lanes_for(S.N, S.frowptr.empty() ? 0 : S.frowptr.back());
    D.fcol = L.take<int32_t>(S.fcol.size());
    D.fslot = L.take<int32_t>(S.fslot.size());
    D.perm = L.take<int32_t>(S.perm.size());
    D.sn_begin = L.take<int32_t>(S.sn_begin.size());
    D.sn_m = L.take<int32_t>(S.sn_m.size());
    D.sn_front_off = L.take<int64_t>(S.sn_front_off.size());
    D.sn_vec_off = L.take<int64_t>(S.sn_vec_off.size());
    D.sn_rows_ptr = L.take<int64_t>(S.sn_rows_ptr.size());
    D.sn_rows = L.take<int32_t>(S.sn_rows.size());
    D.relmap_off = L.take<int64_t>(S.relmap_off.size());
    D.relmap = L.take<int32_t>(S.relmap.size());
    D.child_ptr = L.take<int32_t>(S.child_ptr.size());
    D.child_list = L.take<int32_t>(S.child_list.size());
    D.var_group_end = L.take<int32_t>(S.var_group_end.size());
    D.solve_sn = L.take<int32_t>(S.solve_sn.size());
    D.panel_ptr = L.take<int32_t>(S.panel_ptr.size());
    D.panel_col = L.take<int32_t>(S.panel_col.size());
    D.panel_tasks = L.take<int64_t>(S.panel_tasks.size());
    D.upd_tasks = L.take<int64_t>(S.upd_tasks.size());
    D.upd_tile_task = L.take<int32_t>(S.upd_tile_task.size());
    D.ea_cols = L.take<int64_t>(S.ea_cols.size());
    D.ea_kids = L.take<int64_t>(S.ea_kid_recs.size());
    D.fill_tasks = L.take<int32_t>(S.fill_tasks.size());
    D.vec_ptr = L.take<int64_t>(S.vec_ptr.size());
    D.vec_src = L.take<int32_t>(S.vec_src.size());
    D.solve_fwd_tasks = L.take<int32_t>(S.solve_fwd_tasks.size());
    D.solve_bwd_tasks = L.take<int32_t>(S.solve_bwd_tasks.size());
    D.solve_ctr = L.take<int>(2 * (size_t)S.nsn);
    D.sn_part_off = L.take<int64_t>(S.sn_part_off.size());
    D.part = L.take<double>(S.part_total);
    D.n_const = (si == 0 && A.mesh.param_kind == 2) ? nx : 0;
    D.const_slots = L.take<int64_t>(D.n_const);
    D.vals = L.take<double>(S.colind.size());
    D.scale = L.take<double>(S.N);
    D.dpiv = L.take<double>(S.N);
    D.epiv = L.take<double>(S.N);
    D.pivtype = L.take<int32_t>(S.N);
    D.lperm = L.take<int32_t>(S.N);
    D.prec = (si == 0 && c->opt.precision == SGN_FP32_IR) ? 1 : 0;
    const size_t esz = D.prec ? sizeof(float) : sizeof(double);
    D.front = L.take<char>(S.front_total * esz + 64);
    D.tv = L.take<double>(S.vec_total);
    D.tp = L.take<double>(S.vec_total);
    D.b = L.take<double>(S.N);
    D.z = L.take<double>(S.N);
    D.r = L.take<double>(S.N);
    D.t = L.take<double>(S.N);
    D.sv = L.take<double>(S.N);
    D.ir_r = L.take<double>(S.N);
    D.ir_d = L.take<double>(S.N);
    D.ir_s = L.take<double>(S.N);
    D.gm_V = L.take<double>((int64_t)(kGmresM + 1) * S.N);
    D.gm_Z = L.take<double>((int64_t)kGmresM * S.N);
    D.gm_t = L.take<double>(S.N);
    if (si == 0) {
      D.ngroups = (int64_t)S.grp_node.size();
      D.grp_ptr = L.take<int32_t>(S.grp_ptr.size());
      D.grp_node = L.take<int32_t>(S.grp_node.size());
      D.grp_vec = L.take<int64_t>(S.grp_vec.size());
      D.pc_w = L.take<double>(S.N);
      D.cur_scale = L.take<double>(S.N);
      for (double*& v : D.mr) v = L.take<double>(S.N);
      if (c->opt.pc_kind == SGN_PC_BLOCK) {
        D.bp_off = L.take<int64_t>(c->bp_off.size());
        D.bp_minv = L.take<double>((size_t)c->bp_off.back());
      }
    }
  }
  {
    const GnnGraph& G = c->G;
    const int64_t nn = A.mesh.n_nodes, E = G.n_edges, H = kGnnH;
    const int64_t rows = std::max<int64_t>(std::max<int64_t>(E, nn), ne);
    auto& g = c->g;
    g.src = L.take<int32_t>(E);
    g.dst = L.take<int32_t>(E);
    g.in_ptr = L.take<int32_t>(nn + 1);
    g.out_ptr = L.take<int32_t>(nn + 1);
    g.out_list = L.take<int32_t>(E);
    g.inc_ptr = L.take<int32_t>(nn + 1);
    g.inc_list = L.take<int32_t>(ne * nv);
    g.nfdof = L.take<int32_t>(nn);
    g.nf = L.take<float>(nn * G.fn);
    g.ef = L.take<float>(E * G.fe);
    for (int l = 0; l <= kGnnLayers; ++l) {
      g.h[l] = L.take<float>(nn * H);
      g.e[l] = L.take<float>(E * H);
    }
    for (int l = 0; l < kGnnLayers; ++l) {
      g.yn[l] = L.take<float>(nn * H);
      g.agg[l] = L.take<float>(nn * H);
      g.ye[l] = L.take<float>(E * H);
    }
    g.dec = L.take<float>(nn * G.nout_node);
    g.emb = L.take<float>(G.param_kind == 0 ? ne * H : 0);
    for (int i = 0; i < 2; ++i) {
      g.dh[i] = L.take<float>(nn * H);
      g.de[i] = L.take<float>(E * H);
    }
    g.dz = L.take<float>(rows * H);
    g.dx = L.take<float>(rows * kGnnMaxK);
    g.dagg = L.take<float>(nn * H);
    g.ddec = L.take<float>(nn * G.nout_node);
    g.demb = L.take<float>(G.param_kind == 0 ? ne * H : 0);
    g.part = L.take<float>((int64_t)wgrad_parts(rows) * (kGnnMaxK + 1) * H);
  }
  c->own_cn = L.take<float>((int64_t)A.mesh.n_nodes * c->G.tri);
  c->own_cp = L.take<float>(np);
  c->g_cn = L.take<float>((int64_t)A.mesh.n_nodes * c->G.tri);
  c->g_cp = L.take<float>(np);
  c->d_x_asm = L.take<double>(nx);
  c->d_p_asm = L.take<double>(np);
  c->d_x_fac = L.take<double>(nx);
  c->d_p_fac = L.take<double>(np);
  c->d_elems = L.take<int32_t>(ne * nv);
  c->d_efdof = L.take<int32_t>(ne * nv);
  c->d_rest = L.take<double>(A.mesh.rest.size());
  c->d_fext = L.take<double>(nx);
  c->d_tdof = L.take<int32_t>(nt);
  c->d_tval = L.take<double>(nt);
  c->d_pref = L.take<double>(np);
  c->d_ebuf = L.take<double>(ne * (int64_t)A.stride);
  c->d_x = L.take<double>(nx);
  c->d_xt = L.take<double>(nx);
  c->d_p = L.take<double>(np);
  c->d_pt = L.take<double>(np);
  c->d_c = L.take<double>(nx);
  c->d_dx = L.take<double>(nx);
  c->d_fx = L.take<double>(nx);
  c->d_fp = L.take<double>(np);
  c->d_lam = L.take<double>(nx);
  c->d_g = L.take<double>(np);
  c->d_old = L.take<double>(A.sgn.N);
  c->d_old2 = L.take<double>(A.sgn.N);
  c->d_rt = L.take<double>(nt);
  c->d_srhs = L.take<double>(A.sgn.N);
  c->d_ssol = L.take<double>(A.sgn.N);
  {
    const int64_t m = std::max(0, c->opt.lbfgs_m);
    c->lb_s = L.take<double>(m * np);
    c->lb_y = L.take<double>(m * np);
    c->lb_pprev = L.take<double>(np);
    c->lb_gprev = L.take<double>(np);
    c->lb_q = L.take<double>(np);
    c->lb_r = L.take<double>(np);
  }
  c->d_seg_x = L.take<int64_t>(c->ncomp + 1);
  c->d_seg_p = L.take<int64_t>(c->ncomp + 1);
  c->d_seg_val = L.take<double>(4 * (int64_t)c->ncomp);
  c->d_seg_alpha = L.take<double>(c->ncomp);
  c->d_seg_mask = L.take<int32_t>(c->ncomp);
  c->d_part = L.take<double>(4 * kRedBlocks);
  c->d_scal = L.take<double>(64);
  c->d_gm = L.take<double>(256);
  c->d_cnt = L.take<int>(64);
  c->d_ull = L.take<unsigned long long>(16);
  return L.off + 256;
}

template <typename T>
hipError_t up(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), bytes_of(src), hipMemcpyHostToDevice, s);
}

// ------------------------------------------------------------------ reductions
// Forget the captured step graph: its nodes hold the workspace addresses and the objective
// weights (target values are read through a pointer, ell and mu by value) of the time of capture.
sgn_status drop_graph(sgn_ctx c) {
  hipError_t e = hipSuccess;
  if (c->graph_exec) e = hipGraphExecDestroy(c->graph_exec);
  if (c->graph) {
    const hipError_t e2 = hipGraphDestroy(c->graph);
    if (e == hipSuccess) e = e2;
  }
  c->graph_exec = nullptr;
  c->graph = nullptr;
  std::fill(c->graph_key, c->graph_key + 4, nullptr);
  c->graph_nir = -1;
  if (e != hipSuccess) return fail(c, SGN_E_HIP, std::string("graph destroy: ") + hipGetErrorString(e));
  return SGN_OK;
}

sgn_status read_scalars(sgn_ctx c, int first, int n, double* out) {
  HIPCHK(hipMemcpyAsync(out, c->d_scal + first, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

void dev_dot(sgn_ctx c, int64_t n, const double* a, const double* b, int slot, int64_t stride = 1,
             int absval = 0) {
  launch_dot_partials(n, a, b, stride, absval, c->d_part, c->stream);
  launch_final_sum(c->d_part, kRedBlocks, c->d_scal + slot, c->stream);
}

void dev_dot_to(sgn_ctx c, int64_t n, const double* a, const double* b, double* out) {
  launch_dot_partials(n, a, b, 1, 0, c->d_part, c->stream);
  launch_final_sum(c->d_part, kRedBlocks, out, c->stream);
}

// ------------------------------------------------------------------ element + assembly
sgn_status run_element(sgn_ctx c, const double* x, const double* p, int mode, int* inverted) {
  const Analysis& A = c->A;
  launch_fill_i32(1, 0, c->d_cnt + 8, c->stream);
  ElemArgs ea{};
  ea.dim = A.mesh.dim;
  ea.ne = A.mesh.n_elems;
  ea.param_kind = A.mesh.param_kind;
  ea.mode = mode;
  ea.elems = c->d_elems;
  ea.efdof = c->d_efdof;
  ea.rest = c->d_rest;
  ea.x = x;
  ea.p = p;
  ea.mu0 = c->mu0;
  ea.lam0 = c->lam0;
  ea.ebuf = c->d_ebuf;
  ea.stride = A.stride;
  ea.off_grad = A.off_grad;
  ea.off_kp = A.off_kp;
  ea.off_energy = A.off_energy;
  ea.inverted = c->d_cnt + 8;
  ea.lam = mode == 3 ? c->d_lam : nullptr;
  ea.off_t = A.off_t;
  ea.off_kl = A.off_kl;
  ea.off_lg = A.off_lg;
  launch_element(ea, c->stream);
  HIPCHK(hipGetLastError());
  int inv = 0;
  HIPCHK(hipMemcpyAsync(&inv, c->d_cnt + 8, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *inverted = inv;
  return SGN_OK;
}

// Kx values (+ shift tau on the diagonal) from the element buffer
void assemble_kx(sgn_ctx c, double tau) {
  const System& S = c->A.kx;
  DevSys& D = c->sys[1];
  launch_gather_slots((int64_t)S.colind.size(), D.slot_ptr, D.slot_src, c->d_ebuf, D.vals, c->stream);
  if (tau != 0.0) launch_diag_add(S.N, D.rowptr, D.diag_kind, 0.0, 0.0, tau, 0.0, D.vals, c->stream);
}

void assemble_sgn(sgn_ctx c) {
  const System& S = c->A.sgn;
  DevSys& D = c->sys[0];
  launch_gather_slots((int64_t)S.colind.size(), D.slot_ptr, D.slot_src, c->d_ebuf, D.vals, c->stream);
  const double a_t = c->target_w / (c->ell * c->ell);
  launch_diag_add(S.N, D.rowptr, D.diag_kind, a_t, c->mu_reg, c->opt.eps_x, c->opt.eps_lambda, D.vals, c->stream);
  if (D.n_const) launch_const_slots(D.n_const, D.const_slots, -1.0, D.vals, c->stream);
}

// residual c = sum g_e - f_ext (- p)
void residual_vec(sgn_ctx c, const double* p, double* out) {
  const System& S = c->A.kx;
  DevSys& D = c->sys[1];
  launch_gather_vec(S.N, D.vec_ptr, D.vec_src, c->d_ebuf, c->d_fext, c->A.mesh.param_kind == 2 ? p : nullptr, out,
                    c->stream);
}

// ------------------------------------------------------------------ factorisation
// update-kernel timing of the last factorisation from its event pairs (ev_pool[0 .. prof_nev))
sgn_status read_update_events(sgn_ctx c) {
  HIPCHK(hipStreamSynchronize(c->stream));
  double ms = 0.0;
  for (size_t k = 0; k < c->prof_nev; k += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, c->ev_pool[k], c->ev_pool[k + 1]));
    ms += t;
  }
  c->stats.update_ms = ms;
  c->stats.update_flops = c->prof_flops;
  c->stats.update_launches = (int64_t)(c->prof_nev / 2);
  return SGN_OK;
}

// Wavefronts per panel's diagonal-block factorisation for a launch of n panels (of up to 64
// columns).  Every wavefront repeats the pivot search, the update of a step is split among them:
// with few panels the step's latency decides (eight), with many the issue of all wavefronts'
// instructions does, since four blocks of a 64-row LDS block fill a compute unit (four from 512
// panels on).  Narrow panels (a 32-row block, 18 blocks per compute unit) do best with one
// wavefront once a step has kNarrowSpread of them.  Measured on the 256-membrane union and the
// 100 x 25 x 25 cantilever; the factor is the same bits whatever the count.
constexpr int64_t kNarrowSpread = 1024;
constexpr int64_t kMediumSpread = 512;
int panel_waves_for(int64_t n) { return n >= 512 ? 4 : 8; }

template <typename T>
sgn_status factor_system(sgn_ctx c, int si, double piv_tol) {
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  DevSys& D = c->sys[si];
  hipStream_t st = c->stream;
  T* front = reinterpret_cast<T*>(D.front);
  HIPCHK(ensure_side(c));
  launch_row_scaling(D.row_lanes, S.N, D.frowptr, D.fslot, D.vals, D.scale, st);
  FrontArgs f;
  f.sn_begin = D.sn_begin;
  f.sn_m = D.sn_m;
  f.sn_front_off = D.sn_front_off;
  f.sn_rows_ptr = D.sn_rows_ptr;
  f.sn_rows = D.sn_rows;
  f.relmap_off = D.relmap_off;
  f.relmap = D.relmap;
  f.var_group_end = D.var_group_end;
  f.dpiv = D.dpiv;
  f.epiv = D.epiv;
  f.pivtype = D.pivtype;
  f.lperm = D.lperm;
  f.counters = c->d_cnt;
  f.piv_tol = piv_tol;
  launch_zero_fronts<T>((int64_t)S.fill_tasks.size() / 2, D.fill_tasks, f, front, st);
  launch_csr_to_fronts<T>((int64_t)S.colind.size(), D.slot_row, D.colind, D.csr_front_pos, D.vals, D.scale, front,
                          st);
  launch_fill_i32(4, 0, c->d_cnt, st);
  const bool prof = c->opt.profile != 0 && si == 0;
  size_t nev = 0;
  double upd_flops = 0.0;
  if (prof) {
    size_t need = 0;
    for (const LevelPlan& P : S.levels)
      for (const PanelStep& ps : P.steps)
        need += 2 * ((ps.upd_tiles > 0) + (ps.outer_tiles > 0) + (ps.far_tiles > 0));
    HIPCHK(ensure_events(c, need));
  }
  auto timed_update = [&](int64_t ntask, int64_t ntiles, const int64_t* tasks, const int32_t* tile_task,
                          double flops, hipStream_t ls) -> hipError_t {
    if (ntask <= 0 || ntiles <= 0) return hipSuccess;
    if (prof) {  // events on the stream the launch goes to
      hipError_t e = hipEventRecord(c->ev_pool[nev], ls);
      if (e != hipSuccess) return e;
    }
    launch_update<T>(ntask, ntiles, tasks, tile_task, f, front, ls);
    if (prof) {
      hipError_t e = hipEventRecord(c->ev_pool[nev + 1], ls);
      if (e != hipSuccess) return e;
      nev += 2;
      upd_flops += flops;
    }
    return hipSuccess;
  };
  for (int L = 0; L < S.nlevels; ++L) {
    const LevelPlan& P = S.levels[L];
    for (size_t r = 0; r < P.ea_work.size(); ++r) {
      launch_extend_add_small<T>(P.ea_kids[r], D.ea_kids + P.ea_kid_begin[r] * 5, f, front, st);
      launch_extend_add<T>(P.ea_work[r], D.ea_cols + P.ea_col_begin[r] * 4, f, front, st);
    }
    // Look-ahead: the delayed update of a block's columns beyond the next block runs on the second
    // stream, beside the next block's panels (which touch only the next block's columns and its W
    // rows).  The main stream waits for it before the next delayed update of the next block's
    // columns (both write the columns after it) and before the next level.
    bool side_busy = false;
    for (const PanelStep& ps : P.steps) {
      const int64_t nt = ps.task_end - ps.task_begin;
      // Width classes (narrow, medium, wide; listed in that order) get launches of their own only
      // when there are enough of them for the smaller block to pay (narrow: one wavefront and a
      // 32-row block; medium: four wavefronts and a 48-row block, eight blocks per compute unit);
      // the rest of the step goes in one launch (another launch on this chain costs more than it
      // saves).
      const int pw = c->A.tune.panel_waves;
      int64_t b = ps.task_begin;
      if (pw == 1 || (pw == 0 && ps.narrow_end - b >= kNarrowSpread)) {
        launch_panel_diag<T>(ps.narrow_end - b, kNarrowPanel, 1, D.panel_tasks + b * 3, f, front, st);
        b = ps.narrow_end;
      }
      if (pw == 4 || (pw == 0 && ps.medium_end - std::max(b, ps.narrow_end) >= kMediumSpread)) {
        // narrow panels not launched above join the medium ones (a 48-row block holds them)
        launch_panel_diag<T>(ps.medium_end - b, kMediumPanel, 4, D.panel_tasks + b * 3, f, front, st);
        b = ps.medium_end;
      }
      launch_panel_diag<T>(ps.task_end - b, kPanel, pw != 0 ? pw : panel_waves_for(ps.task_end - b),
                           D.panel_tasks + b * 3, f, front, st);
      launch_panel_trsm<T>(nt, ps.trsm_rows, D.panel_tasks + ps.task_begin * 3, f, front, st);
      HIPCHK(timed_update(ps.upd_end - ps.upd_begin, ps.upd_tiles, D.upd_tasks + ps.upd_begin * 6,
                          D.upd_tile_task + ps.upd_map, ps.upd_flops, st));
      if (ps.outer_tiles > 0 && side_busy) {
        HIPCHK(hipStreamWaitEvent(st, c->ev_join, 0));
        side_busy = false;
      }
      HIPCHK(timed_update(ps.outer_end - ps.outer_begin, ps.outer_tiles, D.upd_tasks + ps.outer_begin * 6,
                          D.upd_tile_task + ps.outer_map, ps.outer_flops, st));
      if (ps.far_tiles > 0) {  // after everything the main stream has so far; after earlier far updates
        HIPCHK(hipEventRecord(c->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
        HIPCHK(timed_update(ps.far_end - ps.far_begin, ps.far_tiles, D.upd_tasks + ps.far_begin * 6,
                            D.upd_tile_task + ps.far_map, ps.far_flops, c->side));
        HIPCHK(hipEventRecord(c->ev_join, c->side));
        side_busy = true;
      }
    }
    if (side_busy) HIPCHK(hipStreamWaitEvent(st, c->ev_join, 0));
  }
  HIPCHK(hipGetLastError());
  if (prof) {
    c->prof_nev = nev;
    c->prof_flops = upd_flops;
    if (!c->capturing) TRY(read_update_events(c));  // captured events are read after each replay
  }
  launch_fill_i32(8, 0, c->d_ull, st);
  launch_inertia(S.N, D.dpiv, D.epiv, D.pivtype, c->d_ull, c->d_part, st);
  HIPCHK(hipGetLastError());
  D.factored = true;
  D.current = true;
  return SGN_OK;
}

sgn_status factor_dispatch(sgn_ctx c, int si, double piv_tol, sgn_factor_info* info) {
  const double t0 = now_ms();
  DevSys& D = c->sys[si];
  HIPCHK(ensure_events(c, 0));
  if (si == 0) HIPCHK(hipEventRecord(c->ev_a, c->stream));
  if (D.prec) TRY(factor_system<float>(c, si, piv_tol));
  else TRY(factor_system<double>(c, si, piv_tol));
  if (si == 0) {
    HIPCHK(hipEventRecord(c->ev_b, c->stream));
    HIPCHK(hipEventSynchronize(c->ev_b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
    c->stats.factor_ms = ms;
    c->stats.factor_flops = c->A.sgn.flops;
  }
  unsigned long long cnt[3] = {0, 0, 0};
  int pert = 0;
  std::vector<double> part(kRedBlocks);
  HIPCHK(hipMemcpyAsync(cnt, c->d_ull, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(&pert, c->d_cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(part.data(), c->d_part, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double mn = INFINITY;
  for (double v : part) mn = std::min(mn, v);
  D.inertia[0] = (int64_t)cnt[0];
  D.inertia[1] = (int64_t)cnt[1];
  D.inertia[2] = (int64_t)cnt[2];
  if (info) {
    const System& S = si == 0 ? c->A.sgn : c->A.kx;
    info->n_pos = (int64_t)cnt[0];
    info->n_neg = (int64_t)cnt[1];
    info->n_zero = (int64_t)cnt[2];
    info->n_perturbed = pert;
    info->min_abs_pivot = mn;
    info->flops = S.flops;
    info->ms = now_ms() - t0;
  }
  return SGN_OK;
}

SolveArgs solve_args(sgn_ctx c, int si) {
  DevSys& D = c->sys[si];
  SolveArgs a;
  a.f.sn_begin = D.sn_begin;
  a.f.sn_m = D.sn_m;
  a.f.sn_front_off = D.sn_front_off;
  a.f.sn_rows_ptr = D.sn_rows_ptr;
  a.f.sn_rows = D.sn_rows;
  a.f.relmap_off = D.relmap_off;
  a.f.relmap = D.relmap;
  a.f.var_group_end = D.var_group_end;
  a.f.dpiv = D.dpiv;
  a.f.epiv = D.epiv;
  a.f.pivtype = D.pivtype;
  a.f.lperm = D.lperm;
  a.f.counters = c->d_cnt;
  a.f.piv_tol = 0;
  a.child_ptr = D.child_ptr;
  a.child_list = D.child_list;
  a.sn_vec_off = D.sn_vec_off;
  a.panel_ptr = D.panel_ptr;
  a.panel_col = D.panel_col;
  a.tv = D.tv;
  a.tp = D.tp;
  a.sn_part_off = D.sn_part_off;
  a.part = D.part;
  a.wd = nullptr;
  return a;
}

// forward sweep y = L^-1 P b (b in the system's new, scaled order); y is left in the
// per-front vectors tp (pivot order)
template <typename T>
sgn_status fwd_sweep_t(sgn_ctx c, int si, const double* b_new) {
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  DevSys& D = c->sys[si];
  hipStream_t st = c->stream;
  const SolveArgs a = solve_args(c, si);
  const T* front = reinterpret_cast<const T*>(D.front);
  launch_fill_i32(2 * (int64_t)S.nsn, 0, D.solve_ctr, st);
  int* err = c->d_cnt + 12;
  for (int L = 0; L < S.nlevels; ++L) {
    const LevelPlan& P = S.levels[L];
    launch_fwd_level<T>(P.one_begin - P.sn_begin, P.solve_max_u, P.solve_max_s, D.solve_sn + P.sn_begin,
                        D.solve_fwd_tasks + 2 * P.fwd_begin, P.fwd_end - P.fwd_begin, a, front, b_new, D.solve_ctr,
                        err, st);
    launch_fwd_one<T>(P.sn_end - P.one_begin, D.solve_sn + P.one_begin, a, front, b_new, st);
  }
  HIPCHK(hipGetLastError());
  return SGN_OK;
}

// backward sweep x = P^T L^-T w, with w = D^-1 y from tp (wd null) or given in pivot order
template <typename T>
sgn_status bwd_sweep_t(sgn_ctx c, int si, double* x_new, const double* wd) {
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  DevSys& D = c->sys[si];
  hipStream_t st = c->stream;
  SolveArgs a = solve_args(c, si);
  a.wd = wd;
  const T* front = reinterpret_cast<const T*>(D.front);
  launch_fill_i32(2 * (int64_t)S.nsn, 0, D.solve_ctr, st);  // tickets start at 0
  int* err = c->d_cnt + 12;
  for (int L = S.nlevels - 1; L >= 0; --L) {
    const LevelPlan& P = S.levels[L];
    launch_bwd_one<T>(P.sn_end - P.one_begin, D.solve_sn + P.one_begin, a, front, x_new, st);
    launch_bwd_level<T>(P.one_begin - P.sn_begin, P.solve_max_s, D.solve_sn + P.sn_begin,
                        D.solve_bwd_tasks + 2 * P.bwd_begin, P.bwd_end - P.bwd_begin, a, front, x_new,
                        D.solve_ctr + S.nsn, err, st);
  }
  HIPCHK(hipGetLastError());
  return SGN_OK;
}

sgn_status fwd_sweep(sgn_ctx c, int si, const double* b_new) {
  return c->sys[si].prec ? fwd_sweep_t<float>(c, si, b_new) : fwd_sweep_t<double>(c, si, b_new);
}
sgn_status bwd_sweep(sgn_ctx c, int si, double* x_new, const double* wd) {
  return c->sys[si].prec ? bwd_sweep_t<float>(c, si, x_new, wd) : bwd_sweep_t<double>(c, si, x_new, wd);
}

void scale_vec(sgn_ctx c, int64_t n, const double* s, const double* in, double* out);

// x_new = K^-1 b_new with the current factor (x_new may alias b_new; uses D.sv)
sgn_status solve_once(sgn_ctx c, int si, const double* b_new, double* x_new) {
  DevSys& D = c->sys[si];
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  scale_vec(c, S.N, D.scale, b_new, D.sv);
  TRY(fwd_sweep(c, si, D.sv));
  TRY(bwd_sweep(c, si, x_new, nullptr));
  scale_vec(c, S.N, D.scale, x_new, x_new);
  return SGN_OK;
}

PcArgs pc_args(sgn_ctx c) {
  DevSys& D = c->sys[0];
  PcArgs a;
  a.ngroups = D.ngroups;
  a.dim = c->A.mesh.dim;
  a.nx = c->A.mesh.n_x;
  a.grp_ptr = D.grp_ptr;
  a.grp_node = D.grp_node;
  a.grp_vec = D.grp_vec;
  a.perm = D.perm;
  a.dpiv = D.dpiv;
  a.epiv = D.epiv;
  a.pivtype = D.pivtype;
  a.corr_node = c->use_own ? c->own_cn : c->corr_node;
  a.corr_par = c->use_own ? c->own_cp : c->corr_par;
  return a;
}

// out_new = M^-1 in_new with the node-block preconditioner of the reference factor (new order;
// out_new may alias in_new); ysave: optional flat copy of the forward result (pivot order)
sgn_status pc_apply_new(sgn_ctx c, const double* in_new, double* out_new, double* ysave) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  if (c->opt.pc_kind == SGN_PC_BLOCK) {
    launch_blockpc_apply(D.ngroups, D.grp_ptr, D.cur_scale, D.bp_off, D.bp_minv, in_new, out_new, c->stream);
    return SGN_OK;
  }
  scale_vec(c, N, D.scale, in_new, D.sv);
  TRY(fwd_sweep(c, 0, D.sv));
  launch_pc_block(pc_args(c), D.tp, ysave, D.pc_w, c->stream);
  TRY(bwd_sweep(c, 0, out_new, D.pc_w));
  scale_vec(c, N, D.scale, out_new, out_new);
  return SGN_OK;
}

// flat forward result y = L^-1 P S in (pivot order) of the reference factor
sgn_status pc_forward_new(sgn_ctx c, const double* in_new, double* y) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  scale_vec(c, N, D.scale, in_new, D.sv);
  TRY(fwd_sweep(c, 0, D.sv));
  launch_pc_block(pc_args(c), D.tp, y, D.pc_w, c->stream);  // saves y; the block result is not used
  return SGN_OK;
}

void scale_vec(sgn_ctx c, int64_t n, const double* s, const double* in, double* out) {
  launch_scale(n, s, in, out, c->stream);
}

// One cycle of restarted flexible GMRES (Saad's FGMRES(m)) in FP64 on the equilibrated system
// (S K S) u = S b with z = S u, right-preconditioned by the stored factor (the forward and backward
// sweeps approximate (S K S)^-1), starting from z_new whose equilibrated residual is rs = S (b - K z)
// with norm beta.  The Arnoldi vectors are orthogonalised by two passes of classical Gram-Schmidt
// (dot products on the device, one read-back per step); the least-squares problem is reduced by
// Givens rotations on the host.  Stops when the residual estimate falls to `stop` or after m steps;
// z_new += S sum_i y_i Z_i.
sgn_status fgmres_cycle(sgn_ctx c, int si, double* z_new, const double* rs, double beta, double stop, int* iters) {
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  DevSys& D = c->sys[si];
  const int64_t N = S.N;
  const int m = kGmresM;
  hipStream_t st = c->stream;
  double* V = D.gm_V;
  double* Z = D.gm_Z;
  launch_axpby(N, 1.0 / beta, rs, 0.0, nullptr, V, st);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
  auto h = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
  g[0] = beta;
  int k = 0;  // basis vectors used
  std::vector<double> hb(2 * 64 + 1);
  while (k < m) {
    const int j = k;
    double* vj = V + (int64_t)j * N;
    double* zj = Z + (int64_t)j * N;
    double* vn = V + (int64_t)(j + 1) * N;
    TRY(fwd_sweep(c, si, vj));
    TRY(bwd_sweep(c, si, zj, nullptr));
    scale_vec(c, N, D.scale, zj, D.sv);
    launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, D.sv, vn, st);
    scale_vec(c, N, D.scale, vn, vn);
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i <= j; ++i) dev_dot_to(c, N, V + (int64_t)i * N, vn, c->d_gm + 64 * pass + i);
      launch_multi_axpy(N, j + 1, V, N, c->d_gm + 64 * pass, -1.0, vn, st);
    }
    dev_dot_to(c, N, vn, vn, c->d_gm + 128);
    HIPCHK(hipMemcpyAsync(hb.data(), c->d_gm, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i <= j; ++i) h(i, j) = hb[i] + hb[64 + i];
    const double hn = std::sqrt(std::max(hb[128], 0.0));
    h(j + 1, j) = hn;
    for (int i = 0; i < j; ++i) {
      const double a = h(i, j), b = h(i + 1, j);
      h(i, j) = cs[i] * a + sn[i] * b;
      h(i + 1, j) = -sn[i] * a + cs[i] * b;
    }
    const double den = std::hypot(h(j, j), h(j + 1, j));
    if (!(den > 0.0)) break;  // the preconditioned operator is singular on this space
    cs[j] = h(j, j) / den;
    sn[j] = h(j + 1, j) / den;
    h(j, j) = den;
    h(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    k = j + 1;
    ++*iters;
    if (std::fabs(g[j + 1]) <= stop || !(hn > 0.0)) break;
    launch_axpby(N, 1.0 / hn, vn, 0.0, nullptr, vn, st);
  }
  if (k == 0) return SGN_OK;
  c->gm_host.assign(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {  // back substitution with the rotated Hessenberg matrix
    double t = g[i];
    for (int l = i + 1; l < k; ++l) t -= h(i, l) * c->gm_host[l];
    c->gm_host[i] = t / h(i, i);
  }
  HIPCHK(hipMemcpyAsync(c->d_gm + 192, c->gm_host.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
  launch_fill(N, 0.0, D.gm_t, st);
  launch_multi_axpy(N, k, Z, N, c->d_gm + 192, 1.0, D.gm_t, st);
  scale_vec(c, N, D.scale, D.gm_t, D.gm_t);
  launch_axpby(N, 1.0, z_new, 1.0, D.gm_t, z_new, st);
  HIPCHK(hipStreamSynchronize(st));  // gm_host is read by the copy
  return SGN_OK;
}

// Refined solve in new order: K z = b (unscaled), FP64 residuals on the assembled
// matrix.  b_new and z_new are caller buffers (distinct from the internal ones).
// Refinement sweeps continue while each one at least halves the equilibrated residual;
// otherwise (or after max_ir sweeps) FGMRES cycles take over from the current iterate.
sgn_status refined_solve(sgn_ctx c, int si, const double* b_new, double* z_new, sgn_solve_info* info) {
  const System& S = si == 0 ? c->A.sgn : c->A.kx;
  DevSys& D = c->sys[si];
  const double t0 = now_ms();
  launch_fill_i32(1, 0, c->d_cnt + 12, c->stream);
  TRY(solve_once(c, si, b_new, z_new));
  scale_vec(c, S.N, D.scale, b_new, D.ir_s);
  dev_dot(c, S.N, D.ir_s, D.ir_s, 1);
  dev_dot(c, S.N, b_new, b_new, 2);
  double bn[2];
  TRY(read_scalars(c, 1, 2, bn));
  const double sb = std::sqrt(bn[0]), rb = std::sqrt(bn[1]);
  int sweeps = 0, gm_iters = 0, cycles = 0;
  double rel = 0, raw = 0, prev = INFINITY, gprev = INFINITY;
  bool krylov = false;
  const int max_ir = std::max(0, c->opt.max_ir);
  // the Newton solves with Kx need no 1e-10 accuracy (a stalled refinement is accepted there), so the
  // Krylov escalation serves the saddle-point system only
  const int max_gmres = si == 0 ? c->opt.max_gmres : 0;
  for (;;) {
    launch_residual(D.row_lanes, S.N, D.frowptr, D.fcol, D.fslot, D.vals, z_new, b_new, D.ir_r, c->stream);
    scale_vec(c, S.N, D.scale, D.ir_r, D.ir_s);
    dev_dot(c, S.N, D.ir_s, D.ir_s, 1);
    dev_dot(c, S.N, D.ir_r, D.ir_r, 2);
    double rn[2];
    TRY(read_scalars(c, 1, 2, rn));
    rel = sb > 0 ? std::sqrt(rn[0]) / sb : 0.0;
    raw = rb > 0 ? std::sqrt(rn[1]) / rb : 0.0;
    if (rel <= c->opt.solve_rtol) break;
    if (!krylov) {
      const bool slow = sweeps > 0 && !(rel <= 0.5 * prev);
      if ((slow || sweeps >= max_ir) && max_gmres > 0) {
        krylov = true;
      } else {
        if (sweeps >= max_ir || !(rel < prev)) break;
        prev = rel;
        TRY(solve_once(c, si, D.ir_r, D.ir_d));
        launch_axpby(S.N, 1.0, z_new, 1.0, D.ir_d, z_new, c->stream);
        ++sweeps;
        continue;
      }
    }
    if (cycles >= max_gmres || !(rel < gprev)) break;
    gprev = rel;
    TRY(fgmres_cycle(c, si, z_new, D.ir_s, rel * sb, 0.5 * c->opt.solve_rtol * sb, &gm_iters));
    ++cycles;
  }
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (timeout) {
    c->err = "a pipelined triangular solve timed out waiting for a panel";
    return SGN_E_HIP;
  }
  if (info) {
    info->sweeps = sweeps;
    info->fallback = 0;
    info->rel_res = rel;
    info->raw_rel_res = raw;
    info->ms = now_ms() - t0;
    info->gmres_iters = gm_iters;
  }
  if (!(rel <= c->opt.solve_rtol)) {
    char buf[96];
    snprintf(buf, sizeof(buf), "refinement stopped at equilibrated relative residual %.3e", rel);
    c->err = buf;
    return SGN_E_REFINE;
  }
  return SGN_OK;
}

// BiCGSTAB (van der Vorst 1992) on the saddle-point system K z = b, right-preconditioned by the
// stored factor, which is the LDL^T of the stabilised matrix K_eps = K + diag(eps_x 1, 0, -eps_lambda 1)
// (Sec. 5, "Solving the saddle point problem"; the assembled values hold K_eps, and products with K
// subtract the stabilisation diagonal again).  It runs on the equilibrated system (S K S) u = S b,
// z = S u, where the factor's sweeps without their scaling are the preconditioner (S K_eps S)^-1, so
// the recursive residual is the equilibrated residual the tolerance is stated in.  Restarts from
// the true residual whenever the recursion claims convergence that the true residual does not
// confirm, or when the recurrence breaks down.  b_new, z_new as for refined_solve.
sgn_status bicgstab_solve(sgn_ctx c, const double* b_new, double* z_new, sgn_solve_info* info) {
  const System& S = c->A.sgn;
  DevSys& D = c->sys[0];
  const int64_t N = S.N;
  hipStream_t st = c->stream;
  const double t0 = now_ms();
  const double ex = c->opt.eps_x, el = c->opt.eps_lambda;
  double* r = D.gm_V;  // work vectors: the FGMRES bases are not in use during this solve
  double* rt = r + N;
  double* p = rt + N;
  double* v = p + N;
  double* sv = v + N;
  double* t = sv + N;
  double* y = t + N;
  double* zh = y + N;
  double* u = zh + N;
  double* tmp = u + N;
  // out = S K S w (K unstabilised)
  auto matvec = [&](const double* w, double* out) {
    scale_vec(c, N, D.scale, w, tmp);
    launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, tmp, out, st);
    if (ex != 0.0 || el != 0.0) launch_unstabilise(N, D.diag_kind, ex, el, -1.0, tmp, out, st);
    scale_vec(c, N, D.scale, out, out);
  };
  // out = (S K_eps S)^-1 w by the factor's sweeps
  auto precond = [&](const double* w, double* out) -> sgn_status {
    TRY(fwd_sweep(c, 0, w));
    return bwd_sweep(c, 0, out, nullptr);
  };
  // true equilibrated residual r = S b - S K S u, its squared norm into slot 40
  auto true_residual = [&]() {
    matvec(u, r);
    scale_vec(c, N, D.scale, b_new, tmp);
    launch_axpby(N, 1.0, tmp, -1.0, r, r, st);
    dev_dot(c, N, r, r, 40);
  };
  launch_fill_i32(1, 0, c->d_cnt + 12, st);
  launch_fill(N, 0.0, u, st);
  scale_vec(c, N, D.scale, b_new, tmp);
  dev_dot(c, N, tmp, tmp, 41);
  dev_dot(c, N, b_new, b_new, 42);
  double hb[2];
  TRY(read_scalars(c, 41, 2, hb));
  const double sb = std::sqrt(hb[0]), rb = std::sqrt(hb[1]);
  const double tol = c->opt.solve_rtol * sb;
  const int max_it = std::max(1, c->opt.max_bicgstab);
  int it = 0;
  double rel = 1.0;
  HIPCHK(hipMemcpyAsync(r, tmp, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  double rn = sb;
  while (sb > 0.0 && it < max_it) {
    // (re)start from the current residual r
    HIPCHK(hipMemcpyAsync(rt, r, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_fill(N, 0.0, p, st);
    launch_fill(N, 0.0, v, st);
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    bool claimed = false;
    while (it < max_it) {
      dev_dot(c, N, rt, r, 43);
      double rho;
      TRY(read_scalars(c, 43, 1, &rho));
      if (!(std::fabs(rho) > 0.0)) break;  // breakdown: restart from the true residual
      const double beta = (rho / rho_prev) * (alpha / omega);
      launch_axpby(N, 1.0, p, -omega, v, p, st);  // p = r + beta (p - omega v)
      launch_axpby(N, 1.0, r, beta, p, p, st);
      TRY(precond(p, y));
      matvec(y, v);
      dev_dot(c, N, rt, v, 44);
      double rv;
      TRY(read_scalars(c, 44, 1, &rv));
      ++it;
      if (!(std::fabs(rv) > 0.0)) break;
      alpha = rho / rv;
      launch_axpby(N, 1.0, r, -alpha, v, sv, st);  // s = r - alpha v
      dev_dot(c, N, sv, sv, 45);
      double ss;
      TRY(read_scalars(c, 45, 1, &ss));
      if (std::sqrt(std::max(ss, 0.0)) <= tol) {
        launch_axpby(N, 1.0, u, alpha, y, u, st);
        claimed = true;
        break;
      }
      TRY(precond(sv, zh));
      matvec(zh, t);
      dev_dot(c, N, t, sv, 46);
      dev_dot(c, N, t, t, 47);
      double ts[2];
      TRY(read_scalars(c, 46, 2, ts));
      if (!(ts[1] > 0.0)) break;
      omega = ts[0] / ts[1];
      launch_axpby(N, 1.0, u, alpha, y, u, st);  // u += alpha y + omega zh
      launch_axpby(N, 1.0, u, omega, zh, u, st);
      launch_axpby(N, 1.0, sv, -omega, t, r, st);  // r = s - omega t
      dev_dot(c, N, r, r, 45);
      double r2;
      TRY(read_scalars(c, 45, 1, &r2));
      rn = std::sqrt(std::max(r2, 0.0));
      if (rn <= tol) {
        claimed = true;
        break;
      }
      if (!(omega != 0.0)) break;
      rho_prev = rho;
    }
    true_residual();
    double r2;
    TRY(read_scalars(c, 40, 1, &r2));
    rn = std::sqrt(std::max(r2, 0.0));
    rel = rn / sb;
    if (rn <= tol) break;
    (void)claimed;  // not confirmed by the true residual: restart from it
  }
  if (sb == 0.0) rel = 0.0;
  scale_vec(c, N, D.scale, u, z_new);
  // raw residual |b - K z| / |b| for the report
  launch_residual(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, z_new, b_new, D.ir_r, st);
  if (ex != 0.0 || el != 0.0) launch_unstabilise(N, D.diag_kind, ex, el, 1.0, z_new, D.ir_r, st);
  dev_dot(c, N, D.ir_r, D.ir_r, 41);
  double raw2;
  TRY(read_scalars(c, 41, 1, &raw2));
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (timeout) {
    c->err = "a pipelined triangular solve timed out waiting for a panel";
    return SGN_E_HIP;
  }
  if (info) {
    info->sweeps = it;
    info->fallback = 0;
    info->rel_res = rel;
    info->raw_rel_res = rb > 0 ? std::sqrt(std::max(raw2, 0.0)) / rb : 0.0;
    info->ms = now_ms() - t0;
    info->gmres_iters = 0;
  }
  if (!(rel <= c->opt.solve_rtol)) {
    char buf[96];
    snprintf(buf, sizeof(buf), "BiCGSTAB stopped at equilibrated relative residual %.3e", rel);
    c->err = buf;
    return SGN_E_REFINE;
  }
  return SGN_OK;
}

// Preconditioned MINRES on the assembled SGN matrix (new order, unscaled), with the
// node-block preconditioner of the reference factor.  The iterate minimises the
// M^-1-norm of the residual over the Krylov space (Lanczos three-term recurrence with
// M-inner products, QR of the tridiagonal by Givens rotations, three-term update of
// the search directions).  Convergence is judged on the true residual with the same
// equilibrated measure as the direct solve, with the row scaling of the current
// matrix.  Returns SGN_OK with *converged false when it hits max_iter or stagnates
// (less than a tenfold reduction over `window` iterations).
sgn_status minres_new(sgn_ctx c, const double* b, double* x, int max_iter, int window, int* iters, double* rel_out,
                      bool* converged) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  hipStream_t st = c->stream;
  double *v_prev = D.mr[0], *v = D.mr[1], *v_next = D.mr[2], *z = D.mr[3], *z_next = D.mr[4];
  double *w_prev = D.mr[5], *w = D.mr[6], *w_next = D.mr[7], *q = D.mr[8], *r = D.mr[9];
  *converged = false;
  *iters = 0;
  launch_row_scaling(D.row_lanes, N, D.frowptr, D.fslot, D.vals, D.cur_scale, st);
  launch_fill(N, 0.0, x, st);
  launch_fill(N, 0.0, v_prev, st);
  launch_fill(N, 0.0, w_prev, st);
  launch_fill(N, 0.0, w, st);
  HIPCHK(hipMemcpyAsync(v, b, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  scale_vec(c, N, D.cur_scale, b, r);
  dev_dot(c, N, r, r, 20);
  TRY(pc_apply_new(c, v, z, nullptr));
  dev_dot(c, N, v, z, 21);
  double h[2];
  TRY(read_scalars(c, 20, 2, h));
  const double sb = std::sqrt(h[0]);
  if (sb == 0.0) {
    *converged = true;
    *rel_out = 0.0;
    return SGN_OK;
  }
  if (!(h[1] > 0.0)) {
    *rel_out = 1.0;
    return SGN_OK;  // preconditioner not positive on b: let the caller fall back
  }
  double gam = std::sqrt(h[1]), gam_prev = 1.0, eta = gam;
  double c_prev = 1.0, cc = 1.0, s_prev = 0.0, ss = 0.0;
  std::vector<double> hist;
  double rel = 1.0;
  for (int j = 1; j <= max_iter; ++j) {
    launch_lincomb3(N, 1.0 / gam, z, 0.0, nullptr, 0.0, nullptr, z, st);  // z_j normalised
    launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, z, q, st);
    dev_dot(c, N, q, z, 20);
    double dl;
    TRY(read_scalars(c, 20, 1, &dl));
    launch_lincomb3(N, 1.0, q, -dl / gam, v, -gam / gam_prev, v_prev, v_next, st);
    TRY(pc_apply_new(c, v_next, z_next, nullptr));
    dev_dot(c, N, v_next, z_next, 21);
    double g2;
    TRY(read_scalars(c, 21, 1, &g2));
    if (g2 < 0.0) break;  // the preconditioner lost definiteness in rounding
    const double gam_next = std::sqrt(g2);
    const double a0 = cc * dl - c_prev * ss * gam;
    const double a1 = std::sqrt(a0 * a0 + gam_next * gam_next);
    const double a2 = ss * dl + c_prev * cc * gam;
    const double a3 = s_prev * gam;
    if (a1 == 0.0) break;
    const double c_next = a0 / a1, s_next = gam_next / a1;
    launch_lincomb3(N, 1.0 / a1, z, -a3 / a1, w_prev, -a2 / a1, w, w_next, st);
    launch_axpby(N, 1.0, x, c_next * eta, w_next, x, st);
    eta = -s_next * eta;
    // true equilibrated residual of the iterate
    launch_residual(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, x, b, r, st);
    scale_vec(c, N, D.cur_scale, r, r);
    dev_dot(c, N, r, r, 22);
    double rn;
    TRY(read_scalars(c, 22, 1, &rn));
    rel = std::sqrt(rn) / sb;
    hist.push_back(rel);
    *iters = j;
    if (verbose()) fprintf(stderr, "[sgn] minres %d: rel %.3e |eta| %.3e\n", j, rel, std::fabs(eta));
    if (rel <= c->opt.solve_rtol) {
      *converged = true;
      break;
    }
    if (j > window && rel > 0.1 * hist[j - 1 - window]) break;  // stagnation
    if (gam_next == 0.0) break;  // invariant subspace: the iterate is exact in it
    // rotate
    std::swap(v_prev, v);
    std::swap(v, v_next);
    std::swap(z, z_next);
    std::swap(w_prev, w);
    std::swap(w, w_next);
    gam_prev = gam;
    gam = gam_next;
    c_prev = cc;
    cc = c_next;
    s_prev = ss;
    ss = s_next;
  }
  *rel_out = rel;
  return SGN_OK;
}

// ------------------------------------------------------------------ equilibrium
sgn_status potential(sgn_ctx c, const double* x, const double* p, double* pi, double* scale, bool* inverted) {
  int inv = 0;
  TRY(run_element(c, x, p, 0, &inv));
  *inverted = inv > 0;
  if (inv) {
    *pi = INFINITY;
    return SGN_OK;
  }
  const Analysis& A = c->A;
  // element energies: value off_energy of every element, dim apart in the grouped buffer
  const int g = A.mesh.dim;
  const double* energy = c->d_ebuf + ebuf_index(A.off_energy, 0, A.mesh.n_elems, g);
  dev_dot(c, A.mesh.n_elems, energy, nullptr, 4, g, 0);
  dev_dot(c, A.mesh.n_elems, energy, nullptr, 5, g, 1);
  dev_dot(c, A.mesh.n_x, c->d_fext, x, 6);
  int ns = 3;
  if (A.mesh.param_kind == 2) {
    dev_dot(c, A.mesh.n_x, p, x, 7);
    ns = 4;
  }
  double v[4] = {0, 0, 0, 0};
  TRY(read_scalars(c, 4, ns, v));
  const double fx = v[2] + v[3];
  *pi = v[0] - fx;
  *scale = v[1] + std::fabs(fx);
  return SGN_OK;
}

// Newton with backtracking; on success the Kx factor is valid at the returned x.
sgn_status equilibrium_impl(sgn_ctx c, const double* p, double* x, sgn_eq_info* info) {
  const Analysis& A = c->A;
  const int64_t nx = A.mesh.n_x;
  const double tol = c->opt.newton_rtol * c->fext_norm + c->opt.newton_atol;
  int halvings = 0;
  double prev_rn = INFINITY;
  c->kx_valid = false;
  for (int it = 0; it <= c->opt.max_newton; ++it) {
    int inv = 0;
    TRY(run_element(c, x, p, 2, &inv));
    if (inv) {
      c->err = "inverted element at the Newton iterate";
      return SGN_E_INVERTED;
    }
    residual_vec(c, p, c->d_c);
    dev_dot(c, nx, c->d_c, c->d_c, 3);
    double rn2;
    TRY(read_scalars(c, 3, 1, &rn2));
    const double rn = std::sqrt(rn2);
    if (verbose()) fprintf(stderr, "[sgn] newton %d |c| = %.3e (rel %.3e)\n", it, rn, rn / c->fext_norm);
    // factorise Kx at this iterate (also needed at convergence for the adjoint)
    double tau = 0.0;
    double dmax = 0.0;
    for (int attempt = 0;; ++attempt) {
      assemble_kx(c, tau);
      TRY(factor_dispatch(c, 1, 1e-300, nullptr));
      if (c->sys[1].inertia[0] == nx) break;
      if (attempt >= 20) {
        c->err = "Kx stayed indefinite after diagonal shifts";
        return SGN_E_NEWTON;
      }
      if (tau == 0.0) {
        launch_max_abs_partials((int64_t)A.kx.colind.size(), c->sys[1].vals, c->d_part, c->stream);
        launch_final_max(c->d_part, kRedBlocks, c->d_scal + 8, c->stream);
        TRY(read_scalars(c, 8, 1, &dmax));
        tau = 1e-8 * dmax;
      } else {
        tau *= 10.0;
      }
    }
    // converged: below tolerance, or stalled at the rounding floor of the residual
    // (|c| no longer halves once it is below 1e-7 |f_ext|)
    const bool stalled = it > 0 && rn <= 1e-7 * c->fext_norm && rn > 0.5 * prev_rn;
    prev_rn = rn;
    if (rn <= tol || stalled) {
      c->kx_valid = (tau == 0.0);
      if (info) {
        info->iters = it;
        info->halvings = halvings;
        info->res_norm = rn;
        info->f_ext_norm = c->fext_norm;
        info->converged = 1;
      }
      return SGN_OK;
    }
    if (it == c->opt.max_newton) break;
    // dx = -Kx^-1 c, in the Kx ordering
    DevSys& D = c->sys[1];
    launch_gather_perm(nx, D.perm, nullptr, c->d_c, D.b, c->stream);
    launch_axpby(nx, -1.0, D.b, 0.0, nullptr, D.b, c->stream);
    sgn_solve_info si{};
    const double keep = c->opt.solve_rtol;
    c->opt.solve_rtol = 1e-14;
    sgn_status s = refined_solve(c, 1, D.b, D.z, &si);
    c->opt.solve_rtol = keep;
    if (s != SGN_OK && s != SGN_E_REFINE) return s;
    if (verbose())
      fprintf(stderr, "[sgn]   Kx inertia (%lld, %lld, %lld) tau %.2e, solve res %.2e after %d sweeps\n",
              (long long)c->sys[1].inertia[0], (long long)c->sys[1].inertia[1], (long long)c->sys[1].inertia[2],
              tau, si.rel_res, si.sweeps);
    launch_scatter_perm(nx, D.perm, nullptr, D.z, c->d_dx, c->stream);
    // backtracking on Pi
    double pi0, sc0;
    bool inv0;
    TRY(potential(c, x, p, &pi0, &sc0, &inv0));
    dev_dot(c, nx, c->d_c, c->d_dx, 9);
    double slope;
    TRY(read_scalars(c, 9, 1, &slope));
    double alpha = 1.0;
    bool ok = false;
    for (int h = 0; h <= c->opt.max_halvings + 10; ++h) {
      launch_axpby(nx, 1.0, x, alpha, c->d_dx, c->d_xt, c->stream);
      double pi1, sc1;
      bool inv1;
      TRY(potential(c, c->d_xt, p, &pi1, &sc1, &inv1));
      if (!inv1 && pi1 <= pi0 + 1e-4 * alpha * slope + 1e-12 * sc0) {
        ok = true;
        break;
      }
      alpha *= 0.5;
      ++halvings;
    }
    if (verbose()) fprintf(stderr, "[sgn]   alpha %.3e (Pi0 %.6e, slope %.3e)\n", alpha, pi0, slope);
    if (!ok) {
      c->err = "Newton line search failed";
      return SGN_E_NEWTON;
    }
    HIPCHK(hipMemcpyAsync(x, c->d_xt, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  if (info) {
    info->iters = c->opt.max_newton;
    info->halvings = halvings;
    info->res_norm = -1;
    info->f_ext_norm = c->fext_norm;
    info->converged = 0;
  }
  c->err = "Newton did not converge";
  return SGN_E_NEWTON;
}

// f(x, p) on device pointers (sync)
sgn_status objective_value(sgn_ctx c, const double* x, const double* p, double* f) {
  const Analysis& A = c->A;
  const int64_t nt = (int64_t)c->target_dof.size();
  launch_fill(A.mesh.n_x, 0.0, c->d_fx, c->stream);
  launch_objective_fx(nt, c->d_tdof, c->d_tval, x, 1.0, c->d_fx, c->stream);  // x_T - t
  dev_dot(c, A.mesh.n_x, c->d_fx, c->d_fx, 10);
  launch_axpby(A.mesh.n_p, 1.0, p, -1.0, c->d_pref, c->d_fp, c->stream);
  dev_dot(c, A.mesh.n_p, c->d_fp, c->d_fp, 11);
  double v[2];
  TRY(read_scalars(c, 10, 2, v));
  *f = 0.5 * c->target_w * v[0] / (c->ell * c->ell) + 0.5 * c->mu_reg * v[1];
  return SGN_OK;
}

// Assemble K_SGN at (x, p) and the rhs in boundary order into rhs_old (device).
// lam = -Kx^-1 df/dx^T (the adjoint multipliers, Appendix A) with the Kx factor of the last
// equilibrium; df/dx^T in c->d_fx on entry, lam in c->d_lam on exit
sgn_status adjoint_multipliers(sgn_ctx c) {
  const int64_t nx = c->A.mesh.n_x;
  DevSys& K = c->sys[1];
  launch_gather_perm(nx, K.perm, nullptr, c->d_fx, K.b, c->stream);
  launch_axpby(nx, -1.0, K.b, 0.0, nullptr, K.b, c->stream);
  const double keep = c->opt.solve_rtol;
  c->opt.solve_rtol = 1e-14;
  sgn_solve_info si{};
  sgn_status s = refined_solve(c, 1, K.b, K.z, &si);
  c->opt.solve_rtol = keep;
  if (s != SGN_OK && s != SGN_E_REFINE) return s;
  launch_scatter_perm(nx, K.perm, nullptr, K.z, c->d_lam, c->stream);
  return SGN_OK;
}

sgn_status assemble_impl(sgn_ctx c, const double* x, const double* p, double* rhs_old, double* grad, double* obj) {
  const Analysis& A = c->A;
  const int64_t nx = A.mesh.n_x, np = A.mesh.n_p, N = A.sgn.N;
  const bool newton = A.newton;
  int inv = 0;
  HIPCHK(ensure_events(c, 0));
  if (newton) {
    // the Newton blocks contract the third derivatives with lam: solve for it first
    if (!c->kx_valid) {
      c->err = "the Newton form needs the Kx factor of sgn_equilibrium at this state";
      return SGN_E_STATE;
    }
    launch_fill(nx, 0.0, c->d_fx, c->stream);
    launch_objective_fx((int64_t)c->target_dof.size(), c->d_tdof, c->d_tval, x, c->target_w / (c->ell * c->ell),
                        c->d_fx, c->stream);
    TRY(adjoint_multipliers(c));
  }
  HIPCHK(hipEventRecord(c->ev_a, c->stream));
  TRY(run_element(c, x, p, newton ? 3 : 2, &inv));
  if (inv) {
    c->err = "inverted element in the given state";
    return SGN_E_INVERTED;
  }
  assemble_sgn(c);
  HIPCHK(hipEventRecord(c->ev_b, c->stream));
  HIPCHK(hipEventSynchronize(c->ev_b));
  {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_a, c->ev_b));
    c->stats.assemble_ms = ms;
    c->stats.assemble_bytes = 8.0 * (double)(nx + np) + 4.0 * (double)A.mesh.n_elems * (A.mesh.dim + 1) +
                              8.0 * (double)A.mesh.rest.size() + 8.0 * (double)A.sgn.colind.size();
  }
  c->sgn_assembled = true;
  c->sys[0].current = false;
  c->sys[0].bp_ready = false;
  HIPCHK(hipMemcpyAsync(c->d_x_asm, x, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_p_asm, p, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (obj) TRY(objective_value(c, x, p, obj));
  if (rhs_old || grad) {
    const int64_t nt = (int64_t)c->target_dof.size();
    launch_fill(nx, 0.0, c->d_fx, c->stream);
    launch_objective_fx(nt, c->d_tdof, c->d_tval, x, c->target_w / (c->ell * c->ell), c->d_fx, c->stream);
    launch_axpby(np, c->mu_reg, p, -c->mu_reg, c->d_pref, c->d_fp, c->stream);
    if (c->opt.rhs_kind == SGN_RHS_KKT) {
      if (grad) {
        c->err = "the KKT right-hand side does not form the gradient";
        return SGN_E_ARG;
      }
      launch_axpby(nx, -1.0, c->d_fx, 0.0, nullptr, rhs_old, c->stream);
      launch_axpby(np, -1.0, c->d_fp, 0.0, nullptr, rhs_old + nx, c->stream);
      launch_fill(nx, 0.0, rhs_old + nx + np, c->stream);
      return SGN_OK;
    }
    if (!c->kx_valid) {
      c->err = "adjoint right-hand side needs the Kx factor of sgn_equilibrium at this state";
      return SGN_E_STATE;
    }
    if (!newton) TRY(adjoint_multipliers(c));  // the Newton form solved for lam before its element pass
    // Kp^T lam through the assembled K_SGN: w = K [0; 0; lam], g = fp + w_p (the x-p block of the
    // Newton form multiplies the zero x part)
    DevSys& D = c->sys[0];
    launch_fill(N, 0.0, c->d_old, c->stream);
    HIPCHK(hipMemcpyAsync(c->d_old + nx + np, c->d_lam, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    launch_gather_perm(N, D.perm, nullptr, c->d_old, D.t, c->stream);
    launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, D.t, D.r, c->stream);
    launch_scatter_perm(N, D.perm, nullptr, D.r, c->d_old2, c->stream);
    launch_axpby(np, 1.0, c->d_fp, 1.0, c->d_old2 + nx, c->d_g, c->stream);
    if (grad && grad != c->d_g)
      HIPCHK(hipMemcpyAsync(grad, c->d_g, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (rhs_old) {
      launch_fill(N, 0.0, rhs_old, c->stream);
      launch_axpby(np, -1.0, c->d_g, 0.0, nullptr, rhs_old + nx, c->stream);
    }
  }
  return SGN_OK;
}

// ------------------------------------------------------------------ block Gauss-Newton
// y = K_SGN v for vectors in boundary (block) order, with the currently assembled values
void sgn_matvec_boundary(sgn_ctx c, const double* v_old, double* y_old) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_gather_perm(N, D.perm, nullptr, v_old, D.t, c->stream);
  launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, D.t, D.r, c->stream);
  launch_scatter_perm(N, D.perm, nullptr, D.r, y_old, c->stream);
}

// Right-preconditioned restarted GMRES(m) (Saad and Schultz) for A u = b on length-n vectors in
// FP64: u += P (V y) with V an orthonormal basis of the Krylov space of A P built by two passes of
// classical Gram-Schmidt (device dot products, one read-back per step) and y from the Givens-reduced
// least-squares problem on the host.  Cycles restart from the true residual until
// |b - A u| <= rtol |b| or max_cycles.  V holds (m + 1) n, w1 and w2 n each.
sgn_status gmres_right(sgn_ctx c, int64_t n, const std::function<sgn_status(const double*, double*)>& Aop,
                       const std::function<sgn_status(const double*, double*)>& Pop, const double* b, double* u,
                       double rtol, int m, int max_cycles, double* V, double* w1, double* w2, int* iters,
                       double* rel_out) {
  hipStream_t st = c->stream;
  dev_dot(c, n, b, b, 48);
  double b2;
  TRY(read_scalars(c, 48, 1, &b2));
  const double bn = std::sqrt(std::max(b2, 0.0));
  *iters = 0;
  *rel_out = 0.0;
  if (bn == 0.0) {
    launch_fill(n, 0.0, u, st);
    return SGN_OK;
  }
  const double stop = rtol * bn;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hb(2 * 64 + 1), y(m);
  auto h = [&](int i, int j) -> double& { return H[(size_t)j * (m + 1) + i]; };
  for (int cycle = 0; cycle < max_cycles; ++cycle) {
    TRY(Aop(u, w1));
    launch_axpby(n, 1.0, b, -1.0, w1, V, st);  // r = b - A u
    dev_dot(c, n, V, V, 48);
    double r2;
    TRY(read_scalars(c, 48, 1, &r2));
    const double beta = std::sqrt(std::max(r2, 0.0));
    *rel_out = beta / bn;
    if (beta <= stop) return SGN_OK;
    launch_axpby(n, 1.0 / beta, V, 0.0, nullptr, V, st);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    while (k < m) {
      const int j = k;
      double* vj = V + (int64_t)j * n;
      double* vn = V + (int64_t)(j + 1) * n;
      TRY(Pop(vj, w2));
      TRY(Aop(w2, vn));
      for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) dev_dot_to(c, n, V + (int64_t)i * n, vn, c->d_gm + 64 * pass + i);
        launch_multi_axpy(n, j + 1, V, n, c->d_gm + 64 * pass, -1.0, vn, st);
      }
      dev_dot_to(c, n, vn, vn, c->d_gm + 128);
      HIPCHK(hipMemcpyAsync(hb.data(), c->d_gm, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int i = 0; i <= j; ++i) h(i, j) = hb[i] + hb[64 + i];
      const double hn = std::sqrt(std::max(hb[128], 0.0));
      h(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const double a = h(i, j), bb = h(i + 1, j);
        h(i, j) = cs[i] * a + sn[i] * bb;
        h(i + 1, j) = -sn[i] * a + cs[i] * bb;
      }
      const double den = std::hypot(h(j, j), h(j + 1, j));
      if (!(den > 0.0)) break;
      cs[j] = h(j, j) / den;
      sn[j] = h(j + 1, j) / den;
      h(j, j) = den;
      h(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      ++*iters;
      if (std::fabs(g[j + 1]) <= 0.5 * stop || !(hn > 0.0)) break;
      launch_axpby(n, 1.0 / hn, vn, 0.0, nullptr, vn, st);
    }
    if (k == 0) break;
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= h(i, l) * y[l];
      y[i] = t / h(i, i);
    }
    HIPCHK(hipMemcpyAsync(c->d_gm + 192, y.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
    launch_fill(n, 0.0, w1, st);
    launch_multi_axpy(n, k, V, n, c->d_gm + 192, 1.0, w1, st);
    TRY(Pop(w1, w2));
    launch_axpby(n, 1.0, u, 1.0, w2, u, st);
    HIPCHK(hipStreamSynchronize(st));  // y is read by the copy above
  }
  TRY(Aop(u, w1));
  launch_axpby(n, 1.0, b, -1.0, w1, w1, st);
  dev_dot(c, n, w1, w1, 48);
  double r2;
  TRY(read_scalars(c, 48, 1, &r2));
  *rel_out = std::sqrt(std::max(r2, 0.0)) / bn;
  return SGN_OK;
}

// Block Gauss-Newton direction (Sec. 4 "Block Solve", Appendix B) at (x, p) with K_SGN assembled
// there and df/dx^T in c->d_fx:  dx = -A^-1 df/dx^T (A = (w / ell^2) I on every free DOF),
// dp = -Kp^-1 Kx dx (the appendix's sign), dlam = Kx^-1 df/dx^T (adjoint right-hand side; the KKT
// form's multiplier is dlam + lam_adj = 0).  Kp is never factorised: Kp dp = -Kx dx is solved by
// GMRES right-preconditioned with -Kx^-1 through the Kx factor (for rest-position parameters Kp =
// -Kx up to terms of the order of the strain, so few iterations suffice); the products with Kx and
// Kp come from the assembled K_SGN.  sol: [N] boundary order.
sgn_status bgn_solve_assembled(sgn_ctx c, const double* x, const double* p, double* sol, sgn_solve_info* info) {
  const Analysis& A = c->A;
  const int64_t nx = A.mesh.n_x, np = A.mesh.n_p, N = A.sgn.N;
  hipStream_t st = c->stream;
  const double t0 = now_ms();
  DevSys& K = c->sys[1];
  if (!c->kx_valid) {  // the Kx factor at (x, p): the element buffer holds this state's derivatives
    assemble_kx(c, 0.0);
    TRY(factor_dispatch(c, 1, 1e-300, nullptr));
    if (c->sys[1].inertia[0] != nx) return fail(c, SGN_E_PIVOT, "Kx is not positive definite at this state");
    c->kx_valid = true;
  }
  const double a = c->target_w / (c->ell * c->ell);
  double* dx = sol;
  double* dp = sol + nx;
  double* dl = sol + nx + np;
  launch_axpby(nx, -1.0 / a, c->d_fx, 0.0, nullptr, dx, st);
  double* e = c->d_old;
  double* ke = c->d_old2;
  // rhs of the Kp system: v = -Kx dx, the x block of K [0; 0; dx] (Kx symmetric)
  launch_fill(N, 0.0, e, st);
  HIPCHK(hipMemcpyAsync(e + nx + np, dx, nx * sizeof(double), hipMemcpyDeviceToDevice, st));
  sgn_matvec_boundary(c, e, ke);
  double* V = c->sys[0].gm_V;  // (31) x nx fits the SGN system's FGMRES basis (31 x N)
  double* w1 = c->sys[0].gm_Z;
  double* w2 = w1 + nx;
  double* v = w2 + nx;
  launch_axpby(nx, -1.0, ke, 0.0, nullptr, v, st);
  // Kp u: the multiplier block of K [0; u; 0]
  auto Kp = [&](const double* u, double* out) -> sgn_status {
    launch_fill(N, 0.0, e, st);
    HIPCHK(hipMemcpyAsync(e + nx, u, np * sizeof(double), hipMemcpyDeviceToDevice, st));
    sgn_matvec_boundary(c, e, ke);
    HIPCHK(hipMemcpyAsync(out, ke + nx + np, nx * sizeof(double), hipMemcpyDeviceToDevice, st));
    return SGN_OK;
  };
  // -Kx^-1 u by the Kx factor's sweeps
  auto prec = [&](const double* u, double* out) -> sgn_status {
    launch_gather_perm(nx, K.perm, nullptr, u, K.b, st);
    TRY(solve_once(c, 1, K.b, K.z));
    launch_scatter_perm(nx, K.perm, nullptr, K.z, out, st);
    launch_axpby(nx, -1.0, out, 0.0, nullptr, out, st);
    return SGN_OK;
  };
  launch_fill_i32(1, 0, c->d_cnt + 12, st);
  launch_fill(np, 0.0, dp, st);
  int its = 0;
  double rel = 0.0;
  const double rtol = std::min(1e-12, 1e-2 * c->opt.solve_rtol);
  TRY(gmres_right(c, nx, Kp, prec, v, dp, rtol, kGmresM, std::max(1, c->opt.max_gmres), V, w1, w2, &its, &rel));
  if (c->opt.rhs_kind == SGN_RHS_KKT) {
    launch_fill(nx, 0.0, dl, st);
  } else {  // dlam = Kx^-1 df/dx^T, refined on the Kx system
    launch_gather_perm(nx, K.perm, nullptr, c->d_fx, K.b, st);
    const double keep = c->opt.solve_rtol;
    c->opt.solve_rtol = 1e-14;
    sgn_solve_info si{};
    const sgn_status s = refined_solve(c, 1, K.b, K.z, &si);
    c->opt.solve_rtol = keep;
    if (s != SGN_OK && s != SGN_E_REFINE) return s;
    launch_scatter_perm(nx, K.perm, nullptr, K.z, dl, st);
  }
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (timeout) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
  if (info) {
    info->sweeps = its;
    info->fallback = 0;
    info->rel_res = rel;
    info->raw_rel_res = rel;
    info->ms = now_ms() - t0;
    info->gmres_iters = its;
  }
  c->stats.solve_ms = now_ms() - t0;
  if (!(rel <= rtol)) {
    char buf[96];
    snprintf(buf, sizeof(buf), "block solve: GMRES on Kp stopped at relative residual %.3e", rel);
    return fail(c, SGN_E_REFINE, buf);
  }
  return SGN_OK;
}

// Backtracking along dir from the equilibrium (d_p, d_x) with one equilibrium per trial and Armijo
// acceptance f(alpha) <= f(0) + 1e-4 alpha g^T dir (si->f0, si->gtdp set by the caller); on success
// (d_p, d_x) move to the accepted trial.  t_start: host time the search began (ms_linesearch).
sgn_status line_search(sgn_ctx c, double* d_p, double* d_x, const double* dir, double t_start, sgn_step_info* si,
                       sgn_step_info* info) {
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  const double f0 = si->f0, gtdp = si->gtdp;
  double alpha = 1.0;
  bool ok = false;
  int nt_iters = 0;
  for (int h = 0; h <= c->opt.max_halvings; ++h) {
    launch_axpby(np, 1.0, d_p, alpha, dir, c->d_pt, c->stream);
    HIPCHK(hipMemcpyAsync(c->d_xt, d_x, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    sgn_eq_info ei{};
    sgn_status s = equilibrium_impl(c, c->d_pt, c->d_xt, &ei);
    if (s == SGN_OK) {
      nt_iters += ei.iters;
      double f1;
      TRY(objective_value(c, c->d_xt, c->d_pt, &f1));
      if (f1 <= f0 + 1e-4 * alpha * gtdp) {
        si->f1 = f1;
        ok = true;
        break;
      }
    } else if (s == SGN_E_HIP) {
      return fail(c, s, c->err);
    }
    alpha *= 0.5;
    ++si->halvings;
  }
  si->ms_linesearch = now_ms() - t_start;
  si->newton_iters = nt_iters;
  if (!ok && std::fabs(gtdp) <= 1e-12 * std::fabs(f0)) {
    // the predicted decrease of the whole step is below the objective's rounding: the iterate is
    // stationary to working precision and Armijo decisions are noise; stay (alpha = 0)
    si->alpha = 0.0;
    si->f1 = f0;
    c->kx_valid = false;  // the Kx factor and values belong to the last trial, not to d_p
    if (info) *info = *si;
    return SGN_OK;
  }
  si->alpha = alpha;
  if (info) *info = *si;
  if (!ok) {
    c->kx_valid = false;
    return fail(c, SGN_E_LINESEARCH, "line search failed");
  }
  HIPCHK(hipMemcpyAsync(d_p, c->d_pt, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(d_x, c->d_xt, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

// Objective of every problem of a batch at the union state (x, p) into h_f[ncomp]:
// f_k = w/(2 ell^2) sum over k's targets (x - t)^2 + mu/2 sum over k's parameters (p - p_ref)^2.
// Uses c->d_old as scratch.
sgn_status batch_objectives(sgn_ctx c, const double* x, const double* p, double* h_f) {
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  const int nc = c->ncomp;
  hipStream_t st = c->stream;
  double* rx = c->d_old;
  double* rp = c->d_old + nx;
  launch_fill(nx, 0.0, rx, st);
  launch_objective_fx((int64_t)c->target_dof.size(), c->d_tdof, c->d_tval, x, 1.0, rx, st);  // x_T - t
  launch_axpby(np, 1.0, p, -1.0, c->d_pref, rp, st);
  launch_segment_dot(nc, c->d_seg_x, rx, rx, c->d_seg_val, st);
  launch_segment_dot(nc, c->d_seg_p, rp, rp, c->d_seg_val + nc, st);
  std::vector<double> v(2 * (size_t)nc);
  HIPCHK(hipMemcpyAsync(v.data(), c->d_seg_val, v.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double wl = c->target_w / (c->ell * c->ell);
  for (int k = 0; k < nc; ++k) h_f[k] = 0.5 * wl * v[k] + 0.5 * c->mu_reg * v[nc + k];
  return SGN_OK;
}

sgn_status check_ready(sgn_ctx c) {
  if (!c) return SGN_E_ARG;
  if (c->sticky) return SGN_E_STATE;
  if (!c->has_ws) return fail(c, SGN_E_STATE, "no workspace set");
  return SGN_OK;
}

sgn_status sgn_factor_impl(sgn_ctx c, sgn_factor_info* info) {
  if (!c->sgn_assembled) return fail(c, SGN_E_STATE, "sgn_factor before sgn_assemble");
  HIPCHK(hipMemcpyAsync(c->d_x_fac, c->d_x_asm, c->A.mesh.n_x * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_p_fac, c->d_p_asm, c->A.mesh.n_p * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  sgn_factor_info fi{};
  const double tol = c->sys[0].prec ? 1e-12 : 1e-14;
  TRY(factor_dispatch(c, 0, tol, &fi));
  if (info) *info = fi;
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  if (c->sys[0].prec == 0 && (fi.n_pos != nx + np || fi.n_neg != nx || fi.n_zero != 0)) {
    char buf[160];
    snprintf(buf, sizeof(buf), "inertia (%lld, %lld, %lld), expected (%lld, %lld, 0)", (long long)fi.n_pos,
             (long long)fi.n_neg, (long long)fi.n_zero, (long long)(nx + np), (long long)nx);
    return fail(c, SGN_E_PIVOT, buf);
  }
  return SGN_OK;
}

sgn_status sgn_solve_impl(sgn_ctx c, const double* rhs, double* sol, sgn_solve_info* info) {
  DevSys& D = c->sys[0];
  if (!D.current) return fail(c, SGN_E_STATE, "sgn_solve before sgn_factor of the assembled matrix");
  const int64_t N = c->A.sgn.N;
  launch_gather_perm(N, D.perm, nullptr, rhs, c->d_old2, c->stream);
  double* zn = c->d_old;  // new-order solution
  const double t0 = now_ms();
  sgn_status s = c->opt.solver == SGN_BICGSTAB ? bicgstab_solve(c, c->d_old2, zn, info)
                                               : refined_solve(c, 0, c->d_old2, zn, info);
  launch_scatter_perm(N, D.perm, nullptr, zn, sol, c->stream);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->stats.solve_ms = now_ms() - t0;
  if (s != SGN_OK) return fail(c, s, c->err);
  return SGN_OK;
}

sgn_status gnn_forward_impl(sgn_ctx c, const float* w, const double* x_ref, const double* p_ref, const double* x,
                            const double* p, float* cn, float* cp);

// Working memory of one refined solve of the saddle-point system (sgn_solve without the Krylov
// escalation): the scaled right-hand side, both per-front solve vectors, the split-k partials, the
// pipelined solve's tickets, the refinement vectors, the permuted right-hand side and solution, the
// reduction partials and result slots, and the counters.  base == nullptr only measures.
struct SolveScratch {
  double *sv, *tv, *tp, *part, *ir_r, *ir_d, *ir_s, *old, *old2, *red, *scal;
  int *ctr, *cnt;
};

size_t carve_solve_scratch(sgn_ctx c, char* base, SolveScratch* s) {
  Layout L{base};
  const System& S = c->A.sgn;
  s->sv = L.take<double>(S.N);
  s->tv = L.take<double>(S.vec_total);
  s->tp = L.take<double>(S.vec_total);
  s->part = L.take<double>(S.part_total);
  s->ctr = L.take<int>(2 * (size_t)S.nsn);
  s->ir_r = L.take<double>(S.N);
  s->ir_d = L.take<double>(S.N);
  s->ir_s = L.take<double>(S.N);
  s->old = L.take<double>(S.N);
  s->old2 = L.take<double>(S.N);
  s->red = L.take<double>(4 * kRedBlocks);
  s->scal = L.take<double>(64);
  s->cnt = L.take<int>(64);
  return (L.off + 255) & ~size_t(255);
}

// MINRES with the reference factor's preconditioner; on stagnation, on max_minres
// iterations, or without a reference factor: exact factorisation of the current
// matrix (which becomes the new reference) and the refined direct solve.
// |B_i|^-1 of the node groups' diagonal blocks of the assembled matrix (block-diagonal preconditioner)
sgn_status blockpc_setup(sgn_ctx c) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_row_scaling(D.row_lanes, N, D.frowptr, D.fslot, D.vals, D.cur_scale, c->stream);
  launch_blockpc_setup(D.ngroups, D.grp_ptr, D.rowptr, D.colind, D.vals, D.cur_scale, D.bp_off, D.bp_minv, c->stream);
  HIPCHK(hipGetLastError());
  D.bp_ready = true;
  return SGN_OK;
}

sgn_status minres_solve_impl(sgn_ctx c, const double* rhs, double* sol, sgn_solve_info* info) {
  DevSys& D = c->sys[0];
  if (!c->sgn_assembled) return fail(c, SGN_E_STATE, "sgn_solve_minres before sgn_assemble");
  const int64_t N = c->A.sgn.N;
  const double t0 = now_ms();
  launch_gather_perm(N, D.perm, nullptr, rhs, c->d_old2, c->stream);
  double* zn = c->d_old;
  sgn_solve_info si{};
  bool conv = false;
  const bool block = c->opt.pc_kind == SGN_PC_BLOCK;
  if (block) TRY(blockpc_setup(c));
  if (D.factored || block) {
    if (c->pc_weights && !block) {  // corrections for the move from the reference state to the assembled one
      TRY(gnn_forward_impl(c, c->pc_weights, c->d_x_fac, c->d_p_fac, c->d_x_asm, c->d_p_asm, c->own_cn, c->own_cp));
      c->use_own = true;
    }
    launch_fill_i32(1, 0, c->d_cnt + 12, c->stream);
    int it = 0;
    double rel = 1.0;
    TRY(minres_new(c, c->d_old2, zn, c->opt.max_minres, 50, &it, &rel, &conv));
    int timeout = 0;
    HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (timeout) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
    si.sweeps = it;
    si.rel_res = rel;
    si.raw_rel_res = -1.0;
  }
  if (!conv) {
    sgn_factor_info fi{};
    TRY(sgn_factor_impl(c, &fi));
    const int it = si.sweeps;
    sgn_status s = refined_solve(c, 0, c->d_old2, zn, &si);
    if (s != SGN_OK) return fail(c, s, c->err);
    si.sweeps += it;
    si.fallback = 1;
  }
  launch_scatter_perm(N, D.perm, nullptr, zn, sol, c->stream);
  HIPCHK(hipStreamSynchronize(c->stream));
  si.ms = now_ms() - t0;
  c->stats.solve_ms = si.ms;
  if (info) *info = si;
  return SGN_OK;
}

// ------------------------------------------------------------------ preconditioner network
DenseArgs dense_args(const float* w, const GnnDense& L, int64_t rows, int act) {
  DenseArgs a{};
  a.rows = rows;
  a.nseg = 0;
  a.K = 0;
  a.W = w + L.w;
  a.N = L.n;
  a.act = act;
  return a;
}

void add_seg(DenseArgs& a, const float* src, const int32_t* idx, int width, int ld) {
  a.seg[a.nseg++] = DenseSeg{src, idx, width, ld};
  a.K += width;
}

sgn_status gnn_forward_impl(sgn_ctx c, const float* w, const double* x_ref, const double* p_ref, const double* x,
                            const double* p, float* cn, float* cp) {
  const GnnGraph& G = c->G;
  auto& g = c->g;
  hipStream_t st = c->stream;
  const int64_t nn = G.n_nodes, E = G.n_edges, ne = G.n_elems, H = kGnnH;
  GnnFeatArgs fa{};
  fa.n_nodes = nn;
  fa.n_edges = E;
  fa.dim = G.dim;
  fa.param_kind = G.param_kind;
  fa.nfdof = g.nfdof;
  fa.rest = c->d_rest;
  fa.x = x;
  fa.x_ref = x_ref;
  fa.p = p;
  fa.p_ref = p_ref;
  fa.inc_ptr = g.inc_ptr;
  fa.inc_list = g.inc_list;
  fa.ell = c->ell;
  fa.hbar = G.hbar;
  launch_gnn_features(fa, g.src, g.dst, g.nf, g.ef, st);
  {
    DenseArgs a = dense_args(w, G.enc_n, nn, 1);
    add_seg(a, g.nf, nullptr, G.fn, G.fn);
    a.out = g.h[0];
    a.ld_out = H;
    launch_dense_fwd(a, st);
    DenseArgs b = dense_args(w, G.enc_e, E, 1);
    add_seg(b, g.ef, nullptr, G.fe, G.fe);
    b.out = g.e[0];
    b.ld_out = H;
    launch_dense_fwd(b, st);
  }
  for (int l = 0; l < kGnnLayers; ++l) {
    DenseArgs a = dense_args(w, G.edge[l], E, 1);
    add_seg(a, g.h[l], g.dst, H, H);
    add_seg(a, g.h[l], g.src, H, H);
    add_seg(a, g.e[l], nullptr, H, H);
    a.res = g.e[l];
    a.ld_res = H;
    a.out = g.e[l + 1];
    a.ld_out = H;
    a.ysave = g.ye[l];
    launch_dense_fwd(a, st);
    launch_fill_f32(nn * H, 0.0f, g.agg[l], st);
    launch_gather_add(nn, g.in_ptr, nullptr, g.e[l + 1], H, 0, H, 1.0f, 1, g.agg[l], H, st);
    DenseArgs b = dense_args(w, G.node[l], nn, 1);
    add_seg(b, g.h[l], nullptr, H, H);
    add_seg(b, g.agg[l], nullptr, H, H);
    b.res = g.h[l];
    b.ld_res = H;
    b.out = g.h[l + 1];
    b.ld_out = H;
    b.ysave = g.yn[l];
    launch_dense_fwd(b, st);
  }
  {
    DenseArgs a = dense_args(w, G.dec_n, nn, 0);
    add_seg(a, g.h[kGnnLayers], nullptr, H, H);
    a.out = g.dec;
    a.ld_out = G.nout_node;
    launch_dense_fwd(a, st);
    launch_split_out(nn, G.tri, G.nout_node, G.dim, G.param_kind != 0, g.nfdof, g.dec, cn, cp, st);
  }
  if (G.param_kind == 0) {
    launch_elem_mean(ne, G.dim + 1, c->d_elems, g.h[kGnnLayers], g.emb, st);
    DenseArgs a = dense_args(w, G.dec_e, ne, 0);
    add_seg(a, g.emb, nullptr, H, H);
    a.out = cp;
    a.ld_out = 1;
    launch_dense_fwd(a, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  c->gnn_fwd_done = true;
  return SGN_OK;
}

// gw += d(sum gcn . cn + gcp . cp)/dw with the activations of the last forward pass
sgn_status gnn_backward_impl(sgn_ctx c, const float* w, const float* gcn, const float* gcp, float* gw) {
  const GnnGraph& G = c->G;
  auto& g = c->g;
  hipStream_t st = c->stream;
  const int64_t nn = G.n_nodes, E = G.n_edges, ne = G.n_elems, H = kGnnH;
  float* dh = g.dh[0];  // dL/dh of the current layer
  float* de = g.de[0];  // dL/de of the current layer
  launch_fill_f32(nn * H, 0.0f, dh, st);
  launch_fill_f32(E * H, 0.0f, de, st);
  // decoders
  launch_split_bwd(nn, G.tri, G.nout_node, G.dim, G.param_kind != 0, g.nfdof, gcn, gcp, g.ddec, st);
  {
    DenseArgs a = dense_args(w, G.dec_n, nn, 0);
    add_seg(a, g.h[kGnnLayers], nullptr, H, H);
    launch_dense_bwd(a, g.ddec, G.nout_node, nullptr, g.dz, g.dx, st);
    launch_dense_wgrad(a, g.dz, g.part, gw + G.dec_n.w, st);
    launch_gather_add(nn, nullptr, nullptr, g.dx, H, 0, H, 1.0f, 0, dh, H, st);
  }
  if (G.param_kind == 0 && gcp) {
    DenseArgs a = dense_args(w, G.dec_e, ne, 0);
    add_seg(a, g.emb, nullptr, H, H);
    launch_dense_bwd(a, gcp, 1, nullptr, g.dz, g.demb, st);
    launch_dense_wgrad(a, g.dz, g.part, gw + G.dec_e.w, st);
    launch_gather_add(nn, g.inc_ptr, g.inc_list, g.demb, H, 0, H, 1.0f / (float)(G.dim + 1), 0, dh, H, st);
  }
  // message-passing layers in reverse
  for (int l = kGnnLayers - 1; l >= 0; --l) {
    {  // node update: h[l+1] = h[l] + tanh(W [h[l], agg[l]] + b)
      DenseArgs a = dense_args(w, G.node[l], nn, 1);
      add_seg(a, g.h[l], nullptr, H, H);
      add_seg(a, g.agg[l], nullptr, H, H);
      launch_dense_bwd(a, dh, H, g.yn[l], g.dz, g.dx, st);
      launch_dense_wgrad(a, g.dz, g.part, gw + G.node[l].w, st);
      launch_gather_add(nn, nullptr, nullptr, g.dx, 2 * H, 0, H, 1.0f, 0, dh, H, st);  // residual + h input
      launch_edge_mean_bwd(E, g.dst, g.in_ptr, g.dx, 2 * H, H, de, st);                // agg = mean of e[l+1]
    }
    {  // edge update: e[l+1] = e[l] + tanh(W [h[l]_dst, h[l]_src, e[l]] + b)
      DenseArgs a = dense_args(w, G.edge[l], E, 1);
      add_seg(a, g.h[l], g.dst, H, H);
      add_seg(a, g.h[l], g.src, H, H);
      add_seg(a, g.e[l], nullptr, H, H);
      launch_dense_bwd(a, de, H, g.ye[l], g.dz, g.dx, st);
      launch_dense_wgrad(a, g.dz, g.part, gw + G.edge[l].w, st);
      launch_gather_add(E, nullptr, nullptr, g.dx, 3 * H, 2 * H, H, 1.0f, 0, de, H, st);           // residual + e input
      launch_gather_add(nn, g.in_ptr, nullptr, g.dx, 3 * H, 0, H, 1.0f, 0, dh, H, st);           // h as receiver
      launch_gather_add(nn, g.out_ptr, g.out_list, g.dx, 3 * H, H, H, 1.0f, 0, dh, H, st);       // h as sender
    }
  }
  {  // encoders (tanh outputs e[0], h[0])
    DenseArgs a = dense_args(w, G.enc_e, E, 1);
    add_seg(a, g.ef, nullptr, G.fe, G.fe);
    launch_dense_bwd(a, de, H, g.e[0], g.dz, nullptr, st);
    launch_dense_wgrad(a, g.dz, g.part, gw + G.enc_e.w, st);
    DenseArgs b = dense_args(w, G.enc_n, nn, 1);
    add_seg(b, g.nf, nullptr, G.fn, G.fn);
    launch_dense_bwd(b, dh, H, g.h[0], g.dz, nullptr, st);
    launch_dense_wgrad(b, g.dz, g.part, gw + G.enc_n.w, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return SGN_OK;
}

// out = T v (flat, pivot order) with T = (R C)^-1 L^-1 P S K S P^T L^-T (R C)^-T, the symmetric
// matrix similar to M^-1 K; z, q are new-order work vectors
sgn_status t_apply(sgn_ctx c, const PcArgs& pa, const double* v, double* out, double* z, double* q) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_pc_half_bwd(pa, v, D.pc_w, c->stream);
  TRY(bwd_sweep(c, 0, z, D.pc_w));
  scale_vec(c, N, D.scale, z, z);
  launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, z, q, c->stream);
  scale_vec(c, N, D.scale, q, D.sv);
  TRY(fwd_sweep(c, 0, D.sv));
  launch_pc_half_fwd(pa, D.tp, out, c->stream);
  return SGN_OK;
}

// Training loss of the network: mean over probes u of min_gamma |gamma T^2 u - u|^2 / |u|^2, T the
// symmetric form of the preconditioned matrix (same spectrum as M^-1 K), with the network's
// corrections for the move from the reference state to the assembled one.  It vanishes when T^2 is
// a multiple of I (spectrum {+c, -c}), and it does not change when M is scaled, as MINRES does not:
// without the free gamma, inflating M (T -> 0) would be a spurious minimum of loss 1.  With a = T u,
// b = T a, gamma = u^T b / b^T b, e = gamma (gamma b - u), f = T e, g = T f (envelope theorem):
//   dl = (2/|u|^2) [e^T dT a + f^T dT u].
sgn_status pc_train_loss_impl(sgn_ctx c, const float* w, const double* probes, int nprobe, int log_form, float* gw,
                              double* loss) {
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  hipStream_t st = c->stream;
  TRY(gnn_forward_impl(c, w, c->d_x_fac, c->d_p_fac, c->d_x_asm, c->d_p_asm, c->own_cn, c->own_cp));
  c->use_own = true;
  launch_fill_f32((int64_t)c->A.mesh.n_nodes * c->G.tri, 0.0f, c->g_cn, st);
  launch_fill_f32(c->A.mesh.n_p, 0.0f, c->g_cp, st);
  launch_fill_i32(1, 0, c->d_cnt + 12, st);
  double *a = D.mr[0], *b = D.mr[1], *e = D.mr[2], *f = D.mr[3], *g = D.mr[4], *z = D.mr[5], *q = D.mr[6];
  const PcArgs pa = pc_args(c);
  const double wt = 1.0 / (double)nprobe;
  double total = 0.0;
  for (int k = 0; k < nprobe; ++k) {
    const double* u = probes + (int64_t)k * N;
    TRY(t_apply(c, pa, u, a, z, q));
    TRY(t_apply(c, pa, a, b, z, q));
    dev_dot(c, N, u, u, 24);
    dev_dot(c, N, u, b, 25);
    dev_dot(c, N, b, b, 26);
    double h[3];
    TRY(read_scalars(c, 24, 3, h));
    if (!(h[0] > 0.0)) return fail(c, SGN_E_ARG, "zero probe vector");
    const double gam = h[2] > 0.0 ? h[1] / h[2] : 0.0;
    // |gamma b - u|^2 = |u|^2 - (u^T b)^2 / |b|^2
    total += h[2] > 0.0 ? std::max(0.0, 1.0 - h[1] * h[1] / (h[0] * h[2])) : 1.0;
    launch_lincomb3(N, gam * gam, b, -gam, u, 0.0, nullptr, e, st);
    TRY(t_apply(c, pa, e, f, z, q));
    TRY(t_apply(c, pa, f, g, z, q));
    const double s = 2.0 / h[0] * wt;
    launch_pc_sym_grad(pa, e, b, a, f, s, c->g_cn, c->g_cp, st);
    launch_pc_sym_grad(pa, f, a, u, g, s, c->g_cn, c->g_cp, st);
  }
  if (log_form && total > 0.0) {  // gradient of log(loss): scale the correction gradients by 1/loss
    const float sc = (float)(1.0 / (total * wt));
    launch_scale_f32((int64_t)c->A.mesh.n_nodes * c->G.tri, sc, c->g_cn, st);
    launch_scale_f32(c->A.mesh.n_p, sc, c->g_cp, st);
  }
  TRY(gnn_backward_impl(c, w, c->g_cn, c->g_cp, gw));
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (timeout) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
  *loss = total * wt;
  return SGN_OK;
}

// One SGN step at (x, p) enqueued without host synchronisation, for graph capture: element kernel and
// SGN assembly, the KKT right-hand side [-df/dx; -df/dp; 0] (same dp as the adjoint form, Appendix A),
// supernodal LDL^T, the solve and n_ir FP64 refinement sweeps; the final equilibrated relative residual
// and its done flag (<= solve_rtol) land in d_scal[32], d_scal[33]; inverted elements are counted in
// d_cnt[8], timed-out waits flagged in d_cnt[12].
sgn_status enqueue_step(sgn_ctx c, const double* x, const double* p, double* rhs, double* sol, int n_ir) {
  const Analysis& A = c->A;
  const System& S = A.sgn;
  DevSys& D = c->sys[0];
  const int64_t nx = A.mesh.n_x, np = A.mesh.n_p, N = S.N;
  hipStream_t st = c->stream;
  launch_fill_i32(1, 0, c->d_cnt + 8, st);
  launch_fill_i32(1, 0, c->d_cnt + 12, st);
  ElemArgs ea{};
  ea.dim = A.mesh.dim;
  ea.ne = A.mesh.n_elems;
  ea.param_kind = A.mesh.param_kind;
  ea.mode = 2;
  ea.elems = c->d_elems;
  ea.efdof = c->d_efdof;
  ea.rest = c->d_rest;
  ea.x = x;
  ea.p = p;
  ea.mu0 = c->mu0;
  ea.lam0 = c->lam0;
  ea.ebuf = c->d_ebuf;
  ea.stride = A.stride;
  ea.off_grad = A.off_grad;
  ea.off_kp = A.off_kp;
  ea.off_energy = A.off_energy;
  ea.inverted = c->d_cnt + 8;
  launch_element(ea, st);
  assemble_sgn(c);
  launch_fill(nx, 0.0, c->d_fx, st);
  launch_objective_fx((int64_t)c->target_dof.size(), c->d_tdof, c->d_tval, x, c->target_w / (c->ell * c->ell),
                      c->d_fx, st);
  launch_axpby(np, c->mu_reg, p, -c->mu_reg, c->d_pref, c->d_fp, st);
  launch_axpby(nx, -1.0, c->d_fx, 0.0, nullptr, rhs, st);
  launch_axpby(np, -1.0, c->d_fp, 0.0, nullptr, rhs + nx, st);
  launch_fill(nx, 0.0, rhs + nx + np, st);
  const double tol = D.prec ? 1e-12 : 1e-14;
  if (D.prec) TRY(factor_system<float>(c, 0, tol));
  else TRY(factor_system<double>(c, 0, tol));
  double* b = c->d_old2;
  double* z = c->d_old;
  launch_gather_perm(N, D.perm, nullptr, rhs, b, st);
  TRY(solve_once(c, 0, b, z));
  for (int k = 0; k < n_ir; ++k) {
    launch_residual(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, z, b, D.ir_r, st);
    TRY(solve_once(c, 0, D.ir_r, D.ir_d));
    launch_axpby(N, 1.0, z, 1.0, D.ir_d, z, st);
  }
  scale_vec(c, N, D.scale, b, D.ir_s);
  dev_dot(c, N, D.ir_s, D.ir_s, 31);
  launch_residual(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, z, b, D.ir_r, st);
  scale_vec(c, N, D.scale, D.ir_r, D.ir_s);
  dev_dot(c, N, D.ir_s, D.ir_s, 30);
  launch_rel_flag(c->d_scal + 30, c->d_scal + 31, c->opt.solve_rtol, c->d_scal + 32, st);
  launch_scatter_perm(N, D.perm, nullptr, z, sol, st);
  HIPCHK(hipGetLastError());
  return SGN_OK;
}

sgn_status pc_ready(sgn_ctx c) {
  TRY(check_ready(c));
  if (!c->sys[0].factored) return fail(c, SGN_E_STATE, "no reference factor (call sgn_factor first)");
  return SGN_OK;
}

}  // namespace

// Refined solve whose working memory is the caller-designated device region [region, region + cap)
// instead of the context's workspace (the factor, the assembled matrix and the symbolic tables stay
// in the workspace).  Plain refinement only: the FGMRES escalation's Krylov bases do not fit a small
// region, so a solve that refinement alone cannot finish returns SGN_E_REFINE.  lookup: the status of
// obtaining the region (reported as SGN_E_HIP).  Everything the solve reads from the region it has
// written first in the same call (tickets and the timeout flag are cleared by the solve itself).
sgn_status solve_in_region(sgn_ctx c, const double* d_rhs, double* d_sol, sgn_solve_info* info, void* region,
                           size_t cap, hipError_t lookup) {
  TRY(check_ready(c));
  if (!d_rhs || !d_sol) return fail(c, SGN_E_ARG, "null vector");
  if (lookup != hipSuccess || !region)
    return fail(c, SGN_E_HIP, std::string("static scratch address: ") + hipGetErrorString(lookup));
  if (((uintptr_t)region & 255) != 0) return fail(c, SGN_E_ARG, "scratch region must be 256-byte aligned");
  SolveScratch s{};
  const size_t need = carve_solve_scratch(c, nullptr, &s);
  if (need > cap) {
    char buf[160];
    snprintf(buf, sizeof(buf), "this system's solve needs %zu bytes of scratch; the static region holds %zu", need,
             cap);
    return fail(c, SGN_E_NOMEM, buf);
  }
  carve_solve_scratch(c, static_cast<char*>(region), &s);
  DevSys& D = c->sys[0];
  const SolveScratch keep{D.sv, D.tv, D.tp, D.part, D.ir_r, D.ir_d, D.ir_s, c->d_old, c->d_old2, c->d_part,
                          c->d_scal, D.solve_ctr, c->d_cnt};
  const int keep_gmres = c->opt.max_gmres;
  auto point = [&](const SolveScratch& v) {
    D.sv = v.sv;
    D.tv = v.tv;
    D.tp = v.tp;
    D.part = v.part;
    D.ir_r = v.ir_r;
    D.ir_d = v.ir_d;
    D.ir_s = v.ir_s;
    c->d_old = v.old;
    c->d_old2 = v.old2;
    c->d_part = v.red;
    c->d_scal = v.scal;
    D.solve_ctr = v.ctr;
    c->d_cnt = v.cnt;
  };
  point(s);
  c->opt.max_gmres = 0;
  const sgn_status st = sgn_solve_impl(c, d_rhs, d_sol, info);
  c->opt.max_gmres = keep_gmres;
  point(keep);
  return st;
}

// =================================================================== C ABI
extern "C" {

void sgn_default_options(sgn_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SGN_FP64;
  o->solver = SGN_LDLT;
  o->max_bicgstab = 50;
  o->lbfgs_m = 5;
  o->rhs_kind = SGN_RHS_ADJOINT;
  o->newton_rtol = 1e-10;
  o->newton_atol = 0.0;
  o->solve_rtol = 1e-10;
  o->eps_x = 0.0;
  o->eps_lambda = 0.0;
  o->max_newton = 50;
  o->max_ir = 10;
  o->max_gmres = 10;
  o->max_minres = 500;
  o->max_halvings = 30;
  o->profile = 0;
}

sgn_status sgn_create(const sgn_problem* pr, const sgn_options* opt, void* stream, sgn_ctx* out) {
  if (!out) return SGN_E_ARG;
  *out = nullptr;
  if (!pr || !pr->rest_pos || !pr->elems || !pr->node_grid || !pr->fixed || !pr->f_ext) return SGN_E_ARG;
  if (pr->dim != 2 && pr->dim != 3) return SGN_E_ARG;
  if (pr->n_nodes <= 0 || pr->n_elems <= 0) return SGN_E_ARG;
  if (pr->param_kind < 0 || pr->param_kind > 2) return SGN_E_ARG;
  sgn_ctx c = new (std::nothrow) sgn_ctx_s();
  if (!c) return SGN_E_NOMEM;
  *out = c;
  if (opt) c->opt = *opt;
  else sgn_default_options(&c->opt);
  c->stream = (hipStream_t)stream;
  const int d = pr->dim, nv = d + 1;
  Mesh& m = c->A.mesh;
  m.dim = d;
  m.n_nodes = pr->n_nodes;
  m.n_elems = pr->n_elems;
  m.param_kind = pr->param_kind;
  m.rest.assign(pr->rest_pos, pr->rest_pos + (size_t)pr->n_nodes * d);
  m.elems.assign(pr->elems, pr->elems + (size_t)pr->n_elems * nv);
  m.grid.assign(pr->node_grid, pr->node_grid + (size_t)pr->n_nodes * d);
  m.fixed.assign(pr->fixed, pr->fixed + pr->n_nodes);
  m.fext.assign(pr->f_ext, pr->f_ext + (size_t)pr->n_nodes * d);
  for (int32_t v : m.elems)
    if (v < 0 || v >= pr->n_nodes) return fail(c, SGN_E_ARG, "element references a node out of range");
  for (int32_t g : m.grid)
    if (g < 0 || g > 1000000) return fail(c, SGN_E_ARG, "grid coordinate out of range");
  if (pr->n_components > 1) {
    if (!pr->component_ptr) return fail(c, SGN_E_ARG, "component_ptr missing");
    m.comp_ptr.assign(pr->component_ptr, pr->component_ptr + pr->n_components + 1);
    if (m.comp_ptr.front() != 0 || m.comp_ptr.back() != pr->n_nodes)
      return fail(c, SGN_E_ARG, "component_ptr must run from 0 to n_nodes");
    for (int k = 0; k < pr->n_components; ++k)
      if (m.comp_ptr[k + 1] <= m.comp_ptr[k]) return fail(c, SGN_E_ARG, "empty or unordered component");
    std::vector<int32_t> comp(pr->n_nodes);
    for (int k = 0; k < pr->n_components; ++k)
      for (int v = m.comp_ptr[k]; v < m.comp_ptr[k + 1]; ++v) comp[v] = k;
    for (int e = 0; e < pr->n_elems; ++e)
      for (int a = 1; a < nv; ++a)
        if (comp[m.elems[(size_t)e * nv + a]] != comp[m.elems[(size_t)e * nv]])
          return fail(c, SGN_E_ARG, "an element spans two components");
  } else {
    m.comp_ptr = {0, pr->n_nodes};
  }
  if (!(pr->E0 > 0) || !(pr->nu > -1.0 && pr->nu < 0.5)) return fail(c, SGN_E_ARG, "invalid material");
  for (int b = 0; b < kTuneBuckets; ++b) {
    const int v = c->opt.outer_panels[b];
    if (v < 0 || v > 16) return fail(c, SGN_E_ARG, "outer_panels must be 1..16 (0: default)");
    c->A.tune.outer_panels[b] = v == 0 ? kOuterPanels : v;
  }
  if (c->opt.seq_panels < -1 || c->opt.seq_panels > kSolveSeqPanels)
    return fail(c, SGN_E_ARG, "seq_panels must be -1..8 (0: default)");
  if (c->opt.solver < SGN_LDLT || c->opt.solver > SGN_BLOCK_GN) return fail(c, SGN_E_ARG, "unknown solver");
  if (c->opt.lbfgs_m < 0 || c->opt.lbfgs_m > 32) return fail(c, SGN_E_ARG, "lbfgs_m must be 0..32");
  c->lb_rho.assign(std::max(1, c->opt.lbfgs_m), 0.0);
  if (c->opt.solver == SGN_BICGSTAB && c->opt.max_bicgstab < 1)
    return fail(c, SGN_E_ARG, "max_bicgstab must be at least 1");
  if (!(c->opt.eps_x >= 0.0) || !(c->opt.eps_lambda >= 0.0)) return fail(c, SGN_E_ARG, "eps_x, eps_lambda must be >= 0");
  c->A.tune.seq_panels = c->opt.seq_panels == 0 ? kSolveSeqPanels : (c->opt.seq_panels < 0 ? 0 : c->opt.seq_panels);
  if (c->opt.panel_waves != 0 && c->opt.panel_waves != 1 && c->opt.panel_waves != 2 && c->opt.panel_waves != 4 &&
      c->opt.panel_waves != 8)
    return fail(c, SGN_E_ARG, "panel_waves must be 0, 1, 2, 4 or 8");
  c->A.tune.panel_waves = c->opt.panel_waves;
  if (c->opt.hessian != SGN_HESSIAN_GN && c->opt.hessian != SGN_HESSIAN_NEWTON)
    return fail(c, SGN_E_ARG, "unknown hessian");
  if (c->opt.hessian == SGN_HESSIAN_NEWTON) {
    // Sec. 4 "Generalization to Arbitrary Objectives", Appendix A: the Lagrangian Hessian at the adjoint
    // multipliers, which the adjoint right-hand side and the refined direct solve serve
    if (pr->param_kind != SGN_P_LOGE) return fail(c, SGN_E_ARG, "the Newton form is built for log-modulus parameters");
    if (pr->n_components > 1) return fail(c, SGN_E_ARG, "the Newton form takes one problem, not a batch");
    if (c->opt.solver != SGN_LDLT) return fail(c, SGN_E_ARG, "the Newton form needs solver = SGN_LDLT");
    if (c->opt.rhs_kind != SGN_RHS_ADJOINT) return fail(c, SGN_E_ARG, "the Newton form needs rhs_kind = SGN_RHS_ADJOINT");
    if (c->opt.eps_x != 0.0 || c->opt.eps_lambda != 0.0)
      return fail(c, SGN_E_ARG, "the Newton form regularises by itself (eps_x = eps_lambda = 0)");
    c->A.newton = true;
  }
  std::string err = analyse(c->A);
  if (!err.empty()) return fail(c, SGN_E_ARG, "symbolic analysis: " + err);
  if (c->opt.pc_kind != SGN_PC_FACTOR && c->opt.pc_kind != SGN_PC_BLOCK) return fail(c, SGN_E_ARG, "unknown pc_kind");
  if (c->opt.pc_kind == SGN_PC_BLOCK) {
    const std::vector<int32_t>& gp = c->A.sgn.grp_ptr;
    c->bp_off.assign(gp.size(), 0);
    for (size_t q = 0; q + 1 < gp.size(); ++q) {
      const int64_t g = gp[q + 1] - gp[q];
      c->bp_off[q + 1] = c->bp_off[q] + g * g;
    }
  }
  err = build_gnn_graph(m, c->G);
  if (!err.empty()) return fail(c, SGN_E_ARG, "preconditioner graph: " + err);
  const int64_t nx = m.n_x, np = m.n_p;
  if (pr->n_targets < 0 || (pr->n_targets > 0 && !pr->target_dof)) return fail(c, SGN_E_ARG, "targets");
  c->target_dof.assign(pr->target_dof, pr->target_dof + pr->n_targets);
  for (int32_t t : c->target_dof)
    if (t < 0 || t >= nx) return fail(c, SGN_E_ARG, "target DOF out of range");
  c->target_val.assign(pr->n_targets, 0.0);
  if (pr->target_val) c->target_val.assign(pr->target_val, pr->target_val + pr->n_targets);
  c->target_w = pr->target_w;
  c->ell = pr->length_scale > 0 ? pr->length_scale : 1.0;
  c->mu_in = pr->reg_mu;
  // rest-position parameters: the regulariser is measured in units of ell, like the misfit
  c->mu_reg = pr->param_kind == SGN_P_REST_POS ? c->mu_in / (c->ell * c->ell) : c->mu_in;
  c->p_ref.assign(np, 0.0);
  if (pr->p_ref) c->p_ref.assign(pr->p_ref, pr->p_ref + np);
  c->mu0 = pr->E0 / (2.0 * (1.0 + pr->nu));
  c->lam0 = pr->E0 * pr->nu / ((1.0 + pr->nu) * (1.0 - 2.0 * pr->nu));
  c->fext_free.assign(nx, 0.0);
  for (int v = 0; v < m.n_nodes; ++v)
    if (m.fdof[v] >= 0)
      for (int k = 0; k < d; ++k) c->fext_free[m.fdof[v] + k] = m.fext[(size_t)v * d + k];
  double fn = 0;
  for (double v : c->fext_free) fn += v * v;
  c->fext_norm = std::sqrt(fn);
  c->efdof.resize((size_t)m.n_elems * nv);
  for (size_t k = 0; k < c->efdof.size(); ++k) c->efdof[k] = m.fdof[m.elems[k]];
  {
    // per-problem ranges of a batch: free DOFs follow the node order, so each component's are
    // contiguous; log-modulus parameters must be stored problem by problem for sgn_batch_step
    const int nc = (int)m.comp_ptr.size() - 1;
    c->ncomp = nc;
    std::vector<int32_t> comp(m.n_nodes);
    for (int k = 0; k < nc; ++k)
      for (int v = m.comp_ptr[k]; v < m.comp_ptr[k + 1]; ++v) comp[v] = k;
    c->seg_x.assign(nc + 1, 0);
    for (int v = 0; v < m.n_nodes; ++v)
      if (m.fdof[v] >= 0) c->seg_x[comp[v] + 1] += d;
    for (int k = 0; k < nc; ++k) c->seg_x[k + 1] += c->seg_x[k];
    bool ok = true;
    if (m.param_kind == SGN_P_LOGE) {
      c->seg_p.assign(nc + 1, 0);
      int prev = 0;
      for (int e = 0; e < m.n_elems; ++e) {
        const int k = comp[m.elems[(size_t)e * nv]];
        if (k < prev) ok = false;
        prev = k;
        c->seg_p[k + 1] += 1;
      }
      for (int k = 0; k < nc; ++k) c->seg_p[k + 1] += c->seg_p[k];
    } else {
      c->seg_p = c->seg_x;
    }
    c->batch_ok = ok && nc <= 65535;
  }
  // target flags on the SGN diagonal
  {
    System& S = c->A.sgn;
    for (int32_t t : c->target_dof) S.diag_kind[S.iperm[t]] = 1;
  }
  if (c->opt.solver == SGN_BLOCK_GN) {
    // Sec. 4 "Block Solve": no direct parameter term (C = 0; B = 0 always here), a square Kp
    // (rest-position parameters) and an invertible A (every free DOF a target)
    if (m.param_kind != SGN_P_REST_POS) return fail(c, SGN_E_ARG, "block solve needs rest-position parameters");
    if (c->mu_in != 0.0) return fail(c, SGN_E_ARG, "block solve needs reg_mu = 0 (C = 0)");
    std::vector<char> hit(nx, 0);
    for (int32_t t : c->target_dof) hit[t] = 1;
    if ((int64_t)c->target_dof.size() != nx || std::count(hit.begin(), hit.end(), 1) != nx)
      return fail(c, SGN_E_ARG, "block solve needs every free DOF to be a target once (A invertible)");
    if (!(c->target_w > 0)) return fail(c, SGN_E_ARG, "block solve needs target_w > 0");
  }
  c->ws_need = layout(c, nullptr);
  if (verbose()) {
    SolveScratch ss{};
    fprintf(stderr, "[sgn] workspace %zu bytes; sgn_solve_static scratch %zu bytes\n", c->ws_need,
            carve_solve_scratch(c, nullptr, &ss));
  }
  return SGN_OK;
}

sgn_status sgn_workspace_size(sgn_ctx c, size_t* bytes) {
  if (!c || !bytes) return SGN_E_ARG;
  if (c->sticky) return SGN_E_STATE;
  *bytes = c->ws_need;
  return SGN_OK;
}

sgn_status sgn_set_workspace(sgn_ctx c, void* d_ws, size_t bytes) {
  if (!c || !d_ws) return SGN_E_ARG;
  if (c->sticky) return SGN_E_STATE;
  if (((uintptr_t)d_ws & 255) != 0) return fail(c, SGN_E_ARG, "workspace must be 256-byte aligned");
  const size_t need = c->ws_need;
  if (bytes < need) return fail(c, SGN_E_NOMEM, "workspace too small");
  TRY(drop_graph(c));  // a graph captured on the previous workspace must never replay
  layout(c, reinterpret_cast<char*>(d_ws));
  const Analysis& A = c->A;
  hipStream_t st = c->stream;
  for (int si = 0; si < 2; ++si) {
    const System& S = si == 0 ? A.sgn : A.kx;
    DevSys& D = c->sys[si];
    HIPCHK(up(D.rowptr, S.rowptr, st));
    HIPCHK(up(D.colind, S.colind, st));
    HIPCHK(up(D.slot_row, S.slot_row, st));
    HIPCHK(up(D.csr_front_pos, S.csr_front_pos, st));
    HIPCHK(up(D.slot_ptr, S.slot_ptr, st));
    HIPCHK(up(D.slot_src, S.slot_src, st));
    HIPCHK(up(D.diag_kind, S.diag_kind, st));
    HIPCHK(up(D.frowptr, S.frowptr, st));
    HIPCHK(up(D.fcol, S.fcol, st));
    HIPCHK(up(D.fslot, S.fslot, st));
    HIPCHK(up(D.perm, S.perm, st));
    HIPCHK(up(D.sn_begin, S.sn_begin, st));
    HIPCHK(up(D.sn_m, S.sn_m, st));
    HIPCHK(up(D.sn_front_off, S.sn_front_off, st));
    HIPCHK(up(D.sn_vec_off, S.sn_vec_off, st));
    HIPCHK(up(D.sn_rows_ptr, S.sn_rows_ptr, st));
    HIPCHK(up(D.sn_rows, S.sn_rows, st));
    HIPCHK(up(D.relmap_off, S.relmap_off, st));
    HIPCHK(up(D.relmap, S.relmap, st));
    HIPCHK(up(D.child_ptr, S.child_ptr, st));
    HIPCHK(up(D.child_list, S.child_list, st));
    HIPCHK(up(D.var_group_end, S.var_group_end, st));
    HIPCHK(up(D.solve_sn, S.solve_sn, st));
    HIPCHK(up(D.panel_ptr, S.panel_ptr, st));
    HIPCHK(up(D.panel_col, S.panel_col, st));
    HIPCHK(up(D.panel_tasks, S.panel_tasks, st));
    HIPCHK(up(D.upd_tasks, S.upd_tasks, st));
    HIPCHK(up(D.upd_tile_task, S.upd_tile_task, st));
    HIPCHK(up(D.ea_cols, S.ea_cols, st));
    HIPCHK(up(D.ea_kids, S.ea_kid_recs, st));
    HIPCHK(up(D.fill_tasks, S.fill_tasks, st));
    HIPCHK(up(D.vec_ptr, S.vec_ptr, st));
    HIPCHK(up(D.vec_src, S.vec_src, st));
    HIPCHK(up(D.solve_fwd_tasks, S.solve_fwd_tasks, st));
    HIPCHK(up(D.solve_bwd_tasks, S.solve_bwd_tasks, st));
    HIPCHK(up(D.sn_part_off, S.sn_part_off, st));
    if (si == 0) {
      HIPCHK(up(D.grp_ptr, S.grp_ptr, st));
      if (c->opt.pc_kind == SGN_PC_BLOCK) HIPCHK(up(D.bp_off, c->bp_off, st));
      HIPCHK(up(D.grp_node, S.grp_node, st));
      HIPCHK(up(D.grp_vec, S.grp_vec, st));
    }
    if (D.n_const) {
      std::vector<int64_t> cs(D.n_const);
      for (int64_t i = 0; i < D.n_const; ++i) {
        const int64_t r = S.iperm[A.mesh.n_x + A.mesh.n_p + i], q = S.iperm[A.mesh.n_x + i];
        const int64_t hi = std::max(r, q), lo = std::min(r, q);
        auto b = S.colind.begin() + S.rowptr[hi], e = S.colind.begin() + S.rowptr[hi + 1];
        cs[i] = std::lower_bound(b, e, (int32_t)lo) - S.colind.begin();
      }
      HIPCHK(hipMemcpyAsync(D.const_slots, cs.data(), cs.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  {
    const GnnGraph& G = c->G;
    HIPCHK(up(c->g.src, G.e_src, st));
    HIPCHK(up(c->g.dst, G.e_dst, st));
    HIPCHK(up(c->g.in_ptr, G.in_ptr, st));
    HIPCHK(up(c->g.out_ptr, G.out_ptr, st));
    HIPCHK(up(c->g.out_list, G.out_list, st));
    HIPCHK(up(c->g.inc_ptr, G.inc_ptr, st));
    HIPCHK(up(c->g.inc_list, G.inc_list, st));
    HIPCHK(up(c->g.nfdof, A.mesh.fdof, st));
  }
  HIPCHK(up(c->d_elems, A.mesh.elems, st));
  HIPCHK(up(c->d_efdof, c->efdof, st));
  HIPCHK(up(c->d_rest, A.mesh.rest, st));
  HIPCHK(up(c->d_fext, c->fext_free, st));
  HIPCHK(up(c->d_tdof, c->target_dof, st));
  HIPCHK(up(c->d_tval, c->target_val, st));
  HIPCHK(up(c->d_pref, c->p_ref, st));
  HIPCHK(up(c->d_seg_x, c->seg_x, st));
  HIPCHK(up(c->d_seg_p, c->seg_p, st));
  HIPCHK(hipStreamSynchronize(st));
  c->has_ws = true;
  return SGN_OK;
}

sgn_status sgn_set_targets(sgn_ctx c, const double* h_tval, double ell) {
  TRY(check_ready(c));
  if (!h_tval || !(ell > 0)) return fail(c, SGN_E_ARG, "targets");
  TRY(drop_graph(c));  // the captured right-hand side holds ell and mu by value
  c->target_val.assign(h_tval, h_tval + c->target_dof.size());
  c->ell = ell;
  c->mu_reg = c->A.mesh.param_kind == SGN_P_REST_POS ? c->mu_in / (ell * ell) : c->mu_in;
  HIPCHK(up(c->d_tval, c->target_val, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

sgn_status sgn_equilibrium(sgn_ctx c, const double* d_p, double* d_x, sgn_eq_info* info) {
  TRY(check_ready(c));
  if (!d_p || !d_x) return fail(c, SGN_E_ARG, "null state");
  sgn_status s = equilibrium_impl(c, d_p, d_x, info);
  if (s != SGN_OK) return fail(c, s, c->err);
  return SGN_OK;
}

sgn_status sgn_assemble(sgn_ctx c, const double* d_x, const double* d_p, double* d_rhs, double* d_grad,
                        double* h_obj) {
  TRY(check_ready(c));
  if (!d_x || !d_p) return fail(c, SGN_E_ARG, "null state");
  sgn_status s = assemble_impl(c, d_x, d_p, d_rhs, d_grad, h_obj);
  if (s != SGN_OK) return fail(c, s, c->err);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, SGN_E_HIP, hipGetErrorString(e));
  return SGN_OK;
}

sgn_status sgn_block_step(sgn_ctx c, const double* d_x, const double* d_p, double* d_sol, sgn_solve_info* info) {
  TRY(check_ready(c));
  if (!d_x || !d_p || !d_sol) return fail(c, SGN_E_ARG, "null vector");
  if (c->opt.solver != SGN_BLOCK_GN) return fail(c, SGN_E_STATE, "the context was not created with SGN_BLOCK_GN");
  sgn_status s = assemble_impl(c, d_x, d_p, nullptr, nullptr, nullptr);
  if (s != SGN_OK) return fail(c, s, c->err);
  const int64_t nx = c->A.mesh.n_x;
  launch_fill(nx, 0.0, c->d_fx, c->stream);
  launch_objective_fx((int64_t)c->target_dof.size(), c->d_tdof, c->d_tval, d_x, c->target_w / (c->ell * c->ell),
                      c->d_fx, c->stream);
  return bgn_solve_assembled(c, d_x, d_p, d_sol, info);
}

sgn_status sgn_factor(sgn_ctx c, sgn_factor_info* info) {
  TRY(check_ready(c));
  return sgn_factor_impl(c, info);
}

sgn_status sgn_solve(sgn_ctx c, const double* d_rhs, double* d_sol, sgn_solve_info* info) {
  TRY(check_ready(c));
  if (!d_rhs || !d_sol) return fail(c, SGN_E_ARG, "null vector");
  return sgn_solve_impl(c, d_rhs, d_sol, info);
}

sgn_status sgn_step(sgn_ctx c, double* d_p, double* d_x, sgn_step_info* info) {
  TRY(check_ready(c));
  if (!d_p || !d_x) return fail(c, SGN_E_ARG, "null state");
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  sgn_step_info si{};
  double t0 = now_ms();
  const bool kkt = c->opt.rhs_kind == SGN_RHS_KKT;
  if (!c->kx_valid) {
    sgn_status s = equilibrium_impl(c, d_p, d_x, nullptr);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  double f0 = 0;
  double* rhs = c->d_srhs;
  double* sol = c->d_ssol;
  {
    sgn_status s = assemble_impl(c, d_x, d_p, rhs, kkt ? nullptr : c->d_g, &f0);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  double t1 = now_ms();
  si.ms_rhs = 0;
  si.ms_assemble = t1 - t0;
  if (c->opt.solver == SGN_MINRES_LEARNED) {
    sgn_status s = minres_solve_impl(c, rhs, sol, &si.solve);
    if (s != SGN_OK) return s;
  } else if (c->opt.solver != SGN_BLOCK_GN) {
    sgn_factor_info fi{};
    sgn_status s = sgn_factor_impl(c, &fi);
    if (s != SGN_OK) return s;
  }
  double t2 = now_ms();
  si.ms_factor = t2 - t1;
  if (c->opt.solver == SGN_BLOCK_GN) {
    sgn_status s = bgn_solve_assembled(c, d_x, d_p, sol, &si.solve);
    if (s != SGN_OK) return s;
  } else if (c->opt.solver != SGN_MINRES_LEARNED) {
    sgn_status s = sgn_solve_impl(c, rhs, sol, &si.solve);
    if (s != SGN_OK) return s;
  }
  double t3 = now_ms();
  si.ms_solve = t3 - t2;
  // slope g^T dp: adjoint form from g; KKT form as df/dx dx + df/dp dp, equal because the step
  // satisfies Kx dx + Kp dp = 0 and g = df/dp^T + Kp^T lam with Kx^T lam = -df/dx^T
  double v[2];
  if (kkt) {
    dev_dot(c, nx, c->d_fx, sol, 12);
    dev_dot(c, np, c->d_fp, sol + nx, 13);
    sgn_status s = read_scalars(c, 12, 2, v);
    if (s != SGN_OK) return s;
    v[0] += v[1];
    v[1] = -1.0;
  } else {
    dev_dot(c, np, c->d_g, sol + nx, 12);
    dev_dot(c, np, c->d_g, c->d_g, 13);
    sgn_status s = read_scalars(c, 12, 2, v);
    if (s != SGN_OK) return s;
  }
  const double gtdp = v[0];
  si.grad_norm = v[1] >= 0.0 ? std::sqrt(v[1]) : -1.0;
  si.gtdp = gtdp;
  si.f0 = f0;
  return line_search(c, d_p, d_x, sol + nx, t3, &si, info);
}

// Sparse Newton step with inertia control (Sec. 4 "Generalization to Arbitrary Objectives", eq.
// totalHessian; Appendix A, Theorem 2; Sec. 5, the inertia test and diagonal regularisation): the
// saddle-point matrix with the Lagrangian Hessian at the adjoint multipliers is factorised, and while
// its inertia is not (n_x + n_p, n_x, 0) (or a pivot had to be perturbed) delta is added to the x and
// p diagonal and it is factorised again: delta = 0 first, then kNewtonDelta0 (or a third of the last
// step's delta, at least kNewtonDeltaMin), growing eightfold up to kNewtonDeltaMax.  The step solves
// the regularised system with the adjoint right-hand side; the line search is the outer one.
constexpr double kNewtonDelta0 = 1e-4, kNewtonDeltaMin = 1e-20, kNewtonDeltaMax = 1e20;

sgn_status sgn_newton_step(sgn_ctx c, double* d_p, double* d_x, int restart, sgn_step_info* info) {
  TRY(check_ready(c));
  if (!d_p || !d_x) return fail(c, SGN_E_ARG, "null state");
  if (!c->A.newton) return fail(c, SGN_E_STATE, "sgn_newton_step needs a context created with hessian = SGN_HESSIAN_NEWTON");
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  if (restart) c->newton_delta_last = 0.0;
  sgn_step_info si{};
  double t0 = now_ms();
  if (!c->kx_valid) {
    sgn_status s = equilibrium_impl(c, d_p, d_x, nullptr);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  double f0 = 0;
  double* rhs = c->d_srhs;
  double* sol = c->d_ssol;
  {
    sgn_status s = assemble_impl(c, d_x, d_p, rhs, c->d_g, &f0);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  double t1 = now_ms();
  si.ms_assemble = t1 - t0;
  const System& S = c->A.sgn;
  DevSys& D = c->sys[0];
  const double tol = D.prec ? 1e-12 : 1e-14;
  double delta = 0.0;
  const double first = c->newton_delta_last > 0.0 ? std::max(kNewtonDeltaMin, c->newton_delta_last / 3.0) : kNewtonDelta0;
  for (int trial = 1;; ++trial) {
    if (trial > 1) {  // the matrix of this delta from the element buffer: same arithmetic every trial
      launch_gather_slots((int64_t)S.colind.size(), D.slot_ptr, D.slot_src, c->d_ebuf, D.vals, c->stream);
      launch_diag_add(S.N, D.rowptr, D.diag_kind, c->target_w / (c->ell * c->ell), c->mu_reg, 0.0, 0.0, D.vals,
                      c->stream);
      launch_diag_add(S.N, D.rowptr, D.diag_kind, 0.0, delta, delta, 0.0, D.vals, c->stream);
      D.current = false;
    }
    sgn_factor_info fi{};
    sgn_status s = factor_dispatch(c, 0, tol, &fi);
    if (s != SGN_OK) return fail(c, s, c->err);
    si.inertia_trials = trial;
    if (fi.n_pos == nx + np && fi.n_neg == nx && fi.n_zero == 0 && fi.n_perturbed == 0) break;
    delta = trial == 1 ? first : delta * 8.0;
    if (delta > kNewtonDeltaMax) return fail(c, SGN_E_PIVOT, "no diagonal regularisation up to 1e20 gives the inertia of a minimum");
  }
  if (delta > 0.0) c->newton_delta_last = delta;
  si.delta = delta;
  HIPCHK(hipMemcpyAsync(c->d_x_fac, d_x, nx * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_p_fac, d_p, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double t2 = now_ms();
  si.ms_factor = t2 - t1;
  {
    sgn_status s = sgn_solve_impl(c, rhs, sol, &si.solve);
    if (s != SGN_OK) return s;
  }
  double t3 = now_ms();
  si.ms_solve = t3 - t2;
  double v[2];
  dev_dot(c, np, c->d_g, sol + nx, 12);
  dev_dot(c, np, c->d_g, c->d_g, 13);
  TRY(read_scalars(c, 12, 2, v));
  si.gtdp = v[0];
  si.grad_norm = std::sqrt(v[1]);
  si.f0 = f0;
  return line_search(c, d_p, d_x, sol + nx, t3, &si, info);
}

sgn_status sgn_lbfgs_step(sgn_ctx c, double* d_p, double* d_x, int restart, sgn_step_info* info) {
  TRY(check_ready(c));
  if (!d_p || !d_x) return fail(c, SGN_E_ARG, "null state");
  if (c->A.newton) return fail(c, SGN_E_STATE, "L-BFGS is initialised with the Gauss-Newton Hessian (hessian = SGN_HESSIAN_GN)");
  if (c->opt.solver != SGN_LDLT && c->opt.solver != SGN_BICGSTAB)
    return fail(c, SGN_E_STATE, "L-BFGS applies its initial inverse Hessian by the direct solve (SGN_LDLT or SGN_BICGSTAB)");
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p, N = c->A.sgn.N;
  const int m = c->opt.lbfgs_m;
  hipStream_t st = c->stream;
  if (restart) {
    c->lb_count = 0;
    c->lb_head = 0;
    c->lb_have_prev = false;
  }
  sgn_step_info si{};
  const double t0 = now_ms();
  if (!c->kx_valid) {
    sgn_status s = equilibrium_impl(c, d_p, d_x, nullptr);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  // gradient g (adjoint form, eq. totalGradient) and K_SGN at the iterate
  double f0 = 0;
  {
    const int keep = c->opt.rhs_kind;
    c->opt.rhs_kind = SGN_RHS_ADJOINT;
    sgn_status s = assemble_impl(c, d_x, d_p, c->d_srhs, c->d_g, &f0);
    c->opt.rhs_kind = keep;
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  const double t1 = now_ms();
  si.ms_assemble = t1 - t0;
  {
    sgn_factor_info fi{};
    sgn_status s = sgn_factor_impl(c, &fi);
    if (s != SGN_OK) return s;
  }
  const double t2 = now_ms();
  si.ms_factor = t2 - t1;
  // curvature pair of the previous step, kept when s^T y > 1e-12 |s| |y|
  if (c->lb_have_prev && m > 0) {
    double* sn = c->lb_s + (int64_t)c->lb_head * np;
    double* yn = c->lb_y + (int64_t)c->lb_head * np;
    launch_axpby(np, 1.0, d_p, -1.0, c->lb_pprev, sn, st);
    launch_axpby(np, 1.0, c->d_g, -1.0, c->lb_gprev, yn, st);
    dev_dot(c, np, sn, yn, 50);
    dev_dot(c, np, sn, sn, 51);
    dev_dot(c, np, yn, yn, 52);
    double v[3];
    TRY(read_scalars(c, 50, 3, v));
    if (v[0] > 1e-12 * std::sqrt(std::max(v[1], 0.0) * std::max(v[2], 0.0))) {
      c->lb_rho[c->lb_head] = 1.0 / v[0];
      c->lb_head = (c->lb_head + 1) % m;
      c->lb_count = std::min(c->lb_count + 1, m);
    }
  }
  // two-loop recursion (newest pair first, then oldest first) around H0 q = H_GN^-1 q, which is the
  // parameter block of the saddle-point solve with right-hand side [0; q; 0] (eq. sparseSystemGN with
  // -g replaced by q)
  HIPCHK(hipMemcpyAsync(c->lb_q, c->d_g, np * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<double> alpha(c->lb_count);
  for (int k = 0; k < c->lb_count; ++k) {
    const int i = (c->lb_head - 1 - k + 2 * m) % m;
    dev_dot(c, np, c->lb_s + (int64_t)i * np, c->lb_q, 53);
    double sq;
    TRY(read_scalars(c, 53, 1, &sq));
    alpha[k] = c->lb_rho[i] * sq;
    launch_axpby(np, 1.0, c->lb_q, -alpha[k], c->lb_y + (int64_t)i * np, c->lb_q, st);
  }
  launch_fill(N, 0.0, c->d_srhs, st);
  HIPCHK(hipMemcpyAsync(c->d_srhs + nx, c->lb_q, np * sizeof(double), hipMemcpyDeviceToDevice, st));
  {
    sgn_status s = sgn_solve_impl(c, c->d_srhs, c->d_ssol, &si.solve);
    if (s != SGN_OK) return s;
  }
  HIPCHK(hipMemcpyAsync(c->lb_r, c->d_ssol + nx, np * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (int k = c->lb_count - 1; k >= 0; --k) {
    const int i = (c->lb_head - 1 - k + 2 * m) % m;
    dev_dot(c, np, c->lb_y + (int64_t)i * np, c->lb_r, 53);
    double yr;
    TRY(read_scalars(c, 53, 1, &yr));
    const double beta = c->lb_rho[i] * yr;
    launch_axpby(np, 1.0, c->lb_r, alpha[k] - beta, c->lb_s + (int64_t)i * np, c->lb_r, st);
  }
  double* dir = c->lb_q;  // -H g
  launch_axpby(np, -1.0, c->lb_r, 0.0, nullptr, dir, st);
  dev_dot(c, np, c->d_g, dir, 54);
  dev_dot(c, np, c->d_g, c->d_g, 55);
  double v[2];
  TRY(read_scalars(c, 54, 2, v));
  const double t3 = now_ms();
  si.ms_solve = t3 - t2;
  HIPCHK(hipMemcpyAsync(c->lb_pprev, d_p, np * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(c->lb_gprev, c->d_g, np * sizeof(double), hipMemcpyDeviceToDevice, st));
  c->lb_have_prev = true;
  si.f0 = f0;
  si.gtdp = v[0];
  si.grad_norm = std::sqrt(std::max(v[1], 0.0));
  return line_search(c, d_p, d_x, dir, t3, &si, info);
}

sgn_status sgn_batch_create(int n, const sgn_problem* const* probs, const sgn_options* opt, void* stream,
                            sgn_ctx* out) {
  if (!out) return SGN_E_ARG;
  *out = nullptr;
  if (n < 1 || !probs) return SGN_E_ARG;
  for (int i = 0; i < n; ++i) {
    const sgn_problem* q = probs[i];
    if (!q || q->n_components > 1 || q->n_nodes <= 0 || q->n_elems <= 0 || (q->dim != 2 && q->dim != 3))
      return SGN_E_ARG;
    if (!q->rest_pos || !q->elems || !q->node_grid || !q->fixed || !q->f_ext) return SGN_E_ARG;
    if (q->n_targets < 0 || (q->n_targets > 0 && !q->target_dof)) return SGN_E_ARG;
    const sgn_problem* f = probs[0];
    if (q->dim != f->dim || q->param_kind != f->param_kind || q->E0 != f->E0 || q->nu != f->nu ||
        q->target_w != f->target_w || q->reg_mu != f->reg_mu)
      return SGN_E_ARG;
  }
  const int d = probs[0]->dim, nv = d + 1;
  std::vector<double> rest, fext, tval, pref;
  std::vector<int32_t> elems, grid, tdof, cptr{0};
  std::vector<uint8_t> fixed;
  double ell = 0.0;
  int64_t node_off = 0, x_off = 0;
  for (int i = 0; i < n; ++i) {
    const sgn_problem* q = probs[i];
    const int64_t nn = q->n_nodes;
    int64_t nfree = 0;
    for (int64_t v = 0; v < nn; ++v) nfree += q->fixed[v] ? 0 : 1;
    const int64_t nxq = nfree * d;
    const int64_t npq = q->param_kind == SGN_P_LOGE ? q->n_elems : nxq;
    rest.insert(rest.end(), q->rest_pos, q->rest_pos + nn * d);
    fext.insert(fext.end(), q->f_ext, q->f_ext + nn * d);
    grid.insert(grid.end(), q->node_grid, q->node_grid + nn * d);
    fixed.insert(fixed.end(), q->fixed, q->fixed + nn);
    for (int64_t k = 0; k < (int64_t)q->n_elems * nv; ++k) {
      const int32_t v = q->elems[k];
      if (v < 0 || v >= nn) return SGN_E_ARG;
      elems.push_back((int32_t)(v + node_off));
    }
    for (int t = 0; t < q->n_targets; ++t) {
      if (q->target_dof[t] < 0 || q->target_dof[t] >= nxq) return SGN_E_ARG;
      tdof.push_back((int32_t)(q->target_dof[t] + x_off));
      tval.push_back(q->target_val ? q->target_val[t] : 0.0);
    }
    for (int64_t k = 0; k < npq; ++k) pref.push_back(q->p_ref ? q->p_ref[k] : 0.0);
    ell = std::max(ell, q->length_scale);
    node_off += nn;
    x_off += nxq;
    cptr.push_back((int32_t)node_off);
    if (node_off > INT32_MAX / 2) return SGN_E_ARG;
  }
  sgn_problem u = *probs[0];
  u.n_nodes = (int)node_off;
  u.n_elems = (int)(elems.size() / nv);
  u.rest_pos = rest.data();
  u.elems = elems.data();
  u.node_grid = grid.data();
  u.fixed = fixed.data();
  u.f_ext = fext.data();
  u.n_targets = (int)tdof.size();
  u.target_dof = tdof.data();
  u.target_val = tval.data();
  u.length_scale = ell > 0 ? ell : 1.0;
  u.p_ref = pref.data();
  u.n_components = n;
  u.component_ptr = cptr.data();
  return sgn_create(&u, opt, stream, out);
}

sgn_status sgn_batch_step(sgn_ctx c, double* const* d_p, double* const* d_x, sgn_step_info* info) {
  TRY(check_ready(c));
  if (!c->batch_ok) return fail(c, SGN_E_STATE, "parameters are not stored problem by problem (sgn_batch_create does)");
  if (c->opt.solver != SGN_LDLT && c->opt.solver != SGN_BICGSTAB)
    return fail(c, SGN_E_STATE, "the batched step uses the direct solve (SGN_LDLT or SGN_BICGSTAB)");
  const int nc = c->ncomp;
  if (!d_p || !d_x) return fail(c, SGN_E_ARG, "null state arrays");
  for (int k = 0; k < nc; ++k)
    if (!d_p[k] || !d_x[k]) return fail(c, SGN_E_ARG, "null state of a problem");
  const int64_t nx = c->A.mesh.n_x, np = c->A.mesh.n_p;
  hipStream_t st = c->stream;
  const bool kkt = c->opt.rhs_kind == SGN_RHS_KKT;
  const std::vector<int64_t>&sx = c->seg_x, &sp = c->seg_p;
  double* X = c->d_x;
  double* P = c->d_p;
  for (int k = 0; k < nc; ++k) {
    HIPCHK(hipMemcpyAsync(P + sp[k], d_p[k], (sp[k + 1] - sp[k]) * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(X + sx[k], d_x[k], (sx[k + 1] - sx[k]) * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  const double t0 = now_ms();
  // the problems' states are equilibria: the union Newton confirms it (and leaves the Kx factor the
  // adjoint right-hand side needs)
  {
    sgn_status s = equilibrium_impl(c, P, X, nullptr);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  std::vector<double> f0(nc), f1(nc), ft(nc), slope(nc), gn(nc, -1.0), alpha(nc, 1.0);
  std::vector<int> done(nc, 0), halv(nc, 0);
  std::vector<int32_t> mask(nc);
  TRY(batch_objectives(c, X, P, f0.data()));
  {
    sgn_status s = assemble_impl(c, X, P, c->d_srhs, kkt ? nullptr : c->d_g, nullptr);
    if (s != SGN_OK) return fail(c, s, c->err);
  }
  const double t1 = now_ms();
  {
    sgn_factor_info fi{};
    sgn_status s = sgn_factor_impl(c, &fi);
    if (s != SGN_OK) return s;
  }
  const double t2 = now_ms();
  sgn_solve_info sinfo{};
  {
    sgn_status s = sgn_solve_impl(c, c->d_srhs, c->d_ssol, &sinfo);
    if (s != SGN_OK) return s;
  }
  const double t3 = now_ms();
  const double* dx = c->d_ssol;
  const double* dp = c->d_ssol + nx;
  // per-problem slopes g^T dp (KKT form: df/dx dx + df/dp dp, equal since Kx dx + Kp dp = 0)
  {
    std::vector<double> v(3 * (size_t)nc);
    if (kkt) {
      launch_segment_dot(nc, c->d_seg_x, c->d_fx, dx, c->d_seg_val, st);
      launch_segment_dot(nc, c->d_seg_p, c->d_fp, dp, c->d_seg_val + nc, st);
    } else {
      launch_fill(nc, 0.0, c->d_seg_val, st);
      launch_segment_dot(nc, c->d_seg_p, c->d_g, dp, c->d_seg_val + nc, st);
      launch_segment_dot(nc, c->d_seg_p, c->d_g, c->d_g, c->d_seg_val + 2 * nc, st);
    }
    HIPCHK(hipMemcpyAsync(v.data(), c->d_seg_val, (kkt ? 2 : 3) * nc * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < nc; ++k) {
      slope[k] = v[k] + v[nc + k];
      if (!kkt) gn[k] = std::sqrt(std::max(v[2 * nc + k], 0.0));
    }
  }
  // backtracking per problem, all trials of a round in one union equilibrium: problems already
  // accepted keep their step and state (kept in d_old2 and restored before every round)
  double* xacc = c->d_old2;
  int nt_iters = 0;
  // the host mask is rewritten for the next use only after the stream has consumed it
  auto upload_mask = [&](auto pred) -> hipError_t {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int k = 0; k < nc; ++k) mask[k] = pred(k) ? 1 : 0;
    return hipMemcpyAsync(c->d_seg_mask, mask.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, st);
  };
  for (int h = 0; h <= c->opt.max_halvings; ++h) {
    HIPCHK(hipMemcpyAsync(c->d_seg_alpha, alpha.data(), nc * sizeof(double), hipMemcpyHostToDevice, st));
    launch_segment_axpy(nc, c->d_seg_p, c->d_seg_alpha, P, dp, c->d_pt, st);
    HIPCHK(upload_mask([&](int k) { return done[k] == 0; }));
    launch_segment_copy(nc, c->d_seg_x, c->d_seg_mask, X, c->d_xt, st);
    HIPCHK(upload_mask([&](int k) { return done[k] != 0; }));
    launch_segment_copy(nc, c->d_seg_x, c->d_seg_mask, xacc, c->d_xt, st);
    sgn_eq_info ei{};
    const sgn_status s = equilibrium_impl(c, c->d_pt, c->d_xt, &ei);
    if (s == SGN_E_HIP) return fail(c, s, c->err);
    if (s == SGN_OK) {
      nt_iters += ei.iters;
      TRY(batch_objectives(c, c->d_xt, c->d_pt, ft.data()));
      for (int k = 0; k < nc; ++k)
        if (!done[k] && ft[k] <= f0[k] + 1e-4 * alpha[k] * slope[k]) {
          done[k] = 3;  // accepted in this round
          f1[k] = ft[k];
        }
      HIPCHK(upload_mask([&](int k) { return done[k] == 3; }));
      launch_segment_copy(nc, c->d_seg_x, c->d_seg_mask, c->d_xt, xacc, st);
      for (int k = 0; k < nc; ++k)
        if (done[k] == 3) done[k] = 1;
    }
    if (std::all_of(done.begin(), done.end(), [](int v) { return v != 0; })) break;
    if (h == c->opt.max_halvings) break;
    HIPCHK(hipStreamSynchronize(st));  // the uploaded step lengths are consumed before they change
    for (int k = 0; k < nc; ++k)
      if (!done[k]) {
        alpha[k] *= 0.5;
        ++halv[k];
      }
  }
  c->kx_valid = false;  // the last equilibrium was of a trial state
  bool failed = false;
  for (int k = 0; k < nc; ++k)
    if (!done[k]) {
      if (std::fabs(slope[k]) <= 1e-12 * std::fabs(f0[k])) {
        done[k] = 2;  // stationary to working precision: stays (alpha = 0), as sgn_step
        alpha[k] = 0.0;
        f1[k] = f0[k];
      } else {
        failed = true;
      }
    }
  const double t4 = now_ms();
  if (info)
    for (int k = 0; k < nc; ++k) {
      sgn_step_info& o = info[k];
      o = sgn_step_info{};
      o.alpha = done[k] ? alpha[k] : 0.0;
      o.f0 = f0[k];
      o.f1 = done[k] ? f1[k] : f0[k];
      o.grad_norm = gn[k];
      o.gtdp = slope[k];
      o.halvings = halv[k];
      o.newton_iters = nt_iters;
      o.ms_assemble = t1 - t0;
      o.ms_factor = t2 - t1;
      o.ms_solve = t3 - t2;
      o.ms_linesearch = t4 - t3;
      o.solve = sinfo;
    }
  if (failed) return fail(c, SGN_E_LINESEARCH, "line search failed for a problem of the batch");
  // final states: accepted problems at their trial, stationary ones where they were
  HIPCHK(hipMemcpyAsync(c->d_seg_alpha, alpha.data(), nc * sizeof(double), hipMemcpyHostToDevice, st));
  launch_segment_axpy(nc, c->d_seg_p, c->d_seg_alpha, P, dp, c->d_pt, st);
  HIPCHK(upload_mask([&](int k) { return done[k] == 1; }));
  launch_segment_copy(nc, c->d_seg_x, c->d_seg_mask, xacc, c->d_xt, st);
  HIPCHK(upload_mask([&](int k) { return done[k] == 2; }));
  launch_segment_copy(nc, c->d_seg_x, c->d_seg_mask, X, c->d_xt, st);
  for (int k = 0; k < nc; ++k) {
    HIPCHK(hipMemcpyAsync(d_p[k], c->d_pt + sp[k], (sp[k + 1] - sp[k]) * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(d_x[k], c->d_xt + sx[k], (sx[k + 1] - sx[k]) * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  (void)np;
  return SGN_OK;
}

sgn_status sgn_set_pc_correction(sgn_ctx c, const float* d_corr_node, const float* d_corr_par) {
  TRY(check_ready(c));
  c->corr_node = d_corr_node;
  c->corr_par = d_corr_par;
  c->pc_weights = nullptr;
  c->use_own = false;
  return SGN_OK;
}

sgn_status sgn_spmv(sgn_ctx c, const double* d_in, double* d_out) {
  TRY(check_ready(c));
  if (!d_in || !d_out || d_in == d_out) return fail(c, SGN_E_ARG, "sgn_spmv needs distinct vectors");
  if (!c->sgn_assembled) return fail(c, SGN_E_STATE, "sgn_spmv before sgn_assemble");
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_gather_perm(N, D.perm, nullptr, d_in, c->d_old2, c->stream);
  launch_spmv(D.row_lanes, N, D.frowptr, D.fcol, D.fslot, D.vals, c->d_old2, c->d_old, c->stream);
  launch_scatter_perm(N, D.perm, nullptr, c->d_old, d_out, c->stream);
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

sgn_status sgn_pc_apply(sgn_ctx c, const double* d_in, double* d_out, double* d_fwd) {
  if (c && c->opt.pc_kind == SGN_PC_BLOCK) {
    TRY(check_ready(c));
    if (!c->sgn_assembled) return fail(c, SGN_E_STATE, "the block-diagonal preconditioner needs sgn_assemble");
    if (!c->sys[0].bp_ready) TRY(blockpc_setup(c));
  } else {
    TRY(pc_ready(c));
  }
  if (!d_in || !d_out) return fail(c, SGN_E_ARG, "null vector");
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_fill_i32(1, 0, c->d_cnt + 12, c->stream);
  launch_gather_perm(N, D.perm, nullptr, d_in, c->d_old2, c->stream);
  TRY(pc_apply_new(c, c->d_old2, c->d_old, d_fwd));
  launch_scatter_perm(N, D.perm, nullptr, c->d_old, d_out, c->stream);
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (timeout) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
  return SGN_OK;
}

sgn_status sgn_pc_forward(sgn_ctx c, const double* d_in, double* d_fwd) {
  TRY(pc_ready(c));
  if (!d_in || !d_fwd) return fail(c, SGN_E_ARG, "null vector");
  DevSys& D = c->sys[0];
  const int64_t N = c->A.sgn.N;
  launch_fill_i32(1, 0, c->d_cnt + 12, c->stream);
  launch_gather_perm(N, D.perm, nullptr, d_in, c->d_old2, c->stream);
  TRY(pc_forward_new(c, c->d_old2, d_fwd));
  int timeout = 0;
  HIPCHK(hipMemcpyAsync(&timeout, c->d_cnt + 12, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (timeout) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
  return SGN_OK;
}

sgn_status sgn_pc_grad(sgn_ctx c, const double* d_fwd_a, const double* d_fwd_b, double weight, float* d_grad_node,
                       float* d_grad_par) {
  TRY(pc_ready(c));
  if (!d_fwd_a || !d_fwd_b) return fail(c, SGN_E_ARG, "null vector");
  launch_pc_grad(pc_args(c), d_fwd_a, d_fwd_b, weight, d_grad_node, d_grad_par, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

sgn_status sgn_solve_minres(sgn_ctx c, const double* d_rhs, double* d_sol, sgn_solve_info* info) {
  TRY(check_ready(c));
  if (!d_rhs || !d_sol || d_rhs == d_sol) return fail(c, SGN_E_ARG, "sgn_solve_minres needs distinct vectors");
  return minres_solve_impl(c, d_rhs, d_sol, info);
}

sgn_status sgn_gnn_num_weights(sgn_ctx c, int64_t* n) {
  if (!c || !n) return SGN_E_ARG;
  *n = c->G.n_weights;
  return SGN_OK;
}

sgn_status sgn_gnn_init(sgn_ctx c, float* d_w, uint64_t seed) {
  TRY(check_ready(c));
  if (!d_w) return fail(c, SGN_E_ARG, "null weights");
  std::vector<float> w;
  gnn_init_weights(c->G, seed, w);
  HIPCHK(hipMemcpyAsync(d_w, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

sgn_status sgn_gnn_forward(sgn_ctx c, const float* d_w, const double* d_x_ref, const double* d_p_ref,
                           const double* d_x, const double* d_p, float* d_corr_node, float* d_corr_par) {
  TRY(check_ready(c));
  if (!d_w || !d_x_ref || !d_p_ref || !d_x || !d_p || !d_corr_node || !d_corr_par)
    return fail(c, SGN_E_ARG, "null argument");
  return gnn_forward_impl(c, d_w, d_x_ref, d_p_ref, d_x, d_p, d_corr_node, d_corr_par);
}

sgn_status sgn_gnn_backward(sgn_ctx c, const float* d_w, const float* d_gcorr_node, const float* d_gcorr_par,
                            float* d_gw) {
  TRY(check_ready(c));
  if (!d_w || !d_gw) return fail(c, SGN_E_ARG, "null argument");
  if (!c->gnn_fwd_done) return fail(c, SGN_E_STATE, "sgn_gnn_backward before sgn_gnn_forward");
  return gnn_backward_impl(c, d_w, d_gcorr_node, d_gcorr_par, d_gw);
}

sgn_status sgn_adam(int64_t n, float* d_w, const float* d_g, float* d_m, float* d_v, float lr, float beta1,
                    float beta2, float eps, int step, void* stream) {
  if (n < 0 || (n > 0 && (!d_w || !d_g || !d_m || !d_v)) || step < 1) return SGN_E_ARG;
  launch_adam(n, d_w, d_g, d_m, d_v, lr, beta1, beta2, eps, step, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return SGN_E_HIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SGN_E_HIP;
  return SGN_OK;
}

sgn_status sgn_set_pc_weights(sgn_ctx c, const float* d_w) {
  TRY(check_ready(c));
  c->pc_weights = d_w;
  c->use_own = false;
  return SGN_OK;
}

sgn_status sgn_pc_train_loss(sgn_ctx c, const float* d_w, const double* d_probes, int n_probes, int log_form,
                             float* d_gw, double* h_loss) {
  TRY(pc_ready(c));
  if (!c->sgn_assembled) return fail(c, SGN_E_STATE, "sgn_pc_train_loss before sgn_assemble");
  if (!d_w || !d_probes || n_probes < 1 || !d_gw || !h_loss) return fail(c, SGN_E_ARG, "invalid argument");
  const bool keep = c->use_own;
  sgn_status s = pc_train_loss_impl(c, d_w, d_probes, n_probes, log_form, d_gw, h_loss);
  c->use_own = keep && c->pc_weights;
  return s;
}

sgn_status sgn_graph_step(sgn_ctx c, const double* d_x, const double* d_p, double* d_rhs, double* d_sol, int n_ir,
                          double* h_rel) {
  TRY(check_ready(c));
  if (!d_x || !d_p || !d_rhs || !d_sol || n_ir < 0 || n_ir > 16) return fail(c, SGN_E_ARG, "invalid argument");
  if (c->A.newton) return fail(c, SGN_E_STATE, "the captured step assembles the Gauss-Newton form");
  hipStream_t user = c->stream;
  if (!c->gstream) HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  const void* key[4] = {d_x, d_p, d_rhs, d_sol};
  const bool same = c->graph_exec && c->graph_nir == n_ir && std::equal(key, key + 4, c->graph_key);
  HIPCHK(hipStreamSynchronize(user));  // inputs written on the caller's stream are complete
  if (!same) {
    if (c->graph_exec) HIPCHK(hipGraphExecDestroy(c->graph_exec));
    if (c->graph) HIPCHK(hipGraphDestroy(c->graph));
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->stream = c->gstream;
    c->capturing = true;
    if (c->opt.profile) {  // create the update events before capture; their records become graph nodes
      size_t need = 0;
      for (const LevelPlan& P : c->A.sgn.levels)
        for (const PanelStep& ps : P.steps)
        need += 2 * ((ps.upd_tiles > 0) + (ps.outer_tiles > 0) + (ps.far_tiles > 0));
      hipError_t e0 = ensure_events(c, need);
      if (e0 != hipSuccess) {
        c->capturing = false;
        c->stream = user;
        return fail(c, SGN_E_HIP, std::string("events: ") + hipGetErrorString(e0));
      }
    }
    sgn_status s = SGN_OK;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      s = enqueue_step(c, d_x, d_p, d_rhs, d_sol, n_ir);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(c->gstream, &g);
      if (e == hipSuccess) e = e2;
      c->graph = g;
    }
    c->capturing = false;
    c->stream = user;
    c->graph_prof = c->opt.profile != 0;
    if (s != SGN_OK) return s;
    if (e != hipSuccess) return fail(c, SGN_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    HIPCHK(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    std::copy(key, key + 4, c->graph_key);
    c->graph_nir = n_ir;
  }
  const double t0 = now_ms();
  HIPCHK(hipGraphLaunch(c->graph_exec, c->gstream));
  double out[2];
  int cnt[16];
  HIPCHK(hipMemcpyAsync(out, c->d_scal + 32, 2 * sizeof(double), hipMemcpyDeviceToHost, c->gstream));
  HIPCHK(hipMemcpyAsync(cnt, c->d_cnt, 16 * sizeof(int), hipMemcpyDeviceToHost, c->gstream));
  HIPCHK(hipStreamSynchronize(c->gstream));
  c->stats.solve_ms = now_ms() - t0;
  if (c->graph_prof) {
    hipStream_t keep = c->stream;
    c->stream = c->gstream;
    const sgn_status s = read_update_events(c);
    c->stream = keep;
    TRY(s);
  }
  c->sys[0].factored = true;
  c->sys[0].current = true;
  c->sgn_assembled = true;
  if (h_rel) *h_rel = out[0];
  if (cnt[12]) return fail(c, SGN_E_HIP, "a pipelined triangular solve timed out waiting for a panel");
  if (cnt[8] > 0) {
    c->err = "inverted element in the given state";
    return SGN_E_INVERTED;
  }
  if (out[1] != 1.0) {
    char buf[96];
    snprintf(buf, sizeof(buf), "fixed refinement stopped at equilibrated relative residual %.3e", out[0]);
    c->err = buf;
    return SGN_E_REFINE;
  }
  return SGN_OK;
}

sgn_status sgn_get_sizes(sgn_ctx c, int which, int64_t* n, int64_t* nnz, int64_t* nsn, int64_t* fe, double* fl) {
  if (!c || (which != 0 && which != 1)) return SGN_E_ARG;
  const System& S = which == 0 ? c->A.sgn : c->A.kx;
  if (n) *n = S.N;
  if (nnz) *nnz = (int64_t)S.colind.size();
  if (nsn) *nsn = S.nsn;
  if (fe) *fe = S.factor_entries;
  if (fl) *fl = S.flops;
  return SGN_OK;
}

sgn_status sgn_get_symbolic(sgn_ctx c, int which, int32_t* perm, int32_t* etree, int64_t* rowptr, int32_t* colind) {
  if (!c || (which != 0 && which != 1)) return SGN_E_ARG;
  const System& S = which == 0 ? c->A.sgn : c->A.kx;
  if (perm) std::memcpy(perm, S.perm.data(), bytes_of(S.perm));
  if (etree) std::memcpy(etree, S.etree.data(), bytes_of(S.etree));
  if (rowptr) std::memcpy(rowptr, S.rowptr.data(), bytes_of(S.rowptr));
  if (colind) std::memcpy(colind, S.colind.data(), bytes_of(S.colind));
  return SGN_OK;
}

sgn_status sgn_get_values(sgn_ctx c, int which, double* h_vals) {
  TRY(check_ready(c));
  if (!h_vals || (which != 0 && which != 1)) return fail(c, SGN_E_ARG, "values");
  const System& S = which == 0 ? c->A.sgn : c->A.kx;
  HIPCHK(hipMemcpyAsync(h_vals, c->sys[which].vals, S.colind.size() * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return SGN_OK;
}

sgn_status sgn_selftest_mfma(int prec, const double* d_a, const double* d_b, double* d_out, void* stream) {
  if (!d_a || !d_b || !d_out || (prec != 0 && prec != 1)) return SGN_E_ARG;
  launch_mfma_probe(prec, d_a, d_b, d_out, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return SGN_E_HIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SGN_E_HIP;
  return SGN_OK;
}

sgn_status sgn_get_stats(sgn_ctx c, sgn_stats* out) {
  if (!c || !out) return SGN_E_ARG;
  *out = c->stats;
  return SGN_OK;
}

const char* sgn_last_error(sgn_ctx c) {
  if (!c) return "null context";
  return c->err.c_str();
}

namespace {

// One candidate of the autotuner: a context of its own at (d_x, d_p); wall milliseconds per round of
// assembly + factorisation + solve (right-hand side of ones), best of `reps` rounds after a warm-up.
sgn_status time_candidate(const sgn_problem* prob, const sgn_options& o, const double* d_x, const double* d_p,
                          int reps, void* stream, double* ms) {
  sgn_ctx c = nullptr;
  sgn_status st = sgn_create(prob, &o, stream, &c);
  void* ws = nullptr;
  double *rhs = nullptr, *sol = nullptr;
  auto done = [&](sgn_status r) {
    if (ws) (void)hipFree(ws);
    if (rhs) (void)hipFree(rhs);
    if (sol) (void)hipFree(sol);
    sgn_destroy(c);
    return r;
  };
  if (st != SGN_OK) return done(st);
  size_t bytes = 0;
  if ((st = sgn_workspace_size(c, &bytes)) != SGN_OK) return done(st);
  const int64_t N = c->A.sgn.N;
  if (hipMalloc(&ws, bytes) != hipSuccess || hipMalloc((void**)&rhs, N * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&sol, N * sizeof(double)) != hipSuccess)
    return done(SGN_E_NOMEM);
  if ((st = sgn_set_workspace(c, ws, bytes)) != SGN_OK) return done(st);
  launch_fill(N, 1.0, rhs, c->stream);
  double best = 1e300;
  for (int r = 0; r <= reps; ++r) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return done(SGN_E_HIP);
    const double t0 = now_ms();
    if ((st = sgn_assemble(c, d_x, d_p, nullptr, nullptr, nullptr)) != SGN_OK) return done(st);
    if ((st = sgn_factor(c, nullptr)) != SGN_OK) return done(st);
    if ((st = sgn_solve(c, rhs, sol, nullptr)) != SGN_OK) return done(st);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return done(SGN_E_HIP);
    const double t = now_ms() - t0;
    if (r > 0 && t < best) best = t;  // round 0 warms up
  }
  *ms = best;
  return done(SGN_OK);
}

}  // namespace

sgn_status sgn_autotune(const sgn_problem* prob, const sgn_options* base, const double* d_x, const double* d_p,
                        int reps, void* stream, sgn_options* best, double* h_ms, int* n_cand) {
  if (!prob || !base || !d_x || !d_p || !best || reps < 1 || reps > 100) return SGN_E_ARG;
  sgn_options cur = *base;
  int nc = 0;
  double cur_ms = 0.0;
  sgn_status st = time_candidate(prob, cur, d_x, d_p, reps, stream, &cur_ms);
  if (st != SGN_OK) return st;
  constexpr int kRecorded = 24;  // entries of h_ms the caller provides
  if (h_ms) h_ms[nc] = cur_ms;
  ++nc;
  auto consider = [&](const sgn_options& cand) -> sgn_status {
    double ms = 0.0;
    const sgn_status s = time_candidate(prob, cand, d_x, d_p, reps, stream, &ms);
    if (s != SGN_OK) return s;
    if (h_ms && nc < kRecorded) h_ms[nc] = ms;
    ++nc;
    if (ms < 0.99 * cur_ms) {  // a candidate must beat the incumbent by 1%
      cur = cand;
      cur_ms = ms;
    }
    return SGN_OK;
  };
  static const int kSpans[] = {1, 2, 4, 8, 16};
  static const int kSeq[] = {-1, 2, 4, 8};
  for (int b = 0; b < kTuneBuckets; ++b) {
    const int inc = cur.outer_panels[b] == 0 ? kOuterPanels : cur.outer_panels[b];
    for (int v : kSpans) {
      if (v == inc) continue;
      sgn_options cand = cur;
      cand.outer_panels[b] = v;
      if ((st = consider(cand)) != SGN_OK) return st;
    }
  }
  {
    const int inc = cur.seq_panels == 0 ? kSolveSeqPanels : cur.seq_panels;
    for (int v : kSeq) {
      if (v == inc) continue;
      sgn_options cand = cur;
      cand.seq_panels = v;
      if ((st = consider(cand)) != SGN_OK) return st;
    }
  }
  {
    static const int kWaves[] = {0, 8, 4};  // 0: by each launch's panel count
    const int inc = cur.panel_waves;
    for (int v : kWaves) {
      if (v == inc) continue;
      sgn_options cand = cur;
      cand.panel_waves = v;
      if ((st = consider(cand)) != SGN_OK) return st;
    }
  }
  *best = cur;
  if (n_cand) *n_cand = nc;
  return SGN_OK;
}

void sgn_destroy(sgn_ctx c) { delete c; }

}  // extern "C"
