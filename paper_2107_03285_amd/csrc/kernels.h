// Launchers of the gfx950 kernels (all asynchronous on the given stream).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sgn {

constexpr int kRedBlocks = 1024;  // fixed partition of deterministic reductions
constexpr int kUpdTile = 64;      // edge of the trailing-update tile (the symbolic schedule counts these tiles)
constexpr int kUpdGroup = 8;      // column tiles per group of the trailing update's tile order

// Tile lt of a trailing update over R row tiles and ct <= R column tiles (tile (i, j) for j < ct,
// j <= i < R; ct R - ct (ct - 1) / 2 tiles): column tiles go in groups of kUpdGroup, and a group's
// tiles run row by row, so the tiles of one row (sharing their L rows) run side by side and the
// group's W columns serve every row.  Full groups J' before group J hold
// G (G + 1) / 2 + (R - G J' - G) G tiles each.  Returns false past the last tile.
__host__ __device__ inline bool update_tile(int64_t lt, int64_t R, int64_t ct, int64_t& i, int64_t& j) {
  constexpr int64_t G = kUpdGroup;
  if (lt < 0) return false;
  int64_t g0 = 0;  // first column tile of the group
  for (;;) {
    if (g0 >= ct) return false;
    const int64_t w = ct - g0 < G ? ct - g0 : G;
    const int64_t n = w * (w + 1) / 2 + (R - g0 - w) * w;
    if (lt < n) {
      const int64_t head = w * (w + 1) / 2;
      int64_t d;
      if (lt < head) {
        d = 0;
        while ((d + 1) * (d + 2) / 2 <= lt) ++d;
        j = g0 + (lt - d * (d + 1) / 2);
      } else {
        d = w + (lt - head) / w;
        j = g0 + (lt - head) % w;
      }
      i = g0 + d;
      return i < R;
    }
    lt -= n;
    g0 += G;
  }
}

// ---------------------------------------------------------------- element + assembly
struct ElemArgs {
  int dim, ne, param_kind, mode;  // mode 0 energy, 1 energy+gradient, 2 + Hessian (+ Kp), 3 + Newton terms
  const int32_t* elems;           // [ne*(dim+1)]
  const int32_t* efdof;           // [ne*(dim+1)] free DOF of each element node, -1 fixed
  const double* rest;             // [n_nodes*dim]
  const double* x;                // [n_x]
  const double* p;                // [n_p]
  double mu0, lam0;
  double* ebuf;
  int stride, off_grad, off_kp, off_energy;
  int* inverted;                  // counter of elements with J <= 0
  const double* lam;              // mode 3: multipliers [n_x] (free-DOF order)
  int off_t, off_kl, off_lg;      // mode 3: d2(lam.g)/dx2, K lam, lam.g in the element buffer
};
void launch_element(const ElemArgs& a, hipStream_t s);
// vals[t] = sum of ebuf[src] over the slot's sources (fixed order)
void launch_gather_slots(int64_t nnz, const int64_t* ptr, const int32_t* src, const double* ebuf,
                         double* vals, hipStream_t s);
// vals[diag(i)] += diag value of var kind; plus constant slots (nodal-force Kp)
void launch_diag_add(int64_t N, const int64_t* rowptr, const int32_t* kind, double a_target, double c_param,
                     double eps_x, double eps_lambda, double* vals, hipStream_t s);
void launch_const_slots(int64_t n, const int64_t* slots, double value, double* vals, hipStream_t s);
// out[i] += sign e_i z[i], e the stabilisation diagonal (eps_x on x, -eps_lambda on lambda, 0 on parameters)
void launch_unstabilise(int64_t N, const int32_t* kind, double eps_x, double eps_lambda, double sign, const double* z,
                        double* out, hipStream_t s);
// c[i] = sum(ebuf[src]) - fext[i] - (pforce ? p[i] : 0)
void launch_gather_vec(int64_t n, const int64_t* ptr, const int32_t* src, const double* ebuf,
                       const double* fext, const double* pforce, double* out, hipStream_t s);
// deterministic reductions: partials[kRedBlocks], then a single-block final sum
void launch_dot_partials(int64_t n, const double* a, const double* b, int64_t stride_a, int absval, double* partials,
                         hipStream_t s);
void launch_final_sum(const double* partials, int np, double* out, hipStream_t s);
void launch_max_abs_partials(int64_t n, const double* a, double* partials, hipStream_t s);
void launch_final_max(const double* partials, int np, double* out, hipStream_t s);

// per-segment operations on batches (segment s = [off[s], off[s+1]), one block each, nseg <= 65535):
// out[s] = sum a b over the segment; out = x + alpha[s] dir; dst = src where mask[s] != 0
void launch_segment_dot(int nseg, const int64_t* off, const double* a, const double* b, double* out, hipStream_t s);
void launch_segment_axpy(int nseg, const int64_t* off, const double* alpha, const double* x, const double* dir,
                         double* out, hipStream_t s);
void launch_segment_copy(int nseg, const int64_t* off, const int32_t* mask, const double* src, double* dst,
                         hipStream_t s);

// ---------------------------------------------------------------- vectors / permutations
// out[k] = scale[k] * in[perm[k]] (scale may be null)
void launch_gather_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out,
                        hipStream_t s);
// out[perm[k]] = scale[k] * in[k] (scale may be null)
void launch_scatter_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out,
                         hipStream_t s);
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t s);
// w += sign * sum_{t < j} coef[t] V[t * ldv + .] (coef on the device)
void launch_multi_axpy(int64_t n, int j, const double* V, int64_t ldv, const double* coef, double sign, double* w,
                       hipStream_t s);
void launch_fill(int64_t n, double v, double* out, hipStream_t s);
// out = s .* in (elementwise; out may alias in)
void launch_scale(int64_t n, const double* s, const double* in, double* out, hipStream_t st);
void launch_fill_bytes(int64_t nbytes, void* out, hipStream_t s);
// out[0] = sqrt(r2 / b2), out[1] = (out[0] <= rtol): a device-side convergence flag
void launch_rel_flag(const double* r2, const double* b2, double rtol, double* out, hipStream_t s);
// out[0 .. n) = v (32-bit words; a kernel, so it may sit in a captured graph where memset nodes may not)
void launch_fill_i32(int64_t n, int32_t v, void* out, hipStream_t s);
// lanes per row (4, 8 or 16) of the row kernels below for a matrix of N rows and nnz stored entries in
// its full CSR
int row_lanes_for(int64_t N, int64_t nnz);
// y = K x with the symmetric matrix stored as lower slots and addressed through the full CSR
void launch_spmv(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot,
                 const double* vals, const double* x, double* y, hipStream_t s);
// out = b - K x
void launch_residual(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot,
                     const double* vals, const double* x, const double* b, double* out, hipStream_t s);
// scale[i] = 1 / sqrt(max_j |K_ij|) over the full row (1 when the row is empty)
// block-diagonal preconditioner: per node group (grp_ptr, new numbering) |B_i|^-1 of the diagonal block B_i
// of S K S (S = scale) stored densely at minv + off[i]; apply: out = S blockdiag(|B_i|^-1) S in
void launch_blockpc_setup(int64_t ngroups, const int32_t* grp_ptr, const int64_t* rowptr, const int32_t* colind,
                          const double* vals, const double* scale, const int64_t* off, double* minv, hipStream_t s);
void launch_blockpc_apply(int64_t ngroups, const int32_t* grp_ptr, const double* scale, const int64_t* off,
                          const double* minv, const double* in, double* out, hipStream_t s);
void launch_row_scaling(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fslot, const double* vals,
                        double* scale, hipStream_t s);
// objective pieces on free DOFs: fx = w (x_T - t)/ell^2 on targets (else 0)
void launch_objective_fx(int64_t nt, const int32_t* tdof, const double* tval, const double* x, double w_over_ell2,
                         double* fx, hipStream_t s);

// ---------------------------------------------------------------- factorisation
struct FrontArgs {
  const int32_t* sn_begin;
  const int32_t* sn_m;
  const int64_t* sn_front_off;
  const int64_t* sn_rows_ptr;
  const int32_t* sn_rows;
  const int64_t* relmap_off;
  const int32_t* relmap;
  const int32_t* var_group_end;
  double* dpiv;      // [N] diagonal of D
  double* epiv;      // [N] off-diagonal of a 2x2 block (stored at its first index)
  int32_t* pivtype;  // [N] 0 = 1x1, 1 = first of 2x2, 2 = second of 2x2
  int32_t* lperm;    // [N] local pivot order: position -> original local index
  int* counters;     // [0] perturbed pivots
  double piv_tol;
};
template <typename T>
void launch_csr_to_fronts(int64_t nnz, const int32_t* slot_row, const int32_t* colind, const int64_t* pos,
                          const double* vals, const double* scale, T* front, hipStream_t s);
// zeroes rows >= column - 63 of every front (the lower triangle and a band above the diagonal);
// ntasks (sn, first column) pairs
template <typename T>
void launch_zero_fronts(int64_t ntasks, const int32_t* tasks, const FrontArgs& f, T* front, hipStream_t s);
// Extend-add of whole small children (u <= kSmallChild), one block each: kids holds 5 int64 per
// child (see System::ea_kid_recs).
template <typename T>
void launch_extend_add_small(int64_t nkids, const int64_t* kids, const FrontArgs& f, T* front, hipStream_t s);
template <typename T>
void launch_extend_add(int64_t ncols, const int64_t* cols, const FrontArgs& f, T* front, hipStream_t s);
template <typename T>
void launch_panel_diag(int64_t ntasks, int max_w, int waves, const int64_t* tasks, const FrontArgs& f, T* front,
                       hipStream_t s);
template <typename T>
void launch_panel_trsm(int64_t ntasks, int64_t max_rows, const int64_t* tasks, const FrontArgs& f, T* front,
                       hipStream_t s);
template <typename T>
void launch_update(int64_t ntasks, int64_t ntiles, const int64_t* tasks, const int32_t* tile_task,
                   const FrontArgs& f, T* front, hipStream_t s);
// inertia: counts[0..2] += (pos, neg, zero); minabs via partial mins
void launch_inertia(int64_t N, const double* dpiv, const double* epiv, const int32_t* pivtype,
                    unsigned long long* counts, double* minabs_partials, hipStream_t s);

// ---------------------------------------------------------------- solves
struct SolveArgs {
  FrontArgs f;
  const int32_t* child_ptr;
  const int32_t* child_list;
  const int64_t* sn_vec_off;
  const int32_t* panel_ptr;
  const int32_t* panel_col;
  const int64_t* sn_part_off;
  double* part;  // split-k partial sums of L21 y
  double* tv;  // per-front accumulation vectors
  double* tp;  // per-front permuted working vectors
  const double* wd;  // null: the backward solve applies D^-1; else it takes D^-1 y from here (pivot order)
};
// One tree level of the forward / backward solve.  tasks: (front, panel) pairs, one per panel of
// each front of the level (the block serves the front, the panel comes from the front's ticket);
// counter: zeroed per-front ticket counters [nsn]; err: set when a bounded wait runs out.
template <typename T>
void launch_fwd_level(int64_t nsn, int64_t max_u, int64_t max_s, const int32_t* level_sn, const int32_t* tasks, int64_t ntasks,
                      const SolveArgs& a, const T* front, const double* b, int* counter, int* err, hipStream_t s);
template <typename T>
void launch_bwd_level(int64_t nsn, int64_t max_s, const int32_t* level_sn, const int32_t* tasks, int64_t ntasks,
                      const SolveArgs& a, const T* front, double* x, int* counter, int* err, hipStream_t s);
// The same level step for fronts of one panel (s <= 64) and u = m - s <= kOneMaxU, one wavefront each:
// forward gather, permutation, unit lower solve and contribution vector; backward D^-1 y (or wd),
// the rows-below product and the transposed unit lower solve.
template <typename T>
void launch_fwd_one(int64_t n, const int32_t* fronts, const SolveArgs& a, const T* front, const double* b,
                    hipStream_t s);
template <typename T>
void launch_bwd_one(int64_t n, const int32_t* fronts, const SolveArgs& a, const T* front, double* x, hipStream_t s);

// ---------------------------------------------------------------- node-block preconditioner
struct PcArgs {
  int64_t ngroups;
  int dim;
  int64_t nx;
  const int32_t* grp_ptr;    // [ngroups+1] first pivot position of each node group
  const int32_t* grp_node;   // [ngroups] mesh node of the group
  const int64_t* grp_vec;    // [ngroups] solve-vector index of the group's first position
  const int32_t* perm;       // new -> old variable (owned parameter positions -> parameter id)
  const double* dpiv;
  const double* epiv;
  const int32_t* pivtype;
  const float* corr_node;    // [n_nodes * (2d)(2d+1)/2] raw lower-triangular corrections, or null
  const float* corr_par;     // [n_p] raw parameter corrections, or null
};
// w = B^-1 y per node group (y from the forward solve's vectors tp; ysave: optional flat copy of y)
void launch_pc_block(const PcArgs& a, const double* tp, double* ysave, double* w, hipStream_t s);
// gn, gp += weight * d(ya^T B^-1 yb)/d(raw corrections)
void launch_pc_grad(const PcArgs& a, const double* ya, const double* yb, double weight, float* gn, float* gp,
                    hipStream_t s);
// halves of B^-1 = (R C)^-T (R C)^-1: u = C^-1 R^-1 y (y from tp), w = R^-T C^-T v (flat, pivot order)
void launch_pc_half_fwd(const PcArgs& a, const double* tp, double* u, hipStream_t s);
void launch_pc_half_bwd(const PcArgs& a, const double* v, double* w, hipStream_t s);
// gn, gp += weight * d(x^T T y)/d(raw corrections), T = (RC)^-1 L^-1 P S K S P^T L^-T (RC)^-T
void launch_pc_sym_grad(const PcArgs& a, const double* x, const double* ty, const double* y, const double* tx,
                        double weight, float* gn, float* gp, hipStream_t s);
// out = a x + b y + c z (y, z may be null)
void launch_lincomb3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* z,
                     double* out, hipStream_t s);

// ---------------------------------------------------------------- preconditioner network (FP32)
struct DenseSeg {
  const float* src;     // row r of the segment: src[(idx ? idx[r] : r) * ld + 0 .. width)
  const int32_t* idx;
  int width, ld;
};
struct DenseArgs {
  int64_t rows;
  DenseSeg seg[3];
  int nseg, K;          // K = sum of segment widths (<= 192)
  const float* W;       // [K x N] row-major, bias [N] right after
  int N;                // outputs (<= 64)
  int act;              // 1: tanh, 0: identity
  const float* res;     // optional residual added to the output
  int ld_res;
  float* out;
  int ld_out;
  float* ysave;         // optional [rows x N] activation outputs (for the backward pass)
};
struct GnnFeatArgs {
  int64_t n_nodes, n_edges;
  int dim, param_kind;
  const int32_t* nfdof;     // [n_nodes] first free DOF, -1 fixed
  const double* rest;       // [n_nodes * dim]
  const double* x;          // current state [n_x]
  const double* x_ref;      // reference state [n_x]
  const double* p;          // [n_p]
  const double* p_ref;      // [n_p]
  const int32_t* inc_ptr;   // node -> elements
  const int32_t* inc_list;
  double ell, hbar;
};
void launch_dense_fwd(const DenseArgs& a, hipStream_t s);
void launch_dense_bwd(const DenseArgs& a, const float* dout, int ld_dout, const float* y, float* dz, float* dx,
                      hipStream_t s);
int wgrad_parts(int64_t rows);
// gw[(K+1) x N] += sum over rows of [x_r; 1] dz_r^T (part: wgrad_parts(rows) * (K+1) * N floats)
void launch_dense_wgrad(const DenseArgs& a, const float* dz, float* part, float* gw, hipStream_t s);
// dst[v, 0:width] += scale * sum_{k in [ptr[v], ptr[v+1])} src[list ? list[k] : k, col : col + width]
// (without ptr: the single row v; divide_by_count: mean instead of sum)
void launch_gather_add(int64_t nv, const int32_t* ptr, const int32_t* list, const float* src, int ld_src, int col,
                       int width, float scale, int divide_by_count, float* dst, int ld_dst, hipStream_t s);
// dE[e, :] += dagg[dst_e, col : col + 64] / deg(dst_e)
void launch_edge_mean_bwd(int64_t ne, const int32_t* dst, const int32_t* in_ptr, const float* dagg, int ld, int col,
                          float* dE, hipStream_t s);
void launch_elem_mean(int64_t ne, int nv, const int32_t* elems, const float* h, float* emb, hipStream_t s);
void launch_gnn_features(const GnnFeatArgs& a, const int32_t* src, const int32_t* dst, float* nf, float* ef,
                         hipStream_t s);
void launch_split_out(int64_t n_nodes, int tri, int nout, int d, int per_node_params, const int32_t* nfdof,
                      const float* dec, float* cn, float* cp, hipStream_t s);
void launch_split_bwd(int64_t n_nodes, int tri, int nout, int d, int per_node_params, const int32_t* nfdof,
                      const float* gcn, const float* gcp, float* ddec, hipStream_t s);
void launch_add_f32(int64_t n, const float* src, float* dst, hipStream_t s);
void launch_fill_f32(int64_t n, float v, float* dst, hipStream_t s);
void launch_scale_f32(int64_t n, float a, float* dst, hipStream_t s);
void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 int t, hipStream_t s);

// ---------------------------------------------------------------- self test
// C(16x16) = A(16x4) B(4x16) on one MFMA; out holds D row-major (double or float)
void launch_mfma_probe(int prec, const double* a, const double* b, double* out, hipStream_t s);

}  // namespace sgn
