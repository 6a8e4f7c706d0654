// Host-side symbolic analysis of the SGN saddle-point system and of the
// Kx system used by the Newton equilibrium solve.  Plain C++17, no HIP: it
// runs once per mesh (the sparsity pattern is fixed) and produces the tables
// the device kernels consume.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sgn {

constexpr int kPanel = 64;        // panel width of the blocked front factorisation
constexpr int kNarrowPanel = 32;  // panels this narrow are listed first in each step's task range,
constexpr int kMediumPanel = 48;  // then those of at most this many columns
constexpr int kOneMaxU = 128;     // one-panel fronts with at most this many rows below the pivots are
constexpr int kOneMaxM = kPanel + kOneMaxU;  // solved by one wavefront each (order <= kOneMaxM) when a
constexpr int kOneMinFronts = 1024;          // level has at least kOneMinFronts of them
constexpr int kSmallChild = 128;  // update blocks up to this order are added by one block per child
constexpr int kZeroWhole = 128;   // fronts up to this order are zeroed whole
constexpr int64_t kZeroRun = 16384;  // entries of consecutive whole-zeroed fronts one block zeroes (>= kZeroWhole^2)
constexpr int kOuterPanels = 4;   // panels per delayed trailing update (k = 256)
constexpr int kTile = 64;         // update tile edge (equal to the kernels' kUpdTile)
constexpr int kSolveKC = 256;     // k-chunk of the split-k L21 y product in the forward solve
constexpr int kSolveSeqPanels = 8;  // fronts with at most this many panels are solved by one block

enum SystemKind { SYS_SGN = 0, SYS_KX = 1 };

// Blocking choices of the schedule that leave the mathematics unchanged (tuned per problem family):
// fronts fall in buckets by their order m (below kTuneBucketEdge[0], below kTuneBucketEdge[1], the
// rest); each bucket delays the trailing update beyond a block of outer_panels panels; fronts with
// at most seq_panels panels are solved by one block.
constexpr int kTuneBuckets = 3;
constexpr int64_t kTuneBucketEdge[kTuneBuckets - 1] = {1024, 4096};
struct Tuning {
  int outer_panels[kTuneBuckets] = {kOuterPanels, kOuterPanels, kOuterPanels};
  int seq_panels = kSolveSeqPanels;
  int panel_waves = 0;  // wavefronts per panel factorisation: 1, 8, or 0 (by the step's panel count)
};
inline int tune_bucket(int64_t m) {
  int b = 0;
  while (b < kTuneBuckets - 1 && m >= kTuneBucketEdge[b]) ++b;
  return b;
}

struct Mesh {
  int dim = 0, n_nodes = 0, n_elems = 0;
  std::vector<double> rest;       // [n_nodes*dim]
  std::vector<int32_t> elems;     // [n_elems*(dim+1)]
  std::vector<int32_t> grid;      // [n_nodes*dim]
  std::vector<uint8_t> fixed;     // [n_nodes]
  std::vector<double> fext;       // [n_nodes*dim]
  std::vector<int32_t> comp_ptr;  // node ranges of independent components ({0, n_nodes} for one)
  int param_kind = 0;
  // derived
  std::vector<int32_t> fdof;      // node -> first free DOF (-1 fixed)
  int64_t n_x = 0, n_p = 0;
};

// One launch of the blocked front factorisation: all fronts of one tree level
// that have a panel with index `panel`.
struct PanelStep {
  int64_t task_begin, task_end;    // range in the panel task table
  int64_t upd_begin, upd_end;      // range in the update task table (inner, k = one panel)
  int64_t outer_begin, outer_end;  // range in the update task table (outer, k = block): the next
                                   // block's columns, which its panels need next
  int64_t far_begin, far_end;      // range in the update task table (outer, k = block): the columns
                                   // beyond the next block, free to run beside its panels
  int64_t upd_tiles, outer_tiles, far_tiles;  // tiles of each update launch
  int64_t upd_map, outer_map, far_map;        // where each launch's tiles start in the tile -> task map
  int64_t narrow_end;              // tasks [task_begin, narrow_end) have at most kNarrowPanel columns,
  int64_t medium_end;              // [narrow_end, medium_end) at most kMediumPanel
  int64_t trsm_rows;               // max rows below the panel over the step's tasks
  double upd_flops, outer_flops, far_flops;   // algorithmic flops of the update launches
};

struct LevelPlan {
  int64_t sn_begin, sn_end;            // range in level_sn (supernodes of this level)
  int max_children;                    // extend-add rounds
  std::vector<int64_t> ea_work;                    // per round: child columns (children past kSmallChild)
  std::vector<int64_t> ea_col_begin;               // per round: its first column record in ea_cols
  std::vector<int64_t> ea_kids, ea_kid_begin;      // per round: children of u <= kSmallChild, first record
  std::vector<PanelStep> steps;
  int64_t max_m = 0, max_s = 0, max_u = 0;
  // solves: solve_sn[sn_begin, one_begin) are solved by the level kernels (solve_max_s, solve_max_u
  // over them), solve_sn[one_begin, sn_end) are one-panel fronts solved by one wavefront each
  int64_t one_begin = 0, solve_max_s = 0, solve_max_u = 0;
  int64_t fwd_begin = 0, fwd_end = 0;  // range (pairs) in solve_fwd_tasks: panels ascending per front
  int64_t bwd_begin = 0, bwd_end = 0;  // range (pairs) in solve_bwd_tasks: panels descending per front
};

struct System {
  int kind = SYS_SGN;
  int64_t N = 0;
  std::vector<int32_t> perm, iperm;      // perm[new] = old
  std::vector<int64_t> rowptr;           // lower CSR, new numbering
  std::vector<int32_t> colind;
  std::vector<int32_t> slot_row;         // row of every lower CSR entry
  std::vector<int32_t> etree;
  // full (both triangles) CSR for the symmetric SpMV: column and lower slot
  std::vector<int64_t> frowptr;
  std::vector<int32_t> fcol, fslot;
  // pivot groups (BK pivoting is restricted to a group), new numbering
  std::vector<int32_t> var_group_end;    // per var: end (exclusive) of its group
  // node groups of the SGN system (owned parameters, x_v, lambda_v of one free node), in elimination
  // order: first position, mesh node, and the solve-vector index of the first position
  std::vector<int32_t> grp_ptr;          // [n_free+1]
  std::vector<int32_t> grp_node;         // [n_free]
  std::vector<int64_t> grp_vec;          // [n_free]
  // supernodes (contiguous pivot ranges)
  int nsn = 0;
  std::vector<int32_t> sn_begin;         // [nsn+1]
  std::vector<int64_t> sn_rows_ptr;      // [nsn+1]
  std::vector<int32_t> sn_rows;          // struct rows, ascending
  std::vector<int32_t> sn_parent, sn_level;
  std::vector<int32_t> sn_m;
  std::vector<int64_t> sn_front_off;     // element offset of the m x m column-major front
  std::vector<int64_t> sn_vec_off;       // element offset of the length-m solve vector
  std::vector<int64_t> sn_part_off;      // offset of the split-k partial sums of L21 y (u * ceil(s / kSolveKC))
  int64_t part_total = 0;
  std::vector<int64_t> relmap_off;       // [nsn+1] into relmap
  std::vector<int32_t> relmap;           // struct row r of child -> index in parent front
  std::vector<int32_t> child_ptr, child_list;
  std::vector<int32_t> var_sn;           // supernode of each var
  std::vector<int64_t> csr_front_pos;    // per lower CSR entry: element offset in its front
  int64_t front_total = 0, vec_total = 0;
  std::vector<int32_t> fill_tasks;       // (sn, first column) pairs: 64-column groups of the fronts
  // panels: per supernode a list of local column starts (last = s)
  std::vector<int32_t> panel_ptr;        // [nsn+1]
  std::vector<int32_t> panel_col;        // local starts, with a terminating s per sn
  // schedule
  int nlevels = 0;
  std::vector<int32_t> level_sn;         // supernodes grouped by level
  std::vector<int32_t> solve_sn;         // the same per level, one-panel fronts with u <= kOneMaxU last (in
                                         // levels with at least kOneMinFronts of them)
  std::vector<LevelPlan> levels;
  // task tables (flattened int64 quintuples, see kernels)
  std::vector<int64_t> panel_tasks;      // (sn, c0, c1) per task: 3 entries
  std::vector<int64_t> upd_tasks;        // (sn, k0, k1, cb, ce, tile_prefix): 6 entries
  std::vector<int32_t> upd_tile_task;    // per update tile: its task, counted from its launch's first
  // per child column c of a round, 4 entries: front offset of the child's entry (sC, sC + c) (the
  // column's rows c.. follow), front offset of the parent column it adds into, offset of the child's
  // relative map, (c << 32) | uC
  std::vector<int64_t> ea_cols;
  // per small child of a round, 5 entries: front offset of its entry (sC, sC), front offset of the
  // parent, offset of its relative map, mC, (mP << 32) | uC
  std::vector<int64_t> ea_kid_recs;
  std::vector<int32_t> solve_fwd_tasks;  // (sn, panel index) pairs, per level; (sn, -1): whole front in one block
  std::vector<int32_t> solve_bwd_tasks;
  int64_t n_panels = 0;                  // total panels (ready flags of the pipelined solves)
  // element -> lower CSR slot contributions and their inverse (gather) map
  int elem_stride = 0;                   // values per element in the element buffer
  std::vector<int64_t> slot_ptr;         // [nnz+1]
  std::vector<int32_t> slot_src;         // element-buffer index e*stride + k
  std::vector<int32_t> diag_kind;        // per var (new): 0 none, 1 target x, 2 param, 3 x, 4 lambda
  // vector gather of the residual c (KX only): per x dof, element-buffer sources
  std::vector<int64_t> vec_ptr;
  std::vector<int32_t> vec_src;
  double flops = 0;                      // dense front work of one factorisation
  int64_t factor_entries = 0;            // sum m*s
  int max_front = 0;
};

// Position of value j of element e in the element buffer: values grouped by g (the spatial
// dimension), groups major, elements next, the g values of a group innermost.  The element kernel's
// stores of one group stay coalesced across elements, and the assembly gather, whose neighbouring
// CSR slots take the x, y (, z) values of one element entry, reads them from one cache line.
inline int64_t ebuf_index(int64_t j, int64_t e, int64_t n_elems, int g) {
  return ((j / g) * n_elems + e) * g + j % g;
}

struct Analysis {
  Mesh mesh;
  Tuning tune;
  // Newton form of the saddle-point system (Appendix A; log-modulus parameters only): the objective's
  // blocks plus the second derivatives of lambda^T c, so the x-x block takes the Kx pattern, the x-p
  // block the Kp pattern and the p-p diagonal the element term; false: the Gauss-Newton pattern
  bool newton = false;
  std::vector<int64_t> node_order;  // free nodes in ND order
  System sgn, kx;
  // element buffer layout: values in groups of dim (the coordinates of one node), group-major:
  // value j of element e at ebuf_index(j, e, n_elems, dim); stride is padded to a multiple of dim
  int nd = 0;              // dofs per element (d+1)*d
  int off_hess = 0, off_grad = 0, off_kp = 0, off_energy = 0, stride = 0;
  // Newton form only (else -1): d2(lam.g_e)/dx2 [nd*nd], K_e lam_e [nd] (= d2(lam.g_e)/dx dp_e for
  // log-modulus parameters) and lam_e.g_e (= d2(lam.g_e)/dp_e2)
  int off_t = -1, off_kl = -1, off_lg = -1;
};

// Runs the whole host analysis.  Returns an empty string on success, else an
// error message.
std::string analyse(Analysis& A);

}  // namespace sgn
