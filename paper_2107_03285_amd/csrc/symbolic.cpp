// Host symbolic analysis (see symbolic.h).
//
// The paper hands ordering and symbolic factorisation of the saddle-point
// matrix (eq. sparseSystemGN) to its sparse direct solver; the rules here
// are this library's own:
//  * pattern: A diagonal, C = mu I, B = 0, all diagonals kept; Kx holds
//    (lambda_i, x_j) for free DOFs of nodes sharing an element; Kp holds
//    (lambda_i, p_e) (log-modulus), node-pair blocks (rest positions) or
//    (lambda_i, p_i) (nodal forces);
//  * node order: geometric nested dissection on the grid (largest axis,
//    ties to the lowest axis, mid = lo + ext/2; boxes with <= 8 grid points or
//    largest extent <= 2 are emitted lexicographically, axis 0 fastest);
//  * variable order per node: owned parameters, x_v, lambda_v;
//  * supernodes: the nested-dissection tree itself (each leaf box and each
//    separator plane is one front), with pivoting restricted to the
//    variables of one mesh node.  A leading block made of whole node groups
//    is [[A_II, 0, Kx_II^T], [0, C_PP, Kp_IP^T], [Kx_II, Kp_IP, 0]]; it is
//    nonsingular when Kx is SPD and C = mu I > 0, so the restricted
//    factorisation exists.
#include "symbolic.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <stdexcept>

namespace sgn {

namespace {

struct TreeNode {
  int64_t nb = 0, ne = 0;   // range in the node order
  int parent = -1;
  std::vector<int> children;
};

struct NdResult {
  std::vector<int64_t> order;
  std::vector<TreeNode> tree;  // in creation (post) order
};

NdResult nested_dissection(const Mesh& m) {
  const int d = m.dim;
  NdResult R;
  const int ncomp = m.comp_ptr.size() > 1 ? (int)m.comp_ptr.size() - 1 : 1;
  for (int comp = 0; comp < ncomp; ++comp) {
    const int v0 = m.comp_ptr.size() > 1 ? m.comp_ptr[comp] : 0;
    const int v1 = m.comp_ptr.size() > 1 ? m.comp_ptr[comp + 1] : m.n_nodes;
    int shape[3] = {1, 1, 1};
    for (int v = v0; v < v1; ++v)
      for (int a = 0; a < d; ++a) shape[a] = std::max(shape[a], m.grid[(size_t)v * d + a] + 1);
    // grid point -> node id (-1 if none)
    int64_t npts = (int64_t)shape[0] * shape[1] * shape[2];
    std::vector<int32_t> at(npts, -1);
    for (int v = v0; v < v1; ++v) {
      int c[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) c[a] = m.grid[(size_t)v * d + a];
      at[((int64_t)c[2] * shape[1] + c[1]) * shape[0] + c[0]] = v;
    }
    auto emit = [&](const int* lo, const int* hi) {
      int64_t n0 = (int64_t)R.order.size();
      int lo2 = d == 3 ? lo[2] : 0, hi2 = d == 3 ? hi[2] : 1;
      for (int k = lo2; k < hi2; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            int32_t v = at[((int64_t)k * shape[1] + j) * shape[0] + i];
            if (v >= 0 && !m.fixed[v]) R.order.push_back(v);
          }
      return std::make_pair(n0, (int64_t)R.order.size());
    };
    auto make = [&](std::pair<int64_t, int64_t> r, std::vector<int> ch) {
      TreeNode t;
      t.nb = r.first;
      t.ne = r.second;
      t.children = std::move(ch);
      R.tree.push_back(t);
      return (int)R.tree.size() - 1;
    };
    // returns tree node ids that are the roots of this box's subtree
    std::function<std::vector<int>(const int*, const int*)> rec = [&](const int* lo, const int* hi) {
      int ext[3] = {1, 1, 1};
      int64_t prod = 1;
      int mx = 0;
      for (int a = 0; a < d; ++a) {
        ext[a] = hi[a] - lo[a];
        if (ext[a] <= 0) return std::vector<int>();
        prod *= ext[a];
        mx = std::max(mx, ext[a]);
      }
      if (prod <= 8 || mx <= 2) {
        auto r = emit(lo, hi);
        if (r.second == r.first) return std::vector<int>();
        return std::vector<int>{make(r, {})};
      }
      int ax = 0;
      for (int a = 1; a < d; ++a)
        if (ext[a] > ext[ax]) ax = a;
      int mid = lo[ax] + ext[ax] / 2;
      int hi1[3], lo2[3], los[3], his[3];
      for (int a = 0; a < 3; ++a) {
        hi1[a] = hi[a];
        lo2[a] = lo[a];
        los[a] = lo[a];
        his[a] = hi[a];
      }
      hi1[ax] = mid;
      lo2[ax] = mid + 1;
      los[ax] = mid;
      his[ax] = mid + 1;
      std::vector<int> ch = rec(lo, hi1);
      std::vector<int> ch2 = rec(lo2, hi);
      ch.insert(ch.end(), ch2.begin(), ch2.end());
      auto r = emit(los, his);
      if (r.second == r.first) return ch;  // empty separator: pass the subtrees up
      return std::vector<int>{make(r, ch)};
    };
    int lo[3] = {0, 0, 0};
    int hi[3] = {shape[0], shape[1], shape[2]};
    rec(lo, hi);
  }
  for (int t = 0; t < (int)R.tree.size(); ++t)
    for (int c : R.tree[t].children) R.tree[c].parent = t;
  return R;
}

// Liu's elimination tree with path compression on a lower CSR.
std::vector<int32_t> etree_liu(int64_t N, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci) {
  std::vector<int32_t> parent(N, -1), anc(N, -1);
  for (int64_t i = 0; i < N; ++i) {
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      int64_t j = ci[t];
      while (j != -1 && j < i) {
        int64_t nxt = anc[j];
        anc[j] = (int32_t)i;
        if (nxt == -1) parent[j] = (int32_t)i;
        j = nxt;
      }
    }
  }
  return parent;
}

// Build a sorted, unique lower CSR from (row, col) pairs (row >= col).
void build_csr(int64_t N, std::vector<std::pair<int32_t, int32_t>>& pairs, std::vector<int64_t>& rp,
               std::vector<int32_t>& ci) {
  rp.assign(N + 1, 0);
  for (auto& p : pairs) rp[p.first + 1]++;
  for (int64_t i = 0; i < N; ++i) rp[i + 1] += rp[i];
  std::vector<int32_t> tmp(pairs.size());
  std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
  for (auto& p : pairs) tmp[fill[p.first]++] = p.second;
  std::vector<std::pair<int32_t, int32_t>>().swap(pairs);
  std::vector<int64_t> nrp(N + 1, 0);
  int64_t out = 0;
  for (int64_t i = 0; i < N; ++i) {
    auto b = tmp.begin() + rp[i], e = tmp.begin() + rp[i + 1];
    std::sort(b, e);
    auto ue = std::unique(b, e);
    for (auto it = b; it != ue; ++it) tmp[out++] = *it;
    nrp[i + 1] = out;
  }
  tmp.resize(out);
  ci.swap(tmp);
  rp.swap(nrp);
}

inline int64_t find_slot(const System& S, int64_t r, int64_t c) {
  if (r < c) std::swap(r, c);
  auto b = S.colind.begin() + S.rowptr[r], e = S.colind.begin() + S.rowptr[r + 1];
  auto it = std::lower_bound(b, e, (int32_t)c);
  if (it == e || *it != c) return -1;
  return it - S.colind.begin();
}

// 2 k flops per updated lower-triangle entry: columns [cb, ce), rows [c, m)
double update_flops(int64_t m, int64_t cb, int64_t ce, int64_t k) {
  const double n = (double)(ce - cb);
  const double entries = n * (double)m - (double)(cb + ce - 1) * n / 2.0;
  return 2.0 * (double)k * entries;
}

int64_t update_tiles(int64_t m, int64_t cb, int64_t ce) {
  int64_t R = (m - cb + kTile - 1) / kTile;
  int64_t ct = (ce - cb + kTile - 1) / kTile;
  return ct * R - ct * (ct - 1) / 2;
}

// Everything that depends only on (variable order, pattern, tree).
std::string finish_system(System& S, const std::vector<TreeNode>& tree,
                          const std::vector<int64_t>& node_var_begin,   // per order position: first var
                          const std::vector<int64_t>& node_pub_begin,   // per order position: first public var
                          int pub_per_node, const std::vector<std::vector<int64_t>>& node_adj_rank,
                          const Tuning& tune) {
  const int64_t N = S.N;
  S.etree = etree_liu(N, S.rowptr, S.colind);
  S.slot_row.resize(S.colind.size());
  for (int64_t i = 0; i < N; ++i)
    for (int64_t t = S.rowptr[i]; t < S.rowptr[i + 1]; ++t) S.slot_row[t] = (int32_t)i;
  // full CSR
  {
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t i = 0; i < N; ++i)
      for (int64_t t = S.rowptr[i]; t < S.rowptr[i + 1]; ++t) {
        cnt[i + 1]++;
        if (S.colind[t] != i) cnt[S.colind[t] + 1]++;
      }
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    S.frowptr = cnt;
    S.fcol.resize(cnt[N]);
    S.fslot.resize(cnt[N]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < N; ++i)  // lower parts first (ascending rows keep rows sorted)
      for (int64_t t = S.rowptr[i]; t < S.rowptr[i + 1]; ++t) {
        int64_t p = fill[i]++;
        S.fcol[p] = S.colind[t];
        S.fslot[p] = (int32_t)t;
      }
    for (int64_t i = 0; i < N; ++i)
      for (int64_t t = S.rowptr[i]; t < S.rowptr[i + 1]; ++t) {
        int64_t j = S.colind[t];
        if (j == i) continue;
        int64_t p = fill[j]++;
        S.fcol[p] = (int32_t)i;
        S.fslot[p] = (int32_t)t;
      }
  }
  // supernodes from the tree (tree nodes are in post order = variable order)
  const int nt = (int)tree.size();
  S.nsn = nt;
  S.sn_begin.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) {
    S.sn_begin[t] = (int32_t)node_var_begin[tree[t].nb];
    if (t > 0 && S.sn_begin[t] != (int32_t)node_var_begin[tree[t - 1].ne])
      return "supernode ranges are not contiguous";
  }
  S.sn_begin[nt] = (int32_t)node_var_begin[tree[nt - 1].ne];
  if (S.sn_begin[0] != 0 || S.sn_begin[nt] != N) return "supernodes do not cover all variables";
  S.sn_parent.assign(nt, -1);
  for (int t = 0; t < nt; ++t) S.sn_parent[t] = tree[t].parent;
  S.var_sn.assign(N, 0);
  for (int t = 0; t < nt; ++t)
    for (int64_t v = S.sn_begin[t]; v < S.sn_begin[t + 1]; ++v) S.var_sn[v] = t;
  // node-level structure of every supernode (ranks after the supernode)
  std::vector<std::vector<int64_t>> st(nt);
  for (int t = 0; t < nt; ++t) {
    std::vector<int64_t> s;
    for (int64_t q = tree[t].nb; q < tree[t].ne; ++q)
      for (int64_t w : node_adj_rank[q])
        if (w >= tree[t].ne) s.push_back(w);
    for (int c : tree[t].children)
      for (int64_t w : st[c])
        if (w >= tree[t].ne) s.push_back(w);
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    st[t] = std::move(s);
  }
  S.sn_rows_ptr.assign(nt + 1, 0);
  S.sn_m.assign(nt, 0);
  for (int t = 0; t < nt; ++t) {
    int64_t s = S.sn_begin[t + 1] - S.sn_begin[t];
    int64_t u = (int64_t)st[t].size() * pub_per_node;
    S.sn_rows_ptr[t + 1] = S.sn_rows_ptr[t] + u;
    if (s + u > (int64_t)2000000000) return "front too large";
    S.sn_m[t] = (int32_t)(s + u);
  }
  S.sn_rows.resize(S.sn_rows_ptr[nt]);
  for (int t = 0; t < nt; ++t) {
    int64_t p = S.sn_rows_ptr[t];
    for (int64_t w : st[t])
      for (int k = 0; k < pub_per_node; ++k) S.sn_rows[p++] = (int32_t)(node_pub_begin[w] + k);
  }
  // offsets
  S.sn_front_off.assign(nt + 1, 0);
  S.sn_vec_off.assign(nt + 1, 0);
  S.flops = 0;
  S.factor_entries = 0;
  S.max_front = 0;
  for (int t = 0; t < nt; ++t) {
    int64_t m = S.sn_m[t], s = S.sn_begin[t + 1] - S.sn_begin[t], u = m - s;
    S.sn_front_off[t + 1] = S.sn_front_off[t] + ((m * m + 31) / 32) * 32;
    S.sn_vec_off[t + 1] = S.sn_vec_off[t] + ((m + 31) / 32) * 32;
    S.flops += (double)s * s * s / 3.0 + (double)s * s * u + (double)s * u * u;
    S.factor_entries += m * s;
    S.max_front = std::max<int>(S.max_front, (int)m);
  }
  S.sn_part_off.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) {
    int64_t m = S.sn_m[t], sz = S.sn_begin[t + 1] - S.sn_begin[t];
    S.sn_part_off[t + 1] = S.sn_part_off[t] + (m - sz) * ((sz + kSolveKC - 1) / kSolveKC);
  }
  S.part_total = S.sn_part_off[nt];
  S.front_total = S.sn_front_off[nt];
  // zeroing tasks: the lower triangle and the band above the diagonal of every front, 64 columns
  // per task; fronts of order <= kZeroWhole are zeroed whole, consecutive ones (adjacent in memory)
  // together up to kZeroRun entries per task, written (first front, -count)
  S.fill_tasks.clear();
  for (int t = 0; t < nt;) {
    if (S.sn_m[t] <= kZeroWhole) {
      int e = t + 1;
      while (e < nt && S.sn_m[e] <= kZeroWhole && S.sn_front_off[e + 1] - S.sn_front_off[t] <= kZeroRun) ++e;
      S.fill_tasks.push_back(t);
      S.fill_tasks.push_back(-(e - t));
      t = e;
      continue;
    }
    for (int64_t c0 = 0; c0 < S.sn_m[t]; c0 += 64) {
      S.fill_tasks.push_back(t);
      S.fill_tasks.push_back((int32_t)c0);
    }
    ++t;
  }
  S.vec_total = S.sn_vec_off[nt];
  // relative maps child struct -> parent front index
  S.relmap_off.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t) S.relmap_off[t + 1] = S.relmap_off[t] + (S.sn_rows_ptr[t + 1] - S.sn_rows_ptr[t]);
  S.relmap.resize(S.relmap_off[nt]);
  for (int t = 0; t < nt; ++t) {
    int P = S.sn_parent[t];
    int64_t u = S.sn_rows_ptr[t + 1] - S.sn_rows_ptr[t];
    if (P < 0) {
      if (u != 0) return "root supernode with a nonempty structure";
      continue;
    }
    int64_t sP = S.sn_begin[P + 1] - S.sn_begin[P];
    auto pb = S.sn_rows.begin() + S.sn_rows_ptr[P], pe = S.sn_rows.begin() + S.sn_rows_ptr[P + 1];
    for (int64_t r = 0; r < u; ++r) {
      int32_t v = S.sn_rows[S.sn_rows_ptr[t] + r];
      int64_t pos;
      if (v >= S.sn_begin[P] && v < S.sn_begin[P + 1]) {
        pos = v - S.sn_begin[P];
      } else {
        auto it = std::lower_bound(pb, pe, v);
        if (it == pe || *it != v) return "child structure not contained in parent front";
        pos = sP + (it - pb);
      }
      S.relmap[S.relmap_off[t] + r] = (int32_t)pos;
    }
  }
  // CSR entry -> front position
  S.csr_front_pos.resize(S.colind.size());
  for (int64_t i = 0; i < N; ++i)
    for (int64_t t = S.rowptr[i]; t < S.rowptr[i + 1]; ++t) {
      int64_t j = S.colind[t];
      int J = S.var_sn[j];
      int64_t m = S.sn_m[J], s = S.sn_begin[J + 1] - S.sn_begin[J];
      int64_t col = j - S.sn_begin[J], row;
      if (i < S.sn_begin[J + 1]) {
        row = i - S.sn_begin[J];
      } else {
        auto b = S.sn_rows.begin() + S.sn_rows_ptr[J], e = S.sn_rows.begin() + S.sn_rows_ptr[J + 1];
        auto it = std::lower_bound(b, e, (int32_t)i);
        if (it == e || *it != i) return "matrix entry outside its front";
        row = s + (it - b);
      }
      S.csr_front_pos[t] = S.sn_front_off[J] + row + col * m;
    }
  // children in fixed (ascending) order
  S.child_ptr.assign(nt + 1, 0);
  for (int t = 0; t < nt; ++t)
    if (S.sn_parent[t] >= 0) S.child_ptr[S.sn_parent[t] + 1]++;
  for (int t = 0; t < nt; ++t) S.child_ptr[t + 1] += S.child_ptr[t];
  S.child_list.resize(S.child_ptr[nt]);
  {
    std::vector<int32_t> fill(S.child_ptr.begin(), S.child_ptr.end() - 1);
    for (int t = 0; t < nt; ++t)
      if (S.sn_parent[t] >= 0) S.child_list[fill[S.sn_parent[t]]++] = t;
  }
  // panels: greedy packing of pivot groups, never splitting a group
  S.panel_ptr.assign(nt + 1, 0);
  S.panel_col.clear();
  for (int t = 0; t < nt; ++t) {
    int64_t b = S.sn_begin[t], e = S.sn_begin[t + 1];
    int64_t c0 = b;
    S.panel_col.push_back(0);
    int64_t v = b;
    while (v < e) {
      int64_t ge = S.var_group_end[v];
      if (ge - v > kPanel) return "pivot group wider than a panel";
      if (ge - c0 > kPanel) {
        S.panel_col.push_back((int32_t)(v - b));
        c0 = v;
      }
      v = ge;
    }
    S.panel_col.push_back((int32_t)(e - b));
    S.panel_ptr[t + 1] = (int32_t)S.panel_col.size();
  }
  // levels
  S.sn_level.assign(nt, 0);
  for (int t = 0; t < nt; ++t)
    for (int32_t q = S.child_ptr[t]; q < S.child_ptr[t + 1]; ++q)
      S.sn_level[t] = std::max(S.sn_level[t], S.sn_level[S.child_list[q]] + 1);
  S.nlevels = 0;
  for (int t = 0; t < nt; ++t) S.nlevels = std::max(S.nlevels, S.sn_level[t] + 1);
  S.level_sn.clear();
  S.solve_sn.clear();
  S.levels.assign(S.nlevels, LevelPlan());
  S.panel_tasks.clear();
  S.upd_tasks.clear();
  S.upd_tile_task.clear();
  S.ea_cols.clear();
  S.ea_kid_recs.clear();
  S.solve_fwd_tasks.clear();
  S.solve_bwd_tasks.clear();
  S.n_panels = (int64_t)S.panel_col.size();
  for (int L = 0; L < S.nlevels; ++L) {
    LevelPlan& P = S.levels[L];
    P.sn_begin = (int64_t)S.level_sn.size();
    int maxp = 0;
    P.max_children = 0;
    for (int t = 0; t < nt; ++t)
      if (S.sn_level[t] == L) {
        S.level_sn.push_back(t);
        maxp = std::max(maxp, S.panel_ptr[t + 1] - S.panel_ptr[t] - 1);
        P.max_children = std::max(P.max_children, S.child_ptr[t + 1] - S.child_ptr[t]);
        P.max_m = std::max<int64_t>(P.max_m, S.sn_m[t]);
        P.max_s = std::max<int64_t>(P.max_s, S.sn_begin[t + 1] - S.sn_begin[t]);
        P.max_u = std::max<int64_t>(P.max_u, S.sn_m[t] - (S.sn_begin[t + 1] - S.sn_begin[t]));
      }
    P.sn_end = (int64_t)S.level_sn.size();
    auto one_panel = [&](int t) {
      return S.panel_ptr[t + 1] - S.panel_ptr[t] - 1 == 1 && S.sn_m[t] - (S.sn_begin[t + 1] - S.sn_begin[t]) <= kOneMaxU;
    };
    // the one-wavefront form pays only with many such fronts in the level (with few, the level
    // kernels' several blocks per front finish sooner)
    int64_t n_one = 0;
    for (int64_t q = P.sn_begin; q < P.sn_end; ++q) n_one += one_panel(S.level_sn[q]) ? 1 : 0;
    const bool use_one = n_one >= kOneMinFronts;
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) P.one_begin = (int64_t)S.solve_sn.size();
      for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
        const int t = S.level_sn[q];
        if ((use_one && one_panel(t)) != (pass == 1)) continue;
        S.solve_sn.push_back(t);
        if (pass == 0) {
          P.solve_max_s = std::max<int64_t>(P.solve_max_s, S.sn_begin[t + 1] - S.sn_begin[t]);
          P.solve_max_u = std::max<int64_t>(P.solve_max_u, S.sn_m[t] - (S.sn_begin[t + 1] - S.sn_begin[t]));
        }
      }
    }
    P.fwd_begin = (int64_t)S.solve_fwd_tasks.size() / 2;
    P.bwd_begin = (int64_t)S.solve_bwd_tasks.size() / 2;
    for (int64_t q = P.sn_begin; q < P.one_begin; ++q) {
      const int t = S.solve_sn[q];
      const int np = S.panel_ptr[t + 1] - S.panel_ptr[t] - 1;
      if (np >= 1 && np <= tune.seq_panels) {  // short panel chain: one block walks it
        S.solve_fwd_tasks.push_back(t);
        S.solve_fwd_tasks.push_back(-1);
        S.solve_bwd_tasks.push_back(t);
        S.solve_bwd_tasks.push_back(-1);
        continue;
      }
      for (int k = 0; k < np; ++k) {
        S.solve_fwd_tasks.push_back(t);
        S.solve_fwd_tasks.push_back(k);
        S.solve_bwd_tasks.push_back(t);
        S.solve_bwd_tasks.push_back(np - 1 - k);
      }
    }
    P.fwd_end = (int64_t)S.solve_fwd_tasks.size() / 2;
    P.bwd_end = (int64_t)S.solve_bwd_tasks.size() / 2;
    for (int r = 0; r < P.max_children; ++r) {
      P.ea_col_begin.push_back((int64_t)S.ea_cols.size() / 4);
      P.ea_kid_begin.push_back((int64_t)S.ea_kid_recs.size() / 5);
      int64_t work = 0, kids = 0;
      for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
        int t = S.level_sn[q];
        if (S.child_ptr[t + 1] - S.child_ptr[t] > r) {
          int c = S.child_list[S.child_ptr[t] + r];
          const int64_t uc = S.sn_rows_ptr[c + 1] - S.sn_rows_ptr[c];
          const int64_t sc = S.sn_begin[c + 1] - S.sn_begin[c], mc = S.sn_m[c], mp = S.sn_m[t];
          if (uc == 0) continue;
          if (uc <= kSmallChild) {  // one block per child, its lower triangle flattened
            S.ea_kid_recs.push_back(S.sn_front_off[c] + sc + sc * mc);
            S.ea_kid_recs.push_back(S.sn_front_off[t]);
            S.ea_kid_recs.push_back(S.relmap_off[c]);
            S.ea_kid_recs.push_back(mc);
            S.ea_kid_recs.push_back((mp << 32) | uc);
            ++kids;
            continue;
          }
          for (int64_t j = 0; j < uc; ++j) {  // one wavefront per child column
            S.ea_cols.push_back(S.sn_front_off[c] + sc + (sc + j) * mc);
            S.ea_cols.push_back(S.sn_front_off[t] + (int64_t)S.relmap[S.relmap_off[c] + j] * mp);
            S.ea_cols.push_back(S.relmap_off[c]);
            S.ea_cols.push_back((j << 32) | uc);
          }
          work += uc;
        }
      }
      P.ea_work.push_back(work);
      P.ea_kids.push_back(kids);
    }
    for (int k = 0; k < maxp; ++k) {
      PanelStep ps;
      ps.task_begin = (int64_t)S.panel_tasks.size() / 3;
      // panels by width class: at most kNarrowPanel columns, at most kMediumPanel, the rest (their own
      // launches can use smaller blocks)
      for (int pass = 0; pass < 3; ++pass) {
        for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
          int t = S.level_sn[q];
          int np = S.panel_ptr[t + 1] - S.panel_ptr[t] - 1;
          if (k >= np) continue;
          const int c0 = S.panel_col[S.panel_ptr[t] + k], c1 = S.panel_col[S.panel_ptr[t] + k + 1];
          const int cls = c1 - c0 <= kNarrowPanel ? 0 : (c1 - c0 <= kMediumPanel ? 1 : 2);
          if (cls != pass) continue;
          S.panel_tasks.push_back(t);
          S.panel_tasks.push_back(c0);
          S.panel_tasks.push_back(c1);
        }
        if (pass == 0) ps.narrow_end = (int64_t)S.panel_tasks.size() / 3;
        if (pass == 1) ps.medium_end = (int64_t)S.panel_tasks.size() / 3;
      }
      ps.task_end = (int64_t)S.panel_tasks.size() / 3;
      ps.trsm_rows = 0;
      for (int64_t q = ps.task_begin; q < ps.task_end; ++q)
        ps.trsm_rows = std::max<int64_t>(ps.trsm_rows, S.sn_m[S.panel_tasks[q * 3]] - S.panel_tasks[q * 3 + 2]);
      ps.upd_begin = (int64_t)S.upd_tasks.size() / 6;
      ps.upd_map = (int64_t)S.upd_tile_task.size();
      int64_t tiles = 0;
      double fl = 0.0;
      for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
        int t = S.level_sn[q];
        int np = S.panel_ptr[t + 1] - S.panel_ptr[t] - 1;
        if (k >= np) continue;
        const int span = tune.outer_panels[tune_bucket(S.sn_m[t])];
        int ob = (k / span) * span;
        int oe = std::min(np, ob + span);
        int64_t c0 = S.panel_col[S.panel_ptr[t] + k], c1 = S.panel_col[S.panel_ptr[t] + k + 1];
        int64_t oend = S.panel_col[S.panel_ptr[t] + oe];
        if (c1 < oend) {
          int64_t m = S.sn_m[t];
          S.upd_tasks.insert(S.upd_tasks.end(), {t, c0, c1, c1, oend, tiles});
          tiles += update_tiles(m, c1, oend);
          S.upd_tile_task.resize(ps.upd_map + tiles, (int32_t)(S.upd_tasks.size() / 6 - 1 - ps.upd_begin));
          fl += update_flops(m, c1, oend, c1 - c0);
        }
      }
      ps.upd_end = (int64_t)S.upd_tasks.size() / 6;
      ps.upd_tiles = tiles;
      ps.upd_flops = fl;
      ps.outer_begin = ps.upd_end;
      ps.outer_map = (int64_t)S.upd_tile_task.size();
      tiles = 0;
      fl = 0.0;
      for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
        int t = S.level_sn[q];
        int np = S.panel_ptr[t + 1] - S.panel_ptr[t] - 1;
        if (k >= np) continue;
        const int span = tune.outer_panels[tune_bucket(S.sn_m[t])];
        int ob = (k / span) * span;
        int oe = std::min(np, ob + span);
        if (k != oe - 1) continue;
        int64_t kb = S.panel_col[S.panel_ptr[t] + ob], c1 = S.panel_col[S.panel_ptr[t] + k + 1];
        int64_t m = S.sn_m[t];
        const int64_t nb = S.panel_col[S.panel_ptr[t] + std::min(np, oe + span)];  // end of the next block
        if (c1 < nb) {  // rows c1.. of the next block's columns
          S.upd_tasks.insert(S.upd_tasks.end(), {t, kb, c1, c1, nb, tiles});
          tiles += update_tiles(m, c1, nb);
          S.upd_tile_task.resize(ps.outer_map + tiles, (int32_t)(S.upd_tasks.size() / 6 - 1 - ps.outer_begin));
          fl += update_flops(m, c1, nb, c1 - kb);
        }
      }
      ps.outer_end = (int64_t)S.upd_tasks.size() / 6;
      ps.outer_tiles = tiles;
      ps.outer_flops = fl;
      ps.far_begin = ps.outer_end;
      ps.far_map = (int64_t)S.upd_tile_task.size();
      tiles = 0;
      fl = 0.0;
      for (int64_t q = P.sn_begin; q < P.sn_end; ++q) {
        int t = S.level_sn[q];
        int np = S.panel_ptr[t + 1] - S.panel_ptr[t] - 1;
        if (k >= np) continue;
        const int span = tune.outer_panels[tune_bucket(S.sn_m[t])];
        int ob = (k / span) * span;
        int oe = std::min(np, ob + span);
        if (k != oe - 1) continue;
        int64_t kb = S.panel_col[S.panel_ptr[t] + ob], c1 = S.panel_col[S.panel_ptr[t] + k + 1];
        int64_t m = S.sn_m[t];
        const int64_t nb = S.panel_col[S.panel_ptr[t] + std::min(np, oe + span)];
        if (nb < m) {  // rows nb.. of the columns beyond the next block
          S.upd_tasks.insert(S.upd_tasks.end(), {t, kb, c1, nb, m, tiles});
          tiles += update_tiles(m, nb, m);
          S.upd_tile_task.resize(ps.far_map + tiles, (int32_t)(S.upd_tasks.size() / 6 - 1 - ps.far_begin));
          fl += update_flops(m, nb, m, c1 - kb);
        }
      }
      ps.far_end = (int64_t)S.upd_tasks.size() / 6;
      ps.far_tiles = tiles;
      ps.far_flops = fl;
      P.steps.push_back(ps);
    }
  }
  return "";
}

}  // namespace

std::string analyse(Analysis& A) {
  Mesh& m = A.mesh;
  const int d = m.dim;
  if (d != 2 && d != 3) return "dim must be 2 or 3";
  const int nv = d + 1;
  m.fdof.assign(m.n_nodes, -1);
  int64_t nf = 0;
  for (int v = 0; v < m.n_nodes; ++v)
    if (!m.fixed[v]) m.fdof[v] = (int32_t)(nf++ * d);
  m.n_x = nf * d;
  m.n_p = m.param_kind == 0 ? m.n_elems : m.n_x;
  A.nd = nv * d;
  A.off_hess = 0;
  A.off_grad = A.nd * A.nd;
  A.off_kp = A.off_grad + A.nd;
  A.off_energy = A.off_kp + (m.param_kind == 1 ? A.nd * A.nd : 0);
  A.stride = (A.off_energy + 1 + d - 1) / d * d;  // padded to whole coordinate groups
  A.off_t = A.off_kl = A.off_lg = -1;
  if (A.newton) {
    if (m.param_kind != 0) return "the Newton form is built for log-modulus parameters";
    A.off_t = A.stride;
    A.off_kl = A.off_t + A.nd * A.nd;
    A.off_lg = A.off_kl + A.nd;
    A.stride = (A.off_lg + 1 + d - 1) / d * d;
  }

  NdResult nd = nested_dissection(m);
  A.node_order = nd.order;
  const int64_t nfree = (int64_t)nd.order.size();
  if (nfree != nf) return "nested dissection lost free nodes";
  std::vector<int64_t> rank(m.n_nodes, -1);
  for (int64_t q = 0; q < nfree; ++q) rank[nd.order[q]] = q;
  // node adjacency in ranks
  std::vector<std::vector<int64_t>> adj(nfree);
  for (int e = 0; e < m.n_elems; ++e)
    for (int a = 0; a < nv; ++a) {
      int va = m.elems[(size_t)e * nv + a];
      if (m.fixed[va]) continue;
      for (int b = 0; b < nv; ++b) {
        int vb = m.elems[(size_t)e * nv + b];
        if (!m.fixed[vb] && vb != va) adj[rank[va]].push_back(rank[vb]);
      }
    }
  for (auto& l : adj) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  // parameter ownership
  std::vector<std::vector<int32_t>> owned(nfree);
  if (m.param_kind == 0) {
    for (int e = 0; e < m.n_elems; ++e) {
      int64_t best = -1;
      for (int a = 0; a < nv; ++a) {
        int v = m.elems[(size_t)e * nv + a];
        if (!m.fixed[v] && (best < 0 || rank[v] < best)) best = rank[v];
      }
      if (best < 0) return "element without free nodes (its parameter would be decoupled)";
      owned[best].push_back(e);  // ascending element id
    }
  }
  const int64_t nx = m.n_x, npar = m.n_p;

  // ---------------------------------------------------------------- SGN system
  {
    System& S = A.sgn;
    S.kind = SYS_SGN;
    S.N = 2 * nx + npar;
    const int64_t N = S.N, lam0 = nx + npar;
    S.perm.clear();
    S.perm.reserve(N);
    std::vector<int64_t> vbeg(nfree + 1), pub(nfree);
    S.var_group_end.assign(N, 0);
    for (int64_t q = 0; q < nfree; ++q) {
      int v = (int)nd.order[q];
      int64_t base = m.fdof[v];
      vbeg[q] = (int64_t)S.perm.size();
      if (m.param_kind == 0) {
        for (int32_t e : owned[q]) S.perm.push_back((int32_t)(nx + e));
      } else {
        for (int c = 0; c < d; ++c) S.perm.push_back((int32_t)(nx + base + c));
      }
      pub[q] = (int64_t)S.perm.size();
      for (int c = 0; c < d; ++c) S.perm.push_back((int32_t)(base + c));
      for (int c = 0; c < d; ++c) S.perm.push_back((int32_t)(lam0 + base + c));
      for (int64_t k = vbeg[q]; k < (int64_t)S.perm.size(); ++k) S.var_group_end[k] = (int32_t)S.perm.size();
    }
    vbeg[nfree] = (int64_t)S.perm.size();
    if ((int64_t)S.perm.size() != N) return "SGN variable order incomplete";
    S.iperm.assign(N, -1);
    for (int64_t k = 0; k < N; ++k) S.iperm[S.perm[k]] = (int32_t)k;
    // pattern
    std::vector<std::pair<int32_t, int32_t>> pairs;
    pairs.reserve((size_t)m.n_elems * (A.nd * A.nd + A.nd) + N);
    auto add = [&](int64_t o1, int64_t o2) {
      int64_t r = S.iperm[o1], c = S.iperm[o2];
      if (r < c) std::swap(r, c);
      pairs.emplace_back((int32_t)r, (int32_t)c);
    };
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) {
        int va = m.elems[(size_t)e * nv + a];
        if (m.fixed[va]) continue;
        for (int ca = 0; ca < d; ++ca) {
          int64_t A_ = m.fdof[va] + ca;
          for (int b = 0; b < nv; ++b) {
            int vb = m.elems[(size_t)e * nv + b];
            if (m.fixed[vb]) continue;
            for (int cb = 0; cb < d; ++cb) {
              int64_t B_ = m.fdof[vb] + cb;
              add(lam0 + A_, B_);
              if (m.param_kind == 1) add(lam0 + A_, nx + B_);
              if (A.newton) add(A_, B_);
            }
          }
          if (m.param_kind == 0) add(lam0 + A_, nx + e);
          if (A.newton) add(A_, nx + e);
        }
      }
    if (m.param_kind == 2)
      for (int64_t i = 0; i < nx; ++i) add(lam0 + i, nx + i);
    for (int64_t i = 0; i < N; ++i) pairs.emplace_back((int32_t)i, (int32_t)i);
    build_csr(N, pairs, S.rowptr, S.colind);
    // element contribution slots -> gather map
    const int64_t nnz = (int64_t)S.colind.size();
    std::vector<std::pair<int64_t, int32_t>> contrib;  // (slot, src)
    contrib.reserve((size_t)m.n_elems * (A.nd * A.nd + A.nd));
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) {
        int va = m.elems[(size_t)e * nv + a];
        if (m.fixed[va]) continue;
        for (int ca = 0; ca < d; ++ca) {
          int la = a * d + ca;
          int64_t A_ = m.fdof[va] + ca;
          for (int b = 0; b < nv; ++b) {
            int vb = m.elems[(size_t)e * nv + b];
            if (m.fixed[vb]) continue;
            for (int cb = 0; cb < d; ++cb) {
              int lb = b * d + cb;
              int64_t B_ = m.fdof[vb] + cb;
              int64_t sl = find_slot(S, S.iperm[lam0 + A_], S.iperm[B_]);
              if (sl < 0) return "missing Kx slot";
              contrib.emplace_back(sl, (int32_t)ebuf_index(A.off_hess + la * A.nd + lb, e, m.n_elems, d));
              if (m.param_kind == 1) {
                int64_t s2 = find_slot(S, S.iperm[lam0 + A_], S.iperm[nx + B_]);
                if (s2 < 0) return "missing Kp slot";
                contrib.emplace_back(s2, (int32_t)ebuf_index(A.off_kp + la * A.nd + lb, e, m.n_elems, d));
              }
              // x-x of the Newton form: each lower entry takes one of the two symmetric values
              if (A.newton && S.iperm[A_] >= S.iperm[B_]) {
                int64_t s3 = find_slot(S, S.iperm[A_], S.iperm[B_]);
                if (s3 < 0) return "missing x-x slot";
                contrib.emplace_back(s3, (int32_t)ebuf_index(A.off_t + la * A.nd + lb, e, m.n_elems, d));
              }
            }
          }
          if (m.param_kind == 0) {
            int64_t sl = find_slot(S, S.iperm[lam0 + A_], S.iperm[nx + e]);
            if (sl < 0) return "missing Kp slot";
            contrib.emplace_back(sl, (int32_t)ebuf_index(A.off_grad + la, e, m.n_elems, d));
          }
          if (A.newton) {
            int64_t sl = find_slot(S, S.iperm[A_], S.iperm[nx + e]);
            if (sl < 0) return "missing x-p slot";
            contrib.emplace_back(sl, (int32_t)ebuf_index(A.off_kl + la, e, m.n_elems, d));
          }
        }
      }
    if (A.newton)
      for (int e = 0; e < m.n_elems; ++e) {
        int64_t sl = find_slot(S, S.iperm[nx + e], S.iperm[nx + e]);
        if (sl < 0) return "missing p-p slot";
        contrib.emplace_back(sl, (int32_t)ebuf_index(A.off_lg, e, m.n_elems, d));
      }
    if ((double)m.n_elems * A.stride > 2147483000.0) return "element buffer index overflow";
    S.slot_ptr.assign(nnz + 1, 0);
    for (auto& c : contrib) S.slot_ptr[c.first + 1]++;
    for (int64_t i = 0; i < nnz; ++i) S.slot_ptr[i + 1] += S.slot_ptr[i];
    S.slot_src.resize(contrib.size());
    {
      std::vector<int64_t> fill(S.slot_ptr.begin(), S.slot_ptr.end() - 1);
      for (auto& c : contrib) S.slot_src[fill[c.first]++] = c.second;  // element order kept
    }
    std::vector<std::pair<int64_t, int32_t>>().swap(contrib);
    S.diag_kind.assign(N, 0);
    for (int64_t k = 0; k < N; ++k) {
      int64_t o = S.perm[k];
      S.diag_kind[k] = o < nx ? 3 : (o < lam0 ? 2 : 4);
    }
    S.elem_stride = A.stride;
    // rest-position parameters couple to the multipliers of neighbouring nodes, so they
    // belong to the node's public variables (rows of earlier fronts); other parameter
    // kinds only touch their owner's group
    int pub_n = 2 * d;
    if (m.param_kind == 1) {
      for (int64_t q = 0; q < nfree; ++q) pub[q] = vbeg[q];
      pub_n = 3 * d;
    }
    std::string err = finish_system(S, nd.tree, vbeg, pub, pub_n, adj, A.tune);
    if (!err.empty()) return "SGN: " + err;
    S.grp_ptr.resize(nfree + 1);
    S.grp_node.resize(nfree);
    S.grp_vec.resize(nfree);
    for (int64_t q = 0; q <= nfree; ++q) S.grp_ptr[q] = (int32_t)vbeg[q];
    for (int64_t q = 0; q < nfree; ++q) {
      const int64_t g = vbeg[q];
      const int J = S.var_sn[g];
      if (S.var_sn[vbeg[q + 1] - 1] != J) return "SGN: node group split across supernodes";
      S.grp_node[q] = (int32_t)nd.order[q];
      S.grp_vec[q] = S.sn_vec_off[J] + (g - S.sn_begin[J]);
    }
  }
  // ---------------------------------------------------------------- Kx system
  {
    System& S = A.kx;
    S.kind = SYS_KX;
    S.N = nx;
    const int64_t N = nx;
    S.perm.clear();
    S.var_group_end.assign(N, 0);
    std::vector<int64_t> vbeg(nfree + 1);
    for (int64_t q = 0; q < nfree; ++q) {
      int v = (int)nd.order[q];
      vbeg[q] = (int64_t)S.perm.size();
      for (int c = 0; c < d; ++c) S.perm.push_back((int32_t)(m.fdof[v] + c));
      for (int64_t k = vbeg[q]; k < (int64_t)S.perm.size(); ++k) S.var_group_end[k] = (int32_t)S.perm.size();
    }
    vbeg[nfree] = N;
    S.iperm.assign(N, -1);
    for (int64_t k = 0; k < N; ++k) S.iperm[S.perm[k]] = (int32_t)k;
    std::vector<std::pair<int32_t, int32_t>> pairs;
    pairs.reserve((size_t)m.n_elems * A.nd * A.nd / 2 + N);
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) {
        int va = m.elems[(size_t)e * nv + a];
        if (m.fixed[va]) continue;
        for (int b = 0; b < nv; ++b) {
          int vb = m.elems[(size_t)e * nv + b];
          if (m.fixed[vb]) continue;
          for (int ca = 0; ca < d; ++ca)
            for (int cb = 0; cb < d; ++cb) {
              int64_t r = S.iperm[m.fdof[va] + ca], c = S.iperm[m.fdof[vb] + cb];
              if (r >= c) pairs.emplace_back((int32_t)r, (int32_t)c);
            }
        }
      }
    for (int64_t i = 0; i < N; ++i) pairs.emplace_back((int32_t)i, (int32_t)i);
    build_csr(N, pairs, S.rowptr, S.colind);
    const int64_t nnz = (int64_t)S.colind.size();
    std::vector<std::pair<int64_t, int32_t>> contrib;
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) {
        int va = m.elems[(size_t)e * nv + a];
        if (m.fixed[va]) continue;
        for (int b = 0; b < nv; ++b) {
          int vb = m.elems[(size_t)e * nv + b];
          if (m.fixed[vb]) continue;
          for (int ca = 0; ca < d; ++ca)
            for (int cb = 0; cb < d; ++cb) {
              int64_t r = S.iperm[m.fdof[va] + ca], c = S.iperm[m.fdof[vb] + cb];
              if (r < c) continue;  // each lower entry takes one of the two symmetric products
              int64_t sl = find_slot(S, r, c);
              if (sl < 0) return "missing Kx slot";
              contrib.emplace_back(sl, (int32_t)ebuf_index(A.off_hess + (a * d + ca) * A.nd + b * d + cb, e, m.n_elems, d));
            }
        }
      }
    S.slot_ptr.assign(nnz + 1, 0);
    for (auto& c : contrib) S.slot_ptr[c.first + 1]++;
    for (int64_t i = 0; i < nnz; ++i) S.slot_ptr[i + 1] += S.slot_ptr[i];
    S.slot_src.resize(contrib.size());
    {
      std::vector<int64_t> fill(S.slot_ptr.begin(), S.slot_ptr.end() - 1);
      for (auto& c : contrib) S.slot_src[fill[c.first]++] = c.second;
    }
    // residual gather (free-DOF order, not permuted)
    S.vec_ptr.assign(nx + 1, 0);
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) {
        int va = m.elems[(size_t)e * nv + a];
        if (!m.fixed[va])
          for (int c = 0; c < d; ++c) S.vec_ptr[m.fdof[va] + c + 1]++;
      }
    for (int64_t i = 0; i < nx; ++i) S.vec_ptr[i + 1] += S.vec_ptr[i];
    S.vec_src.resize(S.vec_ptr[nx]);
    {
      std::vector<int64_t> fill(S.vec_ptr.begin(), S.vec_ptr.end() - 1);
      for (int e = 0; e < m.n_elems; ++e)
        for (int a = 0; a < nv; ++a) {
          int va = m.elems[(size_t)e * nv + a];
          if (!m.fixed[va])
            for (int c = 0; c < d; ++c)
              S.vec_src[fill[m.fdof[va] + c]++] = (int32_t)ebuf_index(A.off_grad + a * d + c, e, m.n_elems, d);
        }
    }
    S.diag_kind.assign(N, 3);
    S.elem_stride = A.stride;
    std::vector<int64_t> pub(nfree);
    for (int64_t q = 0; q < nfree; ++q) pub[q] = vbeg[q];
    std::string err = finish_system(S, nd.tree, vbeg, pub, d, adj, A.tune);
    if (!err.empty()) return "Kx: " + err;
  }
  return "";
}

}  // namespace sgn
