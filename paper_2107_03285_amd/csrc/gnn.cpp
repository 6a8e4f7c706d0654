// Host side of the preconditioner network: graph tables and weight layout.
#include "gnn.h"

#include <algorithm>
#include <cmath>

namespace sgn {

namespace {

GnnDense dense(int64_t& off, int k, int n) {
  GnnDense d;
  d.w = off;
  d.k = k;
  d.n = n;
  off += (int64_t)(k + 1) * n;
  return d;
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

std::string build_gnn_graph(const Mesh& m, GnnGraph& g) {
  const int d = m.dim, nv = d + 1;
  g.dim = d;
  g.n_nodes = m.n_nodes;
  g.n_elems = m.n_elems;
  g.param_kind = m.param_kind;
  g.fn = 2 * d + 3;
  g.fe = 2 * d;
  g.tri = (2 * d) * (2 * d + 1) / 2;
  g.nout_node = g.tri + (m.param_kind == 0 ? 0 : d);
  // undirected pairs sharing an element, both directions, sorted by (dst, src)
  std::vector<int64_t> keys;
  keys.reserve((size_t)m.n_elems * nv * (nv - 1));
  for (int e = 0; e < m.n_elems; ++e)
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b) {
        if (a == b) continue;
        const int64_t s = m.elems[(size_t)e * nv + a], t = m.elems[(size_t)e * nv + b];
        keys.push_back(t * m.n_nodes + s);
      }
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  if (keys.size() > (size_t)INT32_MAX) return "too many edges";
  g.n_edges = (int64_t)keys.size();
  g.e_src.resize(keys.size());
  g.e_dst.resize(keys.size());
  g.in_ptr.assign(m.n_nodes + 1, 0);
  g.out_ptr.assign(m.n_nodes + 1, 0);
  double len = 0;
  for (size_t k = 0; k < keys.size(); ++k) {
    const int32_t t = (int32_t)(keys[k] / m.n_nodes), s = (int32_t)(keys[k] % m.n_nodes);
    g.e_src[k] = s;
    g.e_dst[k] = t;
    ++g.in_ptr[t + 1];
    ++g.out_ptr[s + 1];
    double l2 = 0;
    for (int c = 0; c < d; ++c) {
      const double dx = m.rest[(size_t)s * d + c] - m.rest[(size_t)t * d + c];
      l2 += dx * dx;
    }
    len += std::sqrt(l2);
  }
  g.hbar = keys.empty() ? 1.0 : len / (double)keys.size();
  for (int v = 0; v < m.n_nodes; ++v) {
    g.in_ptr[v + 1] += g.in_ptr[v];
    g.out_ptr[v + 1] += g.out_ptr[v];
  }
  g.out_list.assign(keys.size(), 0);
  {
    std::vector<int32_t> fill(g.out_ptr.begin(), g.out_ptr.end() - 1);
    for (size_t k = 0; k < keys.size(); ++k) g.out_list[fill[g.e_src[k]]++] = (int32_t)k;
  }
  // node -> elements
  g.inc_ptr.assign(m.n_nodes + 1, 0);
  for (int32_t v : m.elems) ++g.inc_ptr[v + 1];
  for (int v = 0; v < m.n_nodes; ++v) g.inc_ptr[v + 1] += g.inc_ptr[v];
  g.inc_list.assign(m.elems.size(), 0);
  {
    std::vector<int32_t> fill(g.inc_ptr.begin(), g.inc_ptr.end() - 1);
    for (int e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < nv; ++a) g.inc_list[fill[m.elems[(size_t)e * nv + a]]++] = e;
  }
  // weights
  int64_t off = 0;
  g.enc_n = dense(off, g.fn, kGnnH);
  g.enc_e = dense(off, g.fe, kGnnH);
  for (int l = 0; l < kGnnLayers; ++l) {
    g.edge[l] = dense(off, 3 * kGnnH, kGnnH);
    g.node[l] = dense(off, 2 * kGnnH, kGnnH);
  }
  g.dec_n = dense(off, kGnnH, g.nout_node);
  g.dec_e = m.param_kind == 0 ? dense(off, kGnnH, 1) : GnnDense{off, kGnnH, 0};
  g.n_weights = off;
  return "";
}

void gnn_init_weights(const GnnGraph& g, uint64_t seed, std::vector<float>& w) {
  w.assign(g.n_weights, 0.0f);
  uint64_t s = seed;
  auto glorot = [&](const GnnDense& L) {
    const double a = std::sqrt(6.0 / (double)(L.k + L.n));
    for (int64_t i = 0; i < (int64_t)L.k * L.n; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
      w[L.w + i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  glorot(g.enc_n);
  glorot(g.enc_e);
  for (int l = 0; l < kGnnLayers; ++l) {
    glorot(g.edge[l]);
    glorot(g.node[l]);
  }
}

}  // namespace sgn
