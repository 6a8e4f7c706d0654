// Mesh graph network that predicts the node-block preconditioner's corrections.
//
// Graph: the mesh nodes, with a directed edge each way between two nodes that
// share an element.  Inputs describe how the current state (x, p) differs from
// the reference state (x_a, p_a) whose factor the preconditioner reuses.
//
//   node features (2d+3): (x_v - x_a,v)/ell, (x_v - X_v)/ell (zero on fixed nodes),
//                         fixed flag, then for log-modulus parameters the means
//                         over the node's elements of (p - p_a) and of p, for
//                         per-node parameters |p_v - p_a,v| / ell and |p_v| / ell
//   edge features (2d):   (X_s - X_d)/hbar, ((x_s - x_d) - (X_s - X_d))/ell
//                         (hbar: mean rest length of the edges)
//   encoders:  h = tanh(W f_n + b),  e = tanh(W f_e + b)          (width 64)
//   3 layers:  e <- e + tanh(W [h_dst, h_src, e] + b)
//              a_v = mean of e over the edges into v
//              h <- h + tanh(W [h, a] + b)
//   decoders:  per node  W h + b -> the (2d)(2d+1)/2 raw entries of the node's
//              correction block (+ d parameter corrections for per-node
//              parameters); per element (log-modulus) W mean_{v in e}(h_v) + b.
//
// Weights are one FP32 vector; each dense layer stores W (K x N, row-major,
// W[k*N + j]) followed by its bias b (N), in the order enc_n, enc_e, then per
// layer edge and node, then dec_n and dec_e.  The decoders start at zero, so an
// untrained network leaves the preconditioner at |D|.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "symbolic.h"

namespace sgn {

constexpr int kGnnH = 64;
constexpr int kGnnLayers = 3;
constexpr int kGnnMaxK = 3 * kGnnH;  // widest dense input (edge layer)

struct GnnDense {
  int64_t w = 0;  // offset of W; b follows at w + k * n
  int k = 0, n = 0;
};

struct GnnGraph {
  int dim = 0, n_nodes = 0, n_elems = 0, param_kind = 0;
  int fn = 0, fe = 0;         // input widths
  int tri = 0;                // (2d)(2d+1)/2
  int nout_node = 0;          // tri (+ d for per-node parameters)
  int64_t n_edges = 0;
  std::vector<int32_t> e_src, e_dst;    // sorted by (dst, src)
  std::vector<int32_t> in_ptr;          // [n_nodes+1] edges into v: [in_ptr[v], in_ptr[v+1])
  std::vector<int32_t> out_ptr, out_list;  // edges out of v (ascending edge id)
  std::vector<int32_t> inc_ptr, inc_list;  // elements of v (ascending)
  double hbar = 1.0;
  GnnDense enc_n, enc_e, edge[kGnnLayers], node[kGnnLayers], dec_n, dec_e;
  int64_t n_weights = 0;
};

std::string build_gnn_graph(const Mesh& m, GnnGraph& g);
// Glorot-uniform weights from a counter-based generator (splitmix64), decoders zero.
void gnn_init_weights(const GnnGraph& g, uint64_t seed, std::vector<float>& w);

}  // namespace sgn
