// FP32 kernels of the preconditioner network: input features, gathered dense
// layers (forward and backward), neighbourhood means, and Adam.  Every sum has
// a fixed order (gathers through CSR tables, weight gradients through per-block
// partials reduced in block order), so forward and backward are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

constexpr int kH = 64;
constexpr int kMaxK = 3 * kH;
constexpr int kWgRows = 16;                                  // rows staged per pass of the weight gradient
constexpr int kWgPairs = ((kMaxK + 1) * kH + 255) / 256;     // (k, j) pairs per thread

__device__ inline float gather_x(const DenseArgs& a, int64_t r, int k) {
  for (int s = 0; s < a.nseg; ++s) {
    const DenseSeg& g = a.seg[s];
    if (k < g.width) {
      const int64_t row = g.idx ? (int64_t)g.idx[r] : r;
      return g.src[row * g.ld + k];
    }
    k -= g.width;
  }
  return 0.0f;
}

// out[r, j] = res[r, j] + act(sum_k W[k, j] x_r[k] + b[j]); ysave (optional) keeps act(...)
__global__ void __launch_bounds__(256) k_dense_fwd(DenseArgs a) {
  __shared__ float xs[4][kMaxK];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* b = a.W + (int64_t)a.K * a.N;
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < a.rows; r += (int64_t)gridDim.x * 4) {
    for (int k = lane; k < a.K; k += 64) xs[wave][k] = gather_x(a, r, k);
    __builtin_amdgcn_wave_barrier();
    if (lane < a.N) {
      float acc = b[lane];
      for (int k = 0; k < a.K; ++k) acc += a.W[(int64_t)k * a.N + lane] * xs[wave][k];
      const float y = a.act ? tanhf(acc) : acc;
      if (a.ysave) a.ysave[r * a.N + lane] = y;
      a.out[r * a.ld_out + lane] = (a.res ? a.res[r * a.ld_res + lane] : 0.0f) + y;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// dz = dout * act'(y); dx (optional) = W dz (rows of K)
__global__ void __launch_bounds__(256) k_dense_bwd(DenseArgs a, const float* __restrict__ dout, int ld_dout,
                                                   const float* __restrict__ y, float* __restrict__ dz,
                                                   float* __restrict__ dx) {
  __shared__ float zs[4][kH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < a.rows; r += (int64_t)gridDim.x * 4) {
    float z = 0.0f;
    if (lane < a.N) {
      z = dout[r * ld_dout + lane];
      if (a.act) {
        const float t = y[r * a.N + lane];
        z *= 1.0f - t * t;
      }
      dz[r * a.N + lane] = z;
    }
    zs[wave][lane] = z;
    __builtin_amdgcn_wave_barrier();
    if (dx)
      for (int k = lane; k < a.K; k += 64) {
        float acc = 0.0f;
        for (int j = 0; j < a.N; ++j) acc += a.W[(int64_t)k * a.N + j] * zs[wave][j];
        dx[r * a.K + k] = acc;
      }
    __builtin_amdgcn_wave_barrier();
  }
}

// per-block partial of [x_r; 1] dz_r^T over the block's rows: part[blk][(K+1) * N]
__global__ void __launch_bounds__(256) k_dense_wgrad(DenseArgs a, const float* __restrict__ dz, int64_t chunk,
                                                     float* __restrict__ part) {
  __shared__ float xs[kWgRows][kMaxK + 1];
  __shared__ float zs[kWgRows][kH];
  const int tid = threadIdx.x;
  const int KN = (a.K + 1) * a.N;
  float acc[kWgPairs];
#pragma unroll
  for (int i = 0; i < kWgPairs; ++i) acc[i] = 0.0f;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(a.rows, r0 + chunk);
  for (int64_t rb = r0; rb < r1; rb += kWgRows) {
    const int nr = (int)min<int64_t>(kWgRows, r1 - rb);
    for (int idx = tid; idx < kWgRows * (a.K + 1); idx += 256) {
      const int rr = idx / (a.K + 1), k = idx % (a.K + 1);
      xs[rr][k] = rr < nr ? (k < a.K ? gather_x(a, rb + rr, k) : 1.0f) : 0.0f;
    }
    for (int idx = tid; idx < kWgRows * kH; idx += 256) {
      const int rr = idx / kH, j = idx % kH;
      zs[rr][j] = (rr < nr && j < a.N) ? dz[(rb + rr) * a.N + j] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kWgPairs; ++i) {
      const int p = tid + 256 * i;
      if (p < KN) {
        const int k = p / a.N, j = p % a.N;
        float s = 0.0f;
        for (int rr = 0; rr < nr; ++rr) s += xs[rr][k] * zs[rr][j];
        acc[i] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kWgPairs; ++i) {
    const int p = tid + 256 * i;
    if (p < KN) part[(int64_t)blockIdx.x * KN + p] = acc[i];
  }
}

__global__ void k_reduce_parts(int nparts, int64_t n, const float* __restrict__ part, float* __restrict__ g) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * n + i];
    g[i] += s;
  }
}

// dst[v, j] += scale * sum over the CSR entries of v of src[id, col + j] (id = list[k], or k without list;
// without ptr the single entry v)
__global__ void __launch_bounds__(256) k_gather_add(int64_t nv, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ list, const float* __restrict__ src,
                                                    int ld_src, int col, int width, float scale, int divide_by_count,
                                                    float* __restrict__ dst, int ld_dst) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= nv || lane >= width) return;
  const int32_t k0 = ptr ? ptr[v] : (int32_t)v, k1 = ptr ? ptr[v + 1] : (int32_t)v + 1;
  float s = 0.0f;
  for (int32_t k = k0; k < k1; ++k) s += src[(int64_t)(list ? list[k] : k) * ld_src + col + lane];
  float f = scale;
  if (divide_by_count) f = k1 > k0 ? scale / (float)(k1 - k0) : 0.0f;
  dst[v * ld_dst + lane] += f * s;
}

// dE[e, j] += dagg[dst_e, col + j] / deg(dst_e)   (dagg rows of stride ld)
__global__ void k_edge_mean_bwd(int64_t ne, const int32_t* __restrict__ dst, const int32_t* __restrict__ in_ptr,
                                const float* __restrict__ dagg, int ld, int col, float* __restrict__ dE) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= ne) return;
  const int32_t t = dst[e];
  const float deg = (float)(in_ptr[t + 1] - in_ptr[t]);
  dE[e * kH + lane] += dagg[(int64_t)t * ld + col + lane] / deg;
}

// emb[e, j] = mean over the element's nodes of h[v, j]
__global__ void k_elem_mean(int64_t ne, int nv, const int32_t* __restrict__ elems, const float* __restrict__ h,
                            float* __restrict__ emb) {
  const int lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= ne) return;
  float s = 0.0f;
  for (int a = 0; a < nv; ++a) s += h[(int64_t)elems[e * nv + a] * kH + lane];
  emb[e * kH + lane] = s / (float)nv;
}

__global__ void k_node_features(GnnFeatArgs a, float* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.n_nodes) return;
  const int d = a.dim, fn = 2 * d + 3;
  float* o = out + v * fn;
  const int32_t f = a.nfdof[v];
  const double il = 1.0 / a.ell;
  for (int c = 0; c < d; ++c) {
    const double xb = f >= 0 ? a.x[f + c] : a.rest[v * d + c];
    const double xa = f >= 0 ? a.x_ref[f + c] : a.rest[v * d + c];
    o[c] = (float)((xb - xa) * il);
    o[d + c] = (float)((xb - a.rest[v * d + c]) * il);
  }
  o[2 * d] = f >= 0 ? 0.0f : 1.0f;
  double s0 = 0.0, s1 = 0.0;
  if (a.param_kind == 0) {
    const int32_t k0 = a.inc_ptr[v], k1 = a.inc_ptr[v + 1];
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t e = a.inc_list[k];
      s0 += a.p[e] - a.p_ref[e];
      s1 += a.p[e];
    }
    if (k1 > k0) {
      s0 /= (double)(k1 - k0);
      s1 /= (double)(k1 - k0);
    }
  } else if (f >= 0) {
    for (int c = 0; c < d; ++c) {
      const double dp = a.p[f + c] - a.p_ref[f + c];
      s0 += dp * dp;
      s1 += a.p[f + c] * a.p[f + c];
    }
    s0 = sqrt(s0) * il;
    s1 = sqrt(s1) * il;
  }
  o[2 * d + 1] = (float)s0;
  o[2 * d + 2] = (float)s1;
}

__global__ void k_edge_features(GnnFeatArgs a, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_edges) return;
  const int d = a.dim;
  const int32_t s = src[e], t = dst[e];
  const int32_t fs = a.nfdof[s], ft = a.nfdof[t];
  float* o = out + e * (2 * d);
  for (int c = 0; c < d; ++c) {
    const double Xs = a.rest[s * d + c], Xt = a.rest[t * d + c];
    const double xs = fs >= 0 ? a.x[fs + c] : Xs, xt = ft >= 0 ? a.x[ft + c] : Xt;
    o[c] = (float)((Xs - Xt) / a.hbar);
    o[d + c] = (float)(((xs - xt) - (Xs - Xt)) / a.ell);
  }
}

// decoder rows -> correction arrays, and back (gradients)
__global__ void k_split_out(int64_t n_nodes, int tri, int nout, int d, int per_node_params,
                            const int32_t* __restrict__ nfdof, const float* __restrict__ dec, float* __restrict__ cn,
                            float* __restrict__ cp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  for (int t = 0; t < tri; ++t) cn[v * tri + t] = dec[v * nout + t];
  if (per_node_params && nfdof[v] >= 0)
    for (int c = 0; c < d; ++c) cp[nfdof[v] + c] = dec[v * nout + tri + c];
}

__global__ void k_split_bwd(int64_t n_nodes, int tri, int nout, int d, int per_node_params,
                            const int32_t* __restrict__ nfdof, const float* __restrict__ gcn,
                            const float* __restrict__ gcp, float* __restrict__ ddec) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  for (int t = 0; t < tri; ++t) ddec[v * nout + t] = gcn ? gcn[v * tri + t] : 0.0f;
  if (per_node_params)
    for (int c = 0; c < d; ++c)
      ddec[v * nout + tri + c] = (gcp && nfdof[v] >= 0) ? gcp[nfdof[v] + c] : 0.0f;
}

__global__ void k_add_f32(int64_t n, const float* __restrict__ src, float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

__global__ void k_scale_f32(int64_t n, float a, float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] *= a;
}

__global__ void k_fill_f32(int64_t n, float v, float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

// Adam with bias correction (step t >= 1)
__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

inline unsigned blocks_for(int64_t n, int per, int64_t cap = 65535) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

void launch_dense_fwd(const DenseArgs& a, hipStream_t s) {
  if (a.rows > 0) k_dense_fwd<<<blocks_for(a.rows, 4, 16384), 256, 0, s>>>(a);
}

void launch_dense_bwd(const DenseArgs& a, const float* dout, int ld_dout, const float* y, float* dz, float* dx,
                      hipStream_t s) {
  if (a.rows > 0) k_dense_bwd<<<blocks_for(a.rows, 4, 16384), 256, 0, s>>>(a, dout, ld_dout, y, dz, dx);
}

int wgrad_parts(int64_t rows) {
  int64_t p = (rows + 255) / 256;
  if (p < 1) p = 1;
  if (p > 256) p = 256;
  return (int)p;
}

void launch_dense_wgrad(const DenseArgs& a, const float* dz, float* part, float* gw, hipStream_t s) {
  if (a.rows <= 0) return;
  const int np = wgrad_parts(a.rows);
  const int64_t chunk = (a.rows + np - 1) / np;
  k_dense_wgrad<<<(unsigned)np, 256, 0, s>>>(a, dz, chunk, part);
  const int64_t n = (int64_t)(a.K + 1) * a.N;
  k_reduce_parts<<<blocks_for(n, 256, 4096), 256, 0, s>>>(np, n, part, gw);
}

void launch_gather_add(int64_t nv, const int32_t* ptr, const int32_t* list, const float* src, int ld_src, int col,
                       int width, float scale, int divide_by_count, float* dst, int ld_dst, hipStream_t s) {
  if (nv > 0)
    k_gather_add<<<blocks_for(nv, 4, 1 << 30), 256, 0, s>>>(nv, ptr, list, src, ld_src, col, width, scale,
                                                            divide_by_count, dst, ld_dst);
}

void launch_edge_mean_bwd(int64_t ne, const int32_t* dst, const int32_t* in_ptr, const float* dagg, int ld, int col,
                          float* dE, hipStream_t s) {
  if (ne > 0) k_edge_mean_bwd<<<blocks_for(ne, 4, 1 << 30), 256, 0, s>>>(ne, dst, in_ptr, dagg, ld, col, dE);
}

void launch_elem_mean(int64_t ne, int nv, const int32_t* elems, const float* h, float* emb, hipStream_t s) {
  if (ne > 0) k_elem_mean<<<blocks_for(ne, 4, 1 << 30), 256, 0, s>>>(ne, nv, elems, h, emb);
}

void launch_gnn_features(const GnnFeatArgs& a, const int32_t* src, const int32_t* dst, float* nf, float* ef,
                         hipStream_t s) {
  if (a.n_nodes > 0) k_node_features<<<blocks_for(a.n_nodes, 128, 1 << 30), 128, 0, s>>>(a, nf);
  if (a.n_edges > 0) k_edge_features<<<blocks_for(a.n_edges, 128, 1 << 30), 128, 0, s>>>(a, src, dst, ef);
}

void launch_split_out(int64_t n_nodes, int tri, int nout, int d, int per_node_params, const int32_t* nfdof,
                      const float* dec, float* cn, float* cp, hipStream_t s) {
  if (n_nodes > 0)
    k_split_out<<<blocks_for(n_nodes, 128, 1 << 30), 128, 0, s>>>(n_nodes, tri, nout, d, per_node_params, nfdof, dec,
                                                                  cn, cp);
}

void launch_split_bwd(int64_t n_nodes, int tri, int nout, int d, int per_node_params, const int32_t* nfdof,
                      const float* gcn, const float* gcp, float* ddec, hipStream_t s) {
  if (n_nodes > 0)
    k_split_bwd<<<blocks_for(n_nodes, 128, 1 << 30), 128, 0, s>>>(n_nodes, tri, nout, d, per_node_params, nfdof, gcn,
                                                                  gcp, ddec);
}

void launch_add_f32(int64_t n, const float* src, float* dst, hipStream_t s) {
  if (n > 0) k_add_f32<<<blocks_for(n, 256, 8192), 256, 0, s>>>(n, src, dst);
}

void launch_scale_f32(int64_t n, float a, float* dst, hipStream_t s) {
  if (n > 0) k_scale_f32<<<blocks_for(n, 256, 8192), 256, 0, s>>>(n, a, dst);
}

void launch_fill_f32(int64_t n, float v, float* dst, hipStream_t s) {
  if (n > 0) k_fill_f32<<<blocks_for(n, 256, 8192), 256, 0, s>>>(n, v, dst);
}

void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 int t, hipStream_t s) {
  if (n <= 0) return;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  k_adam<<<blocks_for(n, 256, 8192), 256, 0, s>>>(n, w, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace sgn
