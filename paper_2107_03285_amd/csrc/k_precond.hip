// Node-block preconditioner built from a reference LDL^T factor, and the
// vector kernels of the preconditioned MINRES iteration.
//
// With the reference factor P (S K_ref S) P^T = L D L^T the preconditioner is
//   M = S^-1 P^T L B L^T P S^-1,   B = blockdiag_i( R_i C_i C_i^T R_i^T ),
// where i runs over the node groups (a free node's owned parameters, x_v and
// lambda_v, contiguous in elimination order; Bunch-Kaufman pivots never cross
// a group), R_i R_i^T = |D_i| is the eigen-absolute value of the group's 1x1
// and 2x2 pivots, and C_i is the learned lower-triangular correction in the
// whitened coordinates.  M is symmetric positive definite for every C_i with a
// positive diagonal, which MINRES requires of its preconditioner.
//
// C_i = blockdiag( exp(r_e) for each owned parameter position,
//                  I + Delta_i on the trailing 2d positions (x_v, lambda_v) ),
// where Delta_i is strictly lower triangular from the raw outputs r and its
// diagonal is exp(r_tt) - 1, so raw outputs of zero give C_i = I (B = |D|).
// Raw corrections are FP32 (network outputs); all arithmetic is FP64.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

constexpr int kMaxTri = 21;  // (2d)(2d+1)/2 for d = 3

struct Pair {
  double c, s, l0, l1;  // eigenvector angle and the eigenvalues of the two positions
};

// symmetric 2x2 [[a, b], [b, e]]: first position <-> eigenvalue (a+e)/2 + rho with
// eigenvector (cos t, sin t), t = atan2(b, (a-e)/2) / 2; second <-> the other one with (-sin t, cos t)
__device__ inline Pair eig2(double a, double b, double e) {
  const double half = 0.5 * (a + e), diff = 0.5 * (a - e);
  const double rho = sqrt(diff * diff + b * b);
  const double det = a * e - b * b;
  double lp, lm;
  if (half >= 0.0) {
    lp = half + rho;
    lm = lp != 0.0 ? det / lp : 0.0;
  } else {
    lm = half - rho;
    lp = det / lm;
  }
  const double t = 0.5 * atan2(b, diff);
  Pair p;
  p.c = cos(t);
  p.s = sin(t);
  p.l0 = lp;
  p.l1 = lm;
  return p;
}

// whitening u = R^-1 y (forward = true) or unwhitening w = R^-T v (forward = false) of the group
// [g0, g1), in place on the thread's array
__device__ inline void whiten(const double* dpiv, const double* epiv, const int32_t* pivtype, int g0, int n,
                              double* y, bool forward) {
  for (int k = 0; k < n; ++k) {
    const int t = pivtype[g0 + k];
    if (t == 0) {
      y[k] /= sqrt(fabs(dpiv[g0 + k]));
    } else if (t == 1 && k + 1 < n) {
      const Pair p = eig2(dpiv[g0 + k], epiv[g0 + k], dpiv[g0 + k + 1]);
      const double r0 = sqrt(fabs(p.l0)), r1 = sqrt(fabs(p.l1));
      const double y0 = y[k], y1 = y[k + 1];
      if (forward) {  // |L|^-1/2 Q^T y
        y[k] = (p.c * y0 + p.s * y1) / r0;
        y[k + 1] = (-p.s * y0 + p.c * y1) / r1;
      } else {  // Q |L|^-1/2 v
        const double a0 = y0 / r0, a1 = y1 / r1;
        y[k] = p.c * a0 - p.s * a1;
        y[k + 1] = p.s * a0 + p.c * a1;
      }
      ++k;
    }
  }
}

// correction factor of a group: diagonal scales of the owned parameters and the dense lower 2d x 2d block
struct Corr {
  int nown, nb;
  double blk[6][6];
};

__device__ inline void load_corr(const float* cn, const float* cp, const int32_t* perm, int64_t nx, int g0, int nown,
                                 int nb, int node, double* pscale, Corr& C) {
  C.nown = nown;
  C.nb = nb;
  const int tri = nb * (nb + 1) / 2;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      double v = 0.0;
      if (j < i) v = cn ? (double)cn[(int64_t)node * tri + i * (i + 1) / 2 + j] : 0.0;
      if (j == i) v = cn ? exp((double)cn[(int64_t)node * tri + i * (i + 1) / 2 + i]) : 1.0;
      C.blk[i][j] = v;
    }
  for (int k = 0; k < nown; ++k) pscale[k] = cp ? exp((double)cp[perm[g0 + k] - nx]) : 1.0;
}

// the trailing block: v = C^-1 u (lower solve) and v = C^-T u (upper solve), in place
__device__ inline void blk_lower_solve(const Corr& C, double* u) {
  for (int i = 0; i < C.nb; ++i) {
    double a = u[i];
    for (int j = 0; j < i; ++j) a -= C.blk[i][j] * u[j];
    u[i] = a / C.blk[i][i];
  }
}
__device__ inline void blk_upper_solve(const Corr& C, double* u) {
  for (int i = C.nb - 1; i >= 0; --i) {
    double a = u[i];
    for (int j = i + 1; j < C.nb; ++j) a -= C.blk[j][i] * u[j];
    u[i] = a / C.blk[i][i];
  }
}

// w = B^-1 y per node group; y read from the forward solve's per-front vectors (pivot order),
// optionally saved flat; w written flat in pivot order for the backward solve
__global__ void __launch_bounds__(128) k_pc_block(PcArgs a, const double* __restrict__ tp, double* __restrict__ ysave,
                                                  double* __restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ngroups) return;
  const int g0 = a.grp_ptr[q], n = a.grp_ptr[q + 1] - g0;
  const int nb = 2 * a.dim, nown = n - nb;
  const double* yv = tp + a.grp_vec[q];
  double y[64];
  for (int k = 0; k < n; ++k) {
    y[k] = yv[k];
    if (ysave) ysave[g0 + k] = y[k];
  }
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, y, true);
  Corr C;
  double ps[64];
  load_corr(a.corr_node, a.corr_par, a.perm, a.nx, g0, nown, nb, a.grp_node[q], ps, C);
  for (int k = 0; k < nown; ++k) y[k] /= ps[k] * ps[k];
  blk_lower_solve(C, y + nown);
  blk_upper_solve(C, y + nown);
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, y, false);
  for (int k = 0; k < n; ++k) w[g0 + k] = y[k];
}

// gradient of the bilinear form ya^T B^-1 yb with respect to the raw corrections, scaled by
// `weight` and added to gn (per node, lower triangle) and gp (per parameter).  ya, yb are
// forward-solve results in pivot order (flat).  With u = R^-1 y, eta = C^-1 ua, gam = C^-1 ub, alpha = C^-T eta,
// beta = C^-T gam:  d/dC_ij = -(alpha_i gam_j + beta_i eta_j), lower triangle.
__global__ void __launch_bounds__(128) k_pc_grad(PcArgs a, const double* __restrict__ ya,
                                                 const double* __restrict__ yb, double weight, float* __restrict__ gn,
                                                 float* __restrict__ gp) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ngroups) return;
  const int g0 = a.grp_ptr[q], n = a.grp_ptr[q + 1] - g0;
  const int nb = 2 * a.dim, nown = n - nb;
  const int node = a.grp_node[q];
  double ua[64], ub[64];
  for (int k = 0; k < n; ++k) {
    ua[k] = ya[g0 + k];
    ub[k] = yb[g0 + k];
  }
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, ua, true);
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, ub, true);
  Corr C;
  double ps[64];
  load_corr(a.corr_node, a.corr_par, a.perm, a.nx, g0, nown, nb, node, ps, C);
  // owned parameters: C = s = exp(r), d/dC = -2 ua ub / s^3, d/dr = s d/dC
  for (int k = 0; k < nown; ++k) {
    const double s = ps[k];
    const double g = -2.0 * ua[k] * ub[k] / (s * s * s) * s;
    if (gp) gp[a.perm[g0 + k] - a.nx] += (float)(weight * g);
  }
  if (!gn) return;
  double eta[6], gam[6], al[6], be[6];
  for (int i = 0; i < nb; ++i) {
    eta[i] = ua[nown + i];
    gam[i] = ub[nown + i];
  }
  blk_lower_solve(C, eta);
  blk_lower_solve(C, gam);
  for (int i = 0; i < nb; ++i) {
    al[i] = eta[i];
    be[i] = gam[i];
  }
  blk_upper_solve(C, al);
  blk_upper_solve(C, be);
  const int tri = nb * (nb + 1) / 2;
  float* g = gn + (int64_t)node * tri;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = -(al[i] * gam[j] + be[i] * eta[j]);
      if (i == j) v *= C.blk[i][i];  // diagonal: C_ii = exp(r_ii)
      g[i * (i + 1) / 2 + j] += (float)(weight * v);
    }
}

// Halves of B^-1 = (R C)^-T (R C)^-1 for the symmetric form of the preconditioned matrix,
// T = (R C)^-1 L^-1 P S K S P^T L^-T (R C)^-T, which is similar to M^-1 K:
//   k_pc_half_fwd:  u = C^-1 R^-1 y   (y from the forward solve's vectors, u flat in pivot order)
//   k_pc_half_bwd:  w = R^-T C^-T v   (flat to flat; w feeds the backward solve)
__global__ void __launch_bounds__(128) k_pc_half_fwd(PcArgs a, const double* __restrict__ tp, double* __restrict__ u) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ngroups) return;
  const int g0 = a.grp_ptr[q], n = a.grp_ptr[q + 1] - g0;
  const int nb = 2 * a.dim, nown = n - nb;
  const double* yv = tp + a.grp_vec[q];
  double y[64];
  for (int k = 0; k < n; ++k) y[k] = yv[k];
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, y, true);
  Corr C;
  double ps[64];
  load_corr(a.corr_node, a.corr_par, a.perm, a.nx, g0, nown, nb, a.grp_node[q], ps, C);
  for (int k = 0; k < nown; ++k) y[k] /= ps[k];
  blk_lower_solve(C, y + nown);
  for (int k = 0; k < n; ++k) u[g0 + k] = y[k];
}

__global__ void __launch_bounds__(128) k_pc_half_bwd(PcArgs a, const double* __restrict__ v, double* __restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ngroups) return;
  const int g0 = a.grp_ptr[q], n = a.grp_ptr[q + 1] - g0;
  const int nb = 2 * a.dim, nown = n - nb;
  double y[64];
  for (int k = 0; k < n; ++k) y[k] = v[g0 + k];
  Corr C;
  double ps[64];
  load_corr(a.corr_node, a.corr_par, a.perm, a.nx, g0, nown, nb, a.grp_node[q], ps, C);
  for (int k = 0; k < nown; ++k) y[k] /= ps[k];
  blk_upper_solve(C, y + nown);
  whiten(a.dpiv, a.epiv, a.pivtype, g0, n, y, false);
  for (int k = 0; k < n; ++k) w[g0 + k] = y[k];
}

// gradient of x^T T y with respect to the raw corrections (x, y, Tx, Ty flat, whitened, pivot order),
// scaled by `weight` and added to gn / gp.  With T = C^-1 A C^-T:
//   d(x^T T y)/dC_ij = -[(C^-T x)_i (T y)_j + (C^-T y)_i (T x)_j]  on the block's lower triangle,
// and the same with the 1x1 scale s on owned-parameter positions; d/dr = C_ii d/dC_ii on diagonals.
__global__ void __launch_bounds__(128) k_pc_sym_grad(PcArgs a, const double* __restrict__ x,
                                                     const double* __restrict__ ty, const double* __restrict__ y,
                                                     const double* __restrict__ tx, double weight,
                                                     float* __restrict__ gn, float* __restrict__ gp) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.ngroups) return;
  const int g0 = a.grp_ptr[q], n = a.grp_ptr[q + 1] - g0;
  const int nb = 2 * a.dim, nown = n - nb;
  const int node = a.grp_node[q];
  Corr C;
  double ps[64];
  load_corr(a.corr_node, a.corr_par, a.perm, a.nx, g0, nown, nb, node, ps, C);
  for (int k = 0; k < nown; ++k) {
    const int i = g0 + k;
    const double g = -(x[i] / ps[k] * ty[i] + y[i] / ps[k] * tx[i]) * ps[k];
    if (gp) gp[a.perm[i] - a.nx] += (float)(weight * g);
  }
  if (!gn) return;
  const int b0 = g0 + nown;
  double cx[6], cy[6];
  for (int i = 0; i < nb; ++i) {
    cx[i] = x[b0 + i];
    cy[i] = y[b0 + i];
  }
  blk_upper_solve(C, cx);  // C^-T x
  blk_upper_solve(C, cy);
  const int tri = nb * (nb + 1) / 2;
  float* g = gn + (int64_t)node * tri;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = -(cx[i] * ty[b0 + j] + cy[i] * tx[b0 + j]);
      if (i == j) v *= C.blk[i][i];
      g[i * (i + 1) / 2 + j] += (float)(weight * v);
    }
}

__global__ void k_lincomb3(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                           double c, const double* __restrict__ z, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (y) v += b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

}  // namespace

static_assert(kMaxTri == 21, "correction block of a 3D node");

void launch_pc_block(const PcArgs& a, const double* tp, double* ysave, double* w, hipStream_t s) {
  if (a.ngroups > 0) k_pc_block<<<(unsigned)((a.ngroups + 127) / 128), 128, 0, s>>>(a, tp, ysave, w);
}

void launch_pc_grad(const PcArgs& a, const double* ya, const double* yb, double weight, float* gn, float* gp,
                    hipStream_t s) {
  if (a.ngroups > 0) k_pc_grad<<<(unsigned)((a.ngroups + 127) / 128), 128, 0, s>>>(a, ya, yb, weight, gn, gp);
}

void launch_pc_half_fwd(const PcArgs& a, const double* tp, double* u, hipStream_t s) {
  if (a.ngroups > 0) k_pc_half_fwd<<<(unsigned)((a.ngroups + 127) / 128), 128, 0, s>>>(a, tp, u);
}

void launch_pc_half_bwd(const PcArgs& a, const double* v, double* w, hipStream_t s) {
  if (a.ngroups > 0) k_pc_half_bwd<<<(unsigned)((a.ngroups + 127) / 128), 128, 0, s>>>(a, v, w);
}

void launch_pc_sym_grad(const PcArgs& a, const double* x, const double* ty, const double* y, const double* tx,
                        double weight, float* gn, float* gp, hipStream_t s) {
  if (a.ngroups > 0)
    k_pc_sym_grad<<<(unsigned)((a.ngroups + 127) / 128), 128, 0, s>>>(a, x, ty, y, tx, weight, gn, gp);
}

void launch_lincomb3(int64_t n, double a, const double* x, double b, const double* y, double c, const double* z,
                     double* out, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  k_lincomb3<<<(unsigned)g, 256, 0, s>>>(n, a, x, b, y, c, z, out);
}

}  // namespace sgn
