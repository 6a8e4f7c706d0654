// Block-diagonal preconditioner of the saddle-point matrix without a reference factor (gfx950).
//
// For MINRES on K (Sec. 5 reports that standard preconditioned Krylov solvers fared poorly on these
// systems; this ablation of the library's learned preconditioner keeps only its block structure):
// with S the row scaling of the current matrix and B_i the diagonal block of S K S over node group i
// (its owned parameters, x_v and lambda_v),
//   M^-1 = S blockdiag_i(|B_i|^-1) S,   |B_i| = V |Lambda| V^T  (B_i = V Lambda V^T),
// symmetric positive definite, as MINRES needs.  One wavefront per group: the block is built from
// the lower CSR in LDS, diagonalised by cyclic Jacobi rotations (rows and columns by lanes), and
// |B_i|^-1 is stored densely, group after group.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

constexpr int kBpMax = 64;  // node groups never exceed a panel

__global__ void __launch_bounds__(64) k_blockpc_setup(const int32_t* __restrict__ grp_ptr,
                                                      const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const double* __restrict__ vals,
                                                      const double* __restrict__ scale,
                                                      const int64_t* __restrict__ off, double* __restrict__ minv) {
  __shared__ double B[kBpMax][kBpMax + 1];
  __shared__ double V[kBpMax][kBpMax + 1];
  const int q = blockIdx.x, lane = threadIdx.x;
  const int g0 = grp_ptr[q], g = grp_ptr[q + 1] - g0;
  for (int j = 0; j < g; ++j) {
    B[lane][j] = 0.0;
    V[lane][j] = lane == j ? 1.0 : 0.0;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < g) {
    // row g0 + lane of the lower CSR: its entries in the group's columns, and their mirror images
    const int64_t i = g0 + lane;
    const double si = scale[i];
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
      const int32_t j = colind[t];
      if (j >= g0) {
        const double v = si * vals[t] * scale[j];
        B[lane][j - g0] = v;
        B[j - g0][lane] = v;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  // cyclic Jacobi: sweeps over all pairs (p, r), each rotation annihilating B[p][r]; stop when the
  // off-diagonal mass is below 1e-30 of the diagonal's (or after 30 sweeps)
  for (int sweep = 0; sweep < 30; ++sweep) {
    double od = 0.0, dg = 0.0;
    if (lane < g) {
      for (int j = 0; j < g; ++j) {
        const double x = B[lane][j];
        if (j == lane) dg += x * x;
        else od += x * x;
      }
    }
    for (int s = 32; s > 0; s >>= 1) {
      od += __shfl_xor(od, s);
      dg += __shfl_xor(dg, s);
    }
    if (!(od > 1e-30 * dg)) break;
    for (int p = 0; p < g - 1; ++p)
      for (int r = p + 1; r < g; ++r) {
        const double apr = B[p][r];
        if (apr == 0.0) continue;
        const double app = B[p][p], arr = B[r][r];
        const double th = (arr - app) / (2.0 * apr);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        __builtin_amdgcn_wave_barrier();
        // columns p and r of B and V (lane = row); then rows p and r of B from the columns (B stays
        // symmetric), with the rotated 2 x 2 block set exactly
        double bp = 0.0, br = 0.0;
        if (lane < g) {
          bp = B[lane][p];
          br = B[lane][r];
          B[lane][p] = c * bp - sn * br;
          B[lane][r] = sn * bp + c * br;
          const double vp = V[lane][p], vr = V[lane][r];
          V[lane][p] = c * vp - sn * vr;
          V[lane][r] = sn * vp + c * vr;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < g && lane != p && lane != r) {
          B[p][lane] = B[lane][p];
          B[r][lane] = B[lane][r];
        }
        if (lane == 0) {
          B[p][p] = app - t * apr;
          B[r][r] = arr + t * apr;
          B[p][r] = 0.0;
          B[r][p] = 0.0;
        }
        __builtin_amdgcn_wave_barrier();
      }
  }
  // |B|^-1 = V |Lambda|^-1 V^T (an eigenvalue below 1e-300 in magnitude is taken as 1e-300)
  __shared__ double il[kBpMax];
  if (lane < g) il[lane] = 1.0 / fmax(fabs(B[lane][lane]), 1e-300);
  __builtin_amdgcn_wave_barrier();
  double* out = minv + off[q];
  if (lane < g) {
    for (int j = 0; j < g; ++j) {
      double acc = 0.0;
      for (int k = 0; k < g; ++k) acc += V[lane][k] * V[j][k] * il[k];
      out[(int64_t)lane * g + j] = acc;
    }
  }
}

// out = S blockdiag(|B_i|^-1) S in, one wavefront per group (vectors in the system's new numbering)
__global__ void __launch_bounds__(64) k_blockpc_apply(const int32_t* __restrict__ grp_ptr,
                                                      const double* __restrict__ scale,
                                                      const int64_t* __restrict__ off, const double* __restrict__ minv,
                                                      const double* __restrict__ in, double* __restrict__ out) {
  __shared__ double xs[kBpMax];
  const int q = blockIdx.x, lane = threadIdx.x;
  const int g0 = grp_ptr[q], g = grp_ptr[q + 1] - g0;
  if (lane < g) xs[lane] = scale[g0 + lane] * in[g0 + lane];
  __builtin_amdgcn_wave_barrier();
  if (lane < g) {
    const double* row = minv + off[q] + (int64_t)lane * g;
    double acc = 0.0;
    for (int j = 0; j < g; ++j) acc += row[j] * xs[j];
    out[g0 + lane] = scale[g0 + lane] * acc;
  }
}

}  // namespace

void launch_blockpc_setup(int64_t ngroups, const int32_t* grp_ptr, const int64_t* rowptr, const int32_t* colind,
                          const double* vals, const double* scale, const int64_t* off, double* minv, hipStream_t s) {
  if (ngroups > 0) k_blockpc_setup<<<(unsigned)ngroups, 64, 0, s>>>(grp_ptr, rowptr, colind, vals, scale, off, minv);
}

void launch_blockpc_apply(int64_t ngroups, const int32_t* grp_ptr, const double* scale, const int64_t* off,
                          const double* minv, const double* in, double* out, hipStream_t s) {
  if (ngroups > 0) k_blockpc_apply<<<(unsigned)ngroups, 64, 0, s>>>(grp_ptr, scale, off, minv, in, out);
}

}  // namespace sgn
