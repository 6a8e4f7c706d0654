// Level-scheduled multifrontal triangular solves with the supernodal factor.
//
// Forward (leaves to root): each front gathers its pivot entries of the
// right-hand side plus its children's contribution vectors (fixed child
// order), applies its pivot permutation, solves with the unit lower panels
// and leaves rows [s, m) as the contribution for its parent; then D^-1
// (1x1 and 2x2 blocks).  Backward (root to leaves): each front reads the
// already-solved ancestor entries of its structure, forms
// z = w - L21^T v with a fixed-order block reduction, solves L11^T and
// scatters through the inverse pivot permutation.  Vectors are FP64 whatever
// the factor precision.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_fwd(const int32_t* __restrict__ level_sn, SolveArgs a,
                                             const T* __restrict__ front, const double* __restrict__ b) {
  const int32_t* panel_ptr = a.panel_ptr;
  const int32_t* panel_col = a.panel_col;
  __shared__ double ys[64];
  const int tid = threadIdx.x;
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J];
  double* tv = a.tv + a.sn_vec_off[J];
  double* tp = a.tp + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  for (int64_t k = tid; k < m; k += 256) tv[k] = k < s ? b[g0 + k] : 0.0;
  __syncthreads();
  for (int32_t q = a.child_ptr[J]; q < a.child_ptr[J + 1]; ++q) {
    const int C = a.child_list[q];
    const int64_t sC = f.sn_begin[C + 1] - f.sn_begin[C], uC = f.sn_m[C] - sC;
    const double* cv = a.tp + a.sn_vec_off[C] + sC;
    const int32_t* rel = f.relmap + f.relmap_off[C];
    for (int64_t r = tid; r < uC; r += 256) tv[rel[r]] += cv[r];
    __syncthreads();
  }
  for (int64_t k = tid; k < m; k += 256) tp[k] = k < s ? tv[f.lperm[g0 + k]] : tv[k];
  __syncthreads();
  for (int32_t pi = panel_ptr[J]; pi + 1 < panel_ptr[J + 1]; ++pi) {
    const int c0 = panel_col[pi], c1 = panel_col[pi + 1];
    for (int k = c0; k < c1; ++k) {
      const double y = tp[k];
      for (int i = k + 1 + tid; i < c1; i += 256) tp[i] -= (double)F[i + (int64_t)k * m] * y;
      __syncthreads();
    }
    if (tid < c1 - c0) ys[tid] = tp[c0 + tid];
    __syncthreads();
    for (int64_t r = c1 + tid; r < m; r += 256) {
      double acc = 0.0;
      for (int k = c0; k < c1; ++k) acc += (double)F[r + (int64_t)k * m] * ys[k - c0];
      tp[r] -= acc;
    }
    __syncthreads();
  }
  for (int64_t k = tid; k < s; k += 256) {
    const int t = f.pivtype[g0 + k];
    if (t == 0) {
      tp[k] = tp[k] / f.dpiv[g0 + k];
    } else if (t == 1) {
      const double A = f.dpiv[g0 + k], B = f.epiv[g0 + k], C = f.dpiv[g0 + k + 1];
      const double det = A * C - B * B;
      const double x0 = tp[k], x1 = tp[k + 1];
      tp[k] = (C * x0 - B * x1) / det;
      tp[k + 1] = (A * x1 - B * x0) / det;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bwd(const int32_t* __restrict__ level_sn, SolveArgs a,
                                             const T* __restrict__ front, double* __restrict__ x) {
  const int32_t* panel_ptr = a.panel_ptr;
  const int32_t* panel_col = a.panel_col;
  __shared__ double red[16][257];
  __shared__ double z[64];
  const int tid = threadIdx.x;
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J];
  double* tp = a.tp + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  const int32_t* rows = f.sn_rows + f.sn_rows_ptr[J];
  for (int64_t r = tid; r < m - s; r += 256) tp[s + r] = x[rows[r]];
  __syncthreads();
  for (int32_t pi = panel_ptr[J + 1] - 2; pi >= panel_ptr[J]; --pi) {
    const int c0 = panel_col[pi], c1 = panel_col[pi + 1];
    const int w = c1 - c0;
    for (int kb = 0; kb < w; kb += 16) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      for (int64_t r = c1 + tid; r < m; r += 256) {
        const double v = tp[r];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (kb + q < w) acc[q] += (double)F[r + (int64_t)(c0 + kb + q) * m] * v;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) red[q][tid] = acc[q];
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
#pragma unroll
          for (int q = 0; q < 16; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
      }
      if (tid < 16 && kb + tid < w) z[kb + tid] = tp[c0 + kb + tid] - red[tid][0];
      __syncthreads();
    }
    for (int k = w - 1; k >= 0; --k) {
      const double v = z[k];
      for (int i = tid; i < k; i += 256) z[i] -= (double)F[(c0 + k) + (int64_t)(c0 + i) * m] * v;
      __syncthreads();
    }
    if (tid < w) tp[c0 + tid] = z[tid];
    __syncthreads();
  }
  for (int64_t k = tid; k < s; k += 256) x[g0 + f.lperm[g0 + k]] = tp[k];
}

}  // namespace

template <typename T>
void launch_fwd_level(int64_t nsn, const int32_t* level_sn, const SolveArgs& a, const T* front, const double* b,
                      hipStream_t s) {
  if (nsn > 0) k_fwd<T><<<(unsigned)nsn, 256, 0, s>>>(level_sn, a, front, b);
}

template <typename T>
void launch_bwd_level(int64_t nsn, const int32_t* level_sn, const SolveArgs& a, const T* front, double* x,
                      hipStream_t s) {
  if (nsn > 0) k_bwd<T><<<(unsigned)nsn, 256, 0, s>>>(level_sn, a, front, x);
}

template void launch_fwd_level<double>(int64_t, const int32_t*, const SolveArgs&, const double*, const double*,
                                       hipStream_t);
template void launch_fwd_level<float>(int64_t, const int32_t*, const SolveArgs&, const float*, const double*,
                                      hipStream_t);
template void launch_bwd_level<double>(int64_t, const int32_t*, const SolveArgs&, const double*, double*,
                                       hipStream_t);
template void launch_bwd_level<float>(int64_t, const int32_t*, const SolveArgs&, const float*, double*, hipStream_t);

}  // namespace sgn
