// Element derivative kernels and deterministic assembly (gfx950).
//
// Per element e with linear shape functions (the paper's inverse elastic
// design example, Sec. 5.1, uses linear tetrahedra with a neo-Hookean
// material): F = Ds Dm^-1, J = det F,
//   Psi = mu/2 (|F|^2 - d) - mu ln J + lam/2 (ln J)^2,
//   P   = mu (F - F^-T) + lam ln J F^-T,
//   dP  = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T,
// energy V0 Psi, gradient V0 P Dm^-T (node 0 takes minus the column sum) and
// the Hessian (dc/dx of Sec. 3.1) column by column from dP along each nodal
// DOF direction, where dF = e_c w^T is rank one.  For log-modulus
// parameters E_e = E0 exp(p_e) the constraint Jacobian column dc/dp_e equals
// the element gradient itself.
//
// Assembly never uses floating-point atomics: every element writes its block
// to an element buffer, and each CSR slot sums its sources in a fixed order
// (ascending element), so the assembled values are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

template <int D>
__device__ inline double det(const double (&M)[D][D]) {
  if constexpr (D == 2) {
    return M[0][0] * M[1][1] - M[0][1] * M[1][0];
  } else {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  }
}

template <int D>
__device__ inline void inverse(const double (&M)[D][D], double dt, double (&R)[D][D]) {
  double id = 1.0 / dt;
  if constexpr (D == 2) {
    R[0][0] = M[1][1] * id;
    R[0][1] = -M[0][1] * id;
    R[1][0] = -M[1][0] * id;
    R[1][1] = M[0][0] * id;
  } else {
    R[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) * id;
    R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
    R[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) * id;
    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) * id;
    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
  }
}

// Newton form (mode 3, log-modulus parameters), with lam_e the element's entries of the multipliers:
// the x-x block of d2(lam.g_e) is the derivative of the Hessian along V = sum_b lam_b w_b^T, column by
// column from the second derivative of P along the rank-one U = e_c w^T and V (G = F^-T):
//   d2P[U, V] = (lam ln J - mu)(G V^T G U^T G + G U^T G V^T G)
//               - lam (tr(F^-1 V) G U^T G + tr(F^-1 V F^-1 U) G + tr(F^-1 U) G V^T G),
// symmetric in U and V; the x-p column is K_e lam_e and the p-p entry lam_e . g_e (both moduli scale
// with exp(p_e)).
template <int D, bool NEWTON>
__global__ void __launch_bounds__(128) k_element(ElemArgs a) {
  constexpr int NV = D + 1;
  constexpr int ND = NV * D;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.ne) return;
  double xe[NV][D], Xe[NV][D];
  for (int v = 0; v < NV; ++v) {
    const int node = a.elems[(int64_t)e * NV + v];
    const int f = a.efdof[(int64_t)e * NV + v];
    for (int c = 0; c < D; ++c) {
      const double r = a.rest[(int64_t)node * D + c];
      Xe[v][c] = (a.param_kind == 1 && f >= 0) ? a.p[f + c] : r;
      xe[v][c] = f >= 0 ? a.x[f + c] : r;
    }
  }
  double Dm[D][D], Ds[D][D], Dmi[D][D];
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      Dm[c][k] = Xe[k + 1][c] - Xe[0][c];
      Ds[c][k] = xe[k + 1][c] - xe[0][c];
    }
  const double dm = det<D>(Dm);
  inverse<D>(Dm, dm, Dmi);
  const double V0 = dm / (D == 2 ? 2.0 : 6.0);
  double mu = a.mu0, lam = a.lam0;
  if (a.param_kind == 0) {
    const double s = exp(a.p[e]);
    mu *= s;
    lam *= s;
  }
  double F[D][D];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
      for (int k = 0; k < D; ++k) acc += Ds[i][k] * Dmi[k][j];
      F[i][j] = acc;
    }
  const double J = det<D>(F);
  // element buffer in coordinate groups: value j of element e at ((j / D) ne + e) D + j % D, so a
  // wavefront's stores of one group cover one contiguous span, and the D values the assembly gathers
  // for neighbouring CSR slots share a cache line
  const int64_t ne = a.ne;
  auto out = [&](int64_t j) -> double& { return a.ebuf[((j / D) * ne + e) * D + j % D]; };
  if (!(J > 0.0)) {
    atomicAdd(a.inverted, 1);
    out(a.off_energy) = __builtin_inf();
    return;
  }
  double Fi[D][D];
  inverse<D>(F, J, Fi);
  const double lnJ = log(J);
  double trC = 0.0;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) trC += F[i][j] * F[i][j];
  out(a.off_energy) = V0 * (0.5 * mu * (trC - D) - mu * lnJ + 0.5 * lam * lnJ * lnJ);
  if (a.mode == 0) return;
  // F^-T[i][j] = Fi[j][i]
  double P[D][D];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) P[i][j] = mu * (F[i][j] - Fi[j][i]) + lam * lnJ * Fi[j][i];
  // multipliers of the element's DOFs (Newton form; 0 on fixed components)
  double lv[NEWTON ? ND : 1];
  if constexpr (NEWTON) {
    for (int v = 0; v < NV; ++v) {
      const int f = a.efdof[(int64_t)e * NV + v];
      for (int c = 0; c < D; ++c) lv[v * D + c] = f >= 0 ? a.lam[f + c] : 0.0;
    }
  }
  // G = V0 P Dm^-T : G[c][k] = V0 sum_j P[c][j] Dmi[k][j]
  {
    double g0[D];
    double lg = 0.0;
    for (int c = 0; c < D; ++c) g0[c] = 0.0;
    for (int k = 0; k < D; ++k)
      for (int c = 0; c < D; ++c) {
        double acc = 0.0;
        for (int j = 0; j < D; ++j) acc += P[c][j] * Dmi[k][j];
        acc *= V0;
        out(a.off_grad + (k + 1) * D + c) = acc;
        g0[c] -= acc;
        if constexpr (NEWTON) lg += acc * lv[(k + 1) * D + c];
      }
    for (int c = 0; c < D; ++c) out(a.off_grad + c) = g0[c];
    if constexpr (NEWTON) {
      for (int c = 0; c < D; ++c) lg += g0[c] * lv[c];
      out(a.off_lg) = lg;
    }
  }
  if (a.mode == 1) return;
  const double cA = mu - lam * lnJ;
  // Newton form: V, W = G V^T G, tr(F^-1 V) and R = F^-1 V F^-1
  double W[D][D], R[D][D], trV = 0.0, kl[NEWTON ? ND : 1];
  if constexpr (NEWTON) {
    double V[D][D];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc += (lv[(k + 1) * D + i] - lv[i]) * Dmi[k][j];
        V[i][j] = acc;  // sum over nodes b of lam_b[i] w_b[j], w_0 = -(sum of the rows of Dm^-1)
      }
    double Q[D][D];  // F^-1 V
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc += Fi[i][k] * V[k][j];
        Q[i][j] = acc;
      }
    for (int i = 0; i < D; ++i) trV += Q[i][i];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc += Q[i][k] * Fi[k][j];
        R[i][j] = acc;
      }
    // W = G V^T G: W[i][j] = sum_{q,r} Fi[q][i] V[r][q] Fi[j][r]
    double VG[D][D];  // V^T G : VG[q][j] = sum_r V[r][q] Fi[j][r]
    for (int q = 0; q < D; ++q)
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
        for (int r = 0; r < D; ++r) acc += V[r][q] * Fi[j][r];
        VG[q][j] = acc;
      }
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double acc = 0.0;
        for (int q = 0; q < D; ++q) acc += Fi[q][i] * VG[q][j];
        W[i][j] = acc;
      }
    for (int r = 0; r < ND; ++r) kl[r] = 0.0;
  }
  for (int b = 0; b < NV; ++b) {
    // w = d(Dm^-1 row) for node b: dF = e_cb w^T
    double w[D];
    for (int j = 0; j < D; ++j) {
      if (b > 0) {
        w[j] = Dmi[b - 1][j];
      } else {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc -= Dmi[k][j];
        w[j] = acc;
      }
    }
    // FinvT w : (F^-T w)_i = sum_a Fi[a][i] w[a]
    double Fw[D];
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int q = 0; q < D; ++q) acc += Fi[q][i] * w[q];
      Fw[i] = acc;
    }
    for (int cb = 0; cb < D; ++cb) {
      // tr(F^-1 dF) = sum_i Fi[i][cb] w[i]
      double tr = 0.0;
      for (int i = 0; i < D; ++i) tr += Fi[i][cb] * w[i];
      double dP[D][D];
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j)
          dP[i][j] = (i == cb ? mu * w[j] : 0.0) + cA * Fw[i] * Fi[j][cb] + lam * tr * Fi[j][i];
      const int col = b * D + cb;
      double h0[D];
      for (int c = 0; c < D; ++c) h0[c] = 0.0;
      for (int k = 0; k < D; ++k)
        for (int c = 0; c < D; ++c) {
          double acc = 0.0;
          for (int j = 0; j < D; ++j) acc += dP[c][j] * Dmi[k][j];
          acc *= V0;
          out(((k + 1) * D + c) * ND + col) = acc;
          h0[c] -= acc;
          if constexpr (NEWTON) kl[(k + 1) * D + c] += acc * lv[col];
        }
      for (int c = 0; c < D; ++c) out(c * ND + col) = h0[c];
      if constexpr (NEWTON) {
        for (int c = 0; c < D; ++c) kl[c] += h0[c] * lv[col];
        // d2P[U, V] for U = e_cb w^T
        double Ww[D];
        for (int i = 0; i < D; ++i) {
          double acc = 0.0;
          for (int q = 0; q < D; ++q) acc += W[i][q] * w[q];
          Ww[i] = acc;
        }
        double trVU = 0.0;  // tr(F^-1 V F^-1 U) = w^T R e_cb
        for (int q = 0; q < D; ++q) trVU += w[q] * R[q][cb];
        double T[D][D];
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j)
            T[i][j] = -cA * (Ww[i] * Fi[j][cb] + Fw[i] * W[cb][j]) -
                      lam * (trV * Fw[i] * Fi[j][cb] + trVU * Fi[j][i] + tr * W[i][j]);
        double t0[D];
        for (int c = 0; c < D; ++c) t0[c] = 0.0;
        for (int k = 0; k < D; ++k)
          for (int c = 0; c < D; ++c) {
            double acc = 0.0;
            for (int j = 0; j < D; ++j) acc += T[c][j] * Dmi[k][j];
            acc *= V0;
            out(a.off_t + ((k + 1) * D + c) * ND + col) = acc;
            t0[c] -= acc;
          }
        for (int c = 0; c < D; ++c) out(a.off_t + c * ND + col) = t0[c];
      }
    }
  }
  if constexpr (NEWTON)
    for (int r = 0; r < ND; ++r) out(a.off_kl + r) = kl[r];
  if (a.param_kind == 1) {
    // d(grad)/dX along each rest DOF: Dm moves, so dDm^-1 = -Dm^-1 dDm Dm^-1,
    // dF = -F dDm Dm^-1, dV0 = V0 tr(Dm^-1 dDm), dG = dV0 P Dm^-T + V0 dP Dm^-T + V0 P d(Dm^-T)
    for (int b = 0; b < NV; ++b) {
      for (int cb = 0; cb < D; ++cb) {
        // dDm = e_cb u^T with u[k] = (b > 0 ? delta(k, b-1) : -1)
        double u[D];
        for (int k = 0; k < D; ++k) u[k] = b > 0 ? (k == b - 1 ? 1.0 : 0.0) : -1.0;
        // (u^T Dm^-1)[j] = sum_k u[k] Dmi[k][j]
        double uD[D];
        for (int j = 0; j < D; ++j) {
          double acc = 0.0;
          for (int k = 0; k < D; ++k) acc += u[k] * Dmi[k][j];
          uD[j] = acc;
        }
        // dDmi = -Dmi e_cb uD^T : dDmi[i][j] = -Dmi[i][cb] uD[j]
        // dF = Ds dDmi = -(Ds Dmi[:, cb]) uD^T = -(F e_cb) uD^T -> column cb of F
        double fc[D];
        for (int i = 0; i < D; ++i) fc[i] = F[i][cb];
        const double dV0 = V0 * uD[cb];  // tr(Dmi dDm) = sum_i Dmi[i][cb] u... = (u^T Dmi)[cb]
        double dF[D][D];
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) dF[i][j] = -fc[i] * uD[j];
        // dP = mu dF + cA F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T
        double trq = 0.0;
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) trq += Fi[i][j] * dF[j][i];
        double T1[D][D];  // dF^T F^-T : T1[q][j] = sum_r dF[r][q] Fi[j][r]
        for (int q = 0; q < D; ++q)
          for (int j = 0; j < D; ++j) {
            double acc = 0.0;
            for (int r = 0; r < D; ++r) acc += dF[r][q] * Fi[j][r];
            T1[q][j] = acc;
          }
        double dP[D][D];
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) {
            double acc = 0.0;
            for (int q = 0; q < D; ++q) acc += Fi[q][i] * T1[q][j];
            dP[i][j] = mu * dF[i][j] + cA * acc + lam * trq * Fi[j][i];
          }
        const int col = b * D + cb;
        double h0[D];
        for (int c = 0; c < D; ++c) h0[c] = 0.0;
        for (int k = 0; k < D; ++k)
          for (int c = 0; c < D; ++c) {
            // G[c][k] = V0 sum_j P[c][j] Dmi[k][j]
            double acc = 0.0;
            for (int j = 0; j < D; ++j)
              acc += dV0 * P[c][j] * Dmi[k][j] + V0 * dP[c][j] * Dmi[k][j] - V0 * P[c][j] * Dmi[k][cb] * uD[j];
            out(a.off_kp + ((k + 1) * D + c) * ND + col) = acc;
            h0[c] -= acc;
          }
        for (int c = 0; c < D; ++c) out(a.off_kp + c * ND + col) = h0[c];
      }
    }
  }
}

// sum of ebuf[src[q]] over q in [q0, q1), ascending; four sources in flight at a time (indices clamped to
// the first source, values past the end masked: adding +0.0 to a sum that starts at +0.0 changes nothing)
__device__ inline double sum_sources(int64_t q0, int64_t q1, const int32_t* __restrict__ src,
                                     const double* __restrict__ ebuf) {
  double acc = 0.0;
  for (int64_t q = q0; q < q1; q += 4) {
    int32_t sq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sq[u] = src[q + u < q1 ? q + u : q0];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = ebuf[sq[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += q + u < q1 ? v[u] : 0.0;
  }
  return acc;
}

// Index of this workgroup once renumbered so that each of the 8 dies (workgroups go to them
// round-robin by index, each die with its own L2) takes one contiguous run of [0, gridDim.x).
__device__ inline int64_t die_contiguous_block() {
  const int64_t n = gridDim.x, x = blockIdx.x & 7;
  int64_t before = 0;
  for (int64_t y = 0; y < x; ++y) before += (n - y + 7) >> 3;
  return before + (blockIdx.x >> 3);
}

// Workgroups go to the 8 dies (each with its own L2) round-robin by index; renumbered, each die takes
// one contiguous run of the slots (rows of the elimination order, so a region of the mesh), and the
// element values of that region are fetched into its L2 once instead of once per die.
__global__ void k_gather_slots(int64_t nnz, const int64_t* __restrict__ ptr, const int32_t* __restrict__ src,
                               const double* __restrict__ ebuf, double* __restrict__ vals) {
  const int64_t b = die_contiguous_block();
  for (int64_t t = b * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x)
    vals[t] = sum_sources(ptr[t], ptr[t + 1], src, ebuf);
}

__global__ void k_diag_add(int64_t N, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ kind,
                           double a_target, double c_param, double eps_x, double eps_lambda, double* vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = kind[i];
    double v = 0.0;
    if (k == 1) v = a_target + eps_x;
    else if (k == 2) v = c_param;
    else if (k == 3) v = eps_x;
    else if (k == 4) v = -eps_lambda;
    vals[rowptr[i + 1] - 1] += v;
  }
}

// out[i] += sign e_i z[i] with e the stabilisation diagonal of the variable kinds (eps_x on x,
// -eps_lambda on lambda, 0 on parameters): sign +1 turns b - K_eps z into b - K z, sign -1 turns
// K_eps z into K z
__global__ void k_unstabilise(int64_t N, const int32_t* __restrict__ kind, double eps_x, double eps_lambda,
                              double sign, const double* __restrict__ z, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = kind[i];
    const double e = (k == 1 || k == 3) ? eps_x : (k == 4 ? -eps_lambda : 0.0);
    out[i] += sign * e * z[i];
  }
}

__global__ void k_const_slots(int64_t n, const int64_t* slots, double value, double* vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    vals[slots[i]] += value;
}

__global__ void k_gather_vec(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ src,
                             const double* __restrict__ ebuf, const double* __restrict__ fext,
                             const double* __restrict__ pforce, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = sum_sources(ptr[i], ptr[i + 1], src, ebuf);
    acc -= fext[i];
    if (pforce) acc -= pforce[i];
    out[i] = acc;
  }
}

// Fixed-shape block reduction: 256 threads, pairwise tree in LDS.
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) k_dot_partials(int64_t n, const double* __restrict__ a,
                                                      const double* __restrict__ b, int64_t sa, int absval,
                                                      double* __restrict__ partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double x = absval ? fabs(a[i * sa]) : a[i * sa];
    acc += b ? x * b[i] : x;
  }
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_final_sum(const double* partials, int np, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += partials[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = r;
}

__global__ void __launch_bounds__(256) k_max_abs_partials(int64_t n, const double* __restrict__ a,
                                                          double* __restrict__ partials) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) acc = fmax(acc, fabs(a[i]));
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_final_max(const double* partials, int np, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc = fmax(acc, partials[i]);
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) *out = r;
}

// Per-segment reductions and updates for batches of independent problems: segment s covers
// [off[s], off[s+1]); one block per segment, fixed summation order (bitwise reproducible).
__global__ void __launch_bounds__(256) k_segment_dot(const int64_t* __restrict__ off, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double sh[256];
  const int64_t lo = off[blockIdx.x], hi = off[blockIdx.x + 1];
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += a[i] * b[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// out[i] = x[i] + alpha[s] dir[i] on segment s
__global__ void __launch_bounds__(256) k_segment_axpy(const int64_t* __restrict__ off, const double* __restrict__ alpha,
                                                      const double* __restrict__ x, const double* __restrict__ dir,
                                                      double* __restrict__ out) {
  const int64_t lo = off[blockIdx.x], hi = off[blockIdx.x + 1];
  const double a = alpha[blockIdx.x];
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) out[i] = x[i] + a * dir[i];
}

// dst[i] = src[i] on the segments whose mask is set
__global__ void __launch_bounds__(256) k_segment_copy(const int64_t* __restrict__ off, const int32_t* __restrict__ mask,
                                                      const double* __restrict__ src, double* __restrict__ dst) {
  if (!mask[blockIdx.x]) return;
  const int64_t lo = off[blockIdx.x], hi = off[blockIdx.x + 1];
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) dst[i] = src[i];
}

__global__ void k_gather_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double v = in[perm[k]];
    out[k] = scale ? scale[k] * v : v;
  }
}

__global__ void k_scatter_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double v = in[k];
    out[perm[k]] = scale ? scale[k] * v : v;
  }
}

__global__ void k_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = a * x[k] + (y ? b * y[k] : 0.0);
}

// w += sign * sum_{t < j} coef[t] V[t], the basis V stored as j vectors of stride ldv; the sum over t
// runs in ascending order (bitwise reproducible)
__global__ void k_multi_axpy(int64_t n, int j, const double* __restrict__ V, int64_t ldv,
                             const double* __restrict__ coef, double sign, double* __restrict__ w) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < j; ++t) acc += coef[t] * V[t * ldv + k];
    w[k] += sign * acc;
  }
}

__global__ void k_scale(int64_t n, const double* sc, const double* in, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = sc[k] * in[k];
}

__global__ void k_fill(int64_t n, double v, double* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = v;
}

__global__ void k_rel_flag(const double* r2, const double* b2, double rtol, double* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double rel = *b2 > 0.0 ? sqrt(*r2 / *b2) : 0.0;
    out[0] = rel;
    out[1] = rel <= rtol ? 1.0 : 0.0;
  }
}

__global__ void k_fill_i32(int64_t n, int32_t v, int32_t* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = v;
}

__global__ void k_fill_bytes(int64_t n16, uint4* out) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n16; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = z;
}

// RL lanes per row (64 / RL rows per wavefront): lane l sums the row's entries l, l + RL, l + 2 RL, ...
// in ascending order, four loads in flight per pass (indices clamped to the row's first entry, products
// masked), then a fixed butterfly over the RL lanes.  RL follows the matrix's mean row length, so that a
// pass of four loads per lane covers about one row: short rows on 16 lanes left most loads idle.
template <int RL>
__global__ void __launch_bounds__(256) k_spmv(int64_t N, const int64_t* __restrict__ frp,
                                              const int32_t* __restrict__ fcol, const int32_t* __restrict__ fslot,
                                              const double* __restrict__ vals, const double* __restrict__ x,
                                              const double* __restrict__ b, double* __restrict__ y) {
  const int sub = threadIdx.x & (RL - 1);
  const int64_t row = (int64_t)blockIdx.x * (256 / RL) + (threadIdx.x / RL);
  if (row >= N) return;  // whole RL-lane groups leave together
  const int64_t t0 = frp[row], t1 = frp[row + 1];
  double acc = 0.0;
  for (int64_t t = t0 + sub; t < t1; t += 4 * RL) {
    int32_t sl[4], cl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t tt = t + q * RL, tc = tt < t1 ? tt : t0;
      sl[q] = fslot[tc];
      cl[q] = fcol[tc];
    }
    double pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) pv[q] = vals[sl[q]] * x[cl[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (t + q * RL < t1) acc += pv[q];
  }
  for (int off = RL / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, RL);
  if (sub == 0) y[row] = b ? b[row] - acc : acc;
}

// max |K_ij| over row i, RL lanes per row as in the SpMV (max is order-independent)
template <int RL>
__global__ void __launch_bounds__(256) k_row_scaling(int64_t N, const int64_t* __restrict__ frp,
                                                     const int32_t* __restrict__ fslot,
                                                     const double* __restrict__ vals, double* __restrict__ scale) {
  const int sub = threadIdx.x & (RL - 1);
  const int64_t row = (int64_t)blockIdx.x * (256 / RL) + (threadIdx.x / RL);
  if (row >= N) return;
  const int64_t t0 = frp[row], t1 = frp[row + 1];
  double m = 0.0;
  for (int64_t t = t0 + sub; t < t1; t += 4 * RL) {
    int32_t sl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t tt = t + q * RL;
      sl[q] = fslot[tt < t1 ? tt : t0];
    }
    double av[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) av[q] = fabs(vals[sl[q]]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (t + q * RL < t1) m = fmax(m, av[q]);
  }
  for (int off = RL / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, RL));
  if (sub == 0) scale[row] = m > 0.0 ? 1.0 / sqrt(m) : 1.0;
}

__global__ void k_objective_fx(int64_t nt, const int32_t* tdof, const double* tval, const double* x, double c,
                               double* fx) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt; k += (int64_t)gridDim.x * blockDim.x)
    fx[tdof[k]] = c * (x[tdof[k]] - tval[k]);
}

inline unsigned grid_for(int64_t n, int bs, int64_t cap = 65536) {
  int64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

void launch_element(const ElemArgs& a, hipStream_t s) {
  if (a.ne <= 0) return;
  const unsigned g = (unsigned)((a.ne + 127) / 128);
  if (a.mode == 3) {
    if (a.dim == 2) k_element<2, true><<<g, 128, 0, s>>>(a);
    else k_element<3, true><<<g, 128, 0, s>>>(a);
  } else {
    if (a.dim == 2) k_element<2, false><<<g, 128, 0, s>>>(a);
    else k_element<3, false><<<g, 128, 0, s>>>(a);
  }
}

void launch_gather_slots(int64_t nnz, const int64_t* ptr, const int32_t* src, const double* ebuf, double* vals,
                         hipStream_t s) {
  if (nnz > 0) k_gather_slots<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, ptr, src, ebuf, vals);
}

void launch_diag_add(int64_t N, const int64_t* rowptr, const int32_t* kind, double a_target, double c_param,
                     double eps_x, double eps_lambda, double* vals, hipStream_t s) {
  if (N > 0) k_diag_add<<<grid_for(N, 256), 256, 0, s>>>(N, rowptr, kind, a_target, c_param, eps_x, eps_lambda, vals);
}

void launch_unstabilise(int64_t N, const int32_t* kind, double eps_x, double eps_lambda, double sign, const double* z,
                        double* out, hipStream_t s) {
  if (N > 0) k_unstabilise<<<grid_for(N, 256), 256, 0, s>>>(N, kind, eps_x, eps_lambda, sign, z, out);
}

void launch_const_slots(int64_t n, const int64_t* slots, double value, double* vals, hipStream_t s) {
  if (n > 0) k_const_slots<<<grid_for(n, 256), 256, 0, s>>>(n, slots, value, vals);
}

void launch_gather_vec(int64_t n, const int64_t* ptr, const int32_t* src, const double* ebuf, const double* fext,
                       const double* pforce, double* out, hipStream_t s) {
  if (n > 0) k_gather_vec<<<grid_for(n, 256), 256, 0, s>>>(n, ptr, src, ebuf, fext, pforce, out);
}

void launch_dot_partials(int64_t n, const double* a, const double* b, int64_t stride_a, int absval, double* partials,
                         hipStream_t s) {
  k_dot_partials<<<kRedBlocks, 256, 0, s>>>(n, a, b, stride_a, absval, partials);
}

void launch_final_sum(const double* partials, int np, double* out, hipStream_t s) {
  k_final_sum<<<1, 256, 0, s>>>(partials, np, out);
}

void launch_max_abs_partials(int64_t n, const double* a, double* partials, hipStream_t s) {
  k_max_abs_partials<<<kRedBlocks, 256, 0, s>>>(n, a, partials);
}

void launch_final_max(const double* partials, int np, double* out, hipStream_t s) {
  k_final_max<<<1, 256, 0, s>>>(partials, np, out);
}

void launch_segment_dot(int nseg, const int64_t* off, const double* a, const double* b, double* out, hipStream_t s) {
  if (nseg > 0) k_segment_dot<<<nseg, 256, 0, s>>>(off, a, b, out);
}

void launch_segment_axpy(int nseg, const int64_t* off, const double* alpha, const double* x, const double* dir,
                         double* out, hipStream_t s) {
  if (nseg > 0) k_segment_axpy<<<nseg, 256, 0, s>>>(off, alpha, x, dir, out);
}

void launch_segment_copy(int nseg, const int64_t* off, const int32_t* mask, const double* src, double* dst,
                         hipStream_t s) {
  if (nseg > 0) k_segment_copy<<<nseg, 256, 0, s>>>(off, mask, src, dst);
}

void launch_gather_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out,
                        hipStream_t s) {
  if (n > 0) k_gather_perm<<<grid_for(n, 256), 256, 0, s>>>(n, perm, scale, in, out);
}

void launch_scatter_perm(int64_t n, const int32_t* perm, const double* scale, const double* in, double* out,
                         hipStream_t s) {
  if (n > 0) k_scatter_perm<<<grid_for(n, 256), 256, 0, s>>>(n, perm, scale, in, out);
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t s) {
  if (n > 0) k_axpby<<<grid_for(n, 256), 256, 0, s>>>(n, a, x, b, y, out);
}

void launch_multi_axpy(int64_t n, int j, const double* V, int64_t ldv, const double* coef, double sign, double* w,
                       hipStream_t s) {
  if (n > 0 && j > 0) k_multi_axpy<<<grid_for(n, 256), 256, 0, s>>>(n, j, V, ldv, coef, sign, w);
}

void launch_scale(int64_t n, const double* sc, const double* in, double* out, hipStream_t s) {
  if (n > 0) k_scale<<<grid_for(n, 256), 256, 0, s>>>(n, sc, in, out);
}

void launch_fill(int64_t n, double v, double* out, hipStream_t s) {
  if (n > 0) k_fill<<<grid_for(n, 256), 256, 0, s>>>(n, v, out);
}

void launch_rel_flag(const double* r2, const double* b2, double rtol, double* out, hipStream_t s) {
  k_rel_flag<<<1, 64, 0, s>>>(r2, b2, rtol, out);
}

void launch_fill_i32(int64_t n, int32_t v, void* out, hipStream_t s) {
  if (n > 0) k_fill_i32<<<grid_for(n, 256, 4096), 256, 0, s>>>(n, v, (int32_t*)out);
}

void launch_fill_bytes(int64_t nbytes, void* out, hipStream_t s) {
  const int64_t n16 = nbytes / 16;  // callers pass 16-byte multiples
  if (n16 > 0) k_fill_bytes<<<grid_for(n16, 256, 1 << 20), 256, 0, s>>>(n16, (uint4*)out);
}

int row_lanes_for(int64_t N, int64_t nnz) {
  const int64_t mean = N > 0 ? nnz / N : 0;
  return mean <= 20 ? 4 : mean <= 48 ? 8 : 16;
}

namespace {
template <int RL>
void spmv_rl(int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot, const double* vals,
             const double* x, const double* b, double* y, hipStream_t s) {
  constexpr int64_t rows = 256 / RL;
  k_spmv<RL><<<(unsigned)((N + rows - 1) / rows), 256, 0, s>>>(N, frowptr, fcol, fslot, vals, x, b, y);
}
void spmv_any(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot,
              const double* vals, const double* x, const double* b, double* y, hipStream_t s) {
  if (N <= 0) return;
  if (row_lanes == 4) spmv_rl<4>(N, frowptr, fcol, fslot, vals, x, b, y, s);
  else if (row_lanes == 8) spmv_rl<8>(N, frowptr, fcol, fslot, vals, x, b, y, s);
  else spmv_rl<16>(N, frowptr, fcol, fslot, vals, x, b, y, s);
}
template <int RL>
void row_scaling_rl(int64_t N, const int64_t* frowptr, const int32_t* fslot, const double* vals, double* scale,
                    hipStream_t s) {
  constexpr int64_t rows = 256 / RL;
  k_row_scaling<RL><<<(unsigned)((N + rows - 1) / rows), 256, 0, s>>>(N, frowptr, fslot, vals, scale);
}
}  // namespace

void launch_spmv(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot,
                 const double* vals, const double* x, double* y, hipStream_t s) {
  spmv_any(row_lanes, N, frowptr, fcol, fslot, vals, x, nullptr, y, s);
}

void launch_residual(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fcol, const int32_t* fslot,
                     const double* vals, const double* x, const double* b, double* out, hipStream_t s) {
  spmv_any(row_lanes, N, frowptr, fcol, fslot, vals, x, b, out, s);
}

void launch_row_scaling(int row_lanes, int64_t N, const int64_t* frowptr, const int32_t* fslot, const double* vals,
                        double* scale, hipStream_t s) {
  if (N <= 0) return;
  if (row_lanes == 4) row_scaling_rl<4>(N, frowptr, fslot, vals, scale, s);
  else if (row_lanes == 8) row_scaling_rl<8>(N, frowptr, fslot, vals, scale, s);
  else row_scaling_rl<16>(N, frowptr, fslot, vals, scale, s);
}

void launch_objective_fx(int64_t nt, const int32_t* tdof, const double* tval, const double* x, double w_over_ell2,
                         double* fx, hipStream_t s) {
  if (nt > 0) k_objective_fx<<<grid_for(nt, 256), 256, 0, s>>>(nt, tdof, tval, x, w_over_ell2, fx);
}

}  // namespace sgn
