// Level-scheduled multifrontal triangular solves with the supernodal factor.
//
// The factorisation does not interchange rows of already factorised columns:
// each panel's Bunch-Kaufman permutation only reorders that panel's own
// columns, so the rows of panel R inside the columns of earlier panels keep
// their original order.  The solves therefore apply each panel's permutation
// at the moment the panel is solved.
//
// Per tree level (forward, leaves to root):
//   F0 (one block per front): gather the pivot entries of the right-hand side
//      and the children's contribution vectors (fixed child order);
//   F1 (one block per panel, pipelined): t_R -= sum_{Q<R} L_RQ y_Q as soon as
//      each earlier panel Q of the same front has published y_Q, then permute
//      and multiply by the inverse of the panel's unit lower block (kept by the
//      factorisation), one wavefront;
//   F2 (many blocks per front): contribution to the parent, t_u - L21 y.
// Backward (root to leaves):
//   B1 (many blocks per front): z = D^-1 y - L21^T v_u, one wavefront per
//      column, v_u read from the solution vector (ancestors are solved); a
//      preconditioner supplies its own block solve of D in place of D^-1 y;
//   B2 (one block per panel, pipelined in reverse): z_R -= sum_{Q>R} L_QR^T v_Q,
//      multiply by the transposed inverse of the panel's block, undo its
//      permutation.
// Pipelined blocks take ordered tickets from their front's atomic counter, so
// a block only ever waits for blocks of its front that started before it;
// every wait is bounded and reports a timeout through an error flag instead of
// hanging.  A panel's results are their own ready signal: before the pipelined
// kernel of a level runs, its values hold a pending marker (a signalling-NaN bit
// pattern that no arithmetic result has), and a consumer polls each value until
// the marker is gone.  Vectors
// are FP64 whatever the factor precision, and every sum has a fixed order,
// so solves are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "symbolic.h"

namespace sgn {

namespace {

constexpr long kSpinLimit = 1L << 22;

__device__ inline int ticket(int* counter) {
  __shared__ int t;
  if (threadIdx.x == 0) t = atomicAdd(counter, 1);
  __syncthreads();
  return t;
}

// Panel results pass between blocks of one launch through device-coherent accesses only: the
// producer writes each value with a device-scope atomic store (written through the per-die caches),
// the consumer polls it with device-scope atomic loads until it is no longer the pending marker.
// Each 8-byte value is written and read whole, so no ordering between values is needed, and no
// whole-cache write-back or invalidation either.
constexpr long long kPending = 0x7ff4d3adbeef5a5all;  // signalling NaN: never an arithmetic result

__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the value at p once it is no longer the pending marker; 0 (and err set) when the bounded wait runs
// out or an earlier wait of the same solve already timed out (so a failure ends every wait fast)
__device__ inline double wait_value(const double* p, int* err) {
  for (long it = 0; it < kSpinLimit; ++it) {
    const double v = ld_dev(p);
    if (__double_as_longlong(v) != kPending) return v;
    if ((it & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0.0;
    __builtin_amdgcn_s_sleep(2);
  }
  atomicExch(err, 1);
  return 0.0;
}

// value of v in lane src (src the same for the whole wavefront): two lane reads into scalar registers
__device__ inline double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Raw buffer loads: a 128-bit resource (base, byte range) plus a per-lane and a scalar byte
// offset; a load outside the range returns 0.  The resource is wavefront-uniform by construction;
// taking base and range through lane reads tells the compiler so even where they were computed
// from vector loads (after an atomic or a store it cannot use scalar loads), and spares a
// per-load loop over distinct resource values.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ inline rsrc_t buffer_rsrc(const void* p, int32_t bytes) {
  const uint64_t u = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(u & 0xffffffffu));
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32));
  void* base = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
template <typename T>
__device__ inline T buffer_load(rsrc_t r, uint32_t voff, int32_t soff) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
  }
}

// Ld[i][j] = F[c0 + i, c0 + j] for i < j < w, else 0 (the upper triangle of the panel's diagonal
// block, where the factorisation keeps the transposed inverse of the unit lower block).  All 16
// loads of a thread are issued before the first LDS store: one memory latency per block, not 16.
template <typename T>
__device__ inline void load_inverse_block(const T* __restrict__ F, int64_t m, int c0, int w, int tid,
                                          double (*Ld)[65]) {
  // every load is unconditional, at a clamped in-block address, and masked afterwards: a
  // predicated load would become a branch with a wait of its own
  const rsrc_t rs = buffer_rsrc(F + c0 + (int64_t)c0 * m, (int32_t)(((int64_t)(w - 1) * m + w) * (int64_t)sizeof(T)));
  const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
  T v[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int idx = tid + 256 * t, i = idx & 63, j = idx >> 6;
    const int ic = i < w ? i : 0, jc = j < w ? j : 0;
    const T val = buffer_load<T>(rs, (uint32_t)(ic * (int)sizeof(T) + jc * cstr), 0);
    v[t] = (i < j && j < w) ? val : (T)0;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int idx = tid + 256 * t;
    Ld[idx & 63][idx >> 6] = (double)v[t];
  }
}

__global__ void __launch_bounds__(256) k_fwd_gather(const int32_t* __restrict__ level_sn, SolveArgs a,
                                                    const double* __restrict__ b) {
  const int tid = threadIdx.x;
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J];
  double* tv = a.tv + a.sn_vec_off[J];
  double* tp = a.tp + a.sn_vec_off[J];
  for (int64_t k = tid; k < m; k += 256) tv[k] = k < s ? b[g0 + k] : 0.0;
  for (int64_t k = tid; k < s; k += 256) tp[k] = __longlong_as_double(kPending);  // y not yet solved
  __syncthreads();
  for (int32_t q = a.child_ptr[J]; q < a.child_ptr[J + 1]; ++q) {
    const int C = a.child_list[q];
    const int64_t sC = f.sn_begin[C + 1] - f.sn_begin[C], uC = f.sn_m[C] - sC;
    const double* cv = a.tp + a.sn_vec_off[C] + sC;
    const int32_t* rel = f.relmap + f.relmap_off[C];
    // eight rows per thread in flight, every load before the first store: the map is injective, so a
    // child's rows land on distinct entries
    for (int64_t r0 = 0; r0 < uC; r0 += 8 * 256) {
      int32_t d[8];
      double c[8], t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t r = r0 + tid + 256 * q, rc = r < uC ? r : 0;
        d[q] = rel[rc];
        c[q] = cv[rc];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = tv[d[q]];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (r0 + tid + 256 * q < uC) tv[d[q]] = t[q] + c[q];
    }
    __syncthreads();
  }
}

// Forward solve of a front with a short panel chain (at most kSolveSeqPanels panels) by one block:
// the panels in order, the y of solved panels kept in LDS, so no flags and no waiting.  Each
// panel's sums, their order and the substitution are those of the pipelined form, so both give
// bitwise the same y.
template <typename T>
__device__ void fwd_front_in_block(int J, const SolveArgs& a, const T* __restrict__ front, double (*part)[64],
                                   double (*Ld)[65], double* ys, int* err) {
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], m = f.sn_m[J], s = f.sn_begin[J + 1] - g0;
  const int32_t pbase = a.panel_ptr[J];
  const int np = a.panel_ptr[J + 1] - pbase - 1;
  if (np > kSolveSeqPanels || s > kSolveSeqPanels * 64) {  // the task table never makes such a task
    if (tid == 0) atomicExch(err, 2);
    return;
  }
  const double* tv = a.tv + a.sn_vec_off[J];
  double* tp = a.tp + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
#pragma unroll 1
  for (int pi = 0; pi < np; ++pi) {
    const int c0 = a.panel_col[pbase + pi], w = a.panel_col[pbase + pi + 1] - c0;
    load_inverse_block(F, m, c0, w, tid, Ld);
    const double tvl = lane < w ? tv[c0 + lane] : 0.0;
    const int src = lane < w ? f.lperm[g0 + c0 + lane] - c0 : 0;
    const uint32_t voff = (uint32_t)((lane < w ? lane : 0) * (int)sizeof(T));
    double acc = 0.0;
#pragma unroll 1
    for (int q = wave; q < pi; q += 4) {
      const int q0 = a.panel_col[pbase + q], nq = a.panel_col[pbase + q + 1] - q0;
      const rsrc_t rs = buffer_rsrc(F + c0 + (int64_t)q0 * m, (int32_t)(((int64_t)(nq - 1) * m + 64) * (int64_t)sizeof(T)));
      T fv[64];
#pragma unroll
      for (int k = 0; k < 64; ++k) fv[k] = buffer_load<T>(rs, voff, (k < nq ? k : 0) * cstr);
      const double tk = lane < nq ? ys[q0 + lane] : 0.0;
#pragma unroll
      for (int k = 0; k < 64; ++k) acc += (double)fv[k] * lane_bcast(tk, k);
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
      double u = 0.0;
      if (lane < w) u = tvl - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
      const double z = __shfl(u, src, 64);
      double y = z;
      // all 64 columns, unpredicated, eight LDS reads in flight at a time: Ld is zero outside its
      // strict triangle and past the panel's width, so the extra terms add nothing
#pragma unroll 8
      for (int j = 0; j < 64; ++j) {
        const double zj = lane_bcast(z, j);
        y += Ld[j][lane] * zj;  // zero unless j < lane < w
      }
      if (lane < w) {
        ys[c0 + lane] = y;
        tp[c0 + lane] = y;
      }
    }
    __syncthreads();
  }
}

// Backward solve of a front with a short panel chain by one block: the panels in reverse order,
// the solved values kept in LDS at their front positions; bitwise the pipelined form's results.
template <typename T>
__device__ void bwd_front_in_block(int J, const SolveArgs& a, const T* __restrict__ front, double* __restrict__ x,
                                   double (*part)[64], double (*Ld)[65], double* xs, int* err) {
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], m = f.sn_m[J], s = f.sn_begin[J + 1] - g0;
  const int32_t pbase = a.panel_ptr[J];
  const int np = a.panel_ptr[J + 1] - pbase - 1;
  if (np > kSolveSeqPanels || s > kSolveSeqPanels * 64) {
    if (tid == 0) atomicExch(err, 2);
    return;
  }
  const double* tv = a.tv + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
#pragma unroll 1
  for (int pi = np - 1; pi >= 0; --pi) {
    const int c0 = a.panel_col[pbase + pi], w = a.panel_col[pbase + pi + 1] - c0;
    load_inverse_block(F, m, c0, w, tid, Ld);
    const double tvl = lane < w ? tv[c0 + lane] : 0.0;
    const int dst = lane < w ? f.lperm[g0 + c0 + lane] : 0;
    double acc = 0.0;
    const uint32_t voff = (uint32_t)((lane < w ? lane : 0) * m * (int64_t)sizeof(T));
#pragma unroll 1
    for (int q = np - 1 - wave; q > pi; q -= 4) {
      const int q0 = a.panel_col[pbase + q], nq = a.panel_col[pbase + q + 1] - q0;
      const rsrc_t rs = buffer_rsrc(F + q0 + (int64_t)c0 * m, (int32_t)(((int64_t)(w - 1) * m + nq) * (int64_t)sizeof(T)));
      T fv[64];
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) fv[kk] = buffer_load<T>(rs, voff, (kk < nq ? kk : 0) * (int)sizeof(T));
      const double vl = lane < nq ? xs[q0 + lane] : 0.0;
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) acc += (double)fv[kk] * lane_bcast(vl, kk);
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
      double z = 0.0;
      if (lane < w) z = tvl - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
      double v = z;
      // all 64 columns, unpredicated, eight LDS reads in flight at a time: Ld is zero outside its
      // strict triangle and past the panel's width, so the extra terms add nothing
#pragma unroll 8
      for (int j = 0; j < 64; ++j) {
        const double zj = lane_bcast(z, j);
        v += Ld[lane][j] * zj;  // zero unless lane < j < w
      }
      if (lane < w) {
        xs[dst] = v;
        x[g0 + dst] = v;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fwd_panels(const int32_t* __restrict__ tasks, int64_t ntasks, SolveArgs a,
                                                    const T* __restrict__ front, int* counter, int* err) {
  __shared__ double part[4][64];
  __shared__ double Ld[64][65];
  __shared__ double ys[kSolveSeqPanels * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (blockIdx.x >= ntasks) return;
  const int J = tasks[2 * blockIdx.x];
  if (tasks[2 * blockIdx.x + 1] < 0) {
    fwd_front_in_block<T>(J, a, front, part, Ld, ys, err);
    return;
  }
  // the task list holds one entry per panel of each front; the block serves that front and takes
  // the front's next panel in start order, so it only ever waits for blocks that started before it
  const int pi = __builtin_amdgcn_readfirstlane(ticket(counter + J));
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], m = f.sn_m[J];
  const int32_t pbase = a.panel_ptr[J];
  const int c0 = a.panel_col[pbase + pi], c1 = a.panel_col[pbase + pi + 1], w = c1 - c0;
  const double* tv = a.tv + a.sn_vec_off[J];
  double* tp = a.tp + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  // the panel's own block does not depend on other panels: load it before waiting.  The factor keeps
  // the inverse of the panel's unit lower block in the diagonal block's upper triangle, transposed:
  // Ld[j][i] = (L11^-1)[i][j] for j < i
  load_inverse_block(F, m, c0, w, tid, Ld);
  // values of this panel that no other panel produces: read before any wait
  const double tvl = lane < w ? tv[c0 + lane] : 0.0;
  const int src = lane < w ? f.lperm[g0 + c0 + lane] - c0 : 0;
  // contributions of the earlier panels, panel Q handled by wave Q % 4
  double acc = 0.0;
  const uint32_t voff = (uint32_t)((lane < w ? lane : 0) * (int)sizeof(T));
  const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
  for (int q = wave; q < pi; q += 4) {
    const int q0 = a.panel_col[pbase + q], nq = a.panel_col[pbase + q + 1] - q0;
    // the factor entries do not depend on the other panel: issue their loads first (rows c0.. of
    // columns q0..q0+nq-1 through one buffer resource, scalar column offsets)
    const rsrc_t rs = buffer_rsrc(F + c0 + (int64_t)q0 * m, (int32_t)(((int64_t)(nq - 1) * m + 64) * (int64_t)sizeof(T)));
    T fv[64];  // factor precision in registers, widened at use
#pragma unroll
    for (int k = 0; k < 64; ++k) fv[k] = buffer_load<T>(rs, voff, (k < nq ? k : 0) * cstr);
    const double tk = lane < nq ? wait_value(tp + q0 + lane, err) : 0.0;
#pragma unroll
    for (int k = 0; k < 64; ++k) acc += (double)fv[k] * lane_bcast(tk, k);
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    // u in original row order, then the panel permutation, then y = L11^-1 (P u): independent
    // products instead of a dependent substitution
    double u = 0.0;
    if (lane < w) u = tvl - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
    const double z = __shfl(u, src, 64);
    double y = z;
    // all 64 columns, unpredicated, eight LDS reads in flight at a time: Ld is zero outside its
    // strict triangle and past the panel's width, so the extra terms add nothing
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
      const double zj = lane_bcast(z, j);
      y += Ld[j][lane] * zj;  // zero unless j < lane < w
    }
    if (lane < w) st_dev(tp + c0 + lane, y);
  }
}

// Split-k partial sums of L21 y: block (front, 256-row strip, k-chunk of 256 columns), one row per
// thread; each column of the strip is one contiguous 1 KB (FP32) piece.  A thread keeps kRectK
// column loads in flight and reads the chunk's y values from LDS, where they are
// staged once per block; the sum over k runs in ascending order.
constexpr int kRectK = 32;
template <typename T>
__global__ void __launch_bounds__(256, 4) k_fwd_rect(const int32_t* __restrict__ level_sn, SolveArgs a,
                                                  const T* __restrict__ front) {
  __shared__ double yk[256];
  const int tid = threadIdx.x;
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J], u = m - s;
  const int64_t r0 = (int64_t)blockIdx.y * 256;
  const int64_t kb = (int64_t)blockIdx.z * 256;
  if (r0 >= u || kb >= s) return;
  const double* tp = a.tp + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  const int64_t r = r0 + tid;
  const int nk = (int)(s - kb < 256 ? s - kb : 256);
  yk[tid] = tid < nk ? tp[kb + tid] : 0.0;
  // the strip's columns through one buffer resource: per-column offsets are scalar, so the
  // loads in flight cost no address registers; rows past u read row r0 and are not stored
  const rsrc_t rs = buffer_rsrc(F + s + r0 + kb * m, (int32_t)(((int64_t)(nk - 1) * m + 256) * (int64_t)sizeof(T)));
  const uint32_t voff = (uint32_t)((r < u ? tid : 0) * (int)sizeof(T));
  const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
  __syncthreads();
  double acc = 0.0;
#pragma unroll 1
  for (int k0 = 0; k0 < nk; k0 += kRectK) {
    T fv[kRectK];
#pragma unroll
    for (int k = 0; k < kRectK; ++k) fv[k] = buffer_load<T>(rs, voff, (k0 + k < nk ? k0 + k : 0) * cstr);
#pragma unroll
    for (int k = 0; k < kRectK; ++k) acc += (double)fv[k] * yk[k0 + k];
  }
  if (r < u) a.part[a.sn_part_off[J] + blockIdx.z * u + r] = acc;
}

// t_u = tv_u - sum over k-chunks (ascending) of the partial sums
__global__ void __launch_bounds__(256) k_fwd_rect_sum(const int32_t* __restrict__ level_sn, SolveArgs a) {
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J], u = m - s;
  const int64_t r = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (r >= u) return;
  const int64_t nkc = (s + 255) / 256;
  const double* pp = a.part + a.sn_part_off[J] + r;
  double acc = 0.0;
  for (int64_t kc = 0; kc < nkc; ++kc) acc += pp[kc * u];
  a.tp[a.sn_vec_off[J] + s + r] = a.tv[a.sn_vec_off[J] + s + r] - acc;
}

// z_k = (D^-1 y)_k - sum_r L21[r, k] x[row_r] into tv[k]; one wavefront per four pivot columns,
// which share the gathered x[row_r].  Per 256 rows a lane issues its 16 factor loads (clamped to
// the front, masked by x = 0) alongside the row-index and x loads, so the factor stream does not
// wait on the gather.  Each column's sum runs over the rows in the same per-lane order as a
// one-column-per-wavefront loop, then across lanes by the same butterfly.
template <typename T>
__global__ void __launch_bounds__(256) k_bwd_rect(const int32_t* __restrict__ level_sn, SolveArgs a,
                                                  const T* __restrict__ front, double* __restrict__ x) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int J = level_sn[blockIdx.x];
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], s = f.sn_begin[J + 1] - g0, m = f.sn_m[J], u = m - s;
  const int64_t k0 = (int64_t)blockIdx.y * 16 + wave * 4;
  if (k0 >= s) return;
  const int nk = (int)(s - k0 < 4 ? s - k0 : 4);
  const double* tp = a.tp + a.sn_vec_off[J];
  double* tv = a.tv + a.sn_vec_off[J];
  const int32_t* rows = f.sn_rows + f.sn_rows_ptr[J];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (u > 0) {
    // rows s.. of columns k0..k0+nk-1
    const rsrc_t rs = buffer_rsrc(front + f.sn_front_off[J] + s + k0 * m,
                                  (int32_t)(((int64_t)(nk - 1) * m + u) * (int64_t)sizeof(T)));
    const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
#pragma unroll 1
    for (int64_t r0 = 0; r0 < u; r0 += 256) {
      double xv[4];
      T fv[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + lane + 64 * q;
        const int64_t rc = r < u ? r : 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) fv[c][q] = buffer_load<T>(rs, (uint32_t)(rc * (int64_t)sizeof(T)), (c < nk ? c : 0) * cstr);
        const double xl = x[rows[rc]];
        xv[q] = r < u ? xl : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)fv[c][q] * xv[q];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = wave_sum(acc[c]);
  if (lane < nk) {
    const int64_t k = k0 + lane;
    const double sum = lane == 0 ? acc[0] : lane == 1 ? acc[1] : lane == 2 ? acc[2] : acc[3];
    const int t = f.pivtype[g0 + k];
    double w;
    if (a.wd) {
      w = a.wd[g0 + k];
    } else if (t == 0) {
      w = tp[k] / f.dpiv[g0 + k];
    } else if (t == 1) {
      const double A = f.dpiv[g0 + k], B = f.epiv[g0 + k], C = f.dpiv[g0 + k + 1];
      w = (C * tp[k] - B * tp[k + 1]) / (A * C - B * B);
    } else {
      const double A = f.dpiv[g0 + k - 1], B = f.epiv[g0 + k - 1], C = f.dpiv[g0 + k];
      w = (A * tp[k] - B * tp[k - 1]) / (A * C - B * B);
    }
    tv[k] = w - sum;
    x[g0 + k] = __longlong_as_double(kPending);  // solved by the panel kernel of this level
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bwd_panels(const int32_t* __restrict__ tasks, int64_t ntasks, SolveArgs a,
                                                    const T* __restrict__ front, double* __restrict__ x,
                                                    int* counter, int* err) {
  __shared__ double part[4][64];
  __shared__ double Ld[64][65];
  __shared__ double xs[kSolveSeqPanels * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (blockIdx.x >= ntasks) return;
  const int J = tasks[2 * blockIdx.x];
  if (tasks[2 * blockIdx.x + 1] < 0) {
    bwd_front_in_block<T>(J, a, front, x, part, Ld, xs, err);
    return;
  }
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J], m = f.sn_m[J];
  const int32_t pbase = a.panel_ptr[J];
  const int np = a.panel_ptr[J + 1] - pbase - 1;
  const int pi = np - 1 - __builtin_amdgcn_readfirstlane(ticket(counter + J));  // the front's panels in reverse start order
  const int c0 = a.panel_col[pbase + pi], c1 = a.panel_col[pbase + pi + 1], w = c1 - c0;
  const double* tv = a.tv + a.sn_vec_off[J];
  const T* F = front + f.sn_front_off[J];
  load_inverse_block(F, m, c0, w, tid, Ld);  // Ld[i][j] = (L11^-1)[j][i] for i < j (see the forward solve)
  const double tvl = lane < w ? tv[c0 + lane] : 0.0;  // read before any wait
  const int dst = lane < w ? f.lperm[g0 + c0 + lane] : 0;
  // contributions of the later panels Q (every fourth one per wave, in the order they are
  // solved): lane = column c0+lane of panel R, summing L[q0 + k', c0 + lane] v[q0 + k']
  double acc = 0.0;
  const uint32_t voff = (uint32_t)((lane < w ? lane : 0) * m * (int64_t)sizeof(T));
  for (int q = np - 1 - wave; q > pi; q -= 4) {  // completion order: last panel first
    const int q0 = a.panel_col[pbase + q], nq = a.panel_col[pbase + q + 1] - q0;
    // rows q0.. of the panel's columns, unconditional loads at clamped rows (masked by v = 0)
    const rsrc_t rs = buffer_rsrc(F + q0 + (int64_t)c0 * m, (int32_t)(((int64_t)(w - 1) * m + nq) * (int64_t)sizeof(T)));
    T fv[64];  // factor precision in registers, widened at use
#pragma unroll
    for (int kk = 0; kk < 64; ++kk) fv[kk] = buffer_load<T>(rs, voff, (kk < nq ? kk : 0) * (int)sizeof(T));
    const double vl = lane < nq ? wait_value(x + g0 + q0 + lane, err) : 0.0;
#pragma unroll
    for (int kk = 0; kk < 64; ++kk) acc += (double)fv[kk] * lane_bcast(vl, kk);
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double z = 0.0;
    if (lane < w) z = tvl - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
    double v = z;  // v = L11^-T z
    // all 64 columns, unpredicated, eight LDS reads in flight at a time: Ld is zero outside its
    // strict triangle and past the panel's width, so the extra terms add nothing
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
      const double zj = lane_bcast(z, j);
      v += Ld[lane][j] * zj;  // zero unless lane < j < w
    }
    if (lane < w) st_dev(x + g0 + dst, v);
  }
}

// ---- fronts of one panel (s <= 64 pivots, u <= kOneMaxU rows below them): one wavefront per front
//
// Forward: the gathered right-hand side t (pivot entries of b, children's contribution vectors
// added in the fixed child order) stays in LDS; y = L11^-1 P t_s by substitution with the unit
// lower block (rows on lanes, so every factor load is one contiguous column piece), then the
// contribution to the parent t_u - L21 y, rows on lanes, the sum over pivot columns in ascending
// order.  Backward: L21^T x_u with rows on lanes (contiguous loads again), per 16 pivot columns a
// butterfly that halves the set of columns a lane carries at each exchange leaves each column's
// sum on the lanes congruent to it mod 16; then v = L11^-T (D^-1 y - L21^T x_u), scattered by the
// panel's permutation.  No flags and no waits: a front's solve is one wavefront's program order.
constexpr int kOneWaves = 4;  // fronts per block
constexpr int kOneChunk = 16;  // factor loads in flight per lane

template <typename T>
__device__ void fwd_one(int J, const SolveArgs& a, const T* __restrict__ front, const double* __restrict__ b,
                        double* tv, double* zy) {
  const int lane = threadIdx.x & 63;
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J];
  const int s = (int)(f.sn_begin[J + 1] - g0), m = f.sn_m[J], u = m - s;
  double* tp = a.tp + a.sn_vec_off[J];
  for (int k = lane; k < m; k += 64) tv[k] = k < s ? b[g0 + k] : 0.0;
  __builtin_amdgcn_wave_barrier();
  for (int32_t q = a.child_ptr[J]; q < a.child_ptr[J + 1]; ++q) {
    const int C = a.child_list[q];
    const int64_t sC = f.sn_begin[C + 1] - f.sn_begin[C], uC = f.sn_m[C] - sC;
    const double* cv = a.tp + a.sn_vec_off[C] + sC;
    const int32_t* rel = f.relmap + f.relmap_off[C];
    for (int64_t r = lane; r < uC; r += 64) tv[rel[r]] += cv[r];  // a child's rows land on distinct entries
    __builtin_amdgcn_wave_barrier();
  }
  const T* F = front + f.sn_front_off[J];
  const double tvl = lane < s ? tv[lane] : 0.0;
  const int src = lane < s ? f.lperm[g0 + lane] : 0;
  const double zs = __shfl(tvl, src, 64);
  const double z = lane < s ? zs : 0.0;
  // y = L11^-1 z: L11[lane][j], j < lane, is kept at F[lane + j m] (below the diagonal of the
  // panel's block); y_j is final once the steps before j are done.  Clamped loads, masked at use;
  // each chunk's loads are issued while the previous chunk is used.
  double y = z;
  {
    const rsrc_t rs = buffer_rsrc(F, (int32_t)(((int64_t)(s - 1) * m + s) * (int64_t)sizeof(T)));
    const uint32_t voff = (uint32_t)((lane < s ? lane : 0) * (int)sizeof(T));
    const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
    T cur[kOneChunk], nxt[kOneChunk];
#pragma unroll
    for (int j = 0; j < kOneChunk; ++j) cur[j] = buffer_load<T>(rs, voff, (j < s ? j : 0) * cstr);
#pragma unroll 1
    for (int j0 = 0; j0 < s; j0 += kOneChunk) {
      const int j1 = j0 + kOneChunk;
      if (j1 < s) {
#pragma unroll
        for (int j = 0; j < kOneChunk; ++j) nxt[j] = buffer_load<T>(rs, voff, (j1 + j < s ? j1 + j : 0) * cstr);
      }
#pragma unroll
      for (int j = 0; j < kOneChunk; ++j)
        if (j0 + j < s) y -= (lane > j0 + j ? (double)cur[j] : 0.0) * lane_bcast(y, j0 + j);
#pragma unroll
      for (int j = 0; j < kOneChunk; ++j) cur[j] = nxt[j];
    }
  }
  if (lane < s) tp[lane] = y;
  __builtin_amdgcn_wave_barrier();
  zy[lane] = lane < s ? y : 0.0;
  __builtin_amdgcn_wave_barrier();
  if (u <= 0) return;
  // rows below: lane = row, columns past s read column 0 and meet y = 0; the (row block, column
  // chunk) pieces in order, each piece's loads issued while the previous one is used
  const rsrc_t rs = buffer_rsrc(F + s, (int32_t)(((int64_t)(s - 1) * m + u) * (int64_t)sizeof(T)));
  const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
  const int nk = (s + kOneChunk - 1) / kOneChunk, npieces = nk * ((u + 63) / 64);
  auto load_piece = [&](int q, T* dst) {
    const int r = (q / nk) * 64 + lane, k0 = (q % nk) * kOneChunk;
    const uint32_t voff = (uint32_t)((r < u ? r : 0) * (int)sizeof(T));
#pragma unroll
    for (int k = 0; k < kOneChunk; ++k) dst[k] = buffer_load<T>(rs, voff, (k0 + k < s ? k0 + k : 0) * cstr);
  };
  T cur[kOneChunk], nxt[kOneChunk];
  load_piece(0, cur);
  double acc = 0.0;
#pragma unroll 1
  for (int q = 0; q < npieces; ++q) {
    if (q + 1 < npieces) load_piece(q + 1, nxt);
    const int k0 = (q % nk) * kOneChunk;  // k0 + k < 64: zy is zero past s
#pragma unroll
    for (int k = 0; k < kOneChunk; ++k) acc += (double)cur[k] * zy[k0 + k];
    if (q % nk == nk - 1) {  // the row block's last chunk
      const int r = (q / nk) * 64 + lane;
      if (r < u) tp[s + r] = tv[s + r] - acc;
      acc = 0.0;
    }
#pragma unroll
    for (int k = 0; k < kOneChunk; ++k) cur[k] = nxt[k];
  }
}

template <typename T>
__device__ void bwd_one(int J, const SolveArgs& a, const T* __restrict__ front, double* __restrict__ x, double* zy) {
  const int lane = threadIdx.x & 63;
  const FrontArgs& f = a.f;
  const int64_t g0 = f.sn_begin[J];
  const int s = (int)(f.sn_begin[J + 1] - g0), m = f.sn_m[J], u = m - s;
  const double* tp = a.tp + a.sn_vec_off[J];
  const int32_t* rows = f.sn_rows + f.sn_rows_ptr[J];
  const T* F = front + f.sn_front_off[J];
  const int kc = lane < s ? lane : 0;  // this lane's pivot column (clamped)
  // sum over the rows of L21[r][lane] x[row r]
  double sum = 0.0;
  if (u > 0) {
    const rsrc_t rs = buffer_rsrc(F + s, (int32_t)(((int64_t)(s - 1) * m + u) * (int64_t)sizeof(T)));
    const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
#pragma unroll 1
    for (int k0 = 0; k0 < s; k0 += kOneChunk) {
      // c[i]: this lane's rows' part of column k0 + i
      double c[kOneChunk];
#pragma unroll
      for (int i = 0; i < kOneChunk; ++i) c[i] = 0.0;
#pragma unroll 1
      for (int r0 = 0; r0 < u; r0 += 64) {
        const int r = r0 + lane;
        const uint32_t voff = (uint32_t)((r < u ? r : 0) * (int)sizeof(T));
        T fv[kOneChunk];
#pragma unroll
        for (int i = 0; i < kOneChunk; ++i) fv[i] = buffer_load<T>(rs, voff, (k0 + i < s ? k0 + i : 0) * cstr);
        const double xr = x[rows[r < u ? r : 0]];
        const double xm = r < u ? xr : 0.0;
#pragma unroll
        for (int i = 0; i < kOneChunk; ++i) c[i] += (double)fv[i] * xm;
      }
      // exchanges across lane bits 3..0: a lane keeps the columns whose bit equals its own and adds
      // the partner's part of them; then the four groups of 16 lanes are added
#pragma unroll
      for (int h = kOneChunk / 2; h >= 1; h >>= 1) {
        const bool up = (lane & h) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
          const double keep = up ? c[i + h] : c[i];
          const double send = up ? c[i] : c[i + h];
          c[i] = keep + __shfl_xor(send, h, 64);
        }
      }
      double t = c[0];  // column k0 + (lane & 15), over this lane's group of 16
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
      if ((lane & ~(kOneChunk - 1)) == k0) sum = t;
    }
  }
  // z = D^-1 y - L21^T x_u on the pivot lanes
  double z = 0.0;
  if (lane < s) {
    const int64_t k = lane;
    const int t = f.pivtype[g0 + k];
    double w;
    if (a.wd) {
      w = a.wd[g0 + k];
    } else if (t == 0) {
      w = tp[k] / f.dpiv[g0 + k];
    } else if (t == 1) {
      const double A = f.dpiv[g0 + k], B = f.epiv[g0 + k], C = f.dpiv[g0 + k + 1];
      w = (C * tp[k] - B * tp[k + 1]) / (A * C - B * B);
    } else {
      const double A = f.dpiv[g0 + k - 1], B = f.epiv[g0 + k - 1], C = f.dpiv[g0 + k];
      w = (A * tp[k] - B * tp[k - 1]) / (A * C - B * B);
    }
    z = w - sum;
  }
  zy[lane] = z;  // read back as broadcasts (zero past s)
  __builtin_amdgcn_wave_barrier();
  // v = L11^-T z: (L11^-1)[j][lane], j > lane, is kept at F[lane + j m]
  double v = z;
  {
    const rsrc_t rs = buffer_rsrc(F, (int32_t)(((int64_t)(s - 1) * m + s) * (int64_t)sizeof(T)));
    const uint32_t voff = (uint32_t)(kc * (int)sizeof(T));
    const int32_t cstr = (int32_t)(m * (int64_t)sizeof(T));
#pragma unroll 1
    for (int j0 = 0; j0 < s; j0 += kOneChunk) {
      T fv[kOneChunk];
#pragma unroll
      for (int j = 0; j < kOneChunk; ++j) fv[j] = buffer_load<T>(rs, voff, (j0 + j < s ? j0 + j : 0) * cstr);
#pragma unroll
      for (int j = 0; j < kOneChunk; ++j) v += (lane < j0 + j ? (double)fv[j] : 0.0) * zy[j0 + j];
    }
  }
  if (lane < s) x[g0 + f.lperm[g0 + lane]] = v;
}

template <typename T>
__global__ void __launch_bounds__(64 * kOneWaves) k_fwd_one(const int32_t* __restrict__ fronts, int64_t n, SolveArgs a,
                                                            const T* __restrict__ front, const double* __restrict__ b) {
  __shared__ double tvs[kOneWaves][kOneMaxM];
  __shared__ double zys[kOneWaves][64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * kOneWaves + wave;
  if (q >= n) return;  // the wavefronts of a block share no data and no barrier
  const int J = fronts[q];
  fwd_one<T>(J, a, front, b, tvs[wave], zys[wave]);
}

template <typename T>
__global__ void __launch_bounds__(64 * kOneWaves) k_bwd_one(const int32_t* __restrict__ fronts, int64_t n, SolveArgs a,
                                                            const T* __restrict__ front, double* __restrict__ x) {
  __shared__ double zys[kOneWaves][64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t q = (int64_t)blockIdx.x * kOneWaves + wave;
  if (q >= n) return;
  const int J = fronts[q];
  bwd_one<T>(J, a, front, x, zys[wave]);
}

}  // namespace

template <typename T>
void launch_fwd_level(int64_t nsn, int64_t max_u, int64_t max_s, const int32_t* level_sn, const int32_t* tasks,
                      int64_t ntasks, const SolveArgs& a, const T* front, const double* b, int* counter, int* err,
                      hipStream_t s) {
  if (nsn <= 0) return;
  k_fwd_gather<<<(unsigned)nsn, 256, 0, s>>>(level_sn, a, b);
  if (ntasks > 0) k_fwd_panels<T><<<(unsigned)ntasks, 256, 0, s>>>(tasks, ntasks, a, front, counter, err);
  if (max_u > 0) {
    if (max_s > 0) {
      dim3 g((unsigned)nsn, (unsigned)((max_u + 255) / 256), (unsigned)((max_s + 255) / 256));
      k_fwd_rect<T><<<g, 256, 0, s>>>(level_sn, a, front);
    }
    dim3 g2((unsigned)nsn, (unsigned)((max_u + 255) / 256));
    k_fwd_rect_sum<<<g2, 256, 0, s>>>(level_sn, a);
  }
}

template <typename T>
void launch_bwd_level(int64_t nsn, int64_t max_s, const int32_t* level_sn, const int32_t* tasks, int64_t ntasks,
                      const SolveArgs& a, const T* front, double* x, int* counter, int* err, hipStream_t s) {
  if (nsn <= 0) return;
  dim3 g((unsigned)nsn, (unsigned)((max_s + 15) / 16));
  k_bwd_rect<T><<<g, 256, 0, s>>>(level_sn, a, front, x);
  if (ntasks > 0)
    k_bwd_panels<T><<<(unsigned)ntasks, 256, 0, s>>>(tasks, ntasks, a, front, x, counter, err);
}

template <typename T>
void launch_fwd_one(int64_t n, const int32_t* fronts, const SolveArgs& a, const T* front, const double* b,
                    hipStream_t s) {
  if (n > 0) k_fwd_one<T><<<(unsigned)((n + kOneWaves - 1) / kOneWaves), 64 * kOneWaves, 0, s>>>(fronts, n, a, front, b);
}

template <typename T>
void launch_bwd_one(int64_t n, const int32_t* fronts, const SolveArgs& a, const T* front, double* x, hipStream_t s) {
  if (n > 0) k_bwd_one<T><<<(unsigned)((n + kOneWaves - 1) / kOneWaves), 64 * kOneWaves, 0, s>>>(fronts, n, a, front, x);
}

template void launch_fwd_one<double>(int64_t, const int32_t*, const SolveArgs&, const double*, const double*,
                                     hipStream_t);
template void launch_fwd_one<float>(int64_t, const int32_t*, const SolveArgs&, const float*, const double*, hipStream_t);
template void launch_bwd_one<double>(int64_t, const int32_t*, const SolveArgs&, const double*, double*, hipStream_t);
template void launch_bwd_one<float>(int64_t, const int32_t*, const SolveArgs&, const float*, double*, hipStream_t);
template void launch_fwd_level<double>(int64_t, int64_t, int64_t, const int32_t*, const int32_t*, int64_t,
                                       const SolveArgs&, const double*, const double*, int*, int*, hipStream_t);
template void launch_fwd_level<float>(int64_t, int64_t, int64_t, const int32_t*, const int32_t*, int64_t,
                                      const SolveArgs&, const float*, const double*, int*, int*, hipStream_t);
template void launch_bwd_level<double>(int64_t, int64_t, const int32_t*, const int32_t*, int64_t, const SolveArgs&,
                                       const double*, double*, int*, int*, hipStream_t);
template void launch_bwd_level<float>(int64_t, int64_t, const int32_t*, const int32_t*, int64_t, const SolveArgs&,
                                      const float*, double*, int*, int*, hipStream_t);

}  // namespace sgn
