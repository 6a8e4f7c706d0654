// Multifrontal supernodal LDL^T of the SGN saddle-point matrix (gfx950).
//
// The paper factorises eq. sparseSystemGN with a sparse direct solver on a
// CPU (Sec. 5, "Solving the saddle point problem"); here every front is a
// dense m x m column-major block (pivot columns first) held in HBM for the
// whole factorisation, processed level by level of the supernode tree:
//   1. original entries of the scaled matrix are scattered into the fronts;
//   2. children's Schur complements are added in a fixed child order
//      (extend-add, one launch per child rank, so sums are deterministic);
//   3. per panel of <= 64 pivot columns (whole node groups):
//        - the panel's diagonal block is factorised in LDS, in the fronts'
//          precision (pivot tests and pivot inverses in FP64), with
//          Bunch-Kaufman 1x1/2x2 pivots restricted to one node's group;
//        - rows below are solved against it (TRSM, one thread per row);
//        - trailing columns are updated with MFMA tiles; updates of columns
//          beyond the current block of 4 panels are delayed and applied
//          with k = 256 (one rank-256 update instead of four rank-64 ones).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sgn {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr double kAlphaBK = 0.6403882032022076;  // (1 + sqrt(17)) / 8

// Output row (M index) held by accumulator register `reg` of `lane` for the
// 16x16x4 matrix-core products; the operand layouts are A[lane%16][lane/16]
// and B[lane/16][lane%16] for both types, the column is lane%16.  Measured on
// gfx950 (the self-test entry point checks it): the FP64 product interleaves
// rows across registers, the FP32 one keeps four consecutive rows per lane.
// Raw buffer loads: a per-lane 32-bit byte offset plus a uniform one from a uniform base held in a
// buffer resource of `bytes` bytes (offsets at or past it read 0; 0x00020000 is the gfx9 descriptor
// word 3 for untyped dword access).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ inline rsrc_t buffer_rsrc(const void* p, int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
template <typename T>
__device__ inline T buffer_load(rsrc_t r, uint32_t voff, int32_t soff) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
  }
}

template <typename T>
__device__ inline int mfma_row(int lane, int reg) {
  return sizeof(T) == 8 ? (lane >> 4) + 4 * reg : 4 * (lane >> 4) + reg;
}

template <typename T>
__global__ void k_csr_to_fronts(int64_t nnz, const int32_t* __restrict__ slot_row, const int32_t* __restrict__ colind,
                                const int64_t* __restrict__ pos, const double* __restrict__ vals,
                                const double* __restrict__ scale, T* __restrict__ front) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = slot_row[t], j = colind[t];
    front[pos[t]] = (T)(scale[i] * vals[t] * scale[j]);
  }
}

// Zeroes rows >= column - 63 of 64 columns of one front (or a whole small front): the lower
// triangle, which the assembly
// and the extend-add accumulate into, and a band of 63 entries above the diagonal.  The trailing
// update reads that band (its diagonal tiles, and the L columns of a partial last k-chunk, which
// are multiplied by zeroed W entries), so the band must hold finite values; entries further above
// the diagonal are never read before the factorisation writes them (the panels' diagonal blocks
// and the W rows of the panel solve), so the rest of the upper triangle is left as it is.
template <typename T>
__global__ void __launch_bounds__(256) k_zero_fronts(const int32_t* __restrict__ tasks, FrontArgs f,
                                                     T* __restrict__ front) {
  // one wavefront per column: scalar stores up to 16-byte alignment, then 16-byte stores, then the
  // scalar tail
  constexpr int64_t V = 16 / sizeof(T);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sn = tasks[2 * blockIdx.x], c0 = tasks[2 * blockIdx.x + 1];
  const int64_t m = f.sn_m[sn];
  T* F = front + f.sn_front_off[sn];
  if (c0 < 0) {
    // -c0 consecutive small fronts whole, from front sn on: they lie back to back, so their entries
    // (and the padding between them) are one contiguous range, zeroed by the block with 16-byte
    // stores (the entries above the band are written before they are read anyway)
    const int tid = threadIdx.x;
    const int64_t n = f.sn_front_off[sn - c0] - f.sn_front_off[sn];
    int64_t head = (int64_t)(((16 - ((uintptr_t)F & 15)) & 15) / sizeof(T));
    if (head > n) head = n;
    if (tid < head) F[tid] = (T)0;
    const int64_t nv = (n - head) / V;
    uint4* vb = reinterpret_cast<uint4*>(F + head);
    for (int64_t v = tid; v < nv; v += 256) vb[v] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t rt = head + nv * V;
    if (rt + tid < n) F[rt + tid] = (T)0;
    return;
  }
  const int64_t c1 = c0 + 64 < m ? c0 + 64 : m;
  for (int64_t c = c0 + wave; c < c1; c += 4) {
    T* col = F + c * m;
    const int64_t r0 = c >= 63 ? c - 63 : 0;
    int64_t head = (int64_t)(((16 - ((uintptr_t)(col + r0) & 15)) & 15) / sizeof(T));
    if (head > m - r0) head = m - r0;
    if (lane < head) col[r0 + lane] = (T)0;
    const int64_t rb = r0 + head, nv = (m - rb) / V;
    uint4* vb = reinterpret_cast<uint4*>(col + rb);
    for (int64_t v = lane; v < nv; v += 64) vb[v] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t rt = rb + nv * V;
    if (rt + lane < m) col[rt + lane] = (T)0;
  }
}

// One wavefront per child column (four per block): adds the child's Schur complement column
// (rows >= column) into the parent front through the child's relative map.  A wavefront rather than
// a block per column keeps the lanes busy on the short columns of small fronts.  The column's
// offsets come from one precomputed record (no chain of table lookups before the data); rows go
// eight per lane at a time, every load (clamped to the column's first row past its end) issued
// before the first store.  The relative map is injective, so the parent entries a wavefront reads
// and writes are distinct.
template <typename T>
__global__ void __launch_bounds__(256) k_extend_add(int64_t ncols, const int64_t* __restrict__ cols, FrontArgs f,
                                                    T* __restrict__ front) {
  constexpr int R = 8;
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= ncols) return;
  const int64_t* rec = cols + 4 * b;
  const int64_t cu = rec[3], c = cu >> 32, uC = cu & 0xffffffffll;
  const T* src = front + rec[0];
  T* dst = front + rec[1];
  const int32_t* rel = f.relmap + rec[2];
  for (int64_t r0 = c; r0 < uC; r0 += 64 * R) {
    T v[R], o[R];
    int32_t d[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t r = r0 + lane + 64 * q;
      const int64_t rc = r < uC ? r : c;
      v[q] = src[rc];
      d[q] = rel[rc];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) o[q] = dst[d[q]];
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (r0 + lane + 64 * q < uC) dst[d[q]] = o[q] + v[q];
  }
}

// Extend-add of a whole small child (u <= kSmallChild) by one block: the lower triangle of its
// update block, column-major, flattened over the threads (short columns would leave most lanes of a
// per-column wavefront idle).  Entry e sits in column c with off(c) <= e < off(c + 1),
// off(c) = c u - c (c - 1) / 2, the smaller root of a quadratic taken in FP32 (exact integers below
// 2^24) and corrected by one step either way.  Every load of a thread (clamped to entry 0) before
// its first store; the relative map is injective, so a block's parent entries are distinct, and
// the children of one round have different parents.
template <typename T>
__global__ void __launch_bounds__(256) k_extend_add_small(const int64_t* __restrict__ kids, FrontArgs f,
                                                          T* __restrict__ front) {
  constexpr int R = 4;
  const int tid = threadIdx.x;
  const int64_t* rec = kids + 5 * (int64_t)blockIdx.x;
  const T* src = front + rec[0];
  T* dst = front + rec[1];
  const int32_t* rel = f.relmap + rec[2];
  const int64_t mc = rec[3];
  const int64_t mp = rec[4] >> 32;
  const int u = (int)(rec[4] & 0xffffffffll);
  const int total = u * (u + 1) / 2;
  const float b2 = 2.0f * (float)u + 1.0f;
  for (int e0 = 0; e0 < total; e0 += 256 * R) {
    T v[R], o[R];
    int64_t d[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int e = e0 + tid + 256 * q, ec = e < total ? e : 0;
      int c = (int)((b2 - sqrtf(b2 * b2 - 8.0f * (float)ec)) * 0.5f);
      c = c < 0 ? 0 : (c > u - 1 ? u - 1 : c);
      c -= (c * u - c * (c - 1) / 2 > ec) ? 1 : 0;
      c += (c + 1 < u && (c + 1) * u - (c + 1) * c / 2 <= ec) ? 1 : 0;
      const int r = c + (ec - (c * u - c * (c - 1) / 2));
      v[q] = src[r + c * mc];
      d[q] = (int64_t)rel[r] + (int64_t)rel[c] * mp;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) o[q] = dst[d[q]];
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (e0 + tid + 256 * q < total) dst[d[q]] = o[q] + v[q];
  }
}

// Factorisation of one panel's diagonal block (w <= WM <= 64) in LDS, 64 * WAVES threads.  The block
// and its updates are in the fronts' precision T (an FP32 block takes half the LDS, so twice the
// blocks share a compute unit, half the lane reads per broadcast and a 32-bit pivot search key); the
// Bunch-Kaufman tests and the 1x1 / 2x2 pivot inverses are in FP64.
// WAVES = 8 shortens a lone panel's step (the update is split over eight wavefronts); WAVES = 1
// leaves no wavefront repeating another's pivot search, which pays when a step holds enough panels
// to fill the chip, and WM = 32 lets more of them share a compute unit's LDS.
// Bunch-Kaufman 1x1/2x2 pivoting restricted to the rows of one node group.  Every
// wavefront reads the pivot column into registers and takes the same pivot decision
// (argmax by a shuffle butterfly over |a| bits with the row index in the low bits, so
// near-ties go to the lower row); the multipliers of the update come from that register
// copy by lane broadcasts.  A step has two barriers (two more for an interchange): one after every
// wavefront has read the pivot columns, before wavefront 0 overwrites them with the multipliers,
// and one at its end.
// The symmetric updates use lane = row, wavefront = every WAVES-th column.
// Alongside L11 the block accumulates X = L11^-1 (unit lower) from the
// elementary column inverses, X <- L_k^-1 X, stored transposed in the upper
// part of the finished rows (X[i][j] at A[j][i]); symmetric interchanges swap
// those entries exactly as X's rows must be swapped.  The rows below the panel
// are then solved by a matrix-core product against X.
__device__ inline double lane_bcast(double v, int src) {  // src uniform across the wavefront
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Maximum over the wavefront: data-parallel-primitive moves within rows of 16 lanes (swap adjacent
// lanes, adjacent pairs, mirrored half rows, mirrored rows), then the four row maxima by lane reads.
template <int CTRL>
__device__ inline unsigned int dpp_u32(unsigned int x) {
  return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
__device__ inline unsigned int wave_max_u32(unsigned int x) {
  x = max(x, dpp_u32<0xB1>(x));   // quad_perm [1, 0, 3, 2]
  x = max(x, dpp_u32<0x4E>(x));   // quad_perm [2, 3, 0, 1]
  x = max(x, dpp_u32<0x141>(x));  // row_half_mirror
  x = max(x, dpp_u32<0x140>(x));  // row_mirror
  unsigned int r = (unsigned int)__builtin_amdgcn_readlane((int)x, 0);
  r = max(r, (unsigned int)__builtin_amdgcn_readlane((int)x, 16));
  r = max(r, (unsigned int)__builtin_amdgcn_readlane((int)x, 32));
  return max(r, (unsigned int)__builtin_amdgcn_readlane((int)x, 48));
}
// 64-bit maximum as two 32-bit ones: the largest high word, then the largest low word among the
// lanes that hold it (the same key as a 64-bit comparison)
__device__ inline unsigned long long wave_max_u64(unsigned long long x) {
  const unsigned int hi = (unsigned int)(x >> 32);
  const unsigned int mh = wave_max_u32(hi);
  const unsigned int ml = wave_max_u32(hi == mh ? (unsigned int)x : 0u);
  return ((unsigned long long)mh << 32) | ml;
}

// The lane holding the largest a >= 0 over the wavefront (-1 if all are 0): the maximum of a key made
// of a's bits with the low 6 replaced by 63 - lane, so near-ties go to the lower row.  An FP32 block
// takes a 32-bit key (one lane reduction), an FP64 block a 64-bit one (two).
__device__ inline int argmax_lane(double a, int lane) {
  const unsigned long long key =
      wave_max_u64(a > 0.0 ? (((unsigned long long)__double_as_longlong(a) & ~63ull) | (unsigned long long)(63 - lane))
                           : 0ull);
  return key ? 63 - (int)(key & 63ull) : -1;
}
__device__ inline int argmax_lane(float a, int lane) {
  const unsigned int key = wave_max_u32(a > 0.0f ? ((__float_as_uint(a) & ~63u) | (unsigned int)(63 - lane)) : 0u);
  return key ? 63 - (int)(key & 63u) : -1;
}
// maximum of a >= 0 over the wavefront (non-negative floats order as their bit patterns)
__device__ inline double wave_max_nonneg(double a) {
  return __longlong_as_double((long long)wave_max_u64((unsigned long long)__double_as_longlong(a)));
}
__device__ inline float wave_max_nonneg(float a) { return __uint_as_float(wave_max_u32(__float_as_uint(a))); }

template <typename T, int WAVES, int WM>
__global__ void __launch_bounds__(64 * WAVES) k_panel_diag(const int64_t* __restrict__ tasks, FrontArgs f,
                                                           T* __restrict__ front) {
  __shared__ T A[WM][WM + 1];  // the block in the fronts' precision; pivot scalars in FP64
  __shared__ int pos[WM];
  constexpr int S = WAVES;  // column stride of a wavefront's share of an update
  const int tid = threadIdx.x, lane = tid & 63, wave = uniform_i(tid >> 6);
  const int sn = (int)tasks[blockIdx.x * 3];
  const int c0 = (int)tasks[blockIdx.x * 3 + 1], c1 = (int)tasks[blockIdx.x * 3 + 2];
  const int w = c1 - c0;
  const int64_t m = f.sn_m[sn];
  const int64_t gbase = f.sn_begin[sn] + c0;
  T* F = front + f.sn_front_off[sn];
  const double tol = f.piv_tol;
  {
    // the panel's lower triangle: all loads of a thread issued unconditionally (clamped to the
    // panel, masked when staged) before the first LDS store
    const int lc = lane < w ? lane : 0;
    constexpr int NL = WM / WAVES;
    T lv[NL];
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int j = wave + WAVES * t, jc = j < w ? j : 0;
      lv[t] = F[(c0 + lc) + (int64_t)(c0 + jc) * m];
    }
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int j = wave + WAVES * t;
      if (j < w && lane >= j && lane < w) {
        const T v = lv[t];
        A[lane][j] = v;
        A[j][lane] = v;
      }
    }
  }
  if (tid < WM) pos[tid] = tid;
  const int gend_r = lane < w ? (int)(f.var_group_end[gbase + lane] - gbase) : w;
  int ptype = 0;
  double dv = 0.0, ev = 0.0;
  __syncthreads();
  int npert = 0;
  int k = 0;
  // lanes past WM hold no row of the block (WM < 64): they read zeros
  const bool row_lane = WM == 64 || lane < WM;
  while (k < w) {
    T v = row_lane ? A[lane][k] : (T)0;
    const int gend = __builtin_amdgcn_readlane(gend_r, k);
    const T cand = (lane > k && lane < gend) ? (T)fabs(v) : (T)0;
    const int am = argmax_lane(cand, lane);
    const int imax = am >= 0 ? am : k;
    const double colmax = am >= 0 ? (double)fabs(lane_bcast(v, imax)) : 0.0;
    const double absakk = (double)fabs(lane_bcast(v, k));
    int kind = 1, p = -1, q = -1;
    bool pert = false;
    if (fmax(absakk, colmax) <= tol) {
      pert = true;
    } else if (absakk < kAlphaBK * colmax) {
      const T u = row_lane ? A[imax][lane] : (T)0;  // row imax
      const T c2 = (lane >= k && lane < gend && lane != imax) ? (T)fabs(u) : (T)0;
      const double rowmax = (double)wave_max_nonneg(c2);
      if (absakk * rowmax >= kAlphaBK * colmax * colmax) {
        kind = 1;
      } else if ((double)fabs(lane_bcast(u, imax)) >= kAlphaBK * rowmax) {
        kind = 1;
        p = k;
        q = imax;
      } else {
        kind = 2;
        p = k + 1;
        q = imax;
      }
    }
    if (p >= 0 && p != q) {
      // symmetric interchange p <-> q in one pass: thread t moves the entries (p,t), (q,t), (t,p), (t,q)
      __syncthreads();  // every wavefront has read column k and row imax
      if (tid < w) {
        const int t = tid;
        if (t != p && t != q) {
          const T apt = A[p][t], aqt = A[q][t], atp = A[t][p], atq = A[t][q];
          A[p][t] = aqt;
          A[q][t] = apt;
          A[t][p] = atq;
          A[t][q] = atp;
        } else if (t == p) {
          const T app = A[p][p], aqq = A[q][q], apq = A[p][q], aqp = A[q][p];
          A[p][p] = aqq;
          A[q][q] = app;
          A[p][q] = aqp;
          A[q][p] = apq;
          const int tp = pos[p];
          pos[p] = pos[q];
          pos[q] = tp;
        }
      }
      __syncthreads();
      v = row_lane ? A[lane][k] : (T)0;
    }
    // every wavefront holds the pivot columns it needs (k, and k + 1 for a 2 x 2 pivot) before any
    // wavefront overwrites them with the step's multipliers
    const T w2 = kind == 2 && row_lane ? A[lane][k + 1] : (T)0;
    __syncthreads();
    if (kind == 1) {
      double d = (double)lane_bcast(v, k);
      if (pert) {
        d = d >= 0.0 ? tol : -tol;
        ++npert;
      } else if (fabs(d) < tol) {
        d = d >= 0.0 ? tol : -tol;
        ++npert;
      }
      const double id = 1.0 / d;
      if (lane > k && lane < w) {
        const T li = (T)((double)v * id);
        // Schur complement and X <- L_k^-1 X; the multipliers A[j][k] are lane j's copy of column k
        int j = k + 1 + wave;
        for (; j + 3 * S < w; j += 4 * S) {
          const T a0 = A[lane][j], a1 = A[lane][j + S], a2 = A[lane][j + 2 * S], a3 = A[lane][j + 3 * S];
          A[lane][j] = a0 - li * lane_bcast(v, j);
          A[lane][j + S] = a1 - li * lane_bcast(v, j + S);
          A[lane][j + 2 * S] = a2 - li * lane_bcast(v, j + 2 * S);
          A[lane][j + 3 * S] = a3 - li * lane_bcast(v, j + 3 * S);
        }
        for (; j < w; j += S) A[lane][j] -= li * lane_bcast(v, j);
        j = wave;
        for (; j + 3 * S < k; j += 4 * S) {
          const T a0 = A[j][lane], a1 = A[j + S][lane], a2 = A[j + 2 * S][lane], a3 = A[j + 3 * S][lane];
          A[j][lane] = a0 - li * lane_bcast(v, j);
          A[j + S][lane] = a1 - li * lane_bcast(v, j + S);
          A[j + 2 * S][lane] = a2 - li * lane_bcast(v, j + 2 * S);
          A[j + 3 * S][lane] = a3 - li * lane_bcast(v, j + 3 * S);
        }
        for (; j < k; j += S) A[j][lane] -= li * lane_bcast(v, j);
        if (wave == 0) {  // column k and row k are read by nobody in this step
          A[lane][k] = li;
          A[k][lane] = -li;
        }
      }
      if (lane == k) {
        ptype = 0;
        dv = d;
        ev = 0.0;
      }
      k += 1;
    } else {
      const double a = (double)lane_bcast(v, k), b = (double)lane_bcast(v, k + 1), c = (double)lane_bcast(w2, k + 1);
      const double det = a * c - b * b;
      const double i00 = c / det, i01 = -b / det, i11 = a / det;
      if (lane > k + 1 && lane < w) {
        const T l0 = (T)((double)v * i00 + (double)w2 * i01), l1 = (T)((double)v * i01 + (double)w2 * i11);
        int j = k + 2 + wave;
        for (; j + 3 * S < w; j += 4 * S) {
          T a4[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) a4[t] = A[lane][j + S * t];
#pragma unroll
          for (int t = 0; t < 4; ++t)
            A[lane][j + S * t] = a4[t] - (l0 * lane_bcast(v, j + S * t) + l1 * lane_bcast(w2, j + S * t));
        }
        for (; j < w; j += S) A[lane][j] -= l0 * lane_bcast(v, j) + l1 * lane_bcast(w2, j);
        j = wave;
        for (; j + 3 * S < k; j += 4 * S) {
          T a4[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) a4[t] = A[j + S * t][lane];
#pragma unroll
          for (int t = 0; t < 4; ++t)
            A[j + S * t][lane] = a4[t] - (l0 * lane_bcast(v, j + S * t) + l1 * lane_bcast(w2, j + S * t));
        }
        for (; j < k; j += S) A[j][lane] -= l0 * lane_bcast(v, j) + l1 * lane_bcast(w2, j);
        if (wave == 0) {
          A[lane][k] = l0;
          A[lane][k + 1] = l1;
          A[k][lane] = -l0;
          A[k + 1][lane] = -l1;
        }
      }
      if (tid == 0) {
        A[k + 1][k] = 0.0;  // L and X are the identity inside a 2x2 block
        A[k][k + 1] = 0.0;
      }
      if (lane == k) {
        ptype = 1;
        dv = a;
        ev = b;
      } else if (lane == k + 1) {
        ptype = 2;
        dv = c;
        ev = 0.0;
      }
      k += 2;
    }
    __syncthreads();
  }
  // A holds L below the diagonal and X[j][i] at (i, j) above it: the transposed
  // placement the rows-below solve reads
  for (int j = wave; j < w; j += WAVES)
    if (lane < w) F[(c0 + lane) + (int64_t)(c0 + j) * m] = (T)(lane == j ? 1.0 : A[lane][j]);
  if (tid < w) {
    f.dpiv[gbase + tid] = dv;
    f.epiv[gbase + tid] = ev;
    f.pivtype[gbase + tid] = ptype;
    f.lperm[gbase + tid] = c0 + pos[tid];
  }
  if (tid == 0 && npert) atomicAdd(&f.counters[0], npert);
}

// Rows [c1, m) of a panel, 64 per block: X = V X11^T on the matrix cores with
// V = F21 P^T (panel columns in pivot order) and X11 = L11^-1 from the diagonal
// block's upper triangle; then W = X goes transposed to the upper triangle and
// L21 = X D^-1 to the lower part.  Precision T throughout (FP32 on the FP32 path).
template <typename T>
__global__ void __launch_bounds__(256) k_panel_trsm(const int64_t* __restrict__ tasks, FrontArgs f,
                                                    T* __restrict__ front) {
  __shared__ T sV[16][68];
  __shared__ T sC[64][65];  // first X11^T (sC[k][c] = X[c][k]), then the block's X tile (sC[c][r])
  __shared__ double dd[64], ee[64];
  __shared__ int ty[64], ps[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t task = blockIdx.x;
  const int sn = (int)tasks[task * 3];
  const int c0 = (int)tasks[task * 3 + 1], c1 = (int)tasks[task * 3 + 2];
  const int w = c1 - c0;
  const int64_t m = f.sn_m[sn];
  const int64_t r0 = c1 + (int64_t)blockIdx.y * 64;
  if (r0 >= m) return;
  const int64_t gbase = f.sn_begin[sn] + c0;
  T* F = front + f.sn_front_off[sn];
  if (tid < 64) {
    const bool in = tid < w;
    dd[tid] = in ? f.dpiv[gbase + tid] : 1.0;
    ee[tid] = in ? f.epiv[gbase + tid] : 0.0;
    ty[tid] = in ? f.pivtype[gbase + tid] : 0;
    ps[tid] = in ? f.lperm[gbase + tid] - c0 : 0;
  }
  __syncthreads();
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  dbl4 accd[2][2];
  flt4 accf[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accd[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
      accf[x][y] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  // every operand the block needs, loaded up front and unconditionally (clamped to in-front
  // addresses, masked when staged): 32 loads in flight per thread instead of one at a time.
  // V element q of a thread is (row rr = tid & 63, k = (tid + 256 q) >> 6); X11 element q is
  // X[c][k] with k = tid & 63 and c = (tid + 256 q) >> 6, kept at (row c0 + k, column c0 + c) for
  // c > k, so consecutive threads read consecutive rows of one column.
  T pv[16], px[16];
  {
    const int rr = tid & 63;
    const int64_t rc = r0 + rr < m ? r0 + rr : r0;
    const int kx = rr < w ? rr : 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = (tid + 256 * q) >> 6;
      const int cx = k < w ? k : 0;
      pv[q] = F[rc + (int64_t)(c0 + ps[k]) * m];  // ps[k] = 0 past w
      px[q] = F[(c0 + kx) + (int64_t)(c0 + cx) * m];
    }
  }
  // X11^T in LDS once: sC[k][c] = X[c][k] (1 on the diagonal, 0 above it and past w)
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = tid & 63, c = (tid + 256 * q) >> 6;
    sC[k][c] = (k < w && c < w) ? (c == k ? (T)1 : (c > k ? px[q] : (T)0)) : (T)0;
  }
#pragma unroll
  for (int kb = 0; kb < 64; kb += 16) {
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      const int q = kb / 4 + q4;
      const int idx = tid + 256 * q;
      const int rr = idx & 63, k = idx >> 6, kk = k - kb;
      const int64_t r = r0 + rr;
      sV[kk][rr] = (k < w && r < m) ? pv[q] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const T av = sC[kb + kr][wc + bj * 16 + (lane & 15)];
          const T bv = sV[kr][wr + bi * 16 + (lane & 15)];
          if constexpr (sizeof(T) == 8) {
            accd[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accd[bi][bj], 0, 0, 0);
          } else {
            accf[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, accf[bi][bj], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
  // X tile -> LDS (sC[c][r])
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int rr = wr + bi * 16 + (lane & 15);
        const int cc = wc + bj * 16 + mfma_row<T>(lane, reg);
        sC[cc][rr] = sizeof(T) == 8 ? (T)accd[bi][bj][reg] : (T)accf[bi][bj][reg];
      }
  __syncthreads();
  // W = X, transposed into the upper triangle: consecutive threads walk the columns c
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int c = idx & 63, rr = idx >> 6;
    const int64_t r = r0 + rr;
    if (c < w && r < m) F[(c0 + c) + r * m] = sC[c][rr];
  }
  // L21 = X D^-1: consecutive threads walk the rows r
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int rr = idx & 63, c = idx >> 6;
    const int64_t r = r0 + rr;
    if (c >= w || r >= m) continue;
    const double x = (double)sC[c][rr];
    double l;
    if (ty[c] == 0) {
      l = x / dd[c];
    } else if (ty[c] == 1) {
      const double a = dd[c], b = ee[c], cc = dd[c + 1];
      l = (cc * x - b * (double)sC[c + 1][rr]) / (a * cc - b * b);
    } else {
      const double a = dd[c - 1], b = ee[c - 1], cc = dd[c];
      l = (a * x - b * (double)sC[c - 1][rr]) / (a * cc - b * b);
    }
    F[r + (int64_t)(c0 + c) * m] = (T)l;
  }
}

// C[r, c] -= sum_{k in [k0,k1)} L[r,k] (L D)[c,k] on one 64 x 64 tile, MFMA 16x16x4.
template <typename T>
__global__ void __launch_bounds__(256) k_update(const int64_t* __restrict__ tasks,
                                                const int32_t* __restrict__ tile_task, FrontArgs f,
                                                T* __restrict__ front) {
  // 64 x 64 tile per block, 32 x 32 per wave (2 x 2 MFMA blocks of 16 x 16); the next k-chunk's loads
  // are in flight while the current one runs on the matrix cores.  (A 128 x 128 tile halves the
  // loads per flop but its register footprint halves the occupancy, which measured slower.)
  // The sum over k is taken in a permuted order: at step s of a chunk, lanes 16 g .. 16 g + 15 feed
  // k = (KC/4) g + s to both operands, so each lane reads its KC/4 W values of a chunk with 16-byte
  // LDS loads.
  constexpr int TM = kUpdTile;
  constexpr int KC = sizeof(T) == 8 ? 16 : 32;  // k per chunk (FP64 halves it to keep the occupancy)
  constexpr int KS = KC / 4;                  // MFMA steps per chunk
  constexpr int NQ = TM * KC / 256;           // loads per thread and chunk, each of L and W
  constexpr int CQ = 256 / KC;                // W columns covered by one load instruction of the block
  // sL rows KS apart (one lane group to the next) start 16 (FP32) or 32 (FP64) banks apart
  constexpr int SL = sizeof(T) == 8 ? TM + 4 : TM + 2;
  constexpr int SW = KC + 16 / (int)sizeof(T);  // 16-byte rows; 16 lanes reading 16 B each cover all banks
  constexpr int VW = 16 / (int)sizeof(T);     // elements per 16-byte LDS read
  typedef T vecw __attribute__((ext_vector_type(VW)));
  __shared__ T sL[KC][SL];                    // sL[k][r]
  __shared__ __attribute__((aligned(16))) T sW[TM][SW];  // sW[c][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Workgroups are handed to the 8 dies (each with its own L2) round-robin by index; renumber so that
  // each die takes one contiguous run of tiles.  In that run the tiles of one row of a column group
  // (same L rows) run side by side, and the group's W columns serve all its rows from that die's L2.
  int64_t b;
  {
    const int64_t n = gridDim.x, x = blockIdx.x & 7;
    int64_t before = 0;
    for (int64_t y = 0; y < x; ++y) before += (n - y + 7) >> 3;
    b = before + (blockIdx.x >> 3);
  }
  // The tile's task from the host-built map: one load, where a search over the tasks' tile offsets
  // took a chain of dependent loads before any of the tile's work could start.
  const int64_t* tk = tasks + (int64_t)tile_task[b] * 6;
  const int sn = (int)tk[0];
  const int64_t k0 = tk[1], k1 = tk[2], cb = tk[3], ce = tk[4];
  const int64_t m = f.sn_m[sn];
  const int64_t lt = b - tk[5];
  const int64_t R = (m - cb + TM - 1) / TM;
  const int64_t ct = (ce - cb + TM - 1) / TM;
  int64_t i, j;
  if (!update_tile(lt, R, ct, i, j)) return;  // beyond the task's tiles (never for a consistent schedule)
  const int64_t r0 = cb + TM * i, cc0 = cb + TM * j;
  T* F = front + f.sn_front_off[sn];
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int64_t cmax = ce < m ? ce : m;
  // Loads: L entries (r0 + rr, kb + kl + 4 q) and W^T entries (kb + kw, cc0 + cw + CQ q), as one
  // per-thread byte offset from a per-chunk base plus a uniform per-q stride.  Rows and columns past
  // the tile's end land on other entries of the front (finite; they only feed outputs that are not
  // stored) or past its end, where the buffer's range check returns 0.
  const int rr = tid & 63, kl = tid >> 6, kw = tid % KC, cw = tid / KC;
  const int64_t szT = (int64_t)sizeof(T);
  const uint32_t offL = (uint32_t)((r0 + rr + (int64_t)kl * m) * szT);
  const uint32_t offW = (uint32_t)((kw + (int64_t)cw * m) * szT);
  const int32_t strL = (int32_t)(4 * m * szT), strW = (int32_t)(CQ * m * szT);
  const int64_t fend = m * m;  // entries in the front
  auto range = [&](int64_t base) -> int32_t {
    const int64_t bytes = (fend - base) * szT;
    return bytes >= 0xffffffffll ? (int32_t)-1 : (int32_t)bytes;
  };
  T rl[NQ], rw[NQ];
  auto load = [&](int64_t kb) {
    const rsrc_t bL = buffer_rsrc(F + kb * m, range(kb * m));
    const rsrc_t bW = buffer_rsrc(F + kb + cc0 * m, range(kb + cc0 * m));
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      rl[q] = buffer_load<T>(bL, offL, q * strL);
      rw[q] = buffer_load<T>(bW, offW, q * strW);
    }
    if (kb + KC > k1 && kw >= (int)(k1 - kb)) {
      // last, partial chunk: k >= k1 contributes zero (its L entries are finite front entries, or 0
      // past the front's end, so zeroing the W side suffices)
#pragma unroll
      for (int q = 0; q < NQ; ++q) rw[q] = (T)0;
    }
  };
  dbl4 accd[2][2];
  flt4 accf[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accd[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
      accf[x][y] = flt4{0.f, 0.f, 0.f, 0.f};
    }
  const int g = lane >> 4, li = lane & 15;
  load(k0);
  for (int64_t kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sL[kl + 4 * q][rr] = rl[q];
      sW[cw + CQ * q][kw] = rw[q];
    }
    __syncthreads();
    if (kb + KC < k1) load(kb + KC);
    T aw[2][KS];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < KS / VW; ++v) {
        const vecw x = *(const vecw*)&sW[wc + bj * 16 + li][KS * g + VW * v];
#pragma unroll
        for (int e = 0; e < VW; ++e) aw[bj][VW * v + e] = x[e];
      }
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      T bv[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) bv[bi] = sL[KS * g + st][wr + bi * 16 + li];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          if constexpr (sizeof(T) == 8) {
            accd[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[bj][st], bv[bi], accd[bi][bj], 0, 0, 0);
          } else {
            accf[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[bj][st], bv[bi], accf[bi][bj], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int64_t r = r0 + wr + bi * 16 + (lane & 15);
        const int64_t c = cc0 + wc + bj * 16 + mfma_row<T>(lane, reg);
        if (r < m && c < cmax) {
          const double a = sizeof(T) == 8 ? (double)accd[bi][bj][reg] : (double)accf[bi][bj][reg];
          F[r + c * m] -= (T)a;
        }
      }
}

__global__ void k_inertia(int64_t N, const double* dpiv, const double* epiv, const int32_t* pivtype,
                          unsigned long long* counts, double* minabs_partials) {
  __shared__ double sh[256];
  __shared__ unsigned long long shc[3][256];
  unsigned long long np = 0, nn = 0, nz = 0;
  double mn = __builtin_inf();
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < N; k += (int64_t)gridDim.x * 256) {
    const int t = pivtype[k];
    if (t == 0) {
      const double d = dpiv[k];
      if (d > 0) ++np;
      else if (d < 0) ++nn;
      else ++nz;
      mn = fmin(mn, fabs(d));
    } else if (t == 1) {
      const double a = dpiv[k], c = dpiv[k + 1], b = epiv[k];
      const double det = a * c - b * b, tr = a + c;
      if (det < 0) {
        ++np;
        ++nn;
      } else if (det > 0) {
        if (tr > 0) np += 2;
        else nn += 2;
      } else {
        nz += 2;
      }
      const double h = 0.5 * tr, r = sqrt(0.25 * (a - c) * (a - c) + b * b);
      mn = fmin(mn, fmin(fabs(h - r), fabs(h + r)));
    }
  }
  // the counts are summed over the block first: one atomic per counter and block, where atomics from
  // every thread on the same three addresses queue up at their memory channel
  sh[threadIdx.x] = mn;
  shc[0][threadIdx.x] = np;
  shc[1][threadIdx.x] = nn;
  shc[2][threadIdx.x] = nz;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    const int t = threadIdx.x;
    if (t < w) {
      sh[t] = fmin(sh[t], sh[t + w]);
      shc[0][t] += shc[0][t + w];
      shc[1][t] += shc[1][t + w];
      shc[2][t] += shc[2][t + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    minabs_partials[blockIdx.x] = sh[0];
    if (shc[0][0]) atomicAdd(&counts[0], shc[0][0]);
    if (shc[1][0]) atomicAdd(&counts[1], shc[1][0]);
    if (shc[2][0]) atomicAdd(&counts[2], shc[2][0]);
  }
}

__global__ void k_mfma_probe_f64(const double* a, const double* b, double* out) {
  const int lane = threadIdx.x;
  const double av = a[(lane & 15) * 4 + (lane >> 4)];  // A[i][k], i = lane % 16, k = lane / 16
  const double bv = b[(lane >> 4) * 16 + (lane & 15)]; // B[k][j], k = lane / 16, j = lane % 16
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[mfma_row<double>(lane, r) * 16 + (lane & 15)] = acc[r];
}

__global__ void k_mfma_probe_f32(const double* a, const double* b, double* out) {
  const int lane = threadIdx.x;
  const float av = (float)a[(lane & 15) * 4 + (lane >> 4)];
  const float bv = (float)b[(lane >> 4) * 16 + (lane & 15)];
  flt4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[mfma_row<float>(lane, r) * 16 + (lane & 15)] = (double)acc[r];
}

}  // namespace

template <typename T>
void launch_csr_to_fronts(int64_t nnz, const int32_t* slot_row, const int32_t* colind, const int64_t* pos,
                          const double* vals, const double* scale, T* front, hipStream_t s) {
  if (nnz <= 0) return;
  int64_t g = (nnz + 255) / 256;
  if (g > 65536) g = 65536;
  k_csr_to_fronts<T><<<(unsigned)g, 256, 0, s>>>(nnz, slot_row, colind, pos, vals, scale, front);
}

template <typename T>
void launch_zero_fronts(int64_t ntasks, const int32_t* tasks, const FrontArgs& f, T* front, hipStream_t s) {
  if (ntasks > 0) k_zero_fronts<T><<<(unsigned)ntasks, 256, 0, s>>>(tasks, f, front);
}

template <typename T>
void launch_extend_add(int64_t ncols, const int64_t* cols, const FrontArgs& f, T* front, hipStream_t s) {
  // ncols: child columns of the round, one wavefront each
  if (ncols > 0) k_extend_add<T><<<(unsigned)((ncols + 3) / 4), 256, 0, s>>>(ncols, cols, f, front);
}

template <typename T>
void launch_extend_add_small(int64_t nkids, const int64_t* kids, const FrontArgs& f, T* front, hipStream_t s) {
  if (nkids > 0) k_extend_add_small<T><<<(unsigned)nkids, 256, 0, s>>>(kids, f, front);
}

template <typename T>
void launch_panel_diag(int64_t ntasks, int max_w, int waves, const int64_t* tasks, const FrontArgs& f, T* front,
                       hipStream_t s) {
  if (ntasks <= 0) return;
  if (waves == 8) k_panel_diag<T, 8, 64><<<(unsigned)ntasks, 512, 0, s>>>(tasks, f, front);
  else if (waves == 4 && max_w <= 48) k_panel_diag<T, 4, 48><<<(unsigned)ntasks, 256, 0, s>>>(tasks, f, front);
  else if (waves == 4) k_panel_diag<T, 4, 64><<<(unsigned)ntasks, 256, 0, s>>>(tasks, f, front);
  else if (waves == 2) k_panel_diag<T, 2, 64><<<(unsigned)ntasks, 128, 0, s>>>(tasks, f, front);
  else if (max_w <= 32) k_panel_diag<T, 1, 32><<<(unsigned)ntasks, 64, 0, s>>>(tasks, f, front);
  else k_panel_diag<T, 1, 64><<<(unsigned)ntasks, 64, 0, s>>>(tasks, f, front);
}

template <typename T>
void launch_panel_trsm(int64_t ntasks, int64_t max_rows, const int64_t* tasks, const FrontArgs& f, T* front,
                       hipStream_t s) {
  if (ntasks <= 0 || max_rows <= 0) return;
  dim3 g((unsigned)ntasks, (unsigned)((max_rows + 63) / 64));
  k_panel_trsm<T><<<g, 256, 0, s>>>(tasks, f, front);
}

template <typename T>
void launch_update(int64_t ntasks, int64_t ntiles, const int64_t* tasks, const int32_t* tile_task,
                   const FrontArgs& f, T* front, hipStream_t s) {
  if (ntasks > 0 && ntiles > 0) k_update<T><<<(unsigned)ntiles, 256, 0, s>>>(tasks, tile_task, f, front);
}

void launch_inertia(int64_t N, const double* dpiv, const double* epiv, const int32_t* pivtype,
                    unsigned long long* counts, double* minabs_partials, hipStream_t s) {
  k_inertia<<<kRedBlocks, 256, 0, s>>>(N, dpiv, epiv, pivtype, counts, minabs_partials);
}

void launch_mfma_probe(int prec, const double* a, const double* b, double* out, hipStream_t s) {
  if (prec == 0) k_mfma_probe_f64<<<1, 64, 0, s>>>(a, b, out);
  else k_mfma_probe_f32<<<1, 64, 0, s>>>(a, b, out);
}

template void launch_csr_to_fronts<double>(int64_t, const int32_t*, const int32_t*, const int64_t*, const double*,
                                           const double*, double*, hipStream_t);
template void launch_csr_to_fronts<float>(int64_t, const int32_t*, const int32_t*, const int64_t*, const double*,
                                          const double*, float*, hipStream_t);
template void launch_zero_fronts<double>(int64_t, const int32_t*, const FrontArgs&, double*, hipStream_t);
template void launch_zero_fronts<float>(int64_t, const int32_t*, const FrontArgs&, float*, hipStream_t);
template void launch_extend_add<double>(int64_t, const int64_t*, const FrontArgs&, double*, hipStream_t);
template void launch_extend_add<float>(int64_t, const int64_t*, const FrontArgs&, float*, hipStream_t);
template void launch_extend_add_small<double>(int64_t, const int64_t*, const FrontArgs&, double*, hipStream_t);
template void launch_extend_add_small<float>(int64_t, const int64_t*, const FrontArgs&, float*, hipStream_t);
template void launch_panel_diag<double>(int64_t, int, int, const int64_t*, const FrontArgs&, double*,
                                         hipStream_t);
template void launch_panel_diag<float>(int64_t, int, int, const int64_t*, const FrontArgs&, float*,
                                        hipStream_t);
template void launch_panel_trsm<double>(int64_t, int64_t, const int64_t*, const FrontArgs&, double*, hipStream_t);
template void launch_panel_trsm<float>(int64_t, int64_t, const int64_t*, const FrontArgs&, float*, hipStream_t);
template void launch_update<double>(int64_t, int64_t, const int64_t*, const int32_t*, const FrontArgs&, double*,
                                    hipStream_t);
template void launch_update<float>(int64_t, int64_t, const int64_t*, const int32_t*, const FrontArgs&, float*,
                                   hipStream_t);

}  // namespace sgn
