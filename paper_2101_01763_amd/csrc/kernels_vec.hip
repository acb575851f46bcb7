// Memory-bound kernels: preconditioner sweeps (batched GEMV and pull
// GEMV over slot lists), BSR SpMV (Algorithms 1/2, line "SpMV") with the
// Newton-basis shift fused in, and the tall-skinny pieces of the s-step
// orthogonalisation (Gram matrices, block updates, triangular scaling).
#include <climits>

#include "internal.h"
#include "kernels_vec.h"

namespace spand {

template <typename T>
__device__ inline T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ GEMV
// out[oslot[r]] = beta*out[oslot[r]] + alpha * sum_c op(A)(r, c) in[islot[c]]
// One workgroup per band of output rows (GemvChunk).  The input is staged
// in LDS.  Bands of one item may run concurrently, so in == out is not
// allowed (in-place sweeps write a scratch vector and copy back).
// Products accumulate in float64 for either factor precision: a float32
// factor stays one fixed linear operator (rounding the vector to float32 in
// every sweep would make M^-1 differ between applications, which
// right-preconditioned GMRES does not tolerate: the update M^-1 Q y would no
// longer match the basis and the true residual would stall above the
// estimate).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using V = float4;
  static constexpr int N = 4;
  __device__ static inline void get(const V &v, float *o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <>
struct Vec16<double> {
  using V = double2;
  static constexpr int N = 2;
  __device__ static inline void get(const V &v, double *o) { o[0] = v.x; o[1] = v.y; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_gemv(const GemvDesc *__restrict__ items,
                                              const GemvChunk *__restrict__ chunks,
                                              const double *__restrict__ in,
                                              double *__restrict__ out, double alpha,
                                              double beta) {
  using VW = Vec16<T>;
  constexpr int VN = VW::N;
  const GemvChunk ch = chunks[blockIdx.x];
  const GemvDesc d = items[ch.item];
  __shared__ double xs[GEMV_MAXC];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = tid; c < d.cols; c += 256) xs[c] = in[d.islot[c]];
  __syncthreads();
  const T *A = (const T *)d.A;
  if (!d.trans) {
    // each wave works on four rows at once (independent sums keep four
    // rows' loads in flight); rows past the band re-read the band's last
    // row and are discarded
    const int cv = d.cols / VN * VN;     // vectorised part (lda is a multiple of 4)
    for (int rr0 = wid * 4; rr0 < ch.nrows; rr0 += 16) {
      const T *row[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        row[q] = A + (int64_t)(ch.row0 + min(rr0 + q, ch.nrows - 1)) * d.lda;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int c = lane * VN; c < cv; c += 64 * VN) {
        typename VW::V v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const typename VW::V *>(row[q] + c);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T e[VN];
          VW::get(v[q], e);
#pragma unroll
          for (int u = 0; u < VN; ++u) acc[q] += double(e[u]) * xs[c + u];
        }
      }
      for (int c = cv + lane; c < d.cols; c += 64)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += double(row[q][c]) * xs[c];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = wsum(acc[q]);
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (rr0 + q >= ch.nrows) break;
          const int o = d.oslot[ch.row0 + rr0 + q];
          double v = alpha * acc[q];
          if (beta != 0.0) v += beta * out[o];
          out[o] = v;
        }
    }
  } else {
    const int r = ch.row0 + tid;
    if (tid < ch.nrows) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      const T *col = A + r;
      int c = 0;
      for (; c + 4 <= d.cols; c += 4) {
        a0 += double(col[(int64_t)c * d.lda]) * xs[c];
        a1 += double(col[(int64_t)(c + 1) * d.lda]) * xs[c + 1];
        a2 += double(col[(int64_t)(c + 2) * d.lda]) * xs[c + 2];
        a3 += double(col[(int64_t)(c + 3) * d.lda]) * xs[c + 3];
      }
      for (; c < d.cols; ++c) a0 += double(col[(int64_t)c * d.lda]) * xs[c];
      const int o = d.oslot[r];
      double v = alpha * ((a0 + a1) + (a2 + a3));
      if (beta != 0.0) v += beta * out[o];
      out[o] = v;
    }
  }
}

int launch_gemv(FType t, const GemvDesc *d_items, const GemvChunk *d_chunks, int nchunks,
                const double *in, double *out, double alpha, double beta, hipStream_t st) {
  if (nchunks <= 0) return SPAND_OK;
  if (t == FType::F64)
    hipLaunchKernelGGL(k_gemv<double>, dim3(nchunks), dim3(256), 0, st, d_items, d_chunks, in, out,
                       alpha, beta);
  else
    hipLaunchKernelGGL(k_gemv<float>, dim3(nchunks), dim3(256), 0, st, d_items, d_chunks, in, out,
                       alpha, beta);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

__global__ void k_slot_copy(const int32_t *__restrict__ slots, int64_t n,
                            const double *__restrict__ src, double *__restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = slots[i];
    dst[s] = src[s];
  }
}

int launch_slot_copy(const int32_t *slots, int64_t n, const double *src, double *dst,
                     hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_slot_copy, dim3((unsigned)std::min<int64_t>(8192, cdiv(n, 256))), dim3(256),
                     0, st, slots, n, src, dst);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ pull
// out[oslot[r]] = beta*out[oslot[r]] + alpha * sum_items op(B_i) in[islot_i]
// One workgroup per chunk of at most 64 output rows of a group; the items of
// the group are accumulated in order, in registers (a row is always owned by
// the same lanes).  Per item the input segment is staged in LDS.
//  * op(B) = B: 4 lanes per row with 16-byte loads from each row's first
//    16-byte boundary on (scalar head and tail); the partial sums combine
//    by shuffles.
//  * op(B) = B^T (B stored cols x rows): one lane per output row, four
//    slices of the columns, combined through LDS at the end.
template <typename T, int TRANS>
__global__ __launch_bounds__(256) void k_pull(const PullGroup *__restrict__ groups,
                                              const PullItem *__restrict__ items,
                                              const PullChunk *__restrict__ chunks,
                                              const double *__restrict__ in,
                                              double *__restrict__ out, double alpha,
                                              double beta) {
  using VW = Vec16<T>;
  constexpr int VN = VW::N;
  const PullChunk ch = chunks[blockIdx.x];
  const PullGroup g = groups[ch.group];
  __shared__ double xs[GEMV_MAXC];
  __shared__ double part[256];
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int it = g.item_begin; it < g.item_end; ++it) {
    const PullItem p = items[it];
    __syncthreads();
    for (int c = tid; c < p.cols; c += 256) xs[c] = in[p.islot[c]];
    __syncthreads();
    const T *B = (const T *)p.B;
    if (!TRANS) {
      // 4 lanes per row, 16-byte loads from the row's first 16-byte
      // boundary on (a row of any leading dimension: the few elements
      // before the boundary and after the last full vector are scalar)
      const int rr = tid >> 2, q = tid & 3;
      double a = 0.0;
      if (rr < ch.nrows) {
        const T *row = B + (int64_t)(ch.row0 + rr) * p.ldb;
        const int mis = int((reinterpret_cast<uintptr_t>(row) / sizeof(T)) % VN);
        const int h = min(mis ? VN - mis : 0, p.cols);
        if (q < h) a += double(row[q]) * xs[q];
        const int cv = h + (p.cols - h) / VN * VN;
#pragma unroll 4
        for (int c = h + q * VN; c < cv; c += 4 * VN) {
          const typename VW::V v = *reinterpret_cast<const typename VW::V *>(row + c);
          T e[VN];
          VW::get(v, e);
#pragma unroll
          for (int u = 0; u < VN; ++u) a += double(e[u]) * xs[c + u];
        }
        for (int c = cv + q; c < p.cols; c += 4) a += double(row[c]) * xs[c];
      }
      a += __shfl_xor(a, 1, 64);
      a += __shfl_xor(a, 2, 64);
      acc[0] += a;
    } else {
      const int rr = tid & 63, cs = tid >> 6;
      if (rr < ch.nrows) {
        const T *col = B + ch.row0 + rr;
        double a0 = 0.0, a1 = 0.0;
        int c = cs;
        for (; c + 4 < p.cols; c += 8) {
          a0 += double(col[(int64_t)c * p.ldb]) * xs[c];
          a1 += double(col[(int64_t)(c + 4) * p.ldb]) * xs[c + 4];
        }
        if (c < p.cols) a0 += double(col[(int64_t)c * p.ldb]) * xs[c];
        acc[0] += a0 + a1;
      }
    }
  }
  auto put = [&](int r, double v) {
    const int o = g.oslot[ch.row0 + r];
    v *= alpha;
    if (beta != 0.0) v += beta * out[o];
    out[o] = v;
  };
  if (!TRANS) {
    const int rr = tid >> 2;
    if ((tid & 3) == 0 && rr < ch.nrows) put(rr, acc[0]);
  } else {
    part[tid] = acc[0];
    __syncthreads();
    if (tid < ch.nrows) put(tid, (part[tid] + part[tid + 64]) + (part[tid + 128] + part[tid + 192]));
  }
}

int launch_pull2(FType t, const PullGroup *d_groups, const PullItem *d_items,
                 const PullChunk *d_chunks, int nchunks, int trans, const double *in,
                 double *out, double alpha, double beta, hipStream_t st) {
  if (nchunks <= 0) return SPAND_OK;
  const dim3 g(nchunks), b(256);
  if (t == FType::F64) {
    if (trans) hipLaunchKernelGGL((k_pull<double, 1>), g, b, 0, st, d_groups, d_items, d_chunks, in, out, alpha, beta);
    else hipLaunchKernelGGL((k_pull<double, 0>), g, b, 0, st, d_groups, d_items, d_chunks, in, out, alpha, beta);
  } else {
    if (trans) hipLaunchKernelGGL((k_pull<float, 1>), g, b, 0, st, d_groups, d_items, d_chunks, in, out, alpha, beta);
    else hipLaunchKernelGGL((k_pull<float, 0>), g, b, 0, st, d_groups, d_items, d_chunks, in, out, alpha, beta);
  }
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ SpMV
// y = alpha*A x + beta*y + gz*z + gw*w  (row-major b x b BSR blocks).
// G lanes per scalar row, 16-byte loads: one instruction of a lane group
// reads 16*G contiguous bytes of the row segment.  G is picked per block
// size by the autotuner (4, 8 or 16).
typedef double spmv_f64x2 __attribute__((ext_vector_type(2)));
template <int G>
__global__ __launch_bounds__(256) void k_spmv(int n_brows, int bs, const int32_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colind,
                                              const double *__restrict__ val,
                                              const double *__restrict__ x, double alpha,
                                              double beta, double *__restrict__ y,
                                              const double *__restrict__ z, double gz,
                                              const double *__restrict__ w, double gw) {
  constexpr int RPB = 256 / G;
  const int64_t N = (int64_t)n_brows * bs;
  const int64_t R = (int64_t)blockIdx.x * RPB + (threadIdx.x / G);
  const int sub = threadIdx.x % G;
  double acc = 0.0;
  if (R < N) {
    const int I = int(R / bs), r = int(R % bs);
    const int64_t b2 = (int64_t)bs * bs;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
      const double *rowv = val + (int64_t)t * b2 + (int64_t)r * bs;
      const double *xv = x + (int64_t)colind[t] * bs;
      for (int c = sub * 2; c < bs; c += 2 * G) {
        // the matrix is streamed once per product: non-temporal, so that
        // the vector's blocks stay in the caches
        const spmv_f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const spmv_f64x2 *>(rowv + c));
        acc += a[0] * xv[c] + a[1] * xv[c + 1];
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (R < N && sub == 0) {
    double v = alpha * acc;
    if (beta != 0.0) v += beta * y[R];
    if (z) v += gz * z[R];
    if (w) v += gw * w[R];
    y[R] = v;
  }
}

static int g_spmv_lanes[65] = {0};   // per block size; 0 = not tuned (default 8)

void set_spmv_lanes(int bs, int G) {
  if (bs >= 0 && bs <= 64) g_spmv_lanes[bs] = G;
}
int get_spmv_lanes(int bs) {
  const int g = (bs >= 0 && bs <= 64) ? g_spmv_lanes[bs] : 0;
  return g ? g : 8;
}

int launch_spmv_g(const spand_bsr_t &A, int G, double alpha, const double *x, double beta,
                  double *y, const double *z, double gz, const double *w, double gw,
                  hipStream_t st) {
  const int64_t N = (int64_t)A.n_brows * A.bs;
  if (N == 0) return SPAND_OK;
  const unsigned nb = (unsigned)cdiv(N, 256 / G);
  if (G == 4)
    hipLaunchKernelGGL(k_spmv<4>, dim3(nb), dim3(256), 0, st, A.n_brows, A.bs, A.d_rowptr,
                       A.d_colind, A.d_val, x, alpha, beta, y, z, gz, w, gw);
  else if (G == 16)
    hipLaunchKernelGGL(k_spmv<16>, dim3(nb), dim3(256), 0, st, A.n_brows, A.bs, A.d_rowptr,
                       A.d_colind, A.d_val, x, alpha, beta, y, z, gz, w, gw);
  else
    hipLaunchKernelGGL(k_spmv<8>, dim3(nb), dim3(256), 0, st, A.n_brows, A.bs, A.d_rowptr,
                       A.d_colind, A.d_val, x, alpha, beta, y, z, gz, w, gw);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// y = alpha*A^T x + beta*y + gz*z + gw*w for a structurally symmetric block
// pattern, without a transposed copy: row R = I*bs + r of A^T x sums
// A_JI(c, r) x_J(c) over the blocks (J, I) mirroring row I's blocks (I, J).
// One lane per output row: for each c the lanes of element I read row c of
// A_JI, bs contiguous doubles, so every load instruction is coalesced.  The
// mirror block is found by binary search in row J (the same search on
// every lane of the element, served by the caches); a missing mirror
// contributes nothing (spmv_t_check reports it before the products).
__global__ __launch_bounds__(256) void k_spmv_t(int n_brows, int bs,
                                                const int32_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ colind,
                                                const double *__restrict__ val,
                                                const double *__restrict__ x, double alpha,
                                                double beta, double *__restrict__ y,
                                                const double *__restrict__ z, double gz,
                                                const double *__restrict__ w, double gw) {
  const int64_t N = (int64_t)n_brows * bs;
  const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (R >= N) return;
  const int I = int(R / bs), r = int(R - (int64_t)I * bs);
  const int64_t b2 = (int64_t)bs * bs;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
    const int J = colind[t];
    int lo = rowptr[J], hi = rowptr[J + 1] - 1, pos = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int cm = colind[mid];
      if (cm == I) { pos = mid; break; }
      if (cm < I) lo = mid + 1; else hi = mid - 1;
    }
    if (pos < 0) continue;
    const double *blk = val + (int64_t)pos * b2 + r;
    const double *xv = x + (int64_t)J * bs;
    int c = 0;
    for (; c + 4 <= bs; c += 4) {
      a0 += __builtin_nontemporal_load(blk + (int64_t)c * bs) * xv[c];
      a1 += __builtin_nontemporal_load(blk + (int64_t)(c + 1) * bs) * xv[c + 1];
      a2 += __builtin_nontemporal_load(blk + (int64_t)(c + 2) * bs) * xv[c + 2];
      a3 += __builtin_nontemporal_load(blk + (int64_t)(c + 3) * bs) * xv[c + 3];
    }
    for (; c < bs; ++c) a0 += __builtin_nontemporal_load(blk + (int64_t)c * bs) * xv[c];
  }
  double v = alpha * ((a0 + a1) + (a2 + a3));
  if (beta != 0.0) v += beta * y[R];
  if (z) v += gz * z[R];
  if (w) v += gw * w[R];
  y[R] = v;
}

// *flag = 1 if some stored block (I, J) has no mirror (J, I)
__global__ __launch_bounds__(256) void k_spmv_t_check(int n_brows, const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colind,
                                                      int *__restrict__ flag) {
  const int I = blockIdx.x * 256 + threadIdx.x;
  if (I >= n_brows) return;
  for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
    const int J = colind[t];
    int lo = rowptr[J], hi = rowptr[J + 1] - 1, pos = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int cm = colind[mid];
      if (cm == I) { pos = mid; break; }
      if (cm < I) lo = mid + 1; else hi = mid - 1;
    }
    if (pos < 0) {
      atomicOr(flag, 1);
      return;
    }
  }
}

int launch_spmv_t_check(const spand_bsr_t &A, int *d_flag, hipStream_t st) {
  if (A.n_brows <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_spmv_t_check, dim3((unsigned)cdiv(A.n_brows, 256)), dim3(256), 0, st,
                     A.n_brows, A.d_rowptr, A.d_colind, d_flag);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

int launch_spmv(const spand_bsr_t &A, int transpose, double alpha, const double *x, double beta,
                double *y, const double *z, double gz, const double *w, double gw,
                hipStream_t st) {
  if (!transpose) return launch_spmv_g(A, get_spmv_lanes(A.bs), alpha, x, beta, y, z, gz, w, gw, st);
  const int64_t N = (int64_t)A.n_brows * A.bs;
  if (N == 0) return SPAND_OK;
  hipLaunchKernelGGL(k_spmv_t, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, st, A.n_brows, A.bs,
                     A.d_rowptr, A.d_colind, A.d_val, x, alpha, beta, y, z, gz, w, gw);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// d_out[t] = alpha * u_I v_J^T for every stored block
__global__ __launch_bounds__(256) void k_pattern_outer(int n_brows, int bs,
                                                       const int32_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ colind,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ v, double alpha,
                                                       double *__restrict__ out) {
  const int I = blockIdx.x;
  if (I >= n_brows) return;
  const int64_t b2 = (int64_t)bs * bs;
  for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
    const int J = colind[t];
    for (int idx = threadIdx.x; idx < bs * bs; idx += 256) {
      const int r = idx / bs, c = idx % bs;
      out[(int64_t)t * b2 + idx] = alpha * u[(int64_t)I * bs + r] * v[(int64_t)J * bs + c];
    }
  }
}

int launch_pattern_outer(const spand_bsr_t &P, const double *u, const double *v, double alpha,
                         double *out, hipStream_t st) {
  if (P.n_brows <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_pattern_outer, dim3(P.n_brows), dim3(256), 0, st, P.n_brows, P.bs,
                     P.d_rowptr, P.d_colind, u, v, alpha, out);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ vectors
__global__ void k_fill(double *x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
__global__ void k_iota(int32_t *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = int32_t(i);
}
// y = a*x + b*y  with a, b optionally read from device scalars:
// a = ca * (pa ? *pa : 1) [* (inva ? 1/ *inva : 1)]
__global__ void k_axpby(int64_t n, const double *__restrict__ x, double *__restrict__ y,
                        double ca, const double *pa, int inva, double cb) {
  double a = ca;
  if (pa) a *= inva ? 1.0 / *pa : *pa;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (cb != 0.0) v += cb * y[i];
    y[i] = v;
  }
}

int vec_fill(double *x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(4096, cdiv(n, 256))), dim3(256), 0,
                     st, x, n, v);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}
int vec_iota(int32_t *x, int64_t n, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)std::min<int64_t>(4096, cdiv(n, 256))), dim3(256), 0,
                     st, x, n);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}
int vec_axpby(int64_t n, const double *x, double *y, double ca, const double *pa, int inva,
              double cb, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)std::min<int64_t>(4096, cdiv(n, 256))), dim3(256), 0,
                     st, n, x, y, ca, pa, inva, cb);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ tall-skinny
// Partial Gram: part[chunk][i][j] = sum_{r in chunk} X[i*ldx + r] * W[j*ldw + r]
// (X: N x a, W: N x s, both column-major).  Chunks of TS_CHUNK rows.
__global__ __launch_bounds__(256) void k_gram_part(int64_t N, const double *__restrict__ X,
                                                   int64_t ldx, int a,
                                                   const double *__restrict__ W, int64_t ldw,
                                                   int s, double *__restrict__ part) {
  __shared__ double ws[TS_CHUNK][TS_MAXS + 1];
  const int64_t r0 = (int64_t)blockIdx.x * TS_CHUNK;
  const int rows = int(std::min<int64_t>(TS_CHUNK, N - r0));
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int idx = tid; idx < TS_CHUNK * s; idx += 256) {
    const int j = idx / TS_CHUNK, r = idx % TS_CHUNK;
    ws[r][j] = r < rows ? W[(int64_t)j * ldw + r0 + r] : 0.0;
  }
  __syncthreads();
  double *outp = part + (int64_t)blockIdx.x * a * s;
  for (int i = wid; i < a; i += 4) {
    double acc[TS_MAXS];
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j) acc[j] = 0.0;
    const double *xc = X + (int64_t)i * ldx + r0;
    for (int r = lane; r < rows; r += 64) {
      const double xv = xc[r];
#pragma unroll
      for (int j = 0; j < TS_MAXS; ++j)
        if (j < s) acc[j] += xv * ws[r][j];
    }
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j) {
      if (j < s) {
        const double v = wsum(acc[j]);
        if (lane == 0) outp[(int64_t)i * s + j] = v;
      }
    }
  }
}

// out[i*ldo + j] = sum over chunks; one workgroup per output, fixed
// partition and tree order (deterministic)
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ part, int nchunk,
                                                     int a, int s, double *__restrict__ out,
                                                     int ldo) {
  __shared__ double red[256];
  const int idx = blockIdx.x;
  double v = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) v += part[(int64_t)c * a * s + idx];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(idx / s) * ldo + idx % s] = red[0];
}

// Wide variant for the single-reduce step (up to 2 * TS_MAXS columns) on the
// FP64 matrix cores: each wave owns TS_WCHUNK rows and accumulates the
// a x s partial Gram matrix as ceil(a/16) tiles of v_mfma_f64_16x16x4f64
// (lane l supplies X(row k + l/16, column l%16) as A and W(row k + l/16,
// column l%16) as B; result register q of lane l is tile row l/16 + 4q,
// column l%16), so the sum over rows needs no cross-lane reduction.  The
// per-wave partials are summed in two deterministic stages (fixed partition
// and order).
constexpr int TS_WCHUNK = 256;     // rows per wave
constexpr int TS_WMAXS = 2 * TS_MAXS;
constexpr int TS_WSPLIT = 64;      // first-stage splits of the partial sums
typedef double gram_f64x4 __attribute__((ext_vector_type(4)));

template <int NT>
__global__ __launch_bounds__(256) void k_gram_part_wide(int64_t N, const double *__restrict__ X,
                                                        int64_t ldx, int a,
                                                        const double *__restrict__ W,
                                                        int64_t ldw, int s, int64_t nchunk,
                                                        int vec4, double *__restrict__ part) {
  const int lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
  const int64_t chunk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= nchunk) return;        // whole wave; no barriers below
  const int64_t rb = chunk * TS_WCHUNK + g;
  gram_f64x4 acc[NT];
  const double *xc[NT];
  bool xok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = gram_f64x4{0.0, 0.0, 0.0, 0.0};
    const int col = t * 16 + m;
    xok[t] = col < a;
    xc[t] = X + (int64_t)(xok[t] ? col : 0) * ldx;
  }
  const bool wok = m < s;
  const double *wc = W + (int64_t)(wok ? m : 0) * ldw;
  if (vec4 && (chunk + 1) * TS_WCHUNK <= N) {
    // full chunk, 32-byte aligned columns: lane group g loads rows
    // 16kk + 4g .. 16kk + 4g + 3 at once and feeds them to four products
    // (k-slot g of product q is row 16kk + 4g + q)
    const int64_t rv = chunk * TS_WCHUNK + 4 * g;
    const gram_f64x4 z4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int kk = 0; kk < TS_WCHUNK / 16; ++kk) {
      const int64_t r = rv + 16 * kk;
      const gram_f64x4 bw = wok ? *(const gram_f64x4 *)(wc + r) : z4;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const gram_f64x4 ax = xok[t] ? *(const gram_f64x4 *)(xc[t] + r) : z4;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[0], bw[0], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[1], bw[1], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[2], bw[2], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[3], bw[3], acc[t], 0, 0, 0);
      }
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < TS_WCHUNK / 4; ++k) {
      const int64_t r = rb + 4 * k;
      const bool in = r < N;
      const double bw = (in && wok) ? wc[r] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double ax = (in && xok[t]) ? xc[t][r] : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bw, acc[t], 0, 0, 0);
      }
    }
  }
  double *outp = part + chunk * a * s;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = t * 16 + g + 4 * q;
      if (i < a && wok) outp[(int64_t)i * s + m] = acc[t][q];
    }
}

// Stage 1: workgroup (x, y) sums chunks [y*nchunk/S, (y+1)*nchunk/S) of the
// 64 outputs from x*64 (one wave per quarter of the range, then in order).
__global__ __launch_bounds__(256) void k_gram_reduce_s1(const double *__restrict__ part,
                                                        int64_t nchunk, int n,
                                                        double *__restrict__ part2) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  const int64_t c0 = nchunk * blockIdx.y / gridDim.y, c1 = nchunk * (blockIdx.y + 1) / gridDim.y;
  const int64_t q0 = c0 + (c1 - c0) * wid / 4, q1 = c0 + (c1 - c0) * (wid + 1) / 4;
  double v = 0.0;
  if (idx < n)
    for (int64_t c = q0; c < q1; ++c) v += part[c * n + idx];
  red[wid][lane] = v;
  __syncthreads();
  if (wid == 0 && idx < n)
    part2[(int64_t)blockIdx.y * n + idx] = (red[0][lane] + red[1][lane]) +
                                           (red[2][lane] + red[3][lane]);
}

// Stage 2: out = sum over the splits, in order.
__global__ __launch_bounds__(64) void k_gram_reduce_s2(const double *__restrict__ part2,
                                                       int nsplit, int n, int s,
                                                       double *__restrict__ out, int ldo) {
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= n) return;
  double v = 0.0;
  for (int y = 0; y < nsplit; ++y) v += part2[(int64_t)y * n + idx];
  out[(idx / s) * ldo + idx % s] = v;
}

int64_t gram_wide_part_elems(int64_t N, int a, int s) {
  return (cdiv(N, TS_WCHUNK) + TS_WSPLIT) * a * s;
}

int launch_gram_wide(int64_t N, const double *X, int64_t ldx, int a, const double *W,
                     int64_t ldw, int s, double *part, double *out, int ldo, hipStream_t st) {
  if (a <= 0 || s <= 0 || N <= 0) return SPAND_OK;
  if (s > TS_WMAXS || a > TS_MAXA) {
    set_error("wide Gram matrix: %d x %d exceeds %d x %d", a, s, TS_MAXA, TS_WMAXS);
    return SPAND_EINVAL;
  }
  const int64_t nchunk = cdiv(N, TS_WCHUNK);
  const dim3 g1((unsigned)cdiv(nchunk, 4));
  // every column start 32-byte aligned: four-row vector loads
  const int vec4 = (ldx % 4 == 0) && (ldw % 4 == 0) && (uintptr_t(X) % 32 == 0) &&
                   (uintptr_t(W) % 32 == 0);
  switch (int(cdiv(a, 16))) {
#define GRAM_NT(nt)                                                                          \
  case nt:                                                                                   \
    hipLaunchKernelGGL(k_gram_part_wide<nt>, g1, dim3(256), 0, st, N, X, ldx, a, W, ldw, s, \
                       nchunk, vec4, part);                                                  \
    break;
    GRAM_NT(1) GRAM_NT(2) GRAM_NT(3) GRAM_NT(4) GRAM_NT(5)
    GRAM_NT(6) GRAM_NT(7) GRAM_NT(8) GRAM_NT(9) GRAM_NT(10)
#undef GRAM_NT
    default:
      set_error("wide Gram matrix: %d rows", a);
      return SPAND_EINVAL;
  }
  SP_HIP(hipGetLastError());
  const int n = a * s;
  double *part2 = part + nchunk * n;
  const int nsplit = int(std::min<int64_t>(TS_WSPLIT, nchunk));
  hipLaunchKernelGGL(k_gram_reduce_s1, dim3(unsigned(cdiv(n, 64)), unsigned(nsplit)), dim3(256),
                     0, st, part, nchunk, n, part2);
  SP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_reduce_s2, dim3(unsigned(cdiv(n, 64))), dim3(64), 0, st, part2,
                     nsplit, n, s, out, ldo);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// One pass over the rows for a single-reduce step, Q_old = Q[:, 0:a] read
// once per row: the pending block P = Q[:, a:a+sp] <- (P - Q_old R1) T^{-1}
// (its second pass) and the new block W = Q[:, a+sp:a+sp+sw] <-
// (W - Q_old C_old - Phat C_P) RV^{-1} (its first pass), coefficients from
// the single-reduce kernel.  bad = 1: nothing; bad = 2: P only.
__global__ __launch_bounds__(256) void k_ts_lag_update(int64_t N, double *__restrict__ Q,
                                                       int64_t ldq, int a, int sp, int sw, int s,
                                                       const KrylovDev *__restrict__ K) {
  __shared__ double RP[TS_MAXA * TS_MAXS];    // R1, ld TS_MAXS
  __shared__ double RW[TS_MAXA * TS_MAXS];    // C_old, ld TS_MAXS
  __shared__ double Ts[TS_MAXS * TS_MAXS], CP[TS_MAXS * TS_MAXS], RV[TS_MAXS * TS_MAXS];
  const int bad = K->bad;
  if (bad == 1) return;
  const int ww = (bad == 0) ? sw : 0;
  if (sp + ww == 0) return;
  for (int idx = threadIdx.x; idx < a * TS_MAXS; idx += 256) {
    const int i = idx / TS_MAXS, c = idx % TS_MAXS;
    RP[idx] = c < sp ? K->Lr1[i * s + c] : 0.0;
    RW[idx] = c < ww ? K->Pra[i * s + c] : 0.0;
  }
  for (int idx = threadIdx.x; idx < TS_MAXS * TS_MAXS; idx += 256) {
    const int r = idx / TS_MAXS, c = idx % TS_MAXS;
    const bool in = r < s && c < s;
    Ts[idx] = in && sp ? K->Lt[r * s + c] : 0.0;
    CP[idx] = in && sp && ww ? K->Pra[(a + r) * s + c] : 0.0;
    RV[idx] = in && ww ? K->Prb[r * s + c] : 0.0;
  }
  __syncthreads();
  // one row per thread (a grid-stride loop would let the compiler keep the
  // triangular factors in registers and spill)
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < N) {
    double ap[TS_MAXS], aw[TS_MAXS];
#pragma unroll
    for (int c = 0; c < TS_MAXS; ++c) ap[c] = aw[c] = 0.0;
#pragma unroll 2
    for (int i = 0; i < a; ++i) {
      const double xv = Q[(int64_t)i * ldq + r];
#pragma unroll
      for (int c = 0; c < TS_MAXS; ++c) {
        if (c < sp) ap[c] += xv * RP[i * TS_MAXS + c];
        if (c < ww) aw[c] += xv * RW[i * TS_MAXS + c];
      }
    }
    double p[TS_MAXS];
#pragma unroll
    for (int c = 0; c < TS_MAXS; ++c) {
      p[c] = 0.0;
      if (c < sp) {
        double v = Q[(int64_t)(a + c) * ldq + r] - ap[c];
#pragma unroll
        for (int q = 0; q < TS_MAXS; ++q)
          if (q < c) v -= p[q] * Ts[q * TS_MAXS + c];
        p[c] = v / Ts[c * TS_MAXS + c];
        Q[(int64_t)(a + c) * ldq + r] = p[c];
      }
    }
    if (ww) {
      double w[TS_MAXS];
#pragma unroll
      for (int c = 0; c < TS_MAXS; ++c) {
        w[c] = 0.0;
        if (c < ww) {
          double v = Q[(int64_t)(a + sp + c) * ldq + r] - aw[c];
#pragma unroll
          for (int q = 0; q < TS_MAXS; ++q)
            if (q < sp) v -= p[q] * CP[q * TS_MAXS + c];
#pragma unroll
          for (int q = 0; q < TS_MAXS; ++q)
            if (q < c) v -= w[q] * RV[q * TS_MAXS + c];
          w[c] = v / RV[c * TS_MAXS + c];
          Q[(int64_t)(a + sp + c) * ldq + r] = w[c];
        }
      }
    }
  }
}

int launch_ts_lag_update(int64_t N, double *Q, int64_t ldq, int a, int sp, int sw, int s,
                         const KrylovDev *K, hipStream_t st) {
  if (N <= 0 || sp + sw == 0) return SPAND_OK;
  if (a > TS_MAXA || s > TS_MAXS || (sp && sp != s) || (sw && sw != s)) {
    set_error("single-reduce update: a = %d, s = %d out of range", a, s);
    return SPAND_EINVAL;
  }
  hipLaunchKernelGGL(k_ts_lag_update, dim3(unsigned(cdiv(N, 256))), dim3(256), 0, st, N, Q, ldq,
                     a, sp, sw, s, K);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

int launch_gram(int64_t N, const double *X, int64_t ldx, int a, const double *W, int64_t ldw,
                int s, double *part, double *out, int ldo, hipStream_t st) {
  if (a <= 0 || s <= 0) return SPAND_OK;
  const int nchunk = int(cdiv(N, TS_CHUNK));
  hipLaunchKernelGGL(k_gram_part, dim3(nchunk), dim3(256), 0, st, N, X, ldx, a, W, ldw, s, part);
  SP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_reduce, dim3(a * s), dim3(256), 0, st, part, nchunk, a, s, out, ldo);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// W[:, j] -= sum_i X[:, i] R[i*ldr + j]
__global__ __launch_bounds__(256) void k_ts_update(int64_t N, const double *__restrict__ X,
                                                   int64_t ldx, int a,
                                                   const double *__restrict__ R, int ldr,
                                                   double *__restrict__ W, int64_t ldw, int s) {
  __shared__ double Rs[TS_MAXA * TS_MAXS];
  for (int idx = threadIdx.x; idx < a * s; idx += 256) Rs[idx] = R[(idx / s) * ldr + idx % s];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * 256) {
    double acc[TS_MAXS];
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j) acc[j] = 0.0;
    for (int i = 0; i < a; ++i) {
      const double xv = X[(int64_t)i * ldx + r];
#pragma unroll
      for (int j = 0; j < TS_MAXS; ++j)
        if (j < s) acc[j] += xv * Rs[i * s + j];
    }
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j)
      if (j < s) W[(int64_t)j * ldw + r] -= acc[j];
  }
}

int launch_ts_update(int64_t N, const double *X, int64_t ldx, int a, const double *R, int ldr,
                     double *W, int64_t ldw, int s, hipStream_t st) {
  if (a <= 0 || s <= 0 || N <= 0) return SPAND_OK;
  const unsigned g = (unsigned)std::min<int64_t>(8192, cdiv(N, 256));
  hipLaunchKernelGGL(k_ts_update, dim3(g), dim3(256), 0, st, N, X, ldx, a, R, ldr, W, ldw, s);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// W <- W T^{-1}, T upper triangular s x s (row-major, ld s); skip if *bad
__global__ __launch_bounds__(256) void k_ts_trsm(int64_t N, double *__restrict__ W, int64_t ldw,
                                                 int s, const double *__restrict__ T,
                                                 const int *__restrict__ bad) {
  if (*bad) return;
  __shared__ double Ts[TS_MAXS * TS_MAXS];
  for (int idx = threadIdx.x; idx < s * s; idx += 256) Ts[idx] = T[idx];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * 256) {
    double x[TS_MAXS];
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j) {
      if (j < s) {
        double v = W[(int64_t)j * ldw + r];
#pragma unroll
        for (int i = 0; i < TS_MAXS; ++i)
          if (i < j) v -= x[i] * Ts[i * s + j];
        x[j] = v / Ts[j * s + j];
      }
    }
#pragma unroll
    for (int j = 0; j < TS_MAXS; ++j)
      if (j < s) W[(int64_t)j * ldw + r] = x[j];
  }
}

int launch_ts_trsm(int64_t N, double *W, int64_t ldw, int s, const double *T, const int *bad,
                   hipStream_t st) {
  if (N <= 0 || s <= 0) return SPAND_OK;
  const unsigned g = (unsigned)std::min<int64_t>(8192, cdiv(N, 256));
  hipLaunchKernelGGL(k_ts_trsm, dim3(g), dim3(256), 0, st, N, W, ldw, s, T, bad);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// y = X[:, 0:k] c   (c on device)
__global__ __launch_bounds__(256) void k_ts_gemv(int64_t N, const double *__restrict__ X,
                                                 int64_t ldx, int k, const double *__restrict__ c,
                                                 double *__restrict__ y) {
  __shared__ double cs[TS_MAXA];
  for (int i = threadIdx.x; i < k; i += 256) cs[i] = c[i];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int i = 0; i < k; ++i) v += X[(int64_t)i * ldx + r] * cs[i];
    y[r] = v;
  }
}

int launch_ts_gemv(int64_t N, const double *X, int64_t ldx, int k, const double *c, double *y,
                   hipStream_t st) {
  if (N <= 0) return SPAND_OK;
  const unsigned g = (unsigned)std::min<int64_t>(8192, cdiv(N, 256));
  hipLaunchKernelGGL(k_ts_gemv, dim3(g), dim3(256), 0, st, N, X, ldx, k, c, y);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

}  // namespace spand
