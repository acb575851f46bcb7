// Dense batched kernels of the spaND factorization (gfx950, wave64).
//
//  * k_gemm          variable-size batched C = a op(A) op(B) + b C
//  * k_elim_panel    one panel (16 columns) of Gauss-Jordan inversion or LU
//                    with partial pivoting, rows held in registers
//  * k_elim_update   the rank-16 update that applies a panel to the rest
//  * k_row_gather    undo the virtual row pivoting
//  * k_schur_elem    level-0 Schur update on b x b element blocks (Eq. 10)
//  * k_qrcp          rank-revealing QR with column pivoting (Eq. 12)
//  * k_copy / k_scale / k_eye  data movement helpers
//
// Matrices are row-major.  Every descriptor is validated on the host before
// upload; kernels trust the sizes they are given.
#include <climits>
#include <type_traits>

#include "internal.h"
#include "factor.h"

namespace spand {

// ------------------------------------------------------------------ utils
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of a double (blockDim multiple of 64, <= 1024)
__device__ inline double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// ------------------------------------------------------------------ GEMM
// Batched GEMMs: 64x64 output tiles, one 256-thread workgroup each (the
// kernels below).  Item of a tile: binary search of tile_start (absolute tile numbers),
// narrowed first by the coarse index when there is one (coarse[c] = item of
// tile tile_base + 64 c, c <= ntiles / 64, relative to this launch's items).
__device__ inline int gemm_item(int tile, int tile_base, const int32_t *__restrict__ tile_start,
                                const int32_t *__restrict__ coarse, int nitems) {
  int lo = 0, hi = nitems;
  if (coarse) {
    const int c = (tile - tile_base) >> 6;
    lo = coarse[c];
    hi = min(nitems, coarse[c + 1] + 1);
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_start[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

// FP32 version on the matrix cores: the same 64x64 tiles, each of the four
// waves owns a 32x32 quarter and accumulates it with v_mfma_f32_32x32x2f32
// (lane l holds A(l%32, k + l/32) and B(k + l/32, l%32); result register r
// of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32 of the quarter).
// K advances in chunks of 32 staged through LDS; the next chunk is fetched
// into registers while the current one is multiplied.  With alpha = 1 the
// accumulators start from beta*C, loaded before the first product.
// Workgroups are dealt round-robin to the 8 XCDs; each XCD is given one
// contiguous range of tiles so that the tiles of a matrix share its L2.
// The register budget is set for 5 waves per SIMD: the K = 64 block updates
// are latency-bound and gain from the extra workgroup per CU (6 spills).
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float __attribute__((address_space(1))) gfloat;   // global memory
constexpr int GK = 32;

__device__ inline int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x * q + min(x, r) + j;
}

template <int TA, int TB>
__global__ __launch_bounds__(256, 5) void k_gemm_f32_mfma(const GemmDesc *__restrict__ items,
                                                       const int32_t *__restrict__ tile_start,
                                                       const int32_t *__restrict__ coarse,
                                                       int nitems, int tile_base, int uniform) {
  const int tile = tile_base + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int lo = uniform > 0 ? (tile - tile_base) / uniform
                             : gemm_item(tile, tile_base, tile_start, coarse, nitems);
  const GemmDesc d = items[lo];
  const int t = tile - tile_start[lo];
  const int ntn = (d.N + 63) >> 6;
  const int m0 = (t / ntn) * 64, n0 = (t % ntn) * 64;
  __shared__ float As[64 * (GK + 1)];   // As[m * (GK + 1) + k]
  __shared__ float Bs[GK * 68];         // Bs[k * 68 + n]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  // global address space and 32-bit element offsets (every operand has
  // fewer than 2^31 elements): a scalar base and one offset register per load
  const gfloat *A = (const gfloat *)d.A;
  const gfloat *B = (const gfloat *)d.B;
  float ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + q * 256;
      int mm, kk;
      if (!TA) { mm = idx >> 5; kk = idx & 31; }
      else { kk = idx >> 6; mm = idx & 63; }
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < d.M && gk < d.K) ? A[TA ? gk * d.lda + gm : gm * d.lda + gk] : 0.f;
      int nn;
      if (!TB) { kk = idx >> 6; nn = idx & 63; }
      else { nn = idx >> 5; kk = idx & 31; }
      const int gn = n0 + nn, gk2 = k0 + kk;
      rb[q] = (gn < d.N && gk2 < d.K) ? B[TB ? gn * d.ldb + gk2 : gk2 * d.ldb + gn] : 0.f;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + q * 256;
      int mm, kk;
      if (!TA) { mm = idx >> 5; kk = idx & 31; }
      else { kk = idx >> 6; mm = idx & 63; }
      As[mm * (GK + 1) + kk] = ra[q];
      int nn;
      if (!TB) { kk = idx >> 6; nn = idx & 63; }
      else { nn = idx >> 5; kk = idx & 31; }
      Bs[kk * 68 + nn] = rb[q];
    }
  };
  // K range of this tile: triangular operands contribute nothing outside
  // it (m0, n0 are multiples of 64, so the range stays in whole chunks)
  const int kb = (d.tri & GEMM_TRI_A_UPPER) ? min(m0, d.K) : 0;
  const int ke = (d.tri & GEMM_TRI_B_UPPER) ? min(d.K, n0 + 64) : d.K;
  if (kb < ke) gload(kb);
  gfloat *C = (gfloat *)d.C;
  const int gn = n0 + wc * 32 + (lane & 31);
  const bool cin = d.alpha == 1.0 && d.beta != 0.0;
  const float al = float(d.alpha), be = float(d.beta);
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gm = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    acc[r] = (cin && gm < d.M && gn < d.N) ? be * C[gm * d.ldc + gn] : 0.f;
  }
  const float *ap = As + (wr * 32 + (lane & 31)) * (GK + 1) + (lane >> 5);
  const float *bp = Bs + (lane >> 5) * 68 + wc * 32 + (lane & 31);
  for (int k0 = kb; k0 < ke; k0 += GK) {
    sstore();
    __syncthreads();
    if (k0 + GK < ke) gload(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[kk], bp[kk * 68], acc, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gm = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (gm < d.M && gn < d.N) {
      gfloat *c = C + gm * d.ldc + gn;
      float v = acc[r];
      if (!cin) {
        v *= al;
        if (d.beta != 0.0) v += be * (*c);
      }
      *c = v;
    }
  }
}

// Accumulating products with a short K (the block updates of the blocked
// eliminations, C += A B with K <= 64, FP32): one workgroup owns a strip of
// up to `tps` 64x64 tiles of C along N that share one 64-row block of A.
// A is staged in LDS once; per tile, the next tile's B and C are fetched into
// registers while the current one is multiplied.  Every output takes the same
// instructions in the same order as in k_gemm_f32_mfma (start from beta*C, K
// in chunks of 32 with zero padding, v_mfma_f32_32x32x2f32 on pairs of k), so
// the results are the same bit for bit.  Items: alpha = 1, no transposes.
constexpr int SK = 64;   // largest K of a strip product
__global__ __launch_bounds__(256, 4) void k_gemm_f32_strip(const GemmDesc *__restrict__ items,
                                                         const int32_t *__restrict__ unit_start,
                                                         const int32_t *__restrict__ coarse,
                                                         int nitems, int unit_base, int uniform,
                                                         int tps) {
  const int unit = unit_base + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int lo = uniform > 0 ? (unit - unit_base) / uniform
                             : gemm_item(unit, unit_base, unit_start, coarse, nitems);
  const GemmDesc d = items[lo];
  const int u = unit - unit_start[lo];
  const int ntn = (d.N + 63) >> 6;
  const int nstrip = (ntn + tps - 1) / tps;
  const int m0 = (u / nstrip) * 64, t0 = (u % nstrip) * tps;
  const int t1 = min(ntn, t0 + tps);
  const int kc = (d.K + GK - 1) / GK * GK;         // K padded to whole chunks (<= SK)
  __shared__ float As[64 * (SK + 1)];   // As[m * (SK + 1) + k]
  __shared__ float Bs[SK * 68];         // Bs[k * 68 + n]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const gfloat *A = (const gfloat *)d.A;
  const gfloat *B = (const gfloat *)d.B;
  gfloat *C = (gfloat *)d.C;
  const float be = float(d.beta);
  // A block: 64 x kc
  for (int idx = tid; idx < 64 * kc; idx += 256) {
    const int mm = idx / kc, kk = idx - mm * kc;
    const int gm = m0 + mm;
    As[mm * (SK + 1) + kk] = (gm < d.M && kk < d.K) ? A[gm * d.lda + kk] : 0.f;
  }
  // B tile (kc x 64) and C tile of column tile t into registers: each thread
  // holds kc/4 B values (k = idx >> 6, n = idx & 63) and its 16 C values
  float rb[SK / 4], rc[16];
  const int gcol = wc * 32 + (lane & 31);
  auto fetch = [&](int t) {
    const int n0 = t * 64;
#pragma unroll
    for (int q = 0; q < SK / 4; ++q) {
      const int idx = tid + q * 256;
      const int kk = idx >> 6, nn = idx & 63;
      const int gn = n0 + nn;
      rb[q] = (kk < kc && kk < d.K && gn < d.N) ? B[kk * d.ldb + gn] : 0.f;
    }
    const int gn = n0 + gcol;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int gm = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      rc[r] = (gm < d.M && gn < d.N) ? C[gm * d.ldc + gn] : 0.f;
    }
  };
  if (t0 < t1) fetch(t0);
  const float *ap = As + (wr * 32 + (lane & 31)) * (SK + 1) + (lane >> 5);
  const float *bp = Bs + (lane >> 5) * 68 + wc * 32 + (lane & 31);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();       // the previous tile's products have read Bs
#pragma unroll
    for (int q = 0; q < SK / 4; ++q) {
      const int idx = tid + q * 256;
      if ((idx >> 6) < kc) Bs[(idx >> 6) * 68 + (idx & 63)] = rb[q];
    }
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = be * rc[r];
    __syncthreads();
    if (t + 1 < t1) fetch(t + 1);
    for (int kk = 0; kk < kc; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[kk], bp[kk * 68], acc, 0, 0, 0);
    const int gn = t * 64 + gcol;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int gm = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (gm < d.M && gn < d.N) C[gm * d.ldc + gn] = acc[r];
    }
  }
}

int launch_gemm_strip(const GemmDesc *d_items, const int32_t *d_unit_start, int nitems,
                      int total_units, hipStream_t st, int unit_base, int uniform,
                      const int32_t *d_coarse, int tps) {
  if (nitems <= 0 || total_units <= 0) return SPAND_OK;
  hipLaunchKernelGGL(k_gemm_f32_strip, dim3(total_units), dim3(256), 0, st, d_items, d_unit_start,
                     d_coarse, nitems, unit_base, uniform, tps);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// FP64 version on the matrix cores: 64x64 tiles, each wave a 32x32 quarter
// as 2x2 blocks of v_mfma_f64_16x16x4f64 (lane l holds A(l%16, k + l/16)
// and B(k + l/16, l%16); result register r of lane l is row l/16 + 4r,
// column l%16 of the block, checked on gfx950).  K advances in chunks of
// 16 through LDS with register prefetch, as in the FP32 kernel.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double __attribute__((address_space(1))) gdouble;

template <int TA, int TB>
__global__ __launch_bounds__(256, 4) void k_gemm_f64_mfma(const GemmDesc *__restrict__ items,
                                                       const int32_t *__restrict__ tile_start,
                                                       const int32_t *__restrict__ coarse,
                                                       int nitems, int tile_base, int uniform) {
  constexpr int DK = 16, LA = DK + 1, LB = 68;
  const int tile = tile_base + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int lo = uniform > 0 ? (tile - tile_base) / uniform
                             : gemm_item(tile, tile_base, tile_start, coarse, nitems);
  const GemmDesc d = items[lo];
  const int t = tile - tile_start[lo];
  const int ntn = (d.N + 63) >> 6;
  const int m0 = (t / ntn) * 64, n0 = (t % ntn) * 64;
  __shared__ double As[64 * LA];   // As[m * LA + k]
  __shared__ double Bs[DK * LB];   // Bs[k * LB + n]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const gdouble *A = (const gdouble *)d.A;
  const gdouble *B = (const gdouble *)d.B;
  double ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + q * 256;
      int mm, kk;
      if (!TA) { mm = idx >> 4; kk = idx & 15; }
      else { kk = idx >> 6; mm = idx & 63; }
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < d.M && gk < d.K) ? A[TA ? gk * d.lda + gm : gm * d.lda + gk] : 0.0;
      int nn;
      if (!TB) { kk = idx >> 6; nn = idx & 63; }
      else { nn = idx >> 4; kk = idx & 15; }
      const int gn = n0 + nn, gk2 = k0 + kk;
      rb[q] = (gn < d.N && gk2 < d.K) ? B[TB ? gn * d.ldb + gk2 : gk2 * d.ldb + gn] : 0.0;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + q * 256;
      int mm, kk;
      if (!TA) { mm = idx >> 4; kk = idx & 15; }
      else { kk = idx >> 6; mm = idx & 63; }
      As[mm * LA + kk] = ra[q];
      int nn;
      if (!TB) { kk = idx >> 6; nn = idx & 63; }
      else { nn = idx >> 4; kk = idx & 15; }
      Bs[kk * LB + nn] = rb[q];
    }
  };
  const int kb = (d.tri & GEMM_TRI_A_UPPER) ? min(m0, d.K) : 0;
  const int ke = (d.tri & GEMM_TRI_B_UPPER) ? min(d.K, n0 + 64) : d.K;
  if (kb < ke) gload(kb);
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  const double *ap = As + (wr * 32 + (lane & 15)) * LA + (lane >> 4);
  const double *bp = Bs + (lane >> 4) * LB + wc * 32 + (lane & 15);
  for (int k0 = kb; k0 < ke; k0 += DK) {
    sstore();
    __syncthreads();
    if (k0 + DK < ke) gload(k0 + DK);
#pragma unroll
    for (int kk = 0; kk < DK; kk += 4) {
      const double a0 = ap[kk], a1 = ap[16 * LA + kk];
      const double b0 = bp[kk * LB], b1 = bp[kk * LB + 16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  gdouble *C = (gdouble *)d.C;
  const double al = d.alpha, be = d.beta;
  // C (when it is accumulated): every load from an in-range (clamped)
  // address, all in one round trip
  double cv[2][2][4];
  if (be != 0.0)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gnc = min(n0 + wc * 32 + j * 16 + (lane & 15), d.N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
          cv[i][j][r] = C[min(gm, d.M - 1) * d.ldc + gnc];
        }
      }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        if (gm < d.M && gn < d.N) {
          double v = al * acc[i][j][r];
          if (be != 0.0) v += be * cv[i][j][r];
          C[gm * d.ldc + gn] = v;
        }
      }
    }
}

int launch_gemm(FType t, const GemmDesc *d_items, const int32_t *d_tile_start, int nitems,
                int total_tiles, hipStream_t st, int tile_base, int tmode, int uniform,
                const int32_t *d_coarse) {
  if (nitems <= 0 || total_tiles <= 0) return SPAND_OK;
  const dim3 g(total_tiles), b(256);
  const int u = uniform;
  const int32_t *cs = d_coarse;
  if (t == FType::F64 && tmode == 0)
    hipLaunchKernelGGL((k_gemm_f64_mfma<0, 0>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (t == FType::F64 && tmode == 1)
    hipLaunchKernelGGL((k_gemm_f64_mfma<0, 1>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (t == FType::F64 && tmode == 2)
    hipLaunchKernelGGL((k_gemm_f64_mfma<1, 0>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (t == FType::F64)
    hipLaunchKernelGGL((k_gemm_f64_mfma<1, 1>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (tmode == 0)
    hipLaunchKernelGGL((k_gemm_f32_mfma<0, 0>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (tmode == 1)
    hipLaunchKernelGGL((k_gemm_f32_mfma<0, 1>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else if (tmode == 2)
    hipLaunchKernelGGL((k_gemm_f32_mfma<1, 0>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  else
    hipLaunchKernelGGL((k_gemm_f32_mfma<1, 1>), g, b, 0, st, d_items, d_tile_start, cs, nitems, tile_base, u);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ copies
// Each thread moves COPY_ILP elements per round, all loads issued before the
// stores: with a few elements per thread the waves would hold too few bytes
// in flight to cover the memory latency (3.3 TB/s measured on the W copies
// with one element per load round).
constexpr int COPY_ILP = 8;
template <typename Ts, typename Td>
__global__ __launch_bounds__(256) void k_copy(const CopyDesc *__restrict__ items) {
  const CopyDesc d = items[blockIdx.x];
  const Ts *src = (const Ts *)d.src;
  Td *dst = (Td *)d.dst;
  const int64_t total = (int64_t)d.rows * d.cols;
  const Ts sc = Ts(d.scale);
  constexpr int PER = 256 * COPY_ILP;
  if (total + int64_t(gridDim.y) * PER <= INT_MAX) {
    // 32-bit index arithmetic (a 64-bit division per element costs more
    // than the element's memory traffic); the bound keeps the last
    // index of a round within int
    const int tot = int(total), cols = d.cols;
    for (int base = blockIdx.y * PER + threadIdx.x; base < tot; base += gridDim.y * PER) {
      Ts v[COPY_ILP];
#pragma unroll
      for (int j = 0; j < COPY_ILP; ++j) {
        const int idx = base + j * 256;
        if (idx < tot) {
          const int r = idx / cols, c = idx - r * cols;
          v[j] = d.trans ? src[(int64_t)c * d.lds + r] : src[(int64_t)r * d.lds + c];
        }
      }
#pragma unroll
      for (int j = 0; j < COPY_ILP; ++j) {
        const int idx = base + j * 256;
        if (idx < tot) {
          const int r = idx / cols, c = idx - r * cols;
          dst[(int64_t)r * d.ldd + c] = Td(v[j] * sc);
        }
      }
    }
    return;
  }
  for (int64_t idx = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.y * blockDim.x) {
    const int r = int(idx / d.cols), c = int(idx % d.cols);
    const Ts v = d.trans ? src[(int64_t)c * d.lds + r] : src[(int64_t)r * d.lds + c];
    dst[(int64_t)r * d.ldd + c] = Td(v * sc);
  }
}

int launch_copy(FType t, int src_is_factor, const CopyDesc *d_items, int n, int64_t max_elems,
                hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  int gy = int(std::min<int64_t>(64, std::max<int64_t>(1, cdiv(max_elems, 256 * COPY_ILP))));
  dim3 grid(n, gy);
  if (t == FType::F64) {
    hipLaunchKernelGGL((k_copy<double, double>), grid, dim3(256), 0, st, d_items);
  } else if (src_is_factor) {
    hipLaunchKernelGGL((k_copy<float, float>), grid, dim3(256), 0, st, d_items);
  } else {
    hipLaunchKernelGGL((k_copy<double, float>), grid, dim3(256), 0, st, d_items);
  }
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// Gather of whole b x b blocks of BSR value arrays (FP64, row-major blocks;
// each item names its source block, so one launch may read the blocks of
// several matrices) into factor-precision matrices: one workgroup per item,
// source read contiguously, destination rows of b at leading dimension ldd.
template <typename Td>
__global__ __launch_bounds__(256) void k_bsr_gather(const GatherItem *__restrict__ items, int b) {
  const GatherItem it = items[blockIdx.x];
  const double *s = it.src;
  Td *d = (Td *)it.dst;
  const int bb = b * b;
  for (int idx = threadIdx.x; idx < bb; idx += 256) {
    const int r = idx / b, c = idx - r * b;
    d[(int64_t)r * it.ldd + c] = Td(s[idx]);
  }
}

int launch_bsr_gather(FType t, const GatherItem *d_items, int n, int b, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  if (t == FType::F64)
    hipLaunchKernelGGL(k_bsr_gather<double>, dim3(n), dim3(256), 0, st, d_items, b);
  else
    hipLaunchKernelGGL(k_bsr_gather<float>, dim3(n), dim3(256), 0, st, d_items, b);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// dst(r, c) = scale * src(c, r): tiles of 64 x 64 read along the source rows
// into LDS (16 loads in flight per thread), written along the destination
// rows (both coalesced).
template <typename Ts, typename Td>
__global__ __launch_bounds__(256) void k_copy_t(const CopyDesc *__restrict__ items, int tiles_c) {
  const CopyDesc d = items[blockIdx.x];
  const int tr = blockIdx.y / tiles_c, tc = blockIdx.y % tiles_c;
  const int r0 = tr * 64, c0 = tc * 64;
  if (r0 >= d.rows || c0 >= d.cols) return;
  __shared__ Ts tile[64][65];
  const Ts *src = (const Ts *)d.src;
  Td *dst = (Td *)d.dst;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;    // 64 x 4
  Ts v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = ty + 4 * q;
    const int c = c0 + k, r = r0 + tx;                      // source row c, column r
    v[q] = (c < d.cols && r < d.rows) ? src[(int64_t)c * d.lds + r] : Ts(0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) tile[ty + 4 * q][tx] = v[q];
  __syncthreads();
  const Ts sc = Ts(d.scale);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = ty + 4 * q;
    const int r = r0 + k, c = c0 + tx;
    if (r < d.rows && c < d.cols) dst[(int64_t)r * d.ldd + c] = Td(tile[tx][k] * sc);
  }
}

int launch_copy_t(FType t, int src_is_factor, const CopyDesc *d_items, int n, int max_rows,
                  int max_cols, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  const int tiles_c = int(cdiv(max_cols, 64));
  dim3 grid(n, unsigned(cdiv(max_rows, 64) * tiles_c));   // tiles <= 32*32 < 65536
  if (t == FType::F64)
    hipLaunchKernelGGL((k_copy_t<double, double>), grid, dim3(256), 0, st, d_items, tiles_c);
  else if (src_is_factor)
    hipLaunchKernelGGL((k_copy_t<float, float>), grid, dim3(256), 0, st, d_items, tiles_c);
  else
    hipLaunchKernelGGL((k_copy_t<double, float>), grid, dim3(256), 0, st, d_items, tiles_c);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale(const ScaleDesc *__restrict__ items) {
  const ScaleDesc d = items[blockIdx.x];
  T *A = (T *)d.A;
  const T *rs = (const T *)d.rs;
  const T *cs = (const T *)d.cs;
  const int64_t total = (int64_t)d.rows * d.cols;
  for (int64_t idx = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.y * blockDim.x) {
    const int r = int(idx / d.cols), c = int(idx % d.cols);
    T v = A[(int64_t)r * d.ld + c];
    if (rs) v *= rs[r];
    if (cs) v *= cs[c];
    A[(int64_t)r * d.ld + c] = v;
  }
}

int launch_scale(FType t, const ScaleDesc *d_items, int n, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  dim3 grid(n, 16);
  if (t == FType::F64)
    hipLaunchKernelGGL(k_scale<double>, grid, dim3(256), 0, st, d_items);
  else
    hipLaunchKernelGGL(k_scale<float>, grid, dim3(256), 0, st, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void k_eye(const EyeDesc *__restrict__ items) {
  const EyeDesc d = items[blockIdx.x];
  T *A = (T *)d.A;
  const int64_t total = (int64_t)d.n * d.n;
  for (int64_t idx = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.y * blockDim.x) {
    const int r = int(idx / d.n), c = int(idx % d.n);
    A[(int64_t)r * d.ld + c] = (r == c) ? T(1) : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(const ZeroDesc *__restrict__ items) {
  const ZeroDesc d = items[blockIdx.x];
  T *A = (T *)d.A;
  const int64_t total = (int64_t)d.rows * d.cols;
  for (int64_t idx = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.y * blockDim.x) {
    const int r = int(idx / d.cols), c = int(idx % d.cols);
    A[(int64_t)r * d.ld + c] = T(0);
  }
}

int launch_zero(FType t, const ZeroDesc *d_items, int n, int64_t max_elems, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  const int gy = int(std::min<int64_t>(64, std::max<int64_t>(1, cdiv(max_elems, 256))));
  const dim3 grid(n, gy);
  if (t == FType::F64)
    hipLaunchKernelGGL(k_zero<double>, grid, dim3(256), 0, st, d_items);
  else
    hipLaunchKernelGGL(k_zero<float>, grid, dim3(256), 0, st, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

int launch_eye(FType t, const EyeDesc *d_items, int n, int max_n, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  int gy = int(std::min<int64_t>(64, std::max<int64_t>(1, cdiv((int64_t)max_n * max_n, 256))));
  dim3 grid(n, gy);
  if (t == FType::F64)
    hipLaunchKernelGGL(k_eye<double>, grid, dim3(256), 0, st, d_items);
  else
    hipLaunchKernelGGL(k_eye<float>, grid, dim3(256), 0, st, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ elimination panel
// One workgroup owns one matrix.  Row r of the panel lives in thread
// r % ELIM_NT, slot r / ELIM_NT.  Virtual pivoting: rows are never swapped;
// piv[k + c] records the row chosen for column k + c, and used[] marks rows
// that already served as pivots.
//   MODE 0 (Gauss-Jordan, pivoting): in-place inversion step; after all
//          panels row piv[j] holds row j of the inverse with its columns in
//          pivot order (undone by k_row_gather with colperm).
//   MODE 1 (LU on [A | I], pivoting): eliminates only rows not yet used as
//          pivots; on exit row piv[j] holds row j of U in the A part and row
//          j of L^{-1} P^T in the identity part.
//   MODE 2 (Gauss-Jordan, no pivoting): pivot of column j is row j.
// The panel's effect on the other columns is the rank-w update
//   A[:, rest] = A[:, rest] with rows piv zeroed + P * A_old[piv, rest]
// where P (n x w) is E e_piv (E = product of the panel's elementary steps):
// for Gauss-Jordan P is the final panel itself, for LU it is tracked in Y.
template <typename T, int MODE>
__global__ __launch_bounds__(ELIM_NT) void k_elim_panel(const ElimDesc *__restrict__ items, int k,
                                                        int *__restrict__ flag, int cw0, int cw1) {
  constexpr int NT = ELIM_NT, RPT = ELIM_RPT, NB = ELIM_NB;
  const ElimDesc d = items[blockIdx.x];
  const int n = d.n;
  if (k >= n) return;
  const int w = min(NB, n - k);
  T *A = (T *)d.A;
  T *P = (T *)d.P;
  T *Tb = (T *)d.T;
  const int64_t ld = d.ld;
  const int tid = threadIdx.x;
  __shared__ T prow_s[NB];
  __shared__ T yrow_s[NB];
  __shared__ double redv[NT / 64];
  __shared__ int redi[NT / 64];
  __shared__ int s_prow;
  __shared__ int s_piv[NB];
  T pan[RPT][NB];
  T Y[RPT][NB];
  bool usedf[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = tid + j * NT;
    usedf[j] = false;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      pan[j][c] = T(0);
      Y[j][c] = T(0);
    }
    if (r < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < w) pan[j][c] = A[(int64_t)r * ld + k + c];
      if (MODE != 2) usedf[j] = d.used[r] != 0;
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < w) {   // w is uniform over the workgroup
    int prow;
    if (MODE == 2) {
      prow = k + c;
    } else {
      double bv = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = tid + j * NT;
        if (r < n && !usedf[j]) {
          double v = fabs((double)pan[j][c]);
          if (v > bv || (v == bv && r < bi)) { bv = v; bi = r; }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(bv, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if ((tid & 63) == 0) { redv[tid >> 6] = bv; redi[tid >> 6] = bi; }
      __syncthreads();
      if (tid == 0) {
        double v = redv[0];
        int ii = redi[0];
        for (int q = 1; q < NT / 64; ++q)
          if (redv[q] > v || (redv[q] == v && redi[q] < ii)) { v = redv[q]; ii = redi[q]; }
        s_prow = ii;
      }
      __syncthreads();
      prow = s_prow;
    }
    if (prow % NT == tid) {
      const int jj = prow / NT;
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        if (j != jj) continue;
        if (MODE == 1) Y[j][c] = T(1);
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
          prow_s[cc] = pan[j][cc];
          yrow_s[cc] = Y[j][cc];
        }
        usedf[j] = true;
      }
      s_piv[c] = prow;
    }
    __syncthreads();
    T p = prow_s[c];
    if (p == T(0)) {
      if (tid == 0) atomicOr(flag, 1);
      p = T(1);
    }
    const T ip = T(1) / p;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = tid + j * NT;
      if (r >= n) continue;
      if (MODE != 1) {
        if (r == prow) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) pan[j][cc] = (cc == c) ? ip : prow_s[cc] * ip;
        } else {
          const T fp = pan[j][c] * ip;
#pragma unroll
          for (int cc = 0; cc < NB; ++cc)
            pan[j][cc] = (cc == c) ? -fp : pan[j][cc] - fp * prow_s[cc];
        }
      } else {
        if (usedf[j]) continue;      // pivot rows (earlier or now) stay as U rows
        const T f = pan[j][c] * ip;
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) {
          if (cc > c) pan[j][cc] -= f * prow_s[cc];
          if (cc <= c) Y[j][cc] -= f * yrow_s[cc];
        }
        pan[j][c] = T(0);
      }
    }
    __syncthreads();
    }
  }
  // write back panel, P, pivots and used flags
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = tid + j * NT;
    if (r >= n) continue;
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      if (cc < w) A[(int64_t)r * ld + k + cc] = pan[j][cc];
      P[(int64_t)r * NB + cc] = (cc < w) ? (MODE == 1 ? Y[j][cc] : pan[j][cc]) : T(0);
    }
    if (MODE != 2) d.used[r] = usedf[j] ? 1 : 0;
  }
  if (tid < w) d.piv[k + tid] = s_piv[tid];
  // pivot rows of the non-panel columns -> T, then zero them in A.  The
  // panel columns of T are zero so the update leaves the panel unchanged.
  // Only the column window [cw0, cw1) is touched (a blocked elimination
  // applies the panels of a block to the columns outside it at once).
  const int c0 = max((MODE == 1) ? k : 0, cw0);
  const int ncol = min(d.ncols, cw1) - c0;
  for (int idx = tid; idx < w * ncol; idx += NT) {
    const int cq = idx / ncol;
    const int col = c0 + idx % ncol;
    const int64_t src = (int64_t)s_piv[cq] * ld + col;
    if (col >= k && col < k + w) {
      Tb[(int64_t)cq * ld + col] = T(0);
    } else {
      Tb[(int64_t)cq * ld + col] = A[src];
      A[src] = T(0);
    }
  }
}

// A[:, c0:ncols] += P[:, 0:w] * T[0:w, c0:ncols]
template <typename T>
__global__ __launch_bounds__(256) void k_elim_update(const ElimDesc *__restrict__ items, int k,
                                                     int lu_mode, int cw0, int cw1) {
  const ElimDesc d = items[blockIdx.x];
  const int n = d.n;
  if (k >= n) return;
  const int w = min(ELIM_NB, n - k);
  const int c0 = max(lu_mode ? k : 0, cw0);
  const int cend = min(d.ncols, cw1);
  const int ncol = cend - c0;
  if (ncol <= 0) return;
  const int ntn = (ncol + 63) >> 6, ntm = (n + 63) >> 6;
  const int t = blockIdx.y;
  if (t >= ntm * ntn) return;
  const int m0 = (t / ntn) * 64, n0 = c0 + (t % ntn) * 64;
  __shared__ T Ps[ELIM_NB][65];
  __shared__ T Ts[ELIM_NB][65];
  const T *P = (const T *)d.P;
  const T *Tb = (const T *)d.T;
  T *A = (T *)d.A;
  const int64_t ld = d.ld;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < ELIM_NB * 64; idx += 256) {
    const int mm = idx / ELIM_NB, kk = idx % ELIM_NB;
    Ps[kk][mm] = (kk < w && m0 + mm < n) ? P[(int64_t)(m0 + mm) * ELIM_NB + kk] : T(0);
    const int kk2 = idx / 64, nn = idx % 64;
    Ts[kk2][nn] = (kk2 < w && n0 + nn < cend) ? Tb[(int64_t)kk2 * ld + n0 + nn] : T(0);
  }
  __syncthreads();
  const int tm = tid >> 4, tn = tid & 15;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
#pragma unroll
  for (int kk = 0; kk < ELIM_NB; ++kk) {
    T a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = Ps[kk][tm + 16 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Ts[kk][tn + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + tm + 16 * i;
    if (gm >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tn + 16 * j;
      if (gn >= cend) continue;
      A[(int64_t)gm * ld + gn] += acc[i][j];
    }
  }
}

int launch_elim_step(FType t, const ElimDesc *d_items, int nactive, int k, int mode,
                     int max_tiles, int *d_flag, int cw0, int cw1, hipStream_t st) {
  if (nactive <= 0) return SPAND_OK;
  const int lu = mode == 1;
  if (t == FType::F64) {
    if (mode == 0)
      hipLaunchKernelGGL((k_elim_panel<double, 0>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    else if (mode == 1)
      hipLaunchKernelGGL((k_elim_panel<double, 1>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    else
      hipLaunchKernelGGL((k_elim_panel<double, 2>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    SP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_elim_update<double>, dim3(nactive, max_tiles), dim3(256), 0, st, d_items, k, lu, cw0, cw1);
  } else {
    if (mode == 0)
      hipLaunchKernelGGL((k_elim_panel<float, 0>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    else if (mode == 1)
      hipLaunchKernelGGL((k_elim_panel<float, 1>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    else
      hipLaunchKernelGGL((k_elim_panel<float, 2>), dim3(nactive), dim3(ELIM_NT), 0, st, d_items, k, d_flag, cw0, cw1);
    SP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_elim_update<float>, dim3(nactive, max_tiles), dim3(256), 0, st, d_items, k, lu, cw0, cw1);
  }
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// Largest of v over the 64 lanes of a wave (every lane active), in every
// lane: DPP max within each row of 16 (quad xor 1, quad xor 2, half-row
// mirror, row mirror), then the four row results through readlane.
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const uint32_t a = __builtin_amdgcn_readlane((int)v, 0), b = __builtin_amdgcn_readlane((int)v, 16);
  const uint32_t c = __builtin_amdgcn_readlane((int)v, 32), d = __builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// Pivot key of a value: the bit pattern of |x| orders like |x| (NaN counts
// as zero, so it still names a valid row).
__device__ inline uint64_t pivot_key(float x) {
  const float a = fabsf(x);
  return a == a ? uint64_t(__float_as_uint(a)) : 0;
}
__device__ inline uint64_t pivot_key(double x) {
  const double a = fabs(x);
  return a == a ? uint64_t(__double_as_longlong(a)) : 0;
}

// Lane of the largest key among the lanes with can set, lowest lane on
// ties; -1 if no lane may pivot.  *kmax receives that key.
template <typename T>
__device__ inline int wave_argmax_key(uint64_t key, bool can, uint64_t *kmax) {
  uint64_t b;
  if (sizeof(T) == 4) {
    const uint32_t m = wave_max_u32(can ? uint32_t(key) : 0u);
    b = __ballot(can && uint32_t(key) == m);
    *kmax = m;
  } else {
    const uint32_t hi = uint32_t(key >> 32), lo = uint32_t(key);
    const uint32_t mh = wave_max_u32(can ? hi : 0u);
    const bool c2 = can && hi == mh;
    const uint32_t ml = wave_max_u32(c2 ? lo : 0u);
    b = __ballot(c2 && lo == ml);
    *kmax = (uint64_t(mh) << 32) | ml;
  }
  return b ? int(__builtin_ctzll(b)) : -1;
}

// ------------------------------------------------------------------ fused block elimination
// One workgroup eliminates the block columns [k0, k0 + wb), wb <= BW, of
// one matrix and applies them to the whole column window [k0, k0 + BW)
// (columns past n exist for LU on [A | I]); one row per thread
// (blockDim.x >= n), the window part of the row in registers.  BW = 64
// (ELIM_BLK), except for FP64 matrices of more than 512 rows: 1024 rows of
// 64 doubles would take the whole register file of a CU, so they take
// blocks of 32 columns.  The
// steps run in groups of 4 columns with the slots fixed inside a group, so
// every register index is a compile-time constant while the group loop
// stays rolled (see the step below).
// Per step: argmax of |a_rc| over the rows that may still pivot (DPP wave
// maximum and ballot, ties to the lowest row; each wave posts its
// candidate's whole row to LDS and one barrier later every thread takes
// the best), then one fused multiply-add per slot.
//   MODE 0/2: Gauss-Jordan (with / without pivoting); every row changes,
//             the pivot row is scaled; on exit the block columns are the
//             block's P_B.
//   MODE 3:   Gauss-Jordan without pivoting on A - S, S = diag(s_c) chosen
//             as each column is reached: s_c = -sign of the current a_cc,
//             so every pivot has modulus >= 1 (the signs go to d.sg).
//   MODE 1:   LU; only rows not yet used as pivots change.  A changed row
//             keeps its multipliers (the block's elimination matrix taken at
//             the pivot rows) in the slots of the columns already
//             eliminated, so PB (n x BW) is written out on exit with
//             no second array: row r of PB is those slots, then 1 at the
//             row's own pivot column for rows pivoted in this block.
template <typename T, int MODE, int MAXT, int BW>
__global__ __launch_bounds__(MAXT) void k_elim_block(const ElimDesc *__restrict__ items, int k0,
                                                     int *__restrict__ flag) {
  constexpr int NWMAX = MAXT / 64, V = 16 / sizeof(T);
  constexpr bool NOPIV = MODE >= 2;        // pivot of block column c is row k0 + c
  static_assert(BW >= 8 && (BW & (BW - 1)) == 0, "slot rotation needs a power-of-two block");
  const ElimDesc d = items[blockIdx.x];
  const int n = d.n;
  if (k0 >= n) return;
  const int wb = min(BW, n - k0);          // columns eliminated
  const int wc = min(BW, d.ncols - k0);    // columns of the window carried along
  const int tid = threadIdx.x, wv = tid >> 6, nw = blockDim.x >> 6;
  T *A = (T *)d.A;
  const int64_t ld = d.ld;
  __shared__ __align__(16) T cand[2][NWMAX][BW];
  __shared__ uint64_t cval[2][NWMAX];
  __shared__ int cidx[2][NWMAX];
  __shared__ unsigned long long ckey[3];   // FP32: (|pivot| bits << 32) | ~row, max over waves
  __shared__ int s_piv[BW];
  const bool live = tid < n;
  // 16-byte row chunks when every row start is aligned and the block is whole
  const bool vec = wb == BW && (ld % V) == 0 && ((uintptr_t)A % 16) == 0;
  T s[BW];
  bool used = false;
  int pc = -1;     // block column this row pivoted at; -2: pivot of an earlier block
#pragma unroll
  for (int i = 0; i < BW; ++i) s[i] = T(0);
  if (live) {
    const T *src = A + (int64_t)tid * ld + k0;
    if (vec) {
#pragma unroll
      for (int i = 0; i < BW; i += V) {
        T tmp[V];
        *(uint4 *)tmp = *(const uint4 *)(src + i);
#pragma unroll
        for (int v = 0; v < V; ++v) s[i + v] = tmp[v];
      }
    } else {
#pragma unroll
      for (int i = 0; i < BW; ++i)
        if (i < wc) s[i] = src[i];
    }
    if (!NOPIV && d.used[tid] != 0) {
      used = true;
      pc = -2;
    }
  }
  constexpr bool KEYED = sizeof(T) == 4 && !NOPIV;
  if (KEYED) {
    if (tid < 3) ckey[tid] = 0;
    __syncthreads();
  }
  // One step per block column.  The steps run in groups of 4: at the start
  // of a group slot i holds block column (c0 + i) mod BW, step k of the
  // group eliminates slot k (a compile-time index), and the slots rotate by
  // 4 between groups.  Inside a group every slot stays in its register, so
  // the candidate rows go to LDS and come back as aligned 16-byte vectors.
  auto step = [&](const int c, const int k) {
    if (c >= wb) return;
    const int buf = c & 1;
    int prow, ws = 0, bi = -1;
    uint64_t kmax = 0;
    if (NOPIV) {
      prow = k0 + c;
      if (tid == prow) {
#pragma unroll
        for (int i = 0; i < BW; i += V) *(uint4 *)&cand[buf][0][i] = *(const uint4 *)&s[i];
      }
      __syncthreads();
    } else {
      const bool can = live && !used;
      const int wl = wave_argmax_key<T>(pivot_key(s[k]), can, &kmax);
      bi = wl < 0 ? -1 : (wv << 6) + wl;
      if (tid == bi) {
#pragma unroll
        for (int i = 0; i < BW; i += V) *(uint4 *)&cand[buf][wv][i] = *(const uint4 *)&s[i];
      }
      // kmax and bi are uniform over the wave
      if (KEYED && bi >= 0 && (tid & 63) == 0)
        atomicMax(&ckey[c % 3], (unsigned long long)((kmax << 32) | uint32_t(~bi)));
    }
    if (KEYED) {
      // the key of step c - 1 is no longer read by anyone: clear it for step c + 2
      __syncthreads();
      if (tid == 0) ckey[(c + 2) % 3] = 0;
      const unsigned long long key = ckey[c % 3];
      prow = key ? int(~uint32_t(key)) : -1;
      ws = prow >> 6;
      if (prow < 0 || prow >= n) {
        if (tid == 0) atomicOr(flag, 1);   // reported as a failed factorization
        prow = k0 + c;
        ws = 0;
      }
    } else if (!NOPIV) {
      if ((tid & 63) == 0) {
        cval[buf][wv] = kmax;
        cidx[buf][wv] = bi;
      }
      __syncthreads();
      // best candidate over the waves; on equal keys the lower wave holds
      // the lower row.  Some row may always pivot (n - k0 - c unused rows),
      // the fallback only keeps a bad key from naming a row out of range.
      uint64_t best = 0;
      ws = -1;
      for (int q = 0; q < nw; ++q) {
        const uint64_t kq = cval[buf][q];
        if (cidx[buf][q] >= 0 && (ws < 0 || kq > best)) { best = kq; ws = q; }
      }
      prow = ws < 0 ? -1 : cidx[buf][ws];
      if (prow < 0 || prow >= n) {
        if (tid == 0) atomicOr(flag, 1);   // reported as a failed factorization
        prow = k0 + c;
        ws = 0;
      }
    }
    const uint4 *pr = (const uint4 *)&cand[buf][ws][0];
    if (tid == 0) s_piv[c] = prow;
    T pq[V];
    *(uint4 *)pq = pr[k / V];
    T p = pq[k % V];
    if (MODE == 3) {
      // shifted pivot a_cc - s_c with s_c = -sign(a_cc): modulus >= 1
      const T sgn = p >= T(0) ? T(-1) : T(1);
      if (tid == 0) ((T *)d.sg)[k0 + c] = sgn;
      p -= sgn;
    } else if (p == T(0)) {
      if (tid == 0) atomicOr(flag, 1);
      p = T(1);
    }
    const T ip = T(1) / p;
    const bool is_piv = tid == prow;
    T h, z;
    if (MODE == 1) {
      const bool upd = live && !used && !is_piv;
      h = upd ? -s[k] * ip : T(0);
      z = upd ? h : s[k];
      if (is_piv) {
        used = true;
        pc = c;
      }
    } else {
      if (is_piv) {
#pragma unroll
        for (int i = 0; i < BW; ++i) s[i] *= ip;
        h = T(0);
        z = ip;
        used = true;
      } else {
        h = -s[k] * ip;
        z = h;
      }
    }
#pragma unroll
    for (int i = 0; i < BW; i += V) {
      T pv[V];
      *(uint4 *)pv = pr[i / V];
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (i + v != k) s[i + v] = fma(h, pv[v], s[i + v]);
    }
    s[k] = z;
  };
  const int nsteps = (wb + 3) & ~3;
  for (int c = 0; c < nsteps; c += 4) {
    step(c, 0);
    step(c + 1, 1);
    step(c + 2, 2);
    step(c + 3, 3);
    T t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = s[i];
#pragma unroll
    for (int i = 0; i < BW - 4; ++i) s[i] = s[i + 4];
#pragma unroll
    for (int i = 0; i < 4; ++i) s[BW - 4 + i] = t[i];
  }
  __syncthreads();
  // slot i now holds block column (nsteps + i) mod BW
  if (live) {
    T *dst = A + (int64_t)tid * ld + k0;
    if (MODE == 1) {
      T *pb = (T *)d.PB + (int64_t)tid * BW;
#pragma unroll
      for (int i = 0; i < BW; ++i) {
        const int col = (nsteps + i) & (BW - 1);
        if (col >= wc) continue;
        if (col >= wb) {            // window column past the last pivot column
          dst[col] = s[i];
          continue;
        }
        T a, y;
        if (pc == -2) {
          a = s[i];
          y = T(0);
        } else if (pc == -1) {
          a = T(0);
          y = s[i];
        } else {
          a = col >= pc ? s[i] : T(0);
          y = col < pc ? s[i] : (col == pc ? T(1) : T(0));
        }
        dst[col] = a;
        pb[col] = y;
      }
    } else if (vec) {
#pragma unroll
      for (int i = 0; i < BW; i += V) {
        T tmp[V];
#pragma unroll
        for (int v = 0; v < V; ++v) tmp[v] = s[i + v];
        *(uint4 *)(dst + i) = *(uint4 *)tmp;
      }
    } else {
#pragma unroll
      for (int i = 0; i < BW; ++i) {
        const int col = (nsteps + i) & (BW - 1);
        if (col < wc) dst[col] = s[i];
      }
    }
    if (!NOPIV) d.used[tid] = used ? 1 : 0;
  }
  if (tid < wb) d.piv[k0 + tid] = s_piv[tid];
}

int elim_block_max_n(FType) { return 1024; }

int elim_block_width(FType t, int n) { return t == FType::F64 && n > 512 ? 32 : ELIM_BLK; }

template <typename T, int MAXT, int BW>
static void elim_block_modes(int mode, dim3 grid, dim3 block, hipStream_t st,
                             const ElimDesc *d_items, int k0, int *d_flag) {
  if (mode == 0)
    hipLaunchKernelGGL((k_elim_block<T, 0, MAXT, BW>), grid, block, 0, st, d_items, k0, d_flag);
  else if (mode == 1)
    hipLaunchKernelGGL((k_elim_block<T, 1, MAXT, BW>), grid, block, 0, st, d_items, k0, d_flag);
  else if (mode == 2)
    hipLaunchKernelGGL((k_elim_block<T, 2, MAXT, BW>), grid, block, 0, st, d_items, k0, d_flag);
  else
    hipLaunchKernelGGL((k_elim_block<T, 3, MAXT, BW>), grid, block, 0, st, d_items, k0, d_flag);
}

int launch_elim_block(FType t, const ElimDesc *d_items, int nactive, int k0, int mode, int nmax,
                      int bw, int *d_flag, hipStream_t st) {
  if (nactive <= 0) return SPAND_OK;
  if (nmax > elim_block_max_n(t) || bw != elim_block_width(t, nmax)) {
    set_error("fused block elimination: n = %d, block width %d (limit %d rows, width %d)", nmax,
              bw, elim_block_max_n(t), elim_block_width(t, nmax));
    return SPAND_EINVAL;
  }
  const dim3 grid(nactive), block(unsigned(cdiv(nmax, 64) * 64));
  if (t == FType::F64) {
    if (bw == 32)
      elim_block_modes<double, 1024, 32>(mode, grid, block, st, d_items, k0, d_flag);
    else
      elim_block_modes<double, 512, ELIM_BLK>(mode, grid, block, st, d_items, k0, d_flag);
  } else {
    elim_block_modes<float, 1024, ELIM_BLK>(mode, grid, block, st, d_items, k0, d_flag);
  }
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// Blocked elimination: after the panels of the block [k0, k0 + wb) have been
// applied to the block's own columns, the pivot rows of the columns the block
// has not touched yet move to TB (wb x ld) and are zeroed in A, so that
// A[:, rest] += P_B TB is the whole block's effect there (P_B = the block
// columns for Gauss-Jordan, the tracked multipliers PB for LU).  Gauss-Jordan
// updates every column outside the block; LU only the columns after it.
template <typename T>
__global__ __launch_bounds__(256) void k_elim_extract(const ElimDesc *__restrict__ items, int k0,
                                                      int bw, int lu) {
  const ElimDesc d = items[blockIdx.x];
  if (k0 >= d.n) return;
  const int wb = min(bw, d.n - k0);
  const int cw1 = k0 + bw;
  T *A = (T *)d.A;
  T *TB = (T *)d.TB;
  const int64_t ld = d.ld;
  for (int q = blockIdx.y; q < wb; q += gridDim.y) {
    T *__restrict__ row = A + (int64_t)d.piv[k0 + q] * ld;
    T *__restrict__ tb = TB + (int64_t)q * ld;
    // four loads in flight per thread before the stores
    for (int c0 = threadIdx.x; c0 < d.ncols; c0 += 4 * 256) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * 256;
        const bool keep = c < cw1 && (lu || c >= k0);   // the block's window stays
        v[u] = (c < d.ncols && !keep) ? row[c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * 256;
        if (c >= d.ncols) break;
        tb[c] = v[u];
        if (!(c < cw1 && (lu || c >= k0))) row[c] = T(0);
      }
    }
  }
}

int launch_elim_extract(FType t, const ElimDesc *d_items, int nactive, int k0, int bw, int lu,
                        hipStream_t st) {
  if (nactive <= 0) return SPAND_OK;
  const dim3 grid(nactive, 16);
  if (t == FType::F64)
    hipLaunchKernelGGL(k_elim_extract<double>, grid, dim3(256), 0, st, d_items, k0, bw, lu);
  else
    hipLaunchKernelGGL(k_elim_extract<float>, grid, dim3(256), 0, st, d_items, k0, bw, lu);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// Blocked LU: fold panel k (multipliers Y = d.P, n x w, pivots piv[k..k+w))
// into the block's multiplier matrix PB (n x ELIM_BLK) of block k0: the
// earlier panels' columns 0..c1 receive this panel's effect (their pivot
// rows of this panel are moved out and zeroed, then PB += Y * those rows),
// and Y becomes columns c1..c1+w.  One workgroup per item.
template <typename T>
__global__ __launch_bounds__(256) void k_elim_pb(const ElimDesc *__restrict__ items, int k, int k0) {
  const ElimDesc d = items[blockIdx.x];
  if (k >= d.n) return;
  const int w = min(ELIM_NB, d.n - k);
  const int c1 = k - k0;                   // columns of earlier panels in PB
  const T *Y = (const T *)d.P;
  T *PB = (T *)d.PB;
  __shared__ double ts[ELIM_NB * ELIM_BLK];
  const int tid = threadIdx.x;
  if (c1 > 0) {
    for (int idx = tid; idx < w * c1; idx += 256) {
      const int t = idx / c1, c = idx % c1;
      ts[idx] = double(PB[(int64_t)d.piv[k + t] * ELIM_BLK + c]);
    }
    __syncthreads();
    for (int idx = tid; idx < w * c1; idx += 256) {
      const int t = idx / c1, c = idx % c1;
      PB[(int64_t)d.piv[k + t] * ELIM_BLK + c] = T(0);
    }
    __syncthreads();
    for (int idx = tid; idx < d.n * c1; idx += 256) {
      const int i = idx / c1, c = idx % c1;
      double v = double(PB[(int64_t)i * ELIM_BLK + c]);
      for (int t = 0; t < w; ++t) v += double(Y[(int64_t)i * ELIM_NB + t]) * ts[t * c1 + c];
      PB[(int64_t)i * ELIM_BLK + c] = T(v);
    }
  }
  for (int idx = tid; idx < d.n * w; idx += 256) {
    const int i = idx / w, t = idx % w;
    PB[(int64_t)i * ELIM_BLK + c1 + t] = Y[(int64_t)i * ELIM_NB + t];
  }
}

int launch_elim_pb(FType t, const ElimDesc *d_items, int nactive, int k, int k0, hipStream_t st) {
  if (nactive <= 0) return SPAND_OK;
  if (t == FType::F64)
    hipLaunchKernelGGL(k_elim_pb<double>, dim3(nactive), dim3(256), 0, st, d_items, k, k0);
  else
    hipLaunchKernelGGL(k_elim_pb<float>, dim3(nactive), dim3(256), 0, st, d_items, k, k0);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// out[j, c] = src[piv[j], colperm ? pinv[c] : c + col_off],  j < n, c < cols
template <typename T>
__global__ __launch_bounds__(256) void k_row_gather(const RowGatherDesc *__restrict__ items) {
  const RowGatherDesc d = items[blockIdx.x];
  __shared__ int pinv[ELIM_MAXN];
  if (d.colperm) {
    for (int j = threadIdx.x; j < d.n; j += blockDim.x) pinv[d.piv[j]] = j;
  }
  __syncthreads();
  const T *src = (const T *)d.src;
  T *dst = (T *)d.dst;
  for (int j = blockIdx.y; j < d.n; j += gridDim.y) {
    const T *srow = src + (int64_t)d.piv[j] * d.lds;
    T *drow = dst + (int64_t)j * d.ldd;
    // four loads in flight per thread before the stores
    for (int c0 = threadIdx.x; c0 < d.cols; c0 += 4 * 256) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * 256;
        if (c < d.cols) v[u] = srow[d.colperm ? pinv[c] : c + d.col_off];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * 256;
        if (c < d.cols) drow[c] = v[u];
      }
    }
  }
}

int launch_row_gather(FType t, const RowGatherDesc *d_items, int n, int max_rows,
                      hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  dim3 grid(n, std::max(1, std::min(max_rows, 64)));
  if (t == FType::F64)
    hipLaunchKernelGGL(k_row_gather<double>, grid, dim3(256), 0, st, d_items);
  else
    hipLaunchKernelGGL(k_row_gather<float>, grid, dim3(256), 0, st, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ level-0 Schur
// target(b x b) -= A1 * Y * A2 for every item of a group, items in order.
// A1, A2: b x b copies of the coupling blocks (factor precision, ld b);
// Y: b x b block of an interior inverse (ld ldy).
__global__ __launch_bounds__(256, 4) void k_schur_elem_mfma(int bs, const SchurGroup *__restrict__ groups,
                                                            const SchurItem *__restrict__ items) {
  constexpr int LS = 65, NE = 16;   // rows of a b x b block per thread (b <= 64)
  const SchurGroup g = groups[blockIdx.x];
  __shared__ float L0[64 * LS];     // A1 (row-major), then -T1
  __shared__ float L1[64 * LS];     // Y, then A2 (both [k][n])
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int kmax = (bs + 1) & ~1;
  float *tg = (float *)g.target;
  const int col = wc * 32 + (lane & 31);
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    acc[r] = (row < bs && col < bs) ? tg[(int64_t)row * g.ldt + col] : 0.f;
  }
  // zero padding rows/columns stay zero in both tiles
  for (int e = tid; e < 64 * LS; e += 256) {
    L0[e] = 0.f;
    L1[e] = 0.f;
  }
  // element (r, c) of a block: this thread takes column c = tid % 64 of the
  // rows r = tid / 64 + 4q; the next pair's blocks are fetched into
  // registers while the current pair is multiplied
  const int c0 = tid & 63, r0 = tid >> 6;
  const bool cin = c0 < bs;
  float ra[NE], ry[NE], r2[NE];
  auto fetch_a1y = [&](int it) {
    const SchurItem s = items[it];
    const float *a1 = (const float *)s.A1 + r0 * bs + c0;
    const float *Y = (const float *)s.Y + (int64_t)r0 * s.ldy + c0;
    const int64_t ys = 4 * (int64_t)s.ldy;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) {
        ra[q] = a1[q * 4 * bs];
        ry[q] = Y[q * ys];
      }
  };
  auto fetch_a2 = [&](int it) {
    const float *a2 = (const float *)items[it].A2 + r0 * bs + c0;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) r2[q] = a2[q * 4 * bs];
  };
  if (g.item_begin < g.item_end) {
    fetch_a1y(g.item_begin);
    fetch_a2(g.item_begin);
  }
  __syncthreads();
  const float *ap = L0 + (wr * 32 + (lane & 31)) * LS + (lane >> 5);
  const float *bp = L1 + (lane >> 5) * LS + wc * 32 + (lane & 31);
  float *l0 = L0 + r0 * LS + c0, *l1 = L1 + r0 * LS + c0;
  for (int it = g.item_begin; it < g.item_end; ++it) {
    const bool more = it + 1 < g.item_end;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) {
        l0[q * 4 * LS] = ra[q];
        l1[q * 4 * LS] = ry[q];
      }
    __syncthreads();
    if (more) fetch_a1y(it + 1);
    f32x16 t1;
#pragma unroll
    for (int r = 0; r < 16; ++r) t1[r] = 0.f;
    for (int kk = 0; kk < kmax; kk += 2)
      t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[kk], bp[kk * LS], t1, 0, 0, 0);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      L0[row * LS + col] = (row < bs && col < bs) ? -t1[r] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) l1[q * 4 * LS] = r2[q];
    __syncthreads();
    if (more) fetch_a2(it + 1);
    for (int kk = 0; kk < kmax; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[kk], bp[kk * LS], acc, 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < bs && col < bs) tg[(int64_t)row * g.ldt + col] = acc[r];
  }
}

// FP64 version on the matrix cores: the same two products per coupling pair
// with v_mfma_f64_16x16x4f64, each wave a 32x32 quarter as 2x2 blocks of
// 16x16 (layout as in k_gemm_f64_mfma); the target stays in the
// accumulators for all its pairs.
__global__ __launch_bounds__(256, 2) void k_schur_elem_mfma64(int bs, const SchurGroup *__restrict__ groups,
                                                              const SchurItem *__restrict__ items) {
  constexpr int LS = 65, NE = 16;
  const SchurGroup g = groups[blockIdx.x];
  __shared__ double L0[64 * LS];     // A1 (row-major), then -T1
  __shared__ double L1[64 * LS];     // Y, then A2 (both [k][n])
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int kmax = (bs + 3) & ~3;
  double *tg = (double *)g.target;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        acc[i][j][r] = (row < bs && col < bs) ? tg[(int64_t)row * g.ldt + col] : 0.0;
      }
    }
  // zero padding rows/columns stay zero in both tiles
  for (int e = tid; e < 64 * LS; e += 256) {
    L0[e] = 0.0;
    L1[e] = 0.0;
  }
  // element mapping and prefetch of the next pair as in k_schur_elem_mfma
  const int c0 = tid & 63, r0 = tid >> 6;
  const bool cin = c0 < bs;
  double ra[NE], ry[NE], r2[NE];
  auto fetch_a1y = [&](int it) {
    const SchurItem s = items[it];
    const double *a1 = (const double *)s.A1 + r0 * bs + c0;
    const double *Y = (const double *)s.Y + (int64_t)r0 * s.ldy + c0;
    const int64_t ys = 4 * (int64_t)s.ldy;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) {
        ra[q] = a1[q * 4 * bs];
        ry[q] = Y[q * ys];
      }
  };
  auto fetch_a2 = [&](int it) {
    const double *a2 = (const double *)items[it].A2 + r0 * bs + c0;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) r2[q] = a2[q * 4 * bs];
  };
  if (g.item_begin < g.item_end) {
    fetch_a1y(g.item_begin);
    fetch_a2(g.item_begin);
  }
  __syncthreads();
  double *l0 = L0 + r0 * LS + c0, *l1 = L1 + r0 * LS + c0;
  const double *ap = L0 + (wr * 32 + (lane & 15)) * LS + (lane >> 4);
  const double *bp = L1 + (lane >> 4) * LS + wc * 32 + (lane & 15);
  auto product = [&](f64x4 (&c)[2][2]) {
    for (int kk = 0; kk < kmax; kk += 4) {
      const double a0 = ap[kk], a1 = ap[16 * LS + kk];
      const double b0 = bp[kk * LS], b1 = bp[kk * LS + 16];
      c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0][0], 0, 0, 0);
      c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[0][1], 0, 0, 0);
      c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[1][0], 0, 0, 0);
      c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[1][1], 0, 0, 0);
    }
  };
  for (int it = g.item_begin; it < g.item_end; ++it) {
    const bool more = it + 1 < g.item_end;
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) {
        l0[q * 4 * LS] = ra[q];
        l1[q * 4 * LS] = ry[q];
      }
    __syncthreads();
    if (more) fetch_a1y(it + 1);
    f64x4 t1[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) t1[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    product(t1);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wc * 32 + j * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr * 32 + i * 16 + (lane >> 4) + 4 * r;
          L0[row * LS + col] = (row < bs && col < bs) ? -t1[i][j][r] : 0.0;
        }
      }
#pragma unroll
    for (int q = 0; q < NE; ++q)
      if (cin && r0 + 4 * q < bs) l1[q * 4 * LS] = r2[q];
    __syncthreads();
    if (more) fetch_a2(it + 1);
    product(acc);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        if (row < bs && col < bs) tg[(int64_t)row * g.ldt + col] = acc[i][j][r];
      }
    }
}

int launch_schur_elem(FType t, int bs, const SchurGroup *d_groups, int ngroups,
                      const SchurItem *d_items, hipStream_t st) {
  if (ngroups <= 0) return SPAND_OK;
  if (bs > 64) {
    set_error("level-0 Schur: element block %d exceeds 64", bs);
    return SPAND_EINVAL;
  }
  if (t == FType::F64)
    hipLaunchKernelGGL(k_schur_elem_mfma64, dim3(ngroups), dim3(256), 0, st, bs, d_groups, d_items);
  else
    hipLaunchKernelGGL(k_schur_elem_mfma, dim3(ngroups), dim3(256), 0, st, bs, d_groups, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ------------------------------------------------------------------ QRCP
// Workgroup GEMM used by the QRCP completion: for i < M, n < N,
// epi(i, n, sum_l A(i, l) B(l, n)), 64 x 64 output tiles, K in chunks of 16,
// 4 x 4 outputs per thread, float64 accumulation.  As/Bs: 1024 doubles each
// in LDS.  BK: load the B tile with l fastest (B(l, n) contiguous in l).
template <bool BK, typename FA, typename FB, typename FE>
__device__ inline void wg_gemm(int M, int N, int K, FA A, FB B, FE epi, double *As, double *Bs) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  for (int i0 = 0; i0 < M; i0 += 64)
    for (int n0 = 0; n0 < N; n0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
      for (int l0 = 0; l0 < K; l0 += 16) {
        __syncthreads();
        for (int e = tid; e < 1024; e += 256) {
          const int i = e & 63, l = e >> 6;
          As[l * 64 + i] = (i0 + i < M && l0 + l < K) ? A(i0 + i, l0 + l) : 0.0;
        }
        for (int e = tid; e < 1024; e += 256) {
          const int n = BK ? (e >> 4) : (e & 63), l = BK ? (e & 15) : (e >> 6);
          Bs[l * 64 + n] = (n0 + n < N && l0 + l < K) ? B(l0 + l, n0 + n) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int l = 0; l < 16; ++l) {
          double a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[q] = As[l * 64 + ty * 4 + q];
            b[q] = Bs[l * 64 + tx * 4 + q];
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
        }
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + ty * 4 + p, n = n0 + tx * 4 + q;
          if (i < M && n < N) epi(i, n, acc[p][q]);
        }
    }
  __syncthreads();
}

// Rank-revealing QR with column pivoting of W (m x nc, row-major), one
// workgroup per interface (Eq. 12).
//  1. Column norms of W.
//  2. Pivoted Gram-Schmidt with re-orthogonalisation (equal in exact
//     arithmetic to Householder QRCP: same pivots, same |R_ii|, same leading
//     columns of Q up to sign).  Column norms are downdated with the
//     LAPACK-style safeguard and recomputed when cancellation is detected.
//     Residual norms never grow, so a column already at or below the
//     stopping threshold eps |R_00| can never be a pivot: it leaves every
//     later pass.  Stops at the first |R_ii| <= eps |R_00| (or at the
//     numerical rank of the stored q's, |R_ii| <= 1e-12 |R_00| in FP64 and
//     1e-4 |R_00| in FP32, whatever eps).  The kept
//     vectors are rows of V (q_t = V[t m .. t m + m)).
//     The steps run in blocks.  A block takes the BQ unselected columns of
//     largest norm as candidates, orthonormalises their residuals into a
//     basis B (BQ x m) and reads W once to form H = B W (BQ values per
//     column, FP64).  While the pivot chosen over all columns is a
//     candidate, its residual and hence q_k lie in span(B), q_k = c^T B,
//     and row k of R is c^T H: the norms of all columns are downdated
//     from H alone.  A pivot outside the candidates ends the block.  The
//     pivots are exactly those of the unblocked method; W is read once per
//     block instead of once per step.
//  3. Completion to an orthogonal Q by Householder reconstruction (Ballard
//     et al., "Reconstructing Householder vectors from tall-skinny QR",
//     IPDPS 2014): with Q_c = [q_0 .. q_{k-1}] = [Q1; Q2] (Q1 k x k) and
//     signs S fixed while inverting Q1 - S (every pivot gets modulus >= 1),
//     H = I + (Q_c S - E) [I, G2^T] with G2 = Q2 (Q1 - S)^-1, E = [I_k; 0],
//     is orthogonal and H E = Q_c S.  Output Q = [Q_c | H(:, k:m)].
//     Rows k.. of V receive G2 S; tau receives S.
template <typename T, int BQ>
__global__ __launch_bounds__(256, 3) void k_qrcp(const QrcpDesc *__restrict__ items, double eps,
                                              int force_full, int MS, int GS, int complete) {
  static_assert(BQ % 2 == 0, "H is read in pairs");
  const QrcpDesc d = items[blockIdx.x];
  const int m = d.m, nc = d.ncols;
  const int64_t ldw = d.ldw;
  constexpr int VN = 16 / sizeof(T);            // columns per 16-byte load
  using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  const int ngrp = (nc + VN - 1) / VN;
  const T *W = (const T *)d.W;      // current layout (packed copies alternate with W2)
  T *Wother = (T *)d.W2;
  T *Q = (T *)d.Q;
  T *Qt = (T *)d.V;
  double *vn1 = d.vn1, *vn2 = d.vn2;
  int *sel = d.sel;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // dynamic LDS: u[MS], cbuf[MS] (or the two GEMM tiles, or the
  // candidates' coefficients P[MS][BQ]), the candidate
  // basis Bm[BQ][MS], the block's coordinates Cc[BQ][BQ] and av[BQ], then
  // the list of active column groups (GS entries) and the candidates
  extern __shared__ double qsm[];
  const int ldsd = max(max(2 * MS, 2048), BQ * MS);
  double *u = qsm, *cbuf = qsm + MS;
  double *Bm = qsm + ldsd, *Cc = Bm + BQ * MS, *av = Cc + BQ * BQ;
  int *act = reinterpret_cast<int *>(av + BQ);
  int *sidx = act + GS;
  double *H = d.H;                  // ldw x BQ: column j of B W at H + j BQ
  __shared__ int s_j, s_nflag, s_nf, s_in;
  __shared__ double rv[4];
  __shared__ int ri[4];
  __shared__ double cnw[BQ];
  __shared__ int wtot[4];
  __shared__ int s_fl[64];
  __shared__ double red[16];
  __shared__ double s_piv;
  const double tol3z = 1.4901161193847656e-08;  // sqrt(2^-52)

  // c[t] = q_t . x for t < n (one wave per 4 consecutive t)
  auto qdots = [&](const double *x, int n, double *c) {
    for (int t0 = wid * 4; t0 < n; t0 += 16) {
      const T *q0 = Qt + (int64_t)t0 * m;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
      for (int r = lane; r < m; r += 64) {
        const double xr = x[r];
        a0 += double(q0[r]) * xr;
        if (t0 + 1 < n) a1 += double(q0[m + r]) * xr;
        if (t0 + 2 < n) a2 += double(q0[2 * m + r]) * xr;
        if (t0 + 3 < n) a3 += double(q0[3 * m + r]) * xr;
      }
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      a2 = wave_sum(a2);
      a3 = wave_sum(a3);
      if (lane == 0) {
        c[t0] = a0;
        if (t0 + 1 < n) c[t0 + 1] = a1;
        if (t0 + 2 < n) c[t0 + 2] = a2;
        if (t0 + 3 < n) c[t0 + 3] = a3;
      }
    }
    __syncthreads();
  };
  // x -= sum_{t<n} c[t] q_t (eight independent sums keep eight loads in flight)
  auto qsub = [&](double *x, int n, const double *c) {
    for (int r = tid; r < m; r += 256) {
      double sv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) sv[q] = 0.0;
      const T *qr = Qt + r;
      int t = 0;
      for (; t + 8 <= n; t += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) sv[q] += double(qr[(int64_t)(t + q) * m]) * c[t + q];
      }
      for (; t < n; ++t) sv[0] += double(qr[(int64_t)t * m]) * c[t];
      x[r] -= ((sv[0] + sv[1]) + (sv[2] + sv[3])) + ((sv[4] + sv[5]) + (sv[6] + sv[7]));
    }
    __syncthreads();
  };

  // ---- 1. column norms, VN adjacent columns per thread with 16-byte loads
  for (int g = tid; g < ngrp; g += 256) {
    double acc[VN];
#pragma unroll
    for (int q = 0; q < VN; ++q) acc[q] = 0.0;
    const T *base = W + (int64_t)g * VN;
    int r = 0;
    for (; r + 4 <= m; r += 4) {
      VT v[4];
#pragma unroll
      for (int u4 = 0; u4 < 4; ++u4) v[u4] = *reinterpret_cast<const VT *>(base + (int64_t)(r + u4) * ldw);
#pragma unroll
      for (int u4 = 0; u4 < 4; ++u4) {
        const T *e = reinterpret_cast<const T *>(&v[u4]);
#pragma unroll
        for (int q = 0; q < VN; ++q) acc[q] += double(e[q]) * double(e[q]);
      }
    }
    for (; r < m; ++r) {
      const VT v = *reinterpret_cast<const VT *>(base + (int64_t)r * ldw);
      const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
      for (int q = 0; q < VN; ++q) acc[q] += double(e[q]) * double(e[q]);
    }
#pragma unroll
    for (int q = 0; q < VN; ++q) {
      const int j = g * VN + q;
      vn1[j] = j < nc ? sqrt(acc[q]) : 0.0;
      vn2[j] = vn1[j];
      sel[j] = j < nc ? 0 : 1;      // padding columns never take part
    }
  }
  __syncthreads();
  double cmax = 0.0;
  for (int j = tid; j < nc; j += 256) cmax = fmax(cmax, vn1[j]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
  if (lane == 0) red[wid] = cmax;
  __syncthreads();
  cmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  // |R_00| is the largest column norm; the 1e-4 margin keeps a column whose
  // norm ties the threshold up to rounding
  const double thr = force_full ? 0.0 : eps * cmax * (1.0 - 1e-4);
  // A group's flags and norms, loaded together (one memory round trip; the
  // empty statement keeps the compiler from moving the loads apart into
  // the branches that use them).
  auto load_group = [&](int g, int (&sg)[VN], double (&vg)[VN]) {
#pragma unroll
    for (int q = 0; q < VN; ++q) {
      sg[q] = sel[g * VN + q];
      vg[q] = vn1[g * VN + q];
    }
#pragma unroll
    for (int q = 0; q < VN; ++q) asm volatile("" ::"v"(sg[q]), "v"(vg[q]));
  };
  auto live_group = [&](int g) {
    int sg[VN];
    double vg[VN];
    load_group(g, sg, vg);
    bool a = false;
#pragma unroll
    for (int q = 0; q < VN; ++q)
      if (!sg[q] && vg[q] > thr) a = true;
    return a;
  };
  // Order-preserving filter of a list of groups (src == nullptr: all groups
  // 0..n-1) into dst; returns the new length (the same on every thread).
  // Stable compaction of the live groups; dst may be src: every thread reads
  // its entry of a round before the round's first barrier and entries are
  // only written at or below the position they are read from.
  auto filter = [&](const int *src, int n, int *dst) {
    int base = 0;
    for (int q0 = 0; q0 < n; q0 += 256) {
      const int qa = q0 + tid;
      const int g = qa < n ? (src ? src[qa] : qa) : 0;
      const bool keep = qa < n && live_group(g);
      const unsigned long long bal = __ballot(keep);
      if (lane == 0) wtot[wid] = __popcll(bal);
      __syncthreads();
      int off = base;
      for (int w = 0; w < wid; ++w) off += wtot[w];
      if (keep) dst[off + __popcll(bal & ((1ull << lane) - 1ull))] = g;
      base += wtot[0] + wtot[1] + wtot[2] + wtot[3];
      __syncthreads();
    }
    return base;
  };
  int nact_cur = filter(nullptr, ngrp, act);   // same value on every thread
  int cur_ngrp = ngrp;                         // groups of the current layout

  // ---- 2. pivoted Gram-Schmidt, in blocks of candidate columns
  double R00 = 0.0;
  int k = 0;
  const int imax = min(m, nc);
  // Numerical rank floor of the stored kept vectors: Gram-Schmidt against q's
  // whose orthogonality is delta (~sqrt(k) u, u the unit roundoff of T)
  // leaves a new residual x with projections ~delta^2 |w| on them, so q_k =
  // x / |x| is orthogonal only to delta^2 |w| / |x|.  Below 1e-12 |R_00|
  // (FP64) or 1e-4 |R_00| (FP32: delta^2 ~ 4e-12 at k = 1024) the residual
  // is rounding noise that cannot be made orthogonal; the completion of Q
  // supplies the remaining orthonormal columns.  Only eps below the floor is
  // affected (eps = 0 still keeps every unknown).
  const double floor_rel = sizeof(T) == 4 ? 1e-4 : 1e-12;
  const double stop_rel = fmax(force_full ? 0.0 : eps, floor_rel);
  // largest vn1 over the unselected columns of the live groups, ties ->
  // smallest index (the packed layouts keep the column order)
  int ncand_in = 0;               // candidates the pivot search checks against
  // block-wide maximum of the threads' (value, index) pairs: s_j, and s_in
  // = whether it is one of the block's candidates
  auto finish_argmax = [&](double bv, int bi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { rv[wid] = bv; ri[wid] = bi; }
    __syncthreads();
    if (tid == 0) {
      double v = rv[0];
      int ii = ri[0];
      for (int q = 1; q < 4; ++q)
        if (rv[q] > v || (rv[q] == v && ri[q] < ii)) { v = rv[q]; ii = ri[q]; }
      s_j = ii;
      int f = 0;                  // is it one of the block's candidates?
      for (int cq = 0; cq < ncand_in; ++cq) f |= sidx[cq] == ii;
      s_in = f;
    }
    __syncthreads();
    return s_j;
  };
  auto argmax_col = [&](int nact) {
    double bv = -1.0;
    int bi = INT_MAX;
    for (int qa = tid; qa < nact; qa += 256) {
      const int g = act[qa];
      int sg[VN];
      double vg[VN];
      load_group(g, sg, vg);
#pragma unroll
      for (int q = 0; q < VN; ++q) {
        const int j = g * VN + q;
        if (sg[q]) continue;
        const double v = vg[q];
        if (v > bv || (v == bv && j < bi)) { bv = v; bi = j; }
      }
    }
    return finish_argmax(bv, bi);
  };
  // c[l] = b_l . x and x -= sum_l c[l] b_l for the basis rows of Bm
  auto bdots = [&](const double *x, int n, double *c) {
    for (int l = wid; l < n; l += 4) {
      double a = 0.0;
      for (int r = lane; r < m; r += 64) a += Bm[l * MS + r] * x[r];
      a = wave_sum(a);
      if (lane == 0) c[l] = a;
    }
    __syncthreads();
  };
  auto bsub = [&](double *x, int n, const double *c) {
    for (int r = tid; r < m; r += 256) {
      double sv = 0.0;
      for (int l = 0; l < n; ++l) sv += Bm[l * MS + r] * c[l];
      x[r] -= sv;
    }
    __syncthreads();
  };
  bool done = false;
  while (!done && k < imax) {
    // keep the groups that can still hold a pivot (pruning never changes a
    // pivot: the largest norm is above the threshold whenever any is)
    if (k > 0) {
      nact_cur = filter(act, nact_cur, act);
      __syncthreads();
    }
    // Once at most half of the groups of the layout are live, pack the live
    // groups to the left of the other buffer (rows keep their stride), so
    // that every later pass reads whole contiguous rows.  The norms and
    // flags move with their columns; the order of columns is kept.
    if (2 * nact_cur <= cur_ngrp) {
      const int na = nact_cur;
      T *dst = Wother;
      for (int r = wid; r < m; r += 4)
        for (int p = lane; p < na; p += 64)
          *reinterpret_cast<VT *>(dst + (int64_t)r * ldw + p * VN) =
              *reinterpret_cast<const VT *>(W + (int64_t)r * ldw + act[p] * VN);
      // norms and flags, in rounds: a source position is never below its
      // destination, so reading a round completely before writing it is safe
      for (int p0 = 0; p0 < na * VN; p0 += 256) {
        const int pos = p0 + tid;
        double a1 = 0.0, a2 = 0.0;
        int sf = 1;
        if (pos < na * VN) {
          const int src = act[pos / VN] * VN + pos % VN;
          a1 = vn1[src];
          a2 = vn2[src];
          sf = sel[src];
        }
        __syncthreads();
        if (pos < na * VN) {
          vn1[pos] = a1;
          vn2[pos] = a2;
          sel[pos] = sf;
        }
        __syncthreads();
      }
      for (int p = tid; p < na; p += 256) act[p] = p;
      Wother = const_cast<T *>(W);
      W = dst;
      cur_ngrp = na;
      __syncthreads();
    }
    // (a) candidates: the BQ unselected columns of largest norm (ties to
    // the smaller index), in that order.  One pass keeps each thread's
    // best BQ sorted in registers; BQ block-wide maxima over the threads'
    // heads then pop them in order.
    ncand_in = 0;
    int ncand = 0;
    {
      double tv[BQ];
      int ti[BQ];
#pragma unroll
      for (int c = 0; c < BQ; ++c) { tv[c] = -1.0; ti[c] = INT_MAX; }
      auto better = [](double v, int j, double w, int i) { return v > w || (v == w && j < i); };
      for (int qa = tid; qa < nact_cur; qa += 256) {
        const int g = act[qa];
#pragma unroll 1
        for (int q = 0; q < VN; ++q) {
          const int j = g * VN + q;
          const int sj = sel[j];
          const double v = vn1[j];
          asm volatile("" ::"v"(sj), "v"(v));   // both loads in one round trip
          if (sj) continue;
          if (better(v, j, tv[BQ - 1], ti[BQ - 1])) {
            tv[BQ - 1] = v;
            ti[BQ - 1] = j;
#pragma unroll
            for (int c = BQ - 1; c > 0; --c)
              if (better(tv[c], ti[c], tv[c - 1], ti[c - 1])) {
                const double x = tv[c]; tv[c] = tv[c - 1]; tv[c - 1] = x;
                const int y = ti[c]; ti[c] = ti[c - 1]; ti[c - 1] = y;
              }
          }
        }
      }
      for (int cq = 0; cq < BQ; ++cq) {
        const int j = finish_argmax(tv[0], ti[0]);
        if (j == INT_MAX) break;
        if (tid == 0) sidx[cq] = j;
        if (ti[0] == j) {
#pragma unroll
          for (int c = 0; c + 1 < BQ; ++c) { tv[c] = tv[c + 1]; ti[c] = ti[c + 1]; }
          tv[BQ - 1] = -1.0;
          ti[BQ - 1] = INT_MAX;
        }
        ++ncand;
      }
    }
    if (ncand == 0) break;
    __syncthreads();
    // (b) their residuals against q_0..q_{k-1} (two block Gram-Schmidt
    // passes over the candidates at once; the k x BQ coefficients go
    // through H, which is free until the pass below), orthonormalised in
    // turn into the rows of Bm.  The first candidate (the next pivot)
    // always enters, like the pivot of the unblocked method.  Another
    // enters only while its row stays well conditioned: a residual above
    // 1e-4 of its column's norm (two passes leave it orthogonal to the q's
    // to ~1e-12) and above 1e-2 of it left after the earlier rows.  The
    // candidates that do not enter are dropped from the block (compacted
    // out of sidx): if one of them becomes the pivot, the block ends and
    // the next one starts with it.
    for (int e = tid; e < ncand * m; e += 256) {
      const int cq = e / m, r = e - cq * m;
      Bm[cq * MS + r] = double(W[(int64_t)r * ldw + sidx[cq]]);
    }
    for (int e = ncand * MS + tid; e < BQ * MS; e += 256) Bm[e] = 0.0;
    __syncthreads();
    for (int cq = wid; cq < ncand; cq += 4) {
      double a2 = 0.0;
      for (int r = lane; r < m; r += 64) a2 += Bm[cq * MS + r] * Bm[cq * MS + r];
      a2 = wave_sum(a2);
      if (lane == 0) cnw[cq] = sqrt(a2);
    }
    // P = Q_k^T U (k x BQ, in the u/cbuf area): lane (tl, rq) of a wave
    // takes row t = 16 tile + tl of Qt and the rows r = rq (mod 4); the four
    // partial sums meet by shuffles.  Then U -= Q_k P, one thread per row.
    double *P = qsm;
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      {
        const int tl = lane & 15, rq = lane >> 4;
        for (int t0 = wid * 16; t0 < k; t0 += 64) {
          const int t = t0 + tl;
          double a[BQ];
#pragma unroll
          for (int cq = 0; cq < BQ; ++cq) a[cq] = 0.0;
          if (t < k) {
            const T *qt = Qt + (int64_t)t * m;
            // eight rows' loads in one round trip, then their products in
            // row order
            int r = rq;
            for (; r + 28 < m; r += 32) {
              T qv[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) qv[u] = qt[r + 4 * u];
#pragma unroll
              for (int u = 0; u < 8; ++u) asm volatile("" ::"v"(qv[u]));
#pragma unroll
              for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int cq = 0; cq < BQ; ++cq) a[cq] += double(qv[u]) * Bm[cq * MS + r + 4 * u];
            }
            for (; r < m; r += 4) {
              const double qv = double(qt[r]);
#pragma unroll
              for (int cq = 0; cq < BQ; ++cq) a[cq] += qv * Bm[cq * MS + r];
            }
          }
#pragma unroll
          for (int cq = 0; cq < BQ; ++cq) {
            a[cq] += __shfl_xor(a[cq], 16, 64);
            a[cq] += __shfl_xor(a[cq], 32, 64);
          }
          if (rq == 0 && t < k)
#pragma unroll
            for (int cq = 0; cq < BQ; ++cq) P[t * BQ + cq] = a[cq];
        }
      }
      __syncthreads();
      for (int r = tid; r < m; r += 256) {
        double sv[BQ];
#pragma unroll
        for (int cq = 0; cq < BQ; ++cq) sv[cq] = 0.0;
        int t = 0;
        for (; t + 8 <= k; t += 8) {       // eight loads per round trip, products in order
          T qv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) qv[u] = Qt[(int64_t)(t + u) * m + r];
#pragma unroll
          for (int u = 0; u < 8; ++u) asm volatile("" ::"v"(qv[u]));
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int cq = 0; cq < BQ; ++cq) sv[cq] += P[(t + u) * BQ + cq] * double(qv[u]);
        }
        for (; t < k; ++t) {
          const double qv = double(Qt[(int64_t)t * m + r]);
#pragma unroll
          for (int cq = 0; cq < BQ; ++cq) sv[cq] += P[t * BQ + cq] * qv;
        }
#pragma unroll
        for (int cq = 0; cq < BQ; ++cq) Bm[cq * MS + r] -= sv[cq];
      }
      __syncthreads();
    }
    int nb = 0;
    for (int cq = 0; cq < ncand; ++cq) {
      double *x = Bm + cq * MS;
      double s0 = 0.0;
      for (int r = tid; r < m; r += 256) s0 += x[r] * x[r];
      const double n0 = sqrt(block_sum(s0, red));
      for (int pass = 0; pass < 2 && nb > 0; ++pass) {
        bdots(x, nb, cbuf);
        bsub(x, nb, cbuf);
      }
      double s1 = 0.0;
      for (int r = tid; r < m; r += 256) s1 += x[r] * x[r];
      const double n1 = sqrt(block_sum(s1, red));
      if (n1 > 0.0 && (cq == 0 || (n1 > 1e-2 * n0 && n0 > 1e-4 * cnw[cq]))) {
        const double inv = 1.0 / n1;
        // row cq moves to row nb <= cq (each thread moves its own entries)
        for (int r = tid; r < m; r += 256) Bm[nb * MS + r] = x[r] * inv;
        if (tid == 0) sidx[nb] = sidx[cq];
        ++nb;
      }
      __syncthreads();
    }
    ncand = nb;
    ncand_in = nb;
    // the next pivot itself has no residual left: the unblocked method stops there
    if (nb == 0) break;
    for (int e = nb * MS + tid; e < BQ * MS; e += 256) Bm[e] = 0.0;
    __syncthreads();
    // (c) H = Bm W for the live columns: one pass over W.  With few active
    // groups, RS adjacent lanes split the rows of one group (in blocks of 4)
    // and combine their sums by shuffles.
    {
      int RS = 1;
      while (RS < 8 && nact_cur * RS * 2 <= 256) RS *= 2;
      const int sl = tid % RS, ga = tid / RS, gpp = 256 / RS;
      const int m4 = m & ~3;
      for (int qa0 = 0; qa0 < nact_cur; qa0 += gpp) {
        const int qa = qa0 + ga;
        const bool live = qa < nact_cur;
        const int g = live ? act[qa] : 0;
        double acc[VN][BQ];
#pragma unroll
        for (int q = 0; q < VN; ++q)
#pragma unroll
          for (int l = 0; l < BQ; ++l) acc[q][l] = 0.0;
        if (live) {
          const T *base = W + (int64_t)g * VN;
          for (int r = sl * 4; r < m4; r += 4 * RS) {
            VT v[4];
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) v[u4] = *reinterpret_cast<const VT *>(base + (int64_t)(r + u4) * ldw);
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) {
              const T *e = reinterpret_cast<const T *>(&v[u4]);
#pragma unroll
              for (int l = 0; l < BQ; ++l) {
                const double bl = Bm[l * MS + r + u4];
#pragma unroll
                for (int q = 0; q < VN; ++q) acc[q][l] += bl * double(e[q]);
              }
            }
          }
          if (sl == 0)
            for (int r = m4; r < m; ++r) {
              const VT v = *reinterpret_cast<const VT *>(base + (int64_t)r * ldw);
              const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
              for (int l = 0; l < BQ; ++l) {
                const double bl = Bm[l * MS + r];
#pragma unroll
                for (int q = 0; q < VN; ++q) acc[q][l] += bl * double(e[q]);
              }
            }
        }
        for (int o = 1; o < RS; o <<= 1)
#pragma unroll
          for (int q = 0; q < VN; ++q)
#pragma unroll
            for (int l = 0; l < BQ; ++l) acc[q][l] += __shfl_xor(acc[q][l], o, 64);
        if (live && sl == 0) {
          double *hg = H + (int64_t)g * VN * BQ;
#pragma unroll
          for (int q = 0; q < VN; ++q)
#pragma unroll
            for (int l = 0; l < BQ; l += 2)
              *reinterpret_cast<double2 *>(hg + q * BQ + l) = make_double2(acc[q][l], acc[q][l + 1]);
        }
      }
    }
    __syncthreads();
    // (d) steps: while the next pivot is a candidate, its residual lies in
    // the span of Bm and so does q_k; row k of R is then c . H for every
    // column, which downdates all norms without reading W
    int nst = 0;
    int js_next = -1;                   // pivot found by the previous downdate
    for (;;) {
      if (k >= imax) { done = true; break; }
      const int js = js_next >= 0 ? js_next : argmax_col(nact_cur);
      if (js == INT_MAX) { done = true; break; }
      if (!s_in) break;                 // next block, with new candidates
      // coordinates of the pivot's residual against q_0..q_{k-1}, then
      // against the block's earlier q's (two passes): lane (t, l) of wave 0
      // holds c_t[l] and coordinate l; the dots reduce over l, the
      // corrections over t.  Its norm is |R_kk|.
      double *ck = Cc + nst * BQ;
      if (wid == 0) {
        const int t = lane / BQ, l = lane % BQ;
        double v = H[(int64_t)js * BQ + l];
        for (int pass = 0; pass < 2 && nst > 0; ++pass) {
          const double ct = t < nst ? Cc[t * BQ + l] : 0.0;
          double dt = ct * v;
#pragma unroll
          for (int o = 1; o < BQ; o <<= 1) dt += __shfl_xor(dt, o, 64);
          double w = dt * ct;
#pragma unroll
          for (int o = BQ; o < 64; o <<= 1) w += __shfl_xor(w, o, 64);
          v -= w;
        }
        const double nrm = sqrt(wave_sum(lane < BQ ? v * v : 0.0));
        if (lane < BQ) ck[lane] = nrm > 0.0 ? v / nrm : 0.0;
        if (lane == 0) s_piv = nrm;
      }
      __syncthreads();
      const double nrm = s_piv;
      if (k == 0) R00 = nrm;
      // below the floor the residual is rounding noise and Gram-Schmidt
      // could no longer make it orthogonal: the completion supplies the rest
      if (nrm == 0.0 || nrm <= stop_rel * R00) { done = true; break; }
      for (int r = tid; r < m; r += 256) {
        double sv = 0.0;
#pragma unroll
        for (int l = 0; l < BQ; ++l) sv += Bm[l * MS + r] * ck[l];
        Qt[(int64_t)k * m + r] = T(sv);
      }
      if (tid == 0) {
        sel[js] = 1;
        s_nflag = 0;
      }
      __syncthreads();
      // row k of R and downdate of the norms (LAPACK's safeguard: a norm
      // that lost too much to cancellation is recomputed below); the next
      // pivot search rides along on the new norms
      double nbv = -1.0;
      int nbi = INT_MAX;
      // one column's downdate from its loaded flag, norms and coordinates
      auto downdate = [&](int j, int sj, double a, double b, const double2 (&h2)[BQ / 2]) {
        if (sj) return;
        double rk = 0.0;
#pragma unroll
        for (int l = 0; l < BQ; l += 2) rk += ck[l] * h2[l / 2].x + ck[l + 1] * h2[l / 2].y;
        double v = a;                   // the column's norm after this step
        if (a != 0.0) {
          double temp = fabs(rk) / a;
          temp = fmax(0.0, (1.0 + temp) * (1.0 - temp));
          const double t2 = temp * (a / b) * (a / b);
          if (t2 <= tol3z) {
            // The estimate fell below sqrt(tol3z) b ~ 1.2e-4 b; with the
            // downdating error the true residual stays below 2e-4 b.  Under
            // the stopping threshold the column can never be a pivot
            // before the method stops: it is dropped, not recomputed.
            if (2e-4 * b < thr) {
              v = 0.0;
            } else {
              v = -1.0;               // recomputed below
              atomicAdd(&s_nflag, 1);
            }
          } else {
            v = a * sqrt(temp);
          }
          vn1[j] = v;
        }
        if (v > nbv || (v == nbv && j < nbi)) { nbv = v; nbi = j; }
      };
      for (int qa = tid; qa < nact_cur; qa += 256) {
        const int g = act[qa];
        const double *hg = H + (int64_t)g * VN * BQ;
#pragma unroll
        for (int q = 0; q < VN; q += 2) {
          // two columns' flags, norms and coordinates are loaded together
          // (every index lies in the arrays); an empty statement that takes
          // every loaded value keeps the loads at this point (one memory
          // round trip) instead of one after another in the branches
          const int j0 = g * VN + q;
          const int s0 = sel[j0], s1 = sel[j0 + 1];
          const double a0 = vn1[j0], a1 = vn1[j0 + 1];
          const double b0 = vn2[j0], b1 = vn2[j0 + 1];
          double2 h0[BQ / 2], h1[BQ / 2];
#pragma unroll
          for (int l = 0; l < BQ; l += 2) {
            h0[l / 2] = *reinterpret_cast<const double2 *>(hg + q * BQ + l);
            h1[l / 2] = *reinterpret_cast<const double2 *>(hg + (q + 1) * BQ + l);
          }
          asm volatile("" ::"v"(s0), "v"(a0), "v"(b0), "v"(s1), "v"(a1), "v"(b1));
#pragma unroll
          for (int l = 0; l < BQ / 2; ++l)
            asm volatile("" ::"v"(h0[l].x), "v"(h0[l].y), "v"(h1[l].x), "v"(h1[l].y));
          downdate(j0, s0, a0, b0, h0);
          downdate(j0 + 1, s1, a1, b1, h1);
        }
      }
      __syncthreads();
      // without recomputed norms the search is complete; otherwise it is
      // repeated after the recomputation
      js_next = s_nflag > 0 ? -1 : finish_argmax(nbv, nbi);
      if (s_nflag > 0) {
        // exact residual norms of the flagged columns against q_0..q_k
        for (;;) {
          if (tid == 0) s_nf = 0;
          __syncthreads();
          for (int qa = tid; qa < nact_cur; qa += 256) {
            const int g = act[qa];
#pragma unroll
            for (int q = 0; q < VN; ++q) {
              const int j = g * VN + q;
              if (!sel[j] && vn1[j] < 0.0) {
                const int p = atomicAdd(&s_nf, 1);
                if (p < 64) s_fl[p] = j;
              }
            }
          }
          __syncthreads();
          const int nf = min(s_nf, 64);
          if (nf == 0) break;
          for (int f = 0; f < nf; ++f) {
            const int j = s_fl[f];
            for (int r = tid; r < m; r += 256) u[r] = double(W[(int64_t)r * ldw + j]);
            __syncthreads();
            qdots(u, k + 1, cbuf);
            qsub(u, k + 1, cbuf);
            double s2 = 0.0;
            for (int r = tid; r < m; r += 256) s2 += u[r] * u[r];
            s2 = block_sum(s2, red);
            if (tid == 0) {
              vn1[j] = sqrt(s2);
              vn2[j] = vn1[j];
            }
            __syncthreads();
          }
        }
      }
      ++nst;
      ++k;
    }
  }
  __syncthreads();

  // ---- 3. complete Q (unless the caller completes it in batched launches
  // from the k_gs kept vectors)
  if (tid == 0) *d.k_gs = k;
  double *As = qsm, *Bs = qsm + 1024;
  if (complete && k == 0) {
    for (int i2 = tid >> 4; i2 < m; i2 += 16)
      for (int c = tid & 15; c < m; c += 16) Q[(int64_t)i2 * m + c] = T(i2 == c ? 1.0 : 0.0);
  } else if (complete) {
    if (k < m) {
      // Q1 into the top-left k x k of Q, then its in-place Gauss-Jordan
      // inversion with the diagonal shifted by -s_j when column j pivots
      for (int i2 = tid >> 4; i2 < k; i2 += 16)
        for (int c = tid & 15; c < k; c += 16) Q[(int64_t)i2 * m + c] = Qt[(int64_t)c * m + i2];
      __syncthreads();
      double *rowj = u, *colj = cbuf;
      for (int j = 0; j < k; ++j) {
        if (tid == 0) {
          const double a = double(Q[(int64_t)j * m + j]);
          const double s = a >= 0.0 ? -1.0 : 1.0;
          s_piv = 1.0 / (a - s);
          d.tau[j] = s;
        }
        __syncthreads();
        const double p = s_piv;
        for (int c = tid; c < k; c += 256) {
          rowj[c] = (c == j ? 1.0 : double(Q[(int64_t)j * m + c])) * p;
          colj[c] = c == j ? 0.0 : double(Q[(int64_t)c * m + j]);
        }
        __syncthreads();
        for (int i2 = tid >> 4; i2 < k; i2 += 16)
          for (int c = tid & 15; c < k; c += 16) {
            double v;
            if (i2 == j) v = rowj[c];
            else v = (c == j ? 0.0 : double(Q[(int64_t)i2 * m + c])) - colj[i2] * rowj[c];
            Q[(int64_t)i2 * m + c] = T(v);
          }
        __syncthreads();
      }
      // G2 S = Q2 (Q1 - S)^-1 S into rows k.. of V
      const double *sg = d.tau;
      wg_gemm<false>(
          m - k, k, k,
          [&](int i2, int l) { return double(Qt[(int64_t)l * m + k + i2]); },
          [&](int l, int t) { return double(Q[(int64_t)l * m + t]); },
          [&](int i2, int t, double v) { Qt[(int64_t)(k + i2) * m + t] = T(v * sg[t]); }, As, Bs);
      // H(:, k:m) = E_c + Q_c (G2 S)^T - [r < k] s_r G2(c, r)
      wg_gemm<true>(
          m, m - k, k,
          [&](int r, int t) { return double(Qt[(int64_t)t * m + r]); },
          [&](int t, int n) { return double(Qt[(int64_t)(k + n) * m + t]); },
          [&](int r, int n, double v) {
            const int c = k + n;
            if (r == c) v += 1.0;
            if (r < k) v -= sg[r] * double(Qt[(int64_t)c * m + r]);
            Q[(int64_t)r * m + c] = T(v);
          },
          As, Bs);
    }
    // Q(:, 0:k) = Q_c
    for (int r = tid >> 4; r < m; r += 16)
      for (int t = tid & 15; t < k; t += 16) Q[(int64_t)r * m + t] = Qt[(int64_t)t * m + r];
  }
  if (tid == 0) *d.k_out = force_full ? m : k;
}

size_t qrcp_lds_bytes(int maxm, int maxgrp, int bq) {
  const size_t MS = size_t(std::max(maxm, 1)), GS = size_t(std::max(maxgrp, 1)), B = size_t(bq);
  return (std::max(std::max<size_t>(2 * MS, 2048), B * MS) + B * MS + B * B + B) * sizeof(double) +
         (GS + B) * sizeof(int);
}

int qrcp_block_width(int maxm, int maxgrp) {
  for (int bq : {8, 4, 2})
    if (qrcp_lds_bytes(maxm, maxgrp, bq) <= QRCP_MAX_LDS) return bq;
  return 0;
}

int launch_qrcp(FType t, const QrcpDesc *d_items, int n, double eps, int force_full, int maxm,
                int maxgrp, int bq, int complete, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  const int MS = std::max(maxm, 1);
  const int GS = std::max(maxgrp, 1);
  const size_t lds = qrcp_lds_bytes(MS, GS, bq);
  if ((bq != 8 && bq != 4 && bq != 2) || lds > QRCP_MAX_LDS) {
    set_error("RRQR launch: block width %d, %zu bytes of LDS", bq, lds);
    return SPAND_EINVAL;
  }
  if (t == FType::F64) {
    if (bq == 8)
      hipLaunchKernelGGL((k_qrcp<double, 8>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
    else if (bq == 4)
      hipLaunchKernelGGL((k_qrcp<double, 4>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
    else
      hipLaunchKernelGGL((k_qrcp<double, 2>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
  } else {
    if (bq == 8)
      hipLaunchKernelGGL((k_qrcp<float, 8>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
    else if (bq == 4)
      hipLaunchKernelGGL((k_qrcp<float, 4>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
    else
      hipLaunchKernelGGL((k_qrcp<float, 2>), dim3(n), dim3(256), lds, st, d_items, eps, force_full, MS, GS, complete);
  }
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

}  // namespace spand

namespace spand {
template <typename T>
__global__ void k_diag_split(const DiagDesc *__restrict__ items) {
  const DiagDesc d = items[blockIdx.x];
  const T *U = (const T *)d.U;
  T *S = (T *)d.S;
  T *Si = (T *)d.Si;
  for (int j = threadIdx.x; j < d.n; j += blockDim.x) {
    const T s = sqrt(fabs(U[(int64_t)j * d.ld + j]));
    S[j] = s;
    Si[j] = s != T(0) ? T(1) / s : T(0);
  }
}

int launch_diag_split(FType t, const DiagDesc *d_items, int n, hipStream_t st) {
  if (n <= 0) return SPAND_OK;
  if (t == FType::F64)
    hipLaunchKernelGGL(k_diag_split<double>, dim3(n), dim3(256), 0, st, d_items);
  else
    hipLaunchKernelGGL(k_diag_split<float>, dim3(n), dim3(256), 0, st, d_items);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}
}  // namespace spand
