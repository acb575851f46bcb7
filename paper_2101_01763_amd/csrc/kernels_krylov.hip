// Small dense kernels of the s-step GMRES (paper Algorithm 2): Cholesky of
// the s x s Gram matrix (CholQR), combination of the two CGS/CholQR passes,
// Hessenberg reconstruction from the Newton change-of-basis matrix, Givens
// rotations and residual estimates, least-squares solve; plus a
// deterministic two-stage dot product.
#include "kernels_vec.h"

namespace spand {

// ---------------------------------------------------------------- dot
__global__ __launch_bounds__(256) void k_dot_part(int64_t N, const double *__restrict__ x,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * 4096;
  const int64_t r1 = std::min<int64_t>(N, r0 + 4096);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) acc += x[r] * y[r];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_dot_reduce(const double *__restrict__ part, int n,
                                                    double *__restrict__ out, int take_sqrt) {
  __shared__ double red[256];
  double acc = 0.0;
  // fixed partition -> deterministic
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = take_sqrt ? sqrt(red[0]) : red[0];
}

int launch_dot(int64_t N, const double *x, const double *y, double *part, double *out,
               int take_sqrt, hipStream_t st) {
  const int nb = int(std::max<int64_t>(1, cdiv(N, 4096)));
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(256), 0, st, N, x, y, part);
  SP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(256), 0, st, part, nb, out, take_sqrt);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- cycle init
__global__ void k_init_cycle(KrylovDev *K, int m) {
  for (int i = threadIdx.x; i < (KRY_MMAX + 1) * KRY_MMAX; i += blockDim.x) {
    K->H[i] = 0.0;
    K->Rm[i] = 0.0;
  }
  for (int i = threadIdx.x; i <= KRY_MMAX; i += blockDim.x) K->g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    K->g[0] = K->scal[0];
    K->bad = 0;
  }
}

int kry_init_cycle(KrylovDev *K, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_init_cycle, dim3(1), dim3(256), 0, st, K, m);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- Cholesky
// G = T^T T, T upper (row-major s x s).  Non-SPD -> K->bad = 1.
__global__ void k_chol(KrylovDev *K, int s, const double *G, double *T) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < s * s; ++i) T[i] = 0.0;
  for (int j = 0; j < s; ++j) {
    double d = G[j * s + j];
    for (int k = 0; k < j; ++k) d -= T[k * s + j] * T[k * s + j];
    if (!(d > 0.0)) {
      K->bad = 1;
      for (int i = 0; i < s; ++i) T[i * s + i] = 1.0;
      return;
    }
    const double tjj = sqrt(d);
    T[j * s + j] = tjj;
    for (int c = j + 1; c < s; ++c) {
      double v = G[j * s + c];
      for (int k = 0; k < j; ++k) v -= T[k * s + j] * T[k * s + c];
      T[j * s + c] = v / tjj;
    }
  }
}

int kry_chol(KrylovDev *K, int s, double *G, double *T, hipStream_t st) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(64), 0, st, K, s, G, T);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- Givens
__device__ void givens_column(KrylovDev *K, int c) {
  // rotate column c of H into Rm using the previous rotations (in place)
  // the rotated entry of row i + 1 is carried in a register (no read back of
  // what was just stored); every other load is of H, cs or sn
  const int ld = KRY_MMAX;
  double hi = K->H[c];
  for (int i = 0; i < c; ++i) {
    const double hn = K->H[(i + 1) * ld + c];
    const double ci = K->cs[i], si = K->sn[i];
    K->Rm[i * ld + c] = ci * hi + si * hn;
    hi = -si * hi + ci * hn;
  }
  const double a = hi, b = K->H[(c + 1) * ld + c];
  double cc = 1.0, ss = 0.0, r = a;
  if (b != 0.0) {
    r = hypot(a, b);
    cc = a / r;
    ss = b / r;
  }
  K->cs[c] = cc;
  K->sn[c] = ss;
  K->Rm[c * ld + c] = r;
  K->Rm[(c + 1) * ld + c] = 0.0;
  K->g[c + 1] = -ss * K->g[c];
  K->g[c] = cc * K->g[c];
  K->est[c] = fabs(K->g[c + 1]);
}

__global__ void k_givens_col(KrylovDev *K, int j) {
  if (threadIdx.x == 0) givens_column(K, j);
}

int kry_givens_col(KrylovDev *K, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_givens_col, dim3(1), dim3(64), 0, st, K, j);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- block finish
// R_a = R1 + R2 T1, R_b = T2 T1;  H[:, j:j+s] = (Rhat Bbar - [H Ctop; 0]) T^{-1}
// with Rhat = [[e_j, R_a], [0, R_b]], Ctop = Rhat[0:j, 0:s], T = Rhat[j:j+s, 0:s];
// then Givens rotations of the new columns.
// passes = 2: W = Q Ra + Wnew Rb with Ra = R1 + R2 T1, Rb = T2 T1 (block
// CGS2 + CholQR2); passes = 1: Ra = R1, Rb = T1.
__global__ __launch_bounds__(256) void k_block_finish(KrylovDev *K, int j, int s, int passes) {
  __shared__ double Ra[TS_MAXA * TS_MAXS];
  __shared__ double Rb[TS_MAXS * TS_MAXS];
  __shared__ double Rhat[TS_MAXA * (TS_MAXS + 1)];
  const int tid = threadIdx.x;
  const int a = j + 1, nr = j + 1 + s, w = s + 1, ld = KRY_MMAX;
  if (K->bad) return;
  for (int idx = tid; idx < a * s; idx += blockDim.x) {
    const int r = idx / s, c = idx % s;
    double v = K->R1[r * s + c];
    if (passes == 2)
      for (int q = 0; q <= c; ++q) v += K->R2[r * s + q] * K->T1[q * s + c];
    Ra[idx] = v;
  }
  for (int idx = tid; idx < s * s; idx += blockDim.x) {
    const int r = idx / s, c = idx % s;
    double v = 0.0;
    if (passes == 2)
      for (int q = r; q <= c; ++q) v += K->T2[r * s + q] * K->T1[q * s + c];
    else
      v = K->T1[r * s + c];
    Rb[idx] = (c >= r) ? v : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < nr * w; idx += blockDim.x) {
    const int r = idx / w, c = idx % w;
    double v = 0.0;
    if (c == 0) v = (r == j) ? 1.0 : 0.0;
    else if (r < a) v = Ra[r * s + c - 1];
    else v = Rb[(r - a) * s + c - 1];
    Rhat[idx] = v;
  }
  __syncthreads();
  // one thread per output row
  for (int r = tid; r < nr; r += blockDim.x) {
    double rb[TS_MAXS];
    for (int c = 0; c < s; ++c) {
      double v = 0.0;
      for (int q = 0; q < w; ++q) v += Rhat[r * w + q] * K->Bb[q * s + c];
      if (j > 0 && r <= j)
        for (int i = 0; i < j; ++i) v -= K->H[r * ld + i] * Rhat[i * w + c];
      rb[c] = v;
    }
    // X T = rb, T[p][c] = Rhat[(j+p)*w + c], upper triangular
    for (int c = 0; c < s; ++c) {
      double v = rb[c];
      for (int p = 0; p < c; ++p) v -= rb[p] * Rhat[(j + p) * w + c];
      rb[c] = v / Rhat[(j + c) * w + c];
    }
    for (int c = 0; c < s; ++c) K->H[r * ld + j + c] = rb[c];
  }
  __syncthreads();
  if (tid == 0)
    for (int c = j; c < j + s; ++c) givens_column(K, c);
}

int kry_block_finish(KrylovDev *K, int j, int s, int passes, hipStream_t st) {
  hipLaunchKernelGGL(k_block_finish, dim3(1), dim3(256), 0, st, K, j, s, passes);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- single reduce
// Upper Cholesky factor of the n x n matrix S (ld TS_MAXS) into T (ld
// TS_MAXS); false if S is not positive definite.  One thread.
__device__ bool chol_small(const double *S, int n, double *T) {
  for (int i = 0; i < TS_MAXS * TS_MAXS; ++i) T[i] = 0.0;
  for (int j = 0; j < n; ++j) {
    double d = S[j * TS_MAXS + j];
    for (int k = 0; k < j; ++k) d -= T[k * TS_MAXS + j] * T[k * TS_MAXS + j];
    if (!(d > 0.0)) return false;
    const double tjj = sqrt(d);
    T[j * TS_MAXS + j] = tjj;
    for (int c = j + 1; c < n; ++c) {
      double v = S[j * TS_MAXS + c];
      for (int k = 0; k < j; ++k) v -= T[k * TS_MAXS + j] * T[k * TS_MAXS + c];
      T[j * TS_MAXS + c] = v / tjj;
    }
  }
  return true;
}

// Columns j..j+s-1 of the Hessenberg matrix from a block's coefficients:
// (Rhat Bbar - [H[0:j+1, 0:j] Rhat[0:j, 0:s]; 0]) T^{-1}, T = Rhat[j:j+s, 0:s],
// Rhat (j+1+s) x (s+1) row-major in LDS; row r goes to out[r * ldo + c].
// One thread per row.
__device__ void hessenberg_cols(const KrylovDev *K, int j, int s, const double *Rhat,
                                double *out, int ldo) {
  const int nr = j + 1 + s, w = s + 1, ld = KRY_MMAX;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) {
    double rb[TS_MAXS];
    for (int c = 0; c < s; ++c) {
      double v = 0.0;
      for (int q = 0; q < w; ++q) v += Rhat[r * w + q] * K->Bb[q * s + c];
      if (j > 0 && r <= j)
        for (int i = 0; i < j; ++i) v -= K->H[r * ld + i] * Rhat[i * w + c];
      rb[c] = v;
    }
    for (int c = 0; c < s; ++c) {
      double v = rb[c];
      for (int p = 0; p < c; ++p) v -= rb[p] * Rhat[(j + p) * w + c];
      rb[c] = v / Rhat[(j + c) * w + c];
    }
    for (int c = 0; c < s; ++c) out[r * ldo + c] = rb[c];
  }
}

// Dense part of one single-reduce step (Algorithm 2 with the second pass
// lagged by one block), from the one Gram matrix G = K->LG =
// Q[:, 0:a+sp+sw]^T Q[:, a:a+sp+sw] (ld sp+sw).  Q[:, 0:a] is final, P =
// Q[:, a:a+sp] the pending block after one pass, W = Q[:, a+sp:a+sp+sw] new.
//  sp: R1 = Q_old^T P, T = chol(P^T P - R1^T R1) (Gram of P - Q_old R1); the
//      pending block's Hessenberg columns j0 = a-1 .. a+s-2 from
//      R_a = Pra + R1 Prb, R_b = T Prb and its starting vector Prho; Givens
//      rotations and residual estimates.  Not positive definite: bad = 1.
//  sw: C = [Q_old^T W; T^{-T}(P^T W - R1^T Q_old^T W)] (coefficients on the
//      re-orthogonalised basis), RV = chol(W^T W - C^T C): the new pending
//      block (Pra = C, Prb = RV, Prho = [R1[:, s-1]; T[:, s-1]], or e_{a-1}
//      with no P), and residual estimates from its one-pass Hessenberg
//      columns in est_t (rotations not kept).  Not positive definite: bad = 2.
__global__ __launch_bounds__(256) void k_lag_block(KrylovDev *K, int a, int sp, int sw, int s) {
  __shared__ double R1s[TS_MAXA * TS_MAXS];
  __shared__ double Cs[TS_MAXA * TS_MAXS];
  __shared__ double Rhat[TS_MAXA * (TS_MAXS + 1)];
  __shared__ double Hn[TS_MAXA * TS_MAXS];
  __shared__ double Ss[TS_MAXS * TS_MAXS], Ts[TS_MAXS * TS_MAXS], RVs[TS_MAXS * TS_MAXS];
  __shared__ int fail;
  const int tid = threadIdx.x, ldg = sp + sw, w = s + 1;
  const double *G = K->LG;
  if (K->bad) return;
  if (tid == 0) fail = 0;
  if (sp) {
    for (int idx = tid; idx < a * TS_MAXS; idx += blockDim.x) {
      const int r = idx / TS_MAXS, c = idx % TS_MAXS;
      R1s[idx] = c < sp ? G[r * ldg + c] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < sp * sp; idx += blockDim.x) {
      const int r = idx / sp, c = idx % sp;
      double v = G[(a + r) * ldg + c];
      for (int q = 0; q < a; ++q) v -= R1s[q * TS_MAXS + r] * R1s[q * TS_MAXS + c];
      Ss[r * TS_MAXS + c] = v;
    }
    __syncthreads();
    if (tid == 0 && !chol_small(Ss, sp, Ts)) {
      K->bad = 1;
      fail = 1;
    }
    __syncthreads();
    if (fail) return;
    for (int idx = tid; idx < a * s; idx += blockDim.x)
      K->Lr1[idx] = R1s[(idx / s) * TS_MAXS + idx % s];
    for (int idx = tid; idx < s * s; idx += blockDim.x)
      K->Lt[idx] = Ts[(idx / s) * TS_MAXS + idx % s];
    // pending block: Rhat = [[rho, Pra + R1 Prb], [0, T Prb]]
    const int j0 = a - 1, nr = a + s;
    for (int idx = tid; idx < nr * w; idx += blockDim.x) {
      const int r = idx / w, c = idx % w;
      double v = 0.0;
      if (c == 0) {
        v = r < a ? K->Prho[r] : 0.0;
      } else if (r < a) {
        v = K->Pra[r * s + c - 1];
        for (int q = 0; q < s; ++q) v += R1s[r * TS_MAXS + q] * K->Prb[q * s + c - 1];
      } else {
        for (int q = 0; q < s; ++q) v += Ts[(r - a) * TS_MAXS + q] * K->Prb[q * s + c - 1];
      }
      Rhat[idx] = v;
    }
    __syncthreads();
    hessenberg_cols(K, j0, s, Rhat, K->H + j0, KRY_MMAX);
    __syncthreads();
    if (tid == 0)
      for (int c = j0; c < j0 + s; ++c) givens_column(K, c);
    __syncthreads();
  }
  if (!sw) return;
  const int a2 = a + sp, j = a2 - 1;
  for (int idx = tid; idx < a * TS_MAXS; idx += blockDim.x) {
    const int r = idx / TS_MAXS, c = idx % TS_MAXS;
    Cs[idx] = c < sw ? G[r * ldg + sp + c] : 0.0;
  }
  __syncthreads();
  if (sp) {
    // M = P^T W - R1^T C_old, then C_P = T^{-T} M (forward substitution)
    for (int idx = tid; idx < sp * sw; idx += blockDim.x) {
      const int r = idx / sw, c = idx % sw;
      double v = G[(a + r) * ldg + sp + c];
      for (int q = 0; q < a; ++q) v -= R1s[q * TS_MAXS + r] * Cs[q * TS_MAXS + c];
      Ss[r * TS_MAXS + c] = v;
    }
    __syncthreads();
    if (tid < sw) {
      const int c = tid;
      for (int r = 0; r < sp; ++r) {
        double v = Ss[r * TS_MAXS + c];
        for (int q = 0; q < r; ++q) v -= Ts[q * TS_MAXS + r] * Cs[(a + q) * TS_MAXS + c];
        Cs[(a + r) * TS_MAXS + c] = v / Ts[r * TS_MAXS + r];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < sw * sw; idx += blockDim.x) {
    const int r = idx / sw, c = idx % sw;
    double v = G[(a2 + r) * ldg + sp + c];
    for (int q = 0; q < a2; ++q) v -= Cs[q * TS_MAXS + r] * Cs[q * TS_MAXS + c];
    Ss[r * TS_MAXS + c] = v;
  }
  __syncthreads();
  if (tid == 0 && !chol_small(Ss, sw, RVs)) {
    K->bad = 2;
    fail = 1;
  }
  __syncthreads();
  if (fail) return;
  // the new pending block
  for (int idx = tid; idx < a2 * s; idx += blockDim.x)
    K->Pra[idx] = Cs[(idx / s) * TS_MAXS + idx % s];
  for (int idx = tid; idx < s * s; idx += blockDim.x)
    K->Prb[idx] = RVs[(idx / s) * TS_MAXS + idx % s];
  for (int r = tid; r < a2; r += blockDim.x) {
    double v;
    if (sp)
      v = r < a ? R1s[r * TS_MAXS + sp - 1] : Ts[(r - a) * TS_MAXS + sp - 1];
    else
      v = (r == a - 1) ? 1.0 : 0.0;
    K->Prho[r] = v;
  }
  const int nr = a2 + s;
  for (int idx = tid; idx < nr * w; idx += blockDim.x) {
    const int r = idx / w, c = idx % w;
    double v = 0.0;
    if (c == 0) {
      if (r < a2) v = sp ? (r < a ? R1s[r * TS_MAXS + sp - 1] : Ts[(r - a) * TS_MAXS + sp - 1])
                         : (r == a - 1 ? 1.0 : 0.0);
    } else {
      v = r < a2 ? Cs[r * TS_MAXS + c - 1] : RVs[(r - a2) * TS_MAXS + c - 1];
    }
    Rhat[idx] = v;
  }
  __syncthreads();
  hessenberg_cols(K, j, s, Rhat, Hn, TS_MAXS);
  __syncthreads();
  if (tid == 0) {
    // Givens rotations of the one-pass columns on a copy: estimates only
    double csl[TS_MAXS], snl[TS_MAXS];
    double gl = K->g[j];
    for (int c = 0; c < s; ++c) {
      const int col = j + c;
      for (int i = 0; i < col; ++i) {
        const double ci = i < j ? K->cs[i] : csl[i - j];
        const double si = i < j ? K->sn[i] : snl[i - j];
        const double hi = Hn[i * TS_MAXS + c], hn = Hn[(i + 1) * TS_MAXS + c];
        Hn[i * TS_MAXS + c] = ci * hi + si * hn;
        Hn[(i + 1) * TS_MAXS + c] = -si * hi + ci * hn;
      }
      const double x = Hn[col * TS_MAXS + c], y = Hn[(col + 1) * TS_MAXS + c];
      double cc = 1.0, ss = 0.0;
      if (y != 0.0) {
        const double r = hypot(x, y);
        cc = x / r;
        ss = y / r;
      }
      csl[c] = cc;
      snl[c] = ss;
      K->est_t[c] = fabs(ss * gl);
      gl = cc * gl;
    }
  }
}

int kry_lag_block(KrylovDev *K, int a, int sp, int sw, int s, hipStream_t st) {
  if (s > TS_MAXS || a + sp + sw > TS_MAXA || a + sp + s > TS_MAXA || a < 1) {
    set_error("single-reduce step: a = %d, s = %d out of range", a, s);
    return SPAND_EINVAL;
  }
  hipLaunchKernelGGL(k_lag_block, dim3(1), dim3(256), 0, st, K, a, sp, sw, s);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

// ---------------------------------------------------------------- least squares
__global__ void k_lsq(KrylovDev *K, int k) {
  if (threadIdx.x != 0) return;
  const int ld = KRY_MMAX;
  for (int i = k - 1; i >= 0; --i) {
    double v = K->g[i];
    for (int c = i + 1; c < k; ++c) v -= K->Rm[i * ld + c] * K->y[c];
    K->y[i] = v / K->Rm[i * ld + i];
  }
}

int kry_lsq(KrylovDev *K, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_lsq, dim3(1), dim3(64), 0, st, K, k);
  SP_HIP(hipGetLastError());
  return SPAND_OK;
}

}  // namespace spand
