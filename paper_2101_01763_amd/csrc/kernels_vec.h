// Launch wrappers of the memory-bound and Krylov kernels.
#pragma once
#include "internal.h"

namespace spand {

constexpr int GEMV_MAXC = 2048;   // largest cluster handled by the sweep kernels
constexpr int PULL_MAXR = 2048;
constexpr int TS_CHUNK = 512;     // rows per partial Gram block
constexpr int TS_MAXS = 8;        // largest s
constexpr int TS_MAXA = 160;      // largest restart + s + 1

constexpr int PULL_ROWS = 64;     // output rows per pull workgroup
int launch_pull2(FType t, const PullGroup *d_groups, const PullItem *d_items,
                 const PullChunk *d_chunks, int nchunks, int trans, const double *in,
                 double *out, double alpha, double beta, hipStream_t st);
int launch_spmv_g(const spand_bsr_t &A, int G, double alpha, const double *x, double beta,
                  double *y, const double *z, double gz, const double *w, double gw,
                  hipStream_t st);
void set_spmv_lanes(int bs, int G);
int get_spmv_lanes(int bs);
int launch_spmv_t_check(const spand_bsr_t &A, int *d_flag, hipStream_t st);   // *d_flag = 1: no mirror block
int launch_pattern_outer(const spand_bsr_t &P, const double *u, const double *v, double alpha,
                         double *out, hipStream_t st);
int vec_fill(double *x, int64_t n, double v, hipStream_t st);
int vec_iota(int32_t *x, int64_t n, hipStream_t st);
int vec_axpby(int64_t n, const double *x, double *y, double ca, const double *pa, int inva,
              double cb, hipStream_t st);
int launch_gram(int64_t N, const double *X, int64_t ldx, int a, const double *W, int64_t ldw,
                int s, double *part, double *out, int ldo, hipStream_t st);
int launch_ts_update(int64_t N, const double *X, int64_t ldx, int a, const double *R, int ldr,
                     double *W, int64_t ldw, int s, hipStream_t st);
int launch_ts_trsm(int64_t N, double *W, int64_t ldw, int s, const double *T, const int *bad,
                   hipStream_t st);
int launch_ts_gemv(int64_t N, const double *X, int64_t ldx, int k, const double *c, double *y,
                   hipStream_t st);
// Gram matrix with up to 2 * TS_MAXS columns (single-reduce step)
int launch_gram_wide(int64_t N, const double *X, int64_t ldx, int a, const double *W,
                     int64_t ldw, int s, double *part, double *out, int ldo, hipStream_t st);
int64_t gram_wide_part_elems(int64_t N, int a, int s);   // size of its partial buffer

// ---- small dense state of the s-step method (device, one workgroup)
constexpr int KRY_MMAX = 128;     // largest restart length
struct KrylovDev {
  double H[(KRY_MMAX + 1) * KRY_MMAX];   // row-major (m+1) x m, ld = KRY_MMAX
  double Rm[(KRY_MMAX + 1) * KRY_MMAX];  // Givens-rotated H (same layout)
  double cs[KRY_MMAX], sn[KRY_MMAX], g[KRY_MMAX + 1];
  double y[KRY_MMAX];
  double est[KRY_MMAX];                  // |g_{c+1}| after column c
  double R1[TS_MAXA * TS_MAXS], R2[TS_MAXA * TS_MAXS];
  double G[TS_MAXS * TS_MAXS], T1[TS_MAXS * TS_MAXS], T2[TS_MAXS * TS_MAXS];
  double Bb[(TS_MAXS + 1) * TS_MAXS];
  double scal[8];                        // [0] beta / norms
  int bad;                               // CholQR breakdown flag (lagged: 1 = P, 2 = W)
  int pad;
  // single-reduce schedule (second pass lagged by one block)
  double LG[TS_MAXA * 2 * TS_MAXS];      // Q[:, 0:a+sp+sw]^T Q[:, a:a+sp+sw], ld sp+sw
  double Lr1[TS_MAXA * TS_MAXS];         // R1 = Q_old^T P (a x s, ld s)
  double Lt[TS_MAXS * TS_MAXS];          // T = chol(P^T P - R1^T R1)
  double Pra[TS_MAXA * TS_MAXS];         // pending block: W = Q[:, 0:a2] Pra + What Prb
  double Prb[TS_MAXS * TS_MAXS];
  double Prho[TS_MAXA];                  // its starting vector on Q[:, 0:a2]
  double est_t[TS_MAXS];                 // residual estimates from its first pass
};

int kry_init_cycle(KrylovDev *K, int m, hipStream_t st);                  // g = beta e0 (beta in scal[0])
int kry_chol(KrylovDev *K, int s, double *G, double *T, hipStream_t st);  // T = chol(G)
int kry_block_finish(KrylovDev *K, int j, int s, int passes, hipStream_t st);         // R, Hessenberg, Givens
int kry_givens_col(KrylovDev *K, int j, hipStream_t st);                  // column j (MGS steps)
int kry_lsq(KrylovDev *K, int k, hipStream_t st);                         // y from Rm, g
int kry_lag_block(KrylovDev *K, int a, int sp, int sw, int s, hipStream_t st);  // from K->LG
int launch_ts_lag_update(int64_t N, double *Q, int64_t ldq, int a, int sp, int sw, int s,
                         const KrylovDev *K, hipStream_t st);
int launch_dot(int64_t N, const double *x, const double *y, double *part, double *out,
               int take_sqrt, hipStream_t st);

}  // namespace spand
