// Internal declarations of libspand: host data structures shared by the
// planning / orchestration code and the launch wrappers of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <array>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/spand.h"

namespace spand {

// ----------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
const char *last_error();

struct Status {
  int code = SPAND_OK;
  bool ok() const { return code == SPAND_OK; }
};

#define SP_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::spand::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,         \
                         hipGetErrorString(e_));                            \
      return SPAND_EHIP;                                                    \
    }                                                                       \
  } while (0)

#define SP_TRY(expr)                                                        \
  do {                                                                      \
    int r_ = (expr);                                                        \
    if (r_ < 0) return r_;                                                  \
  } while (0)

// ----------------------------------------------------------------- device memory
// Cached device blocks (pool.hip).  pool_alloc rounds the size up and
// reports the block's real size in *got; pool_release takes that size back.
// Release a block only after the work that used it has completed.
int pool_alloc(void **p, size_t bytes, size_t *got);
void pool_release(void *p, size_t bytes);
void pool_trim();
size_t pool_cached_bytes();
double pool_driver_ms();   // calling thread's cumulative hipMalloc/hipFree time
// Timing events of the current device, cached (pool.hip); put an event back
// only after its last record has completed and been read.
int event_get(hipEvent_t *e);
void event_put(hipEvent_t e);

// ----------------------------------------------------------------- ND
struct NDCluster {
  int32_t node, box;
  bool interior;
  std::vector<int32_t> elems;   // ascending
};

struct NDResult {
  int nx = 0, ny = 0, L = 0;
  std::vector<int32_t> node_of_elem;
  std::map<int64_t, int> node_level;               // node id -> level
  std::vector<std::vector<NDCluster>> levels;      // per level
  std::vector<std::vector<std::vector<int>>> children;  // [l][cluster] -> ids at l-1
  std::vector<int32_t> perm;
};

int default_levels(int64_t K);
NDResult nested_dissection(int nx, int ny, bool px, bool py, int L);
NDResult nd_union(const std::vector<NDResult> &parts, const std::vector<int64_t> &elem_off);

// ----------------------------------------------------------------- device memory
// Simple owning device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Element type tag for the factor (float or double storage/compute).
enum class FType { F64 = 0, F32 = 1 };
inline size_t fsize(FType t) { return t == FType::F64 ? 8 : 4; }

// ----------------------------------------------------------------- kernel descriptors
// All descriptors hold byte offsets / element pointers into device memory;
// they are built and bounds-checked on the host, then uploaded.

// C = alpha * op(A) op(B) + beta * C  (row-major, per item sizes)
// tri: structural zeros of the operands as used in the product, which the
// kernels skip (exactly: the skipped terms are products with zeros)
//   GEMM_TRI_B_UPPER  op(B)(k, j) = 0 for k > j
//   GEMM_TRI_A_UPPER  op(A)(i, k) = 0 for k < i
constexpr int GEMM_TRI_B_UPPER = 1, GEMM_TRI_A_UPPER = 2;
struct GemmDesc {
  const void *A;
  const void *B;
  void *C;
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t transA, transB;
  double alpha, beta;
  int32_t tri, pad;
};

// Copy of a rows x cols sub-matrix, optional transpose, from src (type Ts)
// to dst (type Td): dst[r*ldd + c] = scale * src(r, c) (or src(c, r)).
struct CopyDesc {
  const void *src;
  void *dst;
  int32_t rows, cols;
  int32_t lds, ldd;
  int32_t trans;
  int32_t pad;
  double scale;
};

// One b x b block of the BSR value array copied to dst (leading dimension
// ldd, factor precision).
struct GatherItem {
  void *dst;
  const double *src;   // b x b block of the input values
  int32_t ldd;
  int32_t pad;
};

// Panel factorisation problem (GJE / LU on an augmented row-major matrix).
struct ElimDesc {
  void *A;          // n x ld row-major (ld >= ncols)
  void *P;          // workspace n x nb  (panel copy)
  void *T;          // workspace nb x ld (pivot rows copy)
  int32_t *piv;     // [n] pivot row per column (virtual pivoting)
  int32_t *used;    // [n] row-used flags
  int32_t n;        // order of the square part
  int32_t ncols;    // total columns (n or 2n)
  int32_t ld;
  int32_t pad;
  void *TB;         // workspace bw x ld (blocked elimination: pivot rows of a block)
  void *PB;         // workspace n x bw (blocked LU: multipliers of a block)
  void *sg;         // [n] factor precision: diagonal shifts of mode 3
};

// Dense GEMV with gather/scatter through slot lists:
// out[oslot[r]] = beta*out[oslot[r]] + alpha * sum_c op(A)(r,c) * in[islot[c]]
struct GemvDesc {
  const void *A;
  const int32_t *islot;
  const int32_t *oslot;
  int32_t rows, cols;      // of op(A)
  int32_t lda;             // of A as stored (a multiple of 4)
  int32_t trans;
};
// a band of output rows of one GEMV item (one workgroup)
struct GemvChunk {
  int32_t item, row0, nrows, pad;
};

// Pull group: out[oslot[r]] += alpha * sum_items op(B_i) in[islot_i[c]].
struct PullItem {
  const void *B;
  const int32_t *islot;
  int32_t rows, cols;      // of op(B)
  int32_t ldb;
  int32_t trans;
};
struct PullGroup {
  const int32_t *oslot;
  int32_t rows;
  int32_t item_begin, item_end;
  int32_t pad;              // bit 0: every block allows 16-byte row loads (set by the host)
};
struct PullChunk {          // up to PULL_ROWS output rows of one group
  int32_t group, row0, nrows, pad;
};

// Level-0 element Schur update: target -= A1 * Y * A2 (b x b blocks)
struct SchurItem {
  const void *A1;      // b x b copy of A[sep elem, leaf elem] (factor precision, ld b)
  const void *Y;       // pointer to the b x b block inside Ainv (ld = ldy)
  const void *A2;      // b x b copy of A[leaf elem, sep elem]
  int32_t ldy;
  int32_t pad;
};
struct SchurGroup {
  void *target;        // b x b sub-block inside a dense interface block
  int32_t ldt;
  int32_t item_begin, item_end;
  int32_t pad;
};

// QRCP problem (rank-revealing QR of a row-major m x ncols matrix W)
struct QrcpDesc {
  const void *W;       // m x ncols row-major (padding columns up to ldw are zero)
  void *W2;            // m x ldw workspace: W with its live column groups packed left
  void *Q;             // m x m row-major output
  void *V;             // m x m workspace: kept vectors q_t = V[t*m ..], then completion terms
  double *tau;         // [m] completion signs
  double *vn1;         // [ldw]
  double *vn2;         // [ldw]
  int32_t *sel;        // [ldw] selected (or padding) flags
  double *H;           // [ldw x block width] candidate-basis coordinates of the columns
  int32_t *k_out;      // rank
  int32_t *k_gs;       // kept Gram-Schmidt vectors (V rows 0..k_gs-1)
  int32_t m, ncols;
  int32_t ldw;         // leading dimension of W (multiple of 4, padding zero)
  int32_t pad;         // LDS stride (largest m of the launch), set by the host
};

// ----------------------------------------------------------------- launches
// Implemented in the .hip files.  Descriptor arrays are device pointers.
// Every wrapper returns SPAND_OK or SPAND_EHIP (launch error).
constexpr int ELIM_NB = 16;        // panel width of the elimination kernels
constexpr int ELIM_BLK = 64;       // block width of the blocked eliminations (4 panels)
constexpr int ELIM_NT = 512;       // threads of a panel workgroup
constexpr int ELIM_RPT = 4;        // rows held per thread -> n <= 2048
constexpr int ELIM_MAXN = ELIM_NT * ELIM_RPT;
constexpr int QRCP_MAXM = 1024;    // largest interface handled by the QRCP kernel

// tmode = 2 * transA + transB, shared by every descriptor of the launch
// (the FP64 kernel reads the flags per descriptor and ignores it)
// uniform > 0: every descriptor of the launch has that many tiles (the item
// of a tile is found by division instead of a search of tile_start)
// d_coarse (may be null): for c = 0 .. ceil(total_tiles / 64), the item (of
// this launch) holding tile tile_base + 64 c, the last entry nitems - 1; it
// narrows each workgroup's search of d_tile_start to a few items.
int launch_gemm(FType t, const GemmDesc *d_items, const int32_t *d_tile_start, int nitems,
                int total_tiles, hipStream_t st, int tile_base, int tmode, int uniform = 0,
                const int32_t *d_coarse = nullptr);
// FP32 C += A B with K <= 64 (alpha = 1, no transposes): work units are
// strips of up to `tps` 64x64 tiles along N (d_unit_start / total_units count
// strips); the same results as launch_gemm, bit for bit
int launch_gemm_strip(const GemmDesc *d_items, const int32_t *d_unit_start, int nitems,
                      int total_units, hipStream_t st, int unit_base, int uniform,
                      const int32_t *d_coarse, int tps);
// host: the coarse index of items [a, b) of a tile_start array (ts[a..b])
void gemm_coarse(const std::vector<int32_t> &ts, size_t a, size_t b, std::vector<int32_t> &out);
// b x b blocks of BSR values (FP64) into factor-precision matrices
int launch_bsr_gather(FType t, const GatherItem *d_items, int n, int b, hipStream_t st);
// src double -> dst factor type (src_is_factor = 0) or factor -> factor (1)
int launch_copy(FType t, int src_is_factor, const CopyDesc *d_items, int n, int64_t max_elems,
                hipStream_t st);
// transposed copies (trans = 1), 32 x 32 tiles through LDS
int launch_copy_t(FType t, int src_is_factor, const CopyDesc *d_items, int n, int max_rows,
                  int max_cols, hipStream_t st);
// mode 0: Gauss-Jordan, partial pivoting; 1: LU (augmented), partial
// pivoting; 2: Gauss-Jordan without pivoting; 3: as 2 on A - S with the
// signs S chosen on the way (fused block path only, signs to ElimDesc::sg).  Items sorted by n descending,
// the first nactive have n > k.
int launch_elim_step(FType t, const ElimDesc *d_items, int nactive, int k, int mode,
                     int max_tiles, int *d_flag, int cw0, int cw1, hipStream_t st);
// block [k0, k0 + bw) (bw = ELIM_BLK on the panel path)
int launch_elim_extract(FType t, const ElimDesc *d_items, int nactive, int k0, int bw, int lu,
                        hipStream_t st);
int launch_elim_pb(FType t, const ElimDesc *d_items, int nactive, int k, int k0, hipStream_t st);
// Whole block [k0, k0 + bw) in one launch, one row per thread: needs
// nmax <= elim_block_max_n(t) and bw = elim_block_width(t, nmax) (32 for
// FP64 matrices of more than 512 rows, else ELIM_BLK).  Writes the block
// columns, piv, used, and for LU (mode 1) the multipliers PB (n x bw); the
// pivot rows' other columns are moved by launch_elim_extract as for the
// panel path.
int elim_block_max_n(FType t);
int elim_block_width(FType t, int n);
int launch_elim_block(FType t, const ElimDesc *d_items, int nactive, int k0, int mode, int nmax,
                      int bw, int *d_flag, hipStream_t st);
// out[j, c] = src[piv[j], colperm ? pinv[c] : c + col_off]
struct RowGatherDesc {
  const void *src;
  void *dst;
  const int32_t *piv;
  int32_t n, cols, lds, ldd, col_off, colperm;
};
int launch_row_gather(FType t, const RowGatherDesc *d_items, int n, int max_rows, hipStream_t st);
int launch_schur_elem(FType t, int bs, const SchurGroup *d_groups, int ngroups,
                      const SchurItem *d_items, hipStream_t st);
// dynamic LDS of one QRCP workgroup with candidate blocks of width bq
size_t qrcp_lds_bytes(int maxm, int maxgrp, int bq);
constexpr size_t QRCP_MAX_LDS = 64 * 1024;
// widest candidate block (8, 4 or 2) whose LDS fits, 0 if none does
int qrcp_block_width(int maxm, int maxgrp);
// every item's H holds ldw x bq doubles.  complete = 0: Q is left to the
// caller (V rows 0..k_gs-1 hold the kept vectors, nothing else is written)
int launch_qrcp(FType t, const QrcpDesc *d_items, int n, double eps, int force_full, int maxm,
                int maxgrp, int bq, int complete, hipStream_t st);
// dst rows/cols scaling: dst[r, c] *= rs[r] * cs[c] (either may be null)
struct ScaleDesc {
  void *A;
  const void *rs;
  const void *cs;
  int32_t rows, cols, ld, pad;
};
int launch_scale(FType t, const ScaleDesc *d_items, int n, hipStream_t st);
// A = I (rows x rows sub-block with leading dimension ld)
struct EyeDesc {
  void *A;
  int32_t n, ld;
};
int launch_eye(FType t, const EyeDesc *d_items, int n, int max_n, hipStream_t st);
// A = 0 (rows x cols sub-block with leading dimension ld)
struct ZeroDesc {
  void *A;
  int32_t rows, cols, ld, pad;
};
int launch_zero(FType t, const ZeroDesc *d_items, int n, int64_t max_elems, hipStream_t st);
int launch_gemv(FType t, const GemvDesc *d_items, const GemvChunk *d_chunks, int nchunks,
                const double *in, double *out, double alpha, double beta, hipStream_t st);
int launch_slot_copy(const int32_t *slots, int64_t n, const double *src, double *dst,
                     hipStream_t st);

int launch_spmv(const spand_bsr_t &A, int transpose, double alpha, const double *x,
                double beta, double *y, const double *z, double gz, const double *w,
                double gw, hipStream_t st);

// s-step GMRES (gmres.hip).  ws == nullptr: device workspace from the block
// cache; otherwise carved from [ws->base, ws->base + ws->bytes) (no device
// allocation, no autotuning, no phase timers).
struct SolveWorkspace {
  void *base;
  size_t bytes;
};
struct Factor;
size_t sstep_workspace_bytes(int64_t N, const sstep_opts_t &o);
// M: the preconditioner (nullptr: none); member >= 0 selects one system of
// a batched factorization
int sstep_solve(const spand_bsr_t &A, Factor *M, int member, const double *b, double *x,
                const sstep_opts_t &o, sstep_stats_t *st, hipStream_t stream,
                const SolveWorkspace *ws = nullptr);

// ----------------------------------------------------------------- helpers
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace spand
