// spaND factor object (host side) and its per-level apply plan.
#pragma once

#include <chrono>
#include <functional>
#include <map>
#include <memory>
#include <initializer_list>
#include <vector>

#include "internal.h"
#include "kernels_vec.h"

namespace spand {

struct Blk {
  void *p = nullptr;   // row-major rows x cols, ld = cols
  int rows = 0, cols = 0;
};

// trailing matrix of one level: clusters (with their slots in the global
// vector) and dense cluster-pair blocks
struct LevelState {
  std::vector<int> size;
  std::vector<char> interior;
  std::vector<std::vector<int32_t>> slots;
  std::vector<int32_t *> d_slots;
  std::map<std::pair<int, int>, Blk> blocks;
};

struct Factor;
struct PullSet {
  PullGroup *d_groups = nullptr;
  PullItem *d_items = nullptr;
  PullChunk *d_chunks = nullptr;
  int n = 0;          // groups
  int nchunks = 0;
  int trans = 0;      // every item of a set has the same orientation
  int set(Factor &F, std::vector<PullGroup> G, const std::vector<PullItem> &I);
};

// batched GEMVs of one sweep step, split into bands of output rows; for
// in-place use the union of output slots is copied back from scratch
struct GemvSet {
  GemvDesc *d_items = nullptr;
  GemvChunk *d_chunks = nullptr;
  int nchunks = 0;
  int n = 0;
  int32_t *d_slots = nullptr;
  int64_t nslots = 0;
  int set(Factor &F, std::vector<GemvDesc> items, const std::vector<const std::vector<int32_t> *> &oslots,
          int trans, int rows = 0);
};

inline int ld4(int n) { return (n + 3) & ~3; }

// apply plan of one level (see Factor::apply)
struct ApplyLevel {
  GemvSet inv, invT;            // interiors: A_ss^-1
  GemvSet F, B, FT, BT;         // interfaces
  PullSet fw;    // x_n -= A_ns t_s          (groups: neighbours)
  PullSet bw;    // x_s -= A_sn x_n          (groups: interiors)
  PullSet tfw;   // x_n -= A_sn^T x_s        (groups: neighbours)
  PullSet tbw;   // t_s  = A_ns^T x_n        (groups: all interiors)
};

struct RankStat {
  int n = 0, kmin = 1 << 30, kmax = 0;
  int64_t ksum = 0, msum = 0;
  void add(int m, int k) {
    ++n;
    kmin = std::min(kmin, k);
    kmax = std::max(kmax, k);
    ksum += k;
    msum += m;
  }
};

enum { PH_GATHER = 0, PH_LU, PH_SCHUR, PH_SCALE, PH_RRQR, PH_COMPRESS, PH_END, PH_COUNT };

// One system of a batched factorization.  The systems of a batch that share
// the block size, the factor precision, eps and the flags are factored as
// one block-diagonal matrix: their elements are numbered one system after
// the other, the nested dissection is the union of the systems' own
// (clusters of one level side by side), and every phase runs one set of
// launches for all of them.  No cluster couples two systems, so every
// system's blocks, ranks and stored operators are those of its own
// factorization.  A system keeps its own sweep plan (the descriptors of its
// clusters only) and graphs, so its apply reads only its own operators.
struct Member {
  int K = 0, L = 0;
  int64_t elem_off = 0, nnz_off = 0, dof_off = 0, N = 0;
  const double *d_val = nullptr;
  std::vector<ApplyLevel> lv;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<RankStat> ranks;
  int top_size = 0;
  double apply_bytes = 0.0, flops = 0.0;
};

// input of a batched factorization: one system
struct BatchSystem {
  spand_bsr_t A;
  spand_grid_t grid;
  int L;
};

// chunked bump allocator over the device block cache
struct Bump {
  std::vector<std::pair<char *, size_t>> chunks;
  size_t used = 0;
  size_t bytes = 0;
  int alloc(void **p, size_t n, size_t chunk);
  void release();
  void absorb(Bump &o);      // take over o's chunks (o becomes empty)
};

struct Factor {
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;      // second stream of the build (forked from and joined to stream)
  hipStream_t side2 = nullptr;     // third one (size classes of a fused elimination block)
  hipEvent_t cls_fork = nullptr, cls_join = nullptr;
  // no second and third stream: set when several builds share the device at
  // once (their extra streams would share the few hardware queues with the
  // other builds' work)
  bool one_stream = false;
  int device = 0;
  FType ft = FType::F64;
  int bs = 0, K = 0, L = 0;
  int64_t N = 0;
  double eps = 0.0;
  std::vector<int32_t> h_rowptr, h_colind;
  // symbolic phase, reused by refactorizations of the same pattern: the
  // validated block pattern above, the nested dissection, grid and options
  std::shared_ptr<const NDResult> nd_sym;
  spand_grid_t grid{};
  spand_opts_t opts{};
  std::vector<ApplyLevel> lv;   // sweeps of all unknowns (every system of a batch)
  // batched factorization: its systems, and the system of every element
  // (empty for a factorization of one system)
  std::vector<Member> members;
  std::vector<int32_t> esys;
  const double *d_val = nullptr;          // values of a one-system factorization
  const double *blk_src(int e, int64_t t) const;   // block t of the input (row element e)
  int csys(int l, int c) const;           // system of cluster c of level l
  void acct(int sys, double bytes, double fl);      // apply bytes and flops of a system
  Bump keep, temp, next_temp;   // next_temp: next level's trailing blocks
  Bump retired;                 // scratch of finished levels, released at the next sync
  size_t keep_bytes = 0;
  int32_t *d_iota = nullptr;
  double *d_tbuf = nullptr;
  int *d_flag = nullptr;
  // statistics
  std::vector<RankStat> ranks;
  int top_size = 0;
  double apply_bytes = 0.0, flops = 0.0, t_host_ms = 0.0;
  double ph_ms[PH_COUNT] = {0};
  double ph_host_ms[PH_COUNT] = {0};   // host time (planning + launches) per phase
  int host_phase = -1;
  std::chrono::steady_clock::time_point trace_t = std::chrono::steady_clock::now();
  void trace(const char *what, int l);
  std::chrono::steady_clock::time_point host_t;
  std::chrono::steady_clock::time_point build_t0;
  double build_drv0 = 0.0;
  bool timing = false;
  std::vector<std::pair<int, hipEvent_t>> events;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> qrcp_events;
  double qrcp_ms = 0.0, qrcp_bytes = 0.0, qrcp_flops = 0.0;
  double alloc_ms = 0.0;
  int n_qrcp = 0;
  // matrix-core products: events around each launch (kind 0 GEMM, 1 the
  // level-0 Schur kernel) with the launch's algorithmic flops and bytes
  struct KTime {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<KTime> kevents;
  double kt_ms[2] = {0, 0}, kt_flops[2] = {0, 0}, kt_bytes[2] = {0, 0};
  int kt_n[2] = {0, 0};
  int timed_launch(int kind, double flops, double bytes, const std::function<int()> &launch);

  int gemv_rows = 64;              // band height of the sweep GEMVs (autotuned)
  bool use_graphs = true;          // replay the sweeps from captured hipGraphs
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  double *d_xg = nullptr;          // the graphs' fixed input/output vector
  ~Factor();
  int sweeps(const std::vector<ApplyLevel> &plan, double *x, int transpose, hipStream_t st);
  int capture(int member, int transpose);
  int capture_graphs(int which = 3, int member = -1);
  // the sweep sets of every system from the sets of all unknowns (gs: the
  // system of each group or item)
  int member_pull(int l, PullSet ApplyLevel::*which, const std::vector<PullGroup> &G,
                  const std::vector<PullItem> &I, const std::vector<int> &gs);
  int member_gemv(int l, GemvSet ApplyLevel::*which, const std::vector<GemvDesc> &gv,
                  const std::vector<const std::vector<int32_t> *> &os, const std::vector<int> &gs,
                  int trans);
  int dalloc(void **p, size_t bytes, bool keep);
  int dalloc_next(void **p, size_t bytes);
  void free_temp();
  void release_retired();
  template <typename D>
  int upload(const std::vector<D> &v, D **out, bool keep);
  // several host arrays in one device allocation and one copy (each part
  // 256-byte aligned; an empty part gets nullptr)
  struct UpPart {
    const void *src;
    size_t bytes;
    void **dst;
  };
  template <typename D>
  static UpPart part(const std::vector<D> &v, D **out) {
    return UpPart{v.data(), v.size() * sizeof(D), (void **)out};
  }
  int upload_parts(std::initializer_list<UpPart> parts, bool keep);
  int upload_slots(const std::vector<int32_t> &v, int32_t **out);
  int upload_level_slots(LevelState &S);
  // Host work that only the apply needs (sweep descriptor sets): queued
  // while the device is busy and run while the host would otherwise wait
  // (before a rank read-back, and at the end of the build).
  std::vector<std::function<int()>> deferred;
  void defer(std::function<int()> f) { deferred.push_back(std::move(f)); }
  int flush_deferred();
  int gemm_batch(const std::vector<GemmDesc> &items);
  int copy_batch(const std::vector<CopyDesc> &items, int src_is_factor);
  int complete_q(int l, const LevelState &S, const std::vector<int> &ifs,
                 const std::vector<int32_t> &kg, const std::vector<void *> &Qm,
                 const std::vector<void *> &Vm);
  int elim_batch(std::vector<ElimDesc> &items, int mode);
  void mark(int phase);
  void collect_events();
  int level0(const NDResult &nd, LevelState &S);
  int eliminate_dense(int l, LevelState &S);
  int sparsify(int l, const NDResult &nd, LevelState &S, LevelState &Nx);
  int build(const spand_bsr_t &A, const spand_grid_t &g, const spand_opts_t &o,
            const Factor *sym = nullptr);
  int build_batch(const std::vector<BatchSystem> &sys, const spand_opts_t &o);
  int numeric();                // buffers, level 0, the levels, the final checks
  // member < 0: all unknowns; otherwise the vectors are those of one system
  int apply(const double *in, double *out, int transpose, hipStream_t st, int member = -1);
  // every system of a batch at once (in[m], out[m]: system m's vectors), one
  // replay of the sweeps of all unknowns
  int apply_batch(const std::vector<const double *> &in, const std::vector<double *> &out,
                  int transpose, hipStream_t st);
  void fill_stats(spand_factor_stats_t *st, int member = -1) const;
};

struct DiagDesc {
  const void *U;
  void *S;
  void *Si;
  int32_t n, ld;
};
int launch_diag_split(FType t, const DiagDesc *d_items, int n, hipStream_t st);

int autotune_spmv(const spand_bsr_t &A, double *x, double *y, hipStream_t st);
int tuned_gemv_rows(FType t, int bs);
int autotune_gemv(FType t, int bs, const std::function<int(int, GemvSet &)> &build, double *in,
                  double *out, hipStream_t st, int *rows_out);

}  // namespace spand
