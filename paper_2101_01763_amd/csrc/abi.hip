// C ABI of libspand (declared in include/spand.h): argument validation,
// handle lifetime, error reporting.  All numerical work is in the kernels.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <atomic>
#include <cstdlib>
#include <thread>
#include <unordered_map>
#include <vector>

#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "factor.h"

// A handle owns a factorization, or shares one with the other systems of a
// batch (member = its index there; -1: the factorization is its own).
struct spand_factor_s {
  std::shared_ptr<spand::Factor> F;
  int member = -1;
  int64_t N() const { return member < 0 ? F->N : F->members[size_t(member)].N; }
};

namespace spand {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char *last_error() { return g_err; }

static int check_bsr(const spand_bsr_t *A) {
  if (!A) {
    set_error("A is NULL");
    return SPAND_EINVAL;
  }
  if (A->n_brows <= 0 || A->bs <= 0 || A->nnzb < A->n_brows) {
    set_error("bad BSR sizes (n_brows=%d bs=%d nnzb=%lld)", A->n_brows, A->bs,
              (long long)A->nnzb);
    return SPAND_EINVAL;
  }
  if (A->bs > 64) {
    set_error("block size %d exceeds 64", A->bs);
    return SPAND_EINVAL;
  }
  if (A->bs % 2 != 0) {
    set_error("block size %d must be even (4 (p+1)^2)", A->bs);
    return SPAND_EINVAL;
  }
  if (!A->d_rowptr || !A->d_colind || !A->d_val) {
    set_error("BSR device pointers must not be NULL");
    return SPAND_EINVAL;
  }
  return SPAND_OK;
}

}  // namespace spand

using namespace spand;

extern "C" {

const char *spand_status_string(int s) {
  switch (s) {
    case SPAND_OK: return "SPAND_OK";
    case SPAND_EINVAL: return "SPAND_EINVAL";
    case SPAND_ENOMEM: return "SPAND_ENOMEM";
    case SPAND_ESINGULAR: return "SPAND_ESINGULAR";
    case SPAND_EHIP: return "SPAND_EHIP";
    case SPAND_ENOTCONV: return "SPAND_ENOTCONV";
    case SPAND_EBREAKDOWN: return "SPAND_EBREAKDOWN";
    default: return "SPAND_UNKNOWN";
  }
}

const char *spand_last_error(void) { return last_error(); }

}  // extern "C"

// Validate, build, and (when `graphs`) capture the sweep graphs.  Batched
// callers build on worker threads with graphs=false and capture afterwards,
// once the workers have joined.
// Builds a factorization on a private stream ordered after `stream`; with
// `sym` the ordering and the validated block pattern (the symbolic phase)
// are taken from that earlier factorization of the same pattern.
static int build_factor(const spand_bsr_t *A, const spand_grid_t *grid, const spand_opts_t *opts,
                        void *stream, const Factor *sym, bool graphs, std::unique_ptr<Factor> &out,
                        bool one_stream = false);

// Arguments of one factorization; *L_out receives the number of levels.
static int check_factor_args(const spand_bsr_t *A, const spand_grid_t *grid,
                             const spand_opts_t *opts, int *L_out) {
  SP_TRY(check_bsr(A));
  if (!grid || !opts) {
    set_error("grid/opts is NULL");
    return SPAND_EINVAL;
  }
  if (grid->nx <= 0 || grid->ny <= 0 || int64_t(grid->nx) * grid->ny != A->n_brows) {
    set_error("grid %dx%d does not match n_brows=%d", grid->nx, grid->ny, A->n_brows);
    return SPAND_EINVAL;
  }
  if (!(opts->eps >= 0.0) || !std::isfinite(opts->eps)) {
    set_error("eps must be a finite number >= 0");
    return SPAND_EINVAL;
  }
  if (opts->nlevels < 0 || opts->nlevels > SPAND_MAX_LEVELS) {
    set_error("nlevels must be in [0, %d]", SPAND_MAX_LEVELS);
    return SPAND_EINVAL;
  }
  if (opts->factor_dtype != SPAND_F64 && opts->factor_dtype != SPAND_F32) {
    set_error("factor_dtype must be SPAND_F64 or SPAND_F32");
    return SPAND_EINVAL;
  }
  int L = opts->nlevels > 0 ? opts->nlevels : default_levels(A->n_brows);
  // every box at depth L-1 must be able to exist: need 2^(L-1) <= K
  if (L > 1 && (int64_t(1) << (L - 1)) > int64_t(A->n_brows)) {
    set_error("nlevels=%d too large for %d elements", L, A->n_brows);
    return SPAND_EINVAL;
  }
  if (L_out) *L_out = L;
  return SPAND_OK;
}

static int factor_one(const spand_bsr_t *A, const spand_grid_t *grid, const spand_opts_t *opts,
                      void *stream, spand_factor_t *out, bool graphs) {
  if (!out) {
    set_error("out is NULL");
    return SPAND_EINVAL;
  }
  *out = nullptr;
  SP_TRY(check_factor_args(A, grid, opts, nullptr));
  auto h = std::make_unique<spand_factor_s>();
  std::unique_ptr<Factor> f;
  SP_TRY(build_factor(A, grid, opts, stream, nullptr, graphs, f));
  h->F = std::move(f);
  *out = h.release();
  return SPAND_OK;
}

// Runs `body` on a new Factor with a private stream ordered after `stream`.
static int run_build(void *stream, const std::function<int(Factor &)> &body,
                     std::unique_ptr<Factor> &out, bool one_stream = false);

static int build_factor(const spand_bsr_t *A, const spand_grid_t *grid, const spand_opts_t *opts,
                        void *stream, const Factor *sym, bool graphs, std::unique_ptr<Factor> &out,
                        bool one_stream) {
  std::unique_ptr<Factor> f;
  SP_TRY(run_build(stream, [&](Factor &F) { return F.build(*A, *grid, *opts, sym); }, f,
                   one_stream));
  if (graphs) SP_TRY(f->capture_graphs(1));
  f->trace("graph capture", -1);
  out = std::move(f);
  return SPAND_OK;
}

static int run_build(void *stream, const std::function<int(Factor &)> &body,
                     std::unique_ptr<Factor> &out, bool one_stream) {
  auto F = std::make_unique<Factor>();
  F->one_stream = one_stream;
  // The build runs on a private non-blocking stream ordered after the
  // caller's: its descriptor uploads (synchronous copies on the null
  // stream) then never wait for the factorization's own kernels, so the
  // host plans the next kernels while the device runs the queued ones.
  hipStream_t ps = nullptr;
  hipEvent_t ready = nullptr;
  SP_HIP(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ready, (hipStream_t)stream) != hipSuccess ||
      hipStreamWaitEvent(ps, ready, 0) != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    (void)hipStreamDestroy(ps);
    set_error("could not order the factorization after the caller's stream");
    return SPAND_EHIP;
  }
  F->stream = ps;
  F->timing = true;
  (void)hipGetDevice(&F->device);
  int r;
  try {
    r = body(*F);
  } catch (const std::exception &ex) {
    set_error("factorization failed: %s", ex.what());
    r = SPAND_EINVAL;
  }
  (void)hipStreamSynchronize(ps);
  (void)hipEventDestroy(ready);
  (void)hipStreamDestroy(ps);
  F->stream = nullptr;
  if (r != SPAND_OK) return r;
  F->trace("build end", -1);
  out = std::move(F);
  return SPAND_OK;
}

extern "C" {

int spand_factor(const spand_bsr_t *A, const spand_grid_t *grid, const spand_opts_t *opts,
                 void *stream, spand_factor_t *out) {
  set_error("");
  return factor_one(A, grid, opts, stream, out, true);
}

int spand_refactor(spand_factor_t F, const spand_bsr_t *A, void *stream) {
  set_error("");
  if (!F || !F->F) {
    set_error("F is NULL");
    return SPAND_EINVAL;
  }
  if (F->member >= 0) {
    set_error("a handle that shares a batched factorization cannot be refactored; factor the "
              "system with spand_factor");
    return SPAND_EINVAL;
  }
  SP_TRY(check_bsr(A));
  Factor &old = *F->F;
  if (A->n_brows != old.K || A->bs != old.bs || A->nnzb != int64_t(old.h_colind.size())) {
    set_error("A (n_brows %d, bs %d, nnzb %lld) does not have the factored pattern (%d, %d, %zu)",
              A->n_brows, A->bs, (long long)A->nnzb, old.K, old.bs, old.h_colind.size());
    return SPAND_EINVAL;
  }
  {
    // the symbolic phase is only valid for the same block pattern
    std::vector<int32_t> rp(size_t(A->n_brows) + 1), ci(size_t(A->nnzb));
    hipStream_t st = (hipStream_t)stream;
    SP_HIP(hipMemcpyAsync(rp.data(), A->d_rowptr, rp.size() * 4, hipMemcpyDeviceToHost, st));
    SP_HIP(hipMemcpyAsync(ci.data(), A->d_colind, ci.size() * 4, hipMemcpyDeviceToHost, st));
    SP_HIP(hipStreamSynchronize(st));
    if (rp != old.h_rowptr || ci != old.h_colind) {
      set_error("A's block pattern differs from the factored one");
      return SPAND_EINVAL;
    }
  }
  std::unique_ptr<Factor> nf;
  try {
    SP_TRY(build_factor(A, &old.grid, &old.opts, stream, &old, old.use_graphs, nf));
  } catch (const std::exception &ex) {
    set_error("refactorization failed: %s", ex.what());
    return SPAND_EINVAL;
  }
  F->F = std::move(nf);        // the previous factorization is released here
  return SPAND_OK;
}

int spand_apply(spand_factor_t F, const double *d_in, double *d_out, void *stream) {
  if (!F || !d_in || !d_out) {
    set_error("NULL argument");
    return SPAND_EINVAL;
  }
  return F->F->apply(d_in, d_out, 0, (hipStream_t)stream, F->member);
}

int spand_apply_T(spand_factor_t F, const double *d_in, double *d_out, void *stream) {
  if (!F || !d_in || !d_out) {
    set_error("NULL argument");
    return SPAND_EINVAL;
  }
  SP_TRY(F->F->capture_graphs(2, F->member));
  return F->F->apply(d_in, d_out, 1, (hipStream_t)stream, F->member);
}

}  // extern "C"

static int check_solve_args(const spand_bsr_t *A, spand_factor_t M, const double *d_b,
                            double *d_x, const sstep_opts_t *opts) {
  SP_TRY(check_bsr(A));
  if (!d_b || !d_x || !opts) {
    set_error("NULL argument");
    return SPAND_EINVAL;
  }
  if (opts->s < 1 || opts->s > TS_MAXS) {
    set_error("s must be in [1, %d]", TS_MAXS);
    return SPAND_EINVAL;
  }
  if (opts->restart < opts->s || opts->restart % opts->s != 0 || opts->restart > KRY_MMAX ||
      opts->restart + 1 + opts->s > TS_MAXA) {
    set_error("restart must be a multiple of s in [s, %d]", KRY_MMAX);
    return SPAND_EINVAL;
  }
  if (opts->maxit < 1 || !(opts->rtol > 0.0) || !std::isfinite(opts->rtol)) {
    set_error("maxit must be >= 1 and rtol > 0");
    return SPAND_EINVAL;
  }
  if (M && (M->N() != int64_t(A->n_brows) * A->bs)) {
    set_error("factor size does not match A");
    return SPAND_EINVAL;
  }
  return SPAND_OK;
}

// ------------------------------------------------- solve without allocation
// Workspace of sstep_gmres_solve_noalloc: one array per device, held from
// the first call on that device until the process ends.  Host code uses its
// device address from hipGetSymbolAddress (taken once per device, with that
// device current), never the array's name.
static __device__ __align__(256) unsigned char scratch[SPAND_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;                 // guards g_scratch_ptr
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_use[kMaxDevices];   // one no-allocation solve per device at a time

static int scratch_address(int dev, void **ptr) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the no-allocation scratch supports", dev, kMaxDevices);
    return SPAND_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return SPAND_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return SPAND_OK;
}

extern "C" {

int sstep_gmres_solve(const spand_bsr_t *A, spand_factor_t M, const double *d_b, double *d_x,
                      const sstep_opts_t *opts, sstep_stats_t *st, void *stream) {
  set_error("");
  SP_TRY(check_solve_args(A, M, d_b, d_x, opts));
  if (st) std::memset(st, 0, sizeof(*st));
  if (M && opts->transpose) SP_TRY(M->F->capture_graphs(2, M->member));
  try {
    return sstep_solve(*A, M ? M->F.get() : nullptr, M ? M->member : -1, d_b, d_x, *opts, st,
                       (hipStream_t)stream);
  } catch (const std::exception &ex) {
    set_error("solve failed: %s", ex.what());
    return SPAND_EINVAL;
  }
}

int sstep_gmres_solve_noalloc(const spand_bsr_t *A, spand_factor_t M, const double *d_b,
                              double *d_x, const sstep_opts_t *opts, sstep_stats_t *st,
                              void *stream) {
  set_error("");
  SP_TRY(check_solve_args(A, M, d_b, d_x, opts));
  const int64_t N = int64_t(A->n_brows) * A->bs;
  const size_t need = sstep_workspace_bytes(N, *opts);
  if (need > SPAND_NOALLOC_SCRATCH_BYTES) {
    set_error("the solve needs %zu bytes of workspace (N = %lld, restart %d); the no-allocation "
              "scratch holds %zu",
              need, (long long)N, opts->restart, (size_t)SPAND_NOALLOC_SCRATCH_BYTES);
    return SPAND_EINVAL;
  }
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  void *ptr = nullptr;
  SP_TRY(scratch_address(dev, &ptr));
  if (st) std::memset(st, 0, sizeof(*st));
  // calls on one device share its scratch: they run one at a time, and each
  // returns only after its work on `stream` has finished
  std::lock_guard<std::mutex> lk(g_scratch_use[dev]);
  const SolveWorkspace ws{ptr, SPAND_NOALLOC_SCRATCH_BYTES};
  try {
    return sstep_solve(*A, M ? M->F.get() : nullptr, M ? M->member : -1, d_b, d_x, *opts, st,
                       (hipStream_t)stream, &ws);
  } catch (const std::exception &ex) {
    set_error("solve failed: %s", ex.what());
    return SPAND_EINVAL;
  }
}

int spand_bsr_spmv(const spand_bsr_t *A, int transpose, double alpha, const double *d_x,
                   double beta, double *d_y, void *stream) {
  set_error("");
  SP_TRY(check_bsr(A));
  if (!d_x || !d_y || d_x == d_y) {
    set_error("x and y must be distinct non-NULL device vectors");
    return SPAND_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  if (!transpose) return launch_spmv(*A, 0, alpha, d_x, beta, d_y, nullptr, 0.0, nullptr, 0.0, st);
  // A^T x reads the mirror blocks in place; the pattern must be symmetric,
  // which is checked (and reported) before the product
  void *fl = nullptr;
  size_t got = 0;
  SP_TRY(pool_alloc(&fl, 64, &got));
  int r = SPAND_OK, flag = 0;
  if (hipMemsetAsync(fl, 0, 64, st) != hipSuccess) r = SPAND_EHIP;
  if (r == SPAND_OK) r = launch_spmv_t_check(*A, (int *)fl, st);
  if (r == SPAND_OK && (hipMemcpyAsync(&flag, fl, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
    r = SPAND_EHIP;
  pool_release(fl, got);
  if (r == SPAND_OK && flag) {
    set_error("transposed SpMV needs a structurally symmetric block pattern");
    r = SPAND_EINVAL;
  }
  if (r == SPAND_OK) r = launch_spmv(*A, 1, alpha, d_x, beta, d_y, nullptr, 0.0, nullptr, 0.0, st);
  return r;
}

int spand_bsr_pattern_outer(const spand_bsr_t *P, const double *d_u, const double *d_v,
                            double alpha, double *d_out, void *stream) {
  set_error("");
  SP_TRY(check_bsr(P));
  if (!d_u || !d_v || !d_out) {
    set_error("NULL argument");
    return SPAND_EINVAL;
  }
  return launch_pattern_outer(*P, d_u, d_v, alpha, d_out, (hipStream_t)stream);
}

// Run job(i, stream) for i < n on a pool of worker threads, each with its own
// non-blocking stream (default priority) ordered after `stream`; `stream`
// then waits for every worker stream.  Items of one group (group[i], equal
// values) run in index order on one worker, so that items sharing state (a
// factor handle and its scratch vectors) never run on two streams at once;
// group == nullptr makes every item its own group.  Returns the per-item
// statuses.
static int run_batched(int n, hipStream_t stream, const std::function<int(int, hipStream_t)> &job,
                       std::vector<int> &status, const std::vector<int> *group = nullptr,
                       int max_workers = 0) {
  status.assign(n, SPAND_OK);
  // work units: lists of items, in order of their first item
  std::vector<std::vector<int>> units;
  {
    std::unordered_map<int, size_t> at;
    for (int i = 0; i < n; ++i) {
      const int g = group ? (*group)[i] : -1;
      if (g < 0) {
        units.push_back({i});
        continue;
      }
      auto it = at.find(g);
      if (it == at.end()) {
        at.emplace(g, units.size());
        units.push_back({i});
      } else {
        units[it->second].push_back(i);
      }
    }
  }
  const int nu = int(units.size());
  int dev = 0;
  SP_HIP(hipGetDevice(&dev));
  int nw = 8;
  if (const char *e = std::getenv("SPAND_BATCH_STREAMS")) nw = std::max(1, std::atoi(e));
  if (max_workers > 0) nw = std::min(nw, max_workers);
  nw = std::min(nw, nu);
  if (nw <= 0) return SPAND_OK;
  hipEvent_t start;
  SP_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  SP_HIP(hipEventRecord(start, stream));
  std::vector<hipStream_t> ss(nw, nullptr);
  for (int w = 0; w < nw; ++w) {
    SP_HIP(hipStreamCreateWithFlags(&ss[w], hipStreamNonBlocking));
    SP_HIP(hipStreamWaitEvent(ss[w], start, 0));
  }
  std::atomic<int> next(0);
  std::vector<std::string> errs(n);
  auto worker = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      const int u = next.fetch_add(1);
      if (u >= nu) break;
      for (const int i : units[u]) {
        int r;
        try {
          r = job(i, ss[w]);
        } catch (const std::exception &ex) {
          set_error("system %d: %s", i, ex.what());
          r = SPAND_EINVAL;
        }
        status[i] = r;
        if (r != SPAND_OK) errs[i] = last_error();
      }
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < nw; ++w) th.emplace_back(worker, w);
  worker(0);
  for (auto &t : th) t.join();
  for (int w = 0; w < nw; ++w) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(e, ss[w]);
      (void)hipStreamWaitEvent(stream, e, 0);
      (void)hipEventDestroy(e);
    }
  }
  (void)hipStreamSynchronize(stream);
  for (auto &q : ss) (void)hipStreamDestroy(q);
  (void)hipEventDestroy(start);
  for (int i = 0; i < n; ++i)
    if (status[i] < 0) {
      set_error("system %d: %s", i, errs[i].c_str());
      break;
    }
  return SPAND_OK;
}

int spand_factor_batched(int32_t n, const spand_bsr_t *A, const spand_grid_t *grids,
                         const spand_opts_t *opts, void *stream, spand_factor_t *out) {
  set_error("");
  if (n < 0 || (n > 0 && (!A || !grids || !opts || !out))) {
    set_error("bad batched arguments");
    return SPAND_EINVAL;
  }
  for (int i = 0; i < n; ++i) out[i] = nullptr;
  std::vector<int> Ls(size_t(n), 0);
  for (int i = 0; i < n; ++i) {
    const int r = check_factor_args(&A[i], &grids[i], &opts[i], &Ls[size_t(i)]);
    if (r != SPAND_OK) {
      set_error("system %d: %s", i, std::string(last_error()).c_str());
      return r;
    }
  }
  // Systems with the same block size, factor precision, eps and flags are
  // factored together (one launch per phase for all of them), in index
  // order, in groups of at most SPAND_BATCH_UNION_DOF unknowns (default 4M,
  // the size that fills the device; a factorization's scratch peaks near
  // 20 kB per unknown in FP32), at most SPAND_BATCH_FACTOR_STREAMS groups
  // (default 2) at a time, each on its own worker stream.
  // SPAND_BATCH_SEPARATE=1 factors every system on its own (for comparisons).
  std::vector<std::vector<int>> groups;
  {
    const bool sep = std::getenv("SPAND_BATCH_SEPARATE") && std::atoi(std::getenv("SPAND_BATCH_SEPARATE"));
    int64_t cap = int64_t(4) << 20;
    if (const char *e = std::getenv("SPAND_BATCH_UNION_DOF")) cap = std::max<int64_t>(1, std::atoll(e));
    std::map<std::tuple<int, int, uint64_t, int>, size_t> gid;   // key -> open group
    std::vector<int64_t> gdof;
    for (int i = 0; i < n; ++i) {
      uint64_t eb;
      std::memcpy(&eb, &opts[i].eps, 8);
      const auto key = std::make_tuple(A[i].bs, opts[i].factor_dtype, eb, opts[i].flags);
      const int64_t dof = int64_t(A[i].n_brows) * A[i].bs;
      auto it = gid.find(key);
      if (sep || it == gid.end() || gdof[it->second] + dof > cap) {
        if (!sep) gid[key] = groups.size();
        groups.push_back({i});
        gdof.push_back(dof);
      } else {
        groups[it->second].push_back(i);
        gdof[it->second] += dof;
      }
    }
  }
  int fw = 2;
  if (const char *e = std::getenv("SPAND_BATCH_FACTOR_STREAMS")) fw = std::max(1, std::atoi(e));
  if (std::getenv("SPAND_BATCH_SEPARATE") && std::atoi(std::getenv("SPAND_BATCH_SEPARATE"))) fw = 0;
  std::vector<std::unique_ptr<Factor>> gf(groups.size());
  std::vector<int> st;
  // with several builds at once each keeps to its worker stream
  const bool conc = groups.size() > 1 && fw != 1;
  SP_TRY(run_batched(int(groups.size()), (hipStream_t)stream, [&](int g, hipStream_t s) {
    set_error("");
    const auto &idx = groups[size_t(g)];
    if (idx.size() == 1) {
      const int i = idx[0];
      return build_factor(&A[i], &grids[i], &opts[i], (void *)s, nullptr, false, gf[size_t(g)],
                          conc);
    }
    std::vector<BatchSystem> sy;
    for (int i : idx) sy.push_back(BatchSystem{A[i], grids[i], Ls[size_t(i)]});
    return run_build((void *)s, [&](Factor &F) { return F.build_batch(sy, opts[idx[0]]); },
                     gf[size_t(g)], conc);
  }, st, nullptr, fw));
  for (size_t g = 0; g < groups.size(); ++g)
    if (st[g] < 0) return st[g];
  std::vector<std::unique_ptr<spand_factor_s>> hs(static_cast<size_t>(n));
  for (size_t g = 0; g < groups.size(); ++g) {
    std::shared_ptr<Factor> f(std::move(gf[g]));
    const auto &idx = groups[g];
    for (size_t k = 0; k < idx.size(); ++k) {
      auto h = std::make_unique<spand_factor_s>();
      h->F = f;
      h->member = idx.size() == 1 ? -1 : int(k);
      hs[size_t(idx[k])] = std::move(h);
    }
  }
  // graphs are captured on the calling thread, with no worker alive
  for (int i = 0; i < n; ++i) {
    const int r = hs[size_t(i)]->F->capture_graphs(1, hs[size_t(i)]->member);
    if (r != SPAND_OK) {
      set_error("system %d: %s", i, std::string(last_error()).c_str());
      return r;
    }
  }
  for (int i = 0; i < n; ++i) out[i] = hs[size_t(i)].release();
  return SPAND_OK;
}

int spand_apply_batched(int32_t n, const spand_factor_t *F, const double *const *d_in,
                        double *const *d_out, int32_t transpose, void *stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!F || !d_in || !d_out)) || (transpose != 0 && transpose != 1)) {
    set_error("bad batched arguments");
    return SPAND_EINVAL;
  }
  for (int i = 0; i < n; ++i)
    if (!F[i] || !d_in[i] || !d_out[i]) {
      set_error("system %d: NULL argument", i);
      return SPAND_EINVAL;
    }
  hipStream_t st = (hipStream_t)stream;
  // the handles that hold every system of one shared factorization, each
  // once, take one replay of that factorization's sweeps
  std::map<Factor *, std::vector<int>> by;
  for (int i = 0; i < n; ++i)
    if (F[i]->member >= 0) by[F[i]->F.get()].push_back(i);
  std::vector<char> done(size_t(n), 0);
  for (auto &kv : by) {
    Factor &f = *kv.first;
    std::vector<int> at(f.members.size(), -1);
    bool full = kv.second.size() == f.members.size();
    for (int i : kv.second) {
      int &a = at[size_t(F[i]->member)];
      if (a >= 0) full = false;
      a = i;
    }
    if (!full) continue;
    std::vector<const double *> in;
    std::vector<double *> out;
    for (int i : at) {
      in.push_back(d_in[i]);
      out.push_back(d_out[i]);
    }
    SP_TRY(f.capture_graphs(1 << transpose, -1));
    SP_TRY(f.apply_batch(in, out, transpose, st));
    for (int i : kv.second) done[size_t(i)] = 1;
  }
  for (int i = 0; i < n; ++i)
    if (!done[size_t(i)]) {
      SP_TRY(F[i]->F->capture_graphs(1 << transpose, F[i]->member));
      SP_TRY(F[i]->F->apply(d_in[i], d_out[i], transpose, st, F[i]->member));
    }
  return SPAND_OK;
}

int sstep_gmres_solve_batched(int32_t n, const spand_bsr_t *A, const spand_factor_t *M,
                              const double *const *d_b, double *const *d_x,
                              const sstep_opts_t *opts, sstep_stats_t *stv, void *stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!A || !d_b || !d_x || !opts))) {
    set_error("bad batched arguments");
    return SPAND_EINVAL;
  }
  // transposed sweeps are captured here, before any worker thread exists
  for (int i = 0; i < n; ++i)
    if (M && M[i] && opts[i].transpose) SP_TRY(M[i]->F->capture_graphs(2, M[i]->member));
  // systems that share a factor handle share its scratch vectors: they run
  // one after the other on one worker stream
  std::vector<int> group(n, -1);
  {
    std::unordered_map<const void *, int> id;
    for (int i = 0; i < n; ++i)
      if (M && M[i]) group[i] = id.emplace((const void *)M[i], int(id.size())).first->second;
  }
  std::vector<int> st;
  SP_TRY(run_batched(n, (hipStream_t)stream, [&](int i, hipStream_t s) {
    return sstep_gmres_solve(&A[i], M ? M[i] : nullptr, d_b[i], d_x[i], &opts[i],
                             stv ? &stv[i] : nullptr, (void *)s);
  }, st, &group));
  int worst = SPAND_OK;
  for (int i = 0; i < n; ++i) {
    if (st[i] < 0) return st[i];
    if (st[i] == SPAND_EBREAKDOWN) worst = SPAND_EBREAKDOWN;
    else if (st[i] == SPAND_ENOTCONV && worst == SPAND_OK) worst = SPAND_ENOTCONV;
  }
  return worst;
}

int spand_pool_trim(void) {
  pool_trim();
  return SPAND_OK;
}

int spand_factor_stats(spand_factor_t F, spand_factor_stats_t *out) {
  if (!F || !out) {
    set_error("NULL argument");
    return SPAND_EINVAL;
  }
  F->F->fill_stats(out, F->member);
  return SPAND_OK;
}

int spand_destroy(spand_factor_t F) {
  if (F) {
    (void)hipDeviceSynchronize();
    delete F;
  }
  return SPAND_OK;
}

int spand_nd(const spand_grid_t *grid, int32_t L, int32_t *L_out, int32_t *h_node_of_elem,
             int32_t *h_perm, int32_t *h_ncl, int32_t *h_cl_ptr, int32_t *h_cl_elems,
             int32_t *h_cl_key, int32_t *h_cl_interior) {
  set_error("");
  if (!grid || grid->nx <= 0 || grid->ny <= 0) {
    set_error("bad grid");
    return SPAND_EINVAL;
  }
  const int64_t K = int64_t(grid->nx) * grid->ny;
  if (L <= 0) L = default_levels(K);
  if (L > SPAND_MAX_LEVELS || (L > 1 && (int64_t(1) << (L - 1)) > K)) {
    set_error("bad number of levels %d", L);
    return SPAND_EINVAL;
  }
  if (L_out) *L_out = L;
  NDResult nd = nested_dissection(grid->nx, grid->ny, grid->periodic_x != 0,
                                  grid->periodic_y != 0, L);
  if (h_node_of_elem) std::memcpy(h_node_of_elem, nd.node_of_elem.data(), K * 4);
  if (h_perm) std::memcpy(h_perm, nd.perm.data(), K * 4);
  if (h_ncl)
    for (int l = 0; l < L; ++l) h_ncl[l] = int32_t(nd.levels[l].size());
  if (h_cl_ptr && h_cl_elems && h_cl_key && h_cl_interior) {
    int64_t pbase = 0, cbase = 0;
    for (int l = 0; l < L; ++l) {
      const auto &cl = nd.levels[l];
      int32_t off = 0;
      for (size_t c = 0; c < cl.size(); ++c) {
        h_cl_ptr[pbase + c] = off;
        for (int32_t e : cl[c].elems) h_cl_elems[int64_t(l) * K + off++] = e;
        h_cl_key[2 * (cbase + c)] = cl[c].node;
        h_cl_key[2 * (cbase + c) + 1] = cl[c].box;
        h_cl_interior[cbase + c] = cl[c].interior ? 1 : 0;
      }
      h_cl_ptr[pbase + cl.size()] = off;
      pbase += int64_t(cl.size()) + 1;
      cbase += int64_t(cl.size());
    }
  }
  return SPAND_OK;
}

}  // extern "C"
