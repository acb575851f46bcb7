// spaND factorization and its application (host orchestration).
//
// Level-synchronous GPU version of the paper's Sec. "Sparsified Nested
// Dissection algorithm": per level, every independent cluster of a phase is
// one item of a batched launch (the GPU counterpart of the per-level task
// graph of Sec. "Parallel implementation using TaskTorrent").
//
//  level 0   leaves: dense A_ss gathered from the BSR input, inverted by
//            blocked Gauss-Jordan with partial pivoting (same pivots as
//            LU with partial pivoting); Schur update A_nm -= A_ns A_ss^-1 A_sm
//            on b x b element blocks (Eq. 10), pulled per target block;
//  every l   interfaces: LU with partial pivoting of A_ss on [A_ss | I] ->
//            U and L^-1 P^T; U^-1 by Gauss-Jordan; diagonal of U split
//            evenly (Eq. 11); all blocks scaled; W = [A_sn A_ns^T] and its
//            column-pivoted QR (Eq. 12); all blocks compressed with the kept
//            columns (Eq. 13) straight into the merged next-level blocks;
//  l >= 1    interiors: dense merged blocks, same inversion, Schur update by
//            batched GEMMs in deterministic rounds;
//  top       inversion of the root separator.
//
// Stored for the apply (factor precision T):
//   interiors  A_ss^-1 and the coupling blocks A_ns, A_sn
//   interfaces F_s = Q_s^T Lh^-1 P^T and B_s = Uh^-1 Q_s
// with the elimination written as L' = [[I,0],[-A_ns A_ss^-1, I]],
// R' = [[A_ss^-1, -A_ss^-1 A_sn],[0, I]]  (L' A R' = diag(I, Schur)).
#include <algorithm>
#include <climits>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <set>

#include "factor.h"

namespace spand {

// ------------------------------------------------------------------ arenas
struct PlanArena {
  std::vector<size_t> offs;
  size_t total = 0;
  char *base = nullptr;
  size_t add(size_t bytes) {
    size_t o = (total + 255) & ~size_t(255);
    total = o + std::max<size_t>(bytes, 1);
    return o;
  }
};

int Bump::alloc(void **p, size_t n, size_t chunk) {
  n = (std::max<size_t>(n, 1) + 255) & ~size_t(255);
  if (chunks.empty() || used + n > chunks.back().second) {
    void *q;
    size_t got = 0;
    SP_TRY(pool_alloc(&q, std::max(n, chunk), &got));
    chunks.push_back({(char *)q, got});
    bytes += got;
    used = 0;
  }
  *p = chunks.back().first + used;
  used += n;
  return SPAND_OK;
}

// Callers have synchronised the work that used the chunks.
void Bump::release() {
  for (auto &c : chunks) pool_release(c.first, c.second);
  chunks.clear();
  used = 0;
  bytes = 0;
}

int Factor::dalloc(void **p, size_t bytes, bool keep) {
  const size_t chunk = size_t(256) << 20;
  return keep ? this->keep.alloc(p, bytes, chunk) : temp.alloc(p, bytes, chunk);
}

int Factor::dalloc_next(void **p, size_t bytes) {
  return next_temp.alloc(p, bytes, size_t(256) << 20);
}

void Bump::absorb(Bump &o) {
  chunks.insert(chunks.end(), o.chunks.begin(), o.chunks.end());
  bytes += o.bytes;
  o.chunks.clear();
  o.used = 0;
  o.bytes = 0;
}

// End of a level: its scratch retires (kernels may still be reading it;
// it returns to the block cache at the next stream synchronisation), and
// the next level's trailing blocks become the current scratch.
void Factor::free_temp() {
  retired.absorb(temp);
  std::swap(temp, next_temp);
}

// Called right after a stream synchronisation: nothing queued uses the
// retired scratch any more.
void Factor::release_retired() { retired.release(); }

Factor::~Factor() {
  // a build that failed may have left work queued on its chunks
  (void)hipDeviceSynchronize();
  collect_events();         // events of a build that stopped early
  for (auto &g : gexec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto &m : members)
    for (auto &g : m.gexec)
      if (g) (void)hipGraphExecDestroy(g);
  temp.release();
  next_temp.release();
  retired.release();
  keep.release();
  if (side) (void)hipStreamDestroy(side);
  if (side2) (void)hipStreamDestroy(side2);
  if (cls_fork) (void)hipEventDestroy(cls_fork);
  if (cls_join) (void)hipEventDestroy(cls_join);
}

// ------------------------------------------------------------------ batch members
const double *Factor::blk_src(int e, int64_t t) const {
  const size_t b2 = size_t(bs) * bs;
  if (members.empty()) return d_val + size_t(t) * b2;
  const Member &M = members[size_t(esys[size_t(e)])];
  return M.d_val + size_t(t - M.nnz_off) * b2;
}

int Factor::csys(int l, int c) const {
  if (members.empty()) return 0;
  return esys[size_t(nd_sym->levels[size_t(l)][size_t(c)].elems[0])];
}

void Factor::acct(int sys, double bytes, double fl) {
  apply_bytes += bytes;
  flops += fl;
  if (!members.empty()) {
    members[size_t(sys)].apply_bytes += bytes;
    members[size_t(sys)].flops += fl;
  }
}

int Factor::member_pull(int l, PullSet ApplyLevel::*which, const std::vector<PullGroup> &G,
                        const std::vector<PullItem> &I, const std::vector<int> &gs) {
  if (members.empty()) return SPAND_OK;
  std::vector<std::vector<PullGroup>> Gm(members.size());
  std::vector<std::vector<PullItem>> Im(members.size());
  for (size_t g = 0; g < G.size(); ++g) {
    const int m = gs[g];
    PullGroup q = G[g];
    q.item_begin = int(Im[size_t(m)].size());
    Im[size_t(m)].insert(Im[size_t(m)].end(), I.begin() + G[g].item_begin, I.begin() + G[g].item_end);
    q.item_end = int(Im[size_t(m)].size());
    Gm[size_t(m)].push_back(q);
  }
  for (size_t m = 0; m < members.size(); ++m)
    SP_TRY((members[m].lv[size_t(l)].*which).set(*this, Gm[m], Im[m]));
  return SPAND_OK;
}

int Factor::member_gemv(int l, GemvSet ApplyLevel::*which, const std::vector<GemvDesc> &gv,
                        const std::vector<const std::vector<int32_t> *> &os,
                        const std::vector<int> &gs, int trans) {
  if (members.empty()) return SPAND_OK;
  std::vector<std::vector<GemvDesc>> gm(members.size());
  std::vector<std::vector<const std::vector<int32_t> *>> om(members.size());
  for (size_t i = 0; i < gv.size(); ++i) {
    gm[size_t(gs[i])].push_back(gv[i]);
    om[size_t(gs[i])].push_back(os[i]);
  }
  for (size_t m = 0; m < members.size(); ++m)
    SP_TRY((members[m].lv[size_t(l)].*which).set(*this, gm[m], om[m], trans));
  return SPAND_OK;
}

template <typename D>
int Factor::upload(const std::vector<D> &v, D **out, bool keep) {
  *out = nullptr;
  if (v.empty()) return SPAND_OK;
  void *p;
  SP_TRY(dalloc(&p, v.size() * sizeof(D), keep));
  SP_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(D), hipMemcpyHostToDevice));
  *out = (D *)p;
  return SPAND_OK;
}

int Factor::upload_parts(std::initializer_list<UpPart> parts, bool keep) {
  size_t tot = 0;
  for (const auto &q : parts) tot += (q.bytes + 255) & ~size_t(255);
  for (const auto &q : parts) *q.dst = nullptr;
  if (tot == 0) return SPAND_OK;
  void *p;
  SP_TRY(dalloc(&p, tot, keep));
  std::vector<char> h(tot);
  size_t off = 0;
  for (const auto &q : parts) {
    if (q.bytes) {
      std::memcpy(h.data() + off, q.src, q.bytes);
      *q.dst = (char *)p + off;
    }
    off += (q.bytes + 255) & ~size_t(255);
  }
  SP_HIP(hipMemcpy(p, h.data(), tot, hipMemcpyHostToDevice));
  return SPAND_OK;
}

int Factor::upload_slots(const std::vector<int32_t> &v, int32_t **out) {
  return upload(v, out, true);
}

// all slot lists of a level in one upload
int Factor::upload_level_slots(LevelState &S) {
  std::vector<int32_t> all;
  std::vector<size_t> off(S.slots.size());
  size_t tot = 0;
  for (const auto &v : S.slots) tot += v.size();
  all.reserve(tot);
  for (size_t c = 0; c < S.slots.size(); ++c) {
    off[c] = all.size();
    all.insert(all.end(), S.slots[c].begin(), S.slots[c].end());
  }
  int32_t *base = nullptr;
  SP_TRY(upload(all, &base, true));
  S.d_slots.assign(S.slots.size(), nullptr);
  for (size_t c = 0; c < S.slots.size(); ++c)
    if (!S.slots[c].empty()) S.d_slots[c] = base + off[c];
  return SPAND_OK;
}

int Factor::flush_deferred() {
  std::vector<std::function<int()>> q;
  q.swap(deferred);
  for (auto &f : q) SP_TRY(f());
  return SPAND_OK;
}

// ------------------------------------------------------------------ host trace
// SPAND_HOST_TRACE set: every planning step prints its host time to stderr
// (diagnostics of the host/device overlap; no effect otherwise).
static bool host_trace_on() {
  static const bool on = std::getenv("SPAND_HOST_TRACE") != nullptr;
  return on;
}

// ------------------------------------------------------------------ batched helpers
void gemm_coarse(const std::vector<int32_t> &ts, size_t a, size_t b, std::vector<int32_t> &out) {
  const int64_t ntiles = ts[b] - ts[a];
  const int64_t nc = ntiles / 64 + 1;
  size_t d = a;
  for (int64_t c = 0; c <= nc; ++c) {
    const int64_t t = ts[a] + std::min<int64_t>(c * 64, ntiles - 1);
    while (d + 1 < b && ts[d + 1] <= t) ++d;
    out.push_back(int32_t(d - a));
  }
}

// Algorithmic work of a batch of products: 2MNK flops per item (for a
// triangular operand only its nonzero half, which is what the tiles read),
// operands read once, C read when accumulated and written.
static void gemm_work(const GemmDesc *d, int n, size_t esz, double *fl, double *by) {
  for (int i = 0; i < n; ++i) {
    const double f = 2.0 * d[i].M * d[i].N * d[i].K;
    *fl += d[i].tri ? 0.5 * f : f;
    *by += (double(d[i].M) * d[i].K * (d[i].tri ? 0.5 : 1.0) + double(d[i].K) * d[i].N +
            double(d[i].M) * d[i].N * (d[i].beta != 0.0 ? 2 : 1)) * double(esz);
  }
}

int Factor::timed_launch(int kind, double flops, double bytes, const std::function<int()> &launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (timing && event_get(&a) == SPAND_OK) {
    if (event_get(&b) != SPAND_OK) {
      event_put(a);
      a = nullptr;
    } else {
      (void)hipEventRecord(a, stream);
    }
  }
  const int r = launch();
  if (a) {
    (void)hipEventRecord(b, stream);
    kevents.push_back({kind, a, b, flops, bytes});
  }
  return r;
}

int Factor::gemm_batch(const std::vector<GemmDesc> &items) {
  if (items.empty()) return SPAND_OK;
  if (host_trace_on()) {
    double fl = 0.0, by = 0.0;
    int64_t tiles = 0;
    for (const auto &d : items) {
      fl += 2.0 * d.M * d.N * d.K;
      by += (double(d.M) * d.K + double(d.K) * d.N + double(d.M) * d.N * (d.beta != 0.0 ? 2 : 1)) * fsize(ft);
      tiles += cdiv(d.M, 64) * cdiv(d.N, 64);
    }
    int modes = 0;
    for (int tm = 0; tm < 4; ++tm) {
      bool any = false;
      for (const auto &d : items) any = any || 2 * (d.transA != 0) + (d.transB != 0) == tm;
      modes += any;
    }
    std::fprintf(stderr, "[spand host] gemm batch: %zu items %lld tiles %.3f TFLOP %.3f GB (operands once), %d launches\n",
                 items.size(), (long long)tiles, fl * 1e-12, by * 1e-9, modes);
  }
  // one launch per transpose mode (the FP32 kernel is specialised on it)
  std::vector<GemmDesc> ord;
  std::vector<int32_t> ts(1, 0);
  int start[5] = {0, 0, 0, 0, 0};
  for (int tm = 0; tm < 4; ++tm) {
    start[tm] = int(ord.size());
    for (const auto &d : items)
      if (2 * (d.transA != 0) + (d.transB != 0) == tm) {
        ord.push_back(d);
        ts.push_back(ts.back() + int32_t(cdiv(d.M, 64) * cdiv(d.N, 64)));
      }
  }
  start[4] = int(ord.size());
  trace("  gemm plan", -2);
  int uni[4] = {0, 0, 0, 0};
  size_t coff[5] = {0, 0, 0, 0, 0};
  std::vector<int32_t> coarse;
  for (int tm = 0; tm < 4; ++tm) {
    const int a = start[tm], b = start[tm + 1];
    coff[tm] = coarse.size();
    if (b > a) {
      int uniform = ts[a + 1] - ts[a];
      for (int q = a; q < b && uniform > 0; ++q)
        if (ts[q + 1] - ts[q] != uniform) uniform = 0;
      uni[tm] = uniform;
      if (!uniform) gemm_coarse(ts, size_t(a), size_t(b), coarse);
    }
  }
  GemmDesc *d_items;
  int32_t *d_ts, *d_coarse;
  SP_TRY(upload_parts({part(ord, &d_items), part(ts, &d_ts), part(coarse, &d_coarse)}, false));
  trace("  gemm upload", -2);
  for (int tm = 0; tm < 4; ++tm) {
    const int a = start[tm], b = start[tm + 1];
    if (b > a) {
      double fl = 0.0, by = 0.0;
      gemm_work(ord.data() + a, b - a, fsize(ft), &fl, &by);
      SP_TRY(timed_launch(0, fl, by, [&]() {
        return launch_gemm(ft, d_items + a, d_ts + a, b - a, ts[b] - ts[a], stream, ts[a], tm,
                           uni[tm], uni[tm] ? nullptr : d_coarse + coff[tm]);
      }));
    }
  }
  return SPAND_OK;
}

int Factor::copy_batch(const std::vector<CopyDesc> &items, int src_is_factor) {
  if (items.empty()) return SPAND_OK;
  // straight copies and transposed copies go to different kernels
  std::vector<CopyDesc> st, tr;
  int64_t mx = 0;
  int mr = 0, mc = 0;
  for (auto &d : items) {
    if (d.trans) {
      tr.push_back(d);
      mr = std::max(mr, d.rows);
      mc = std::max(mc, d.cols);
    } else {
      st.push_back(d);
      mx = std::max<int64_t>(mx, int64_t(d.rows) * d.cols);
    }
  }
  CopyDesc *d_st, *d_tr;
  SP_TRY(upload_parts({part(st, &d_st), part(tr, &d_tr)}, false));
  if (!st.empty()) SP_TRY(launch_copy(ft, src_is_factor, d_st, int(st.size()), mx, stream));
  if (!tr.empty())
    SP_TRY(launch_copy_t(ft, src_is_factor, d_tr, int(tr.size()), mr, mc, stream));
  return SPAND_OK;
}

// Blocked elimination of a batch; items get their n/ncols/ld filled in.
int Factor::elim_batch(std::vector<ElimDesc> &items, int mode) {
  if (items.empty()) return SPAND_OK;
  std::sort(items.begin(), items.end(), [](const ElimDesc &a, const ElimDesc &b) {
    return a.n > b.n;
  });
  // The eliminations are blocked: each block of bw columns is eliminated in
  // its own columns (one fused launch, one row per thread, for matrices of
  // up to elim_block_max_n rows; panels of 16 columns for larger ones); the
  // rest of the matrix receives each block at once as one rank-bw product
  // on the matrix cores.  In-place Gauss-Jordan (modes 0, 2) leaves the
  // block's multipliers in the block columns themselves; LU (mode 1)
  // accumulates them in PB.
  const bool lu = mode == 1;
  // path of a matrix: 0 panels, else the fused block width
  auto path = [&](int n) { return n > elim_block_max_n(ft) ? 0 : elim_block_width(ft, n); };
  // every item takes its own path: matrices of different paths go to
  // separate calls
  if (path(items[0].n) != path(items.back().n)) {
    const int p0 = path(items[0].n);
    const auto cut = std::find_if(items.begin(), items.end(), [&](const ElimDesc &d) {
      return path(d.n) != p0;
    });
    std::vector<ElimDesc> big(items.begin(), cut), small(cut, items.end());
    if (p0 == 0 && !one_stream) {
      // the few matrices beyond the fused limit take a long chain of
      // one-workgroup panel launches: it runs on the side stream, beside the
      // fused launches of the others (independent matrices and scratch)
      if (!side) SP_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
      hipEvent_t fork, join;
      SP_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
      SP_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
      SP_HIP(hipEventRecord(fork, stream));
      SP_HIP(hipStreamWaitEvent(side, fork, 0));
      std::swap(stream, side);
      const int rb = elim_batch(big, mode);
      std::swap(stream, side);
      // joined even when the side call failed, so that nothing it queued
      // outlives the build's scratch
      SP_HIP(hipEventRecord(join, side));
      const int rs = rb == SPAND_OK ? elim_batch(small, mode) : rb;
      SP_HIP(hipStreamWaitEvent(stream, join, 0));
      (void)hipEventDestroy(fork);
      (void)hipEventDestroy(join);
      SP_TRY(rs);
    } else {
      SP_TRY(elim_batch(big, mode));
      SP_TRY(elim_batch(small, mode));
    }
    std::copy(big.begin(), big.end(), items.begin());
    std::copy(small.begin(), small.end(), items.begin() + big.size());
    return SPAND_OK;
  }
  const bool fused = path(items[0].n) != 0;
  const int bw = fused ? path(items[0].n) : ELIM_BLK;
  if (mode == 3 && !fused) {
    set_error("shifted Gauss-Jordan: n = %d exceeds the fused limit %d", items[0].n, elim_block_max_n(ft));
    return SPAND_EINVAL;
  }
  size_t nP = 0, nT = 0, nI = 0, nB = 0, nPB = 0;
  for (auto &d : items) {
    if (!fused) {
      nP += size_t(d.n) * ELIM_NB;
      nT += size_t(ELIM_NB) * d.ld;
    }
    nI += size_t(d.n);
    nB += size_t(bw) * d.ld;
    if (lu) nPB += size_t(d.n) * bw;
  }
  void *P = nullptr, *T = nullptr, *piv, *used, *TB = nullptr, *PB = nullptr;
  if (!fused) {
    SP_TRY(dalloc(&P, nP * fsize(ft), false));
    SP_TRY(dalloc(&T, nT * fsize(ft), false));
  }
  SP_TRY(dalloc(&piv, nI * 4, false));
  SP_TRY(dalloc(&used, nI * 4, false));
  SP_TRY(dalloc(&TB, nB * fsize(ft), false));
  if (lu) SP_TRY(dalloc(&PB, nPB * fsize(ft), false));
  SP_HIP(hipMemsetAsync(used, 0, nI * 4, stream));
  size_t oP = 0, oT = 0, oI = 0, oB = 0, oPB = 0;
  for (auto &d : items) {
    d.P = fused ? nullptr : (char *)P + oP * fsize(ft);
    d.T = fused ? nullptr : (char *)T + oT * fsize(ft);
    d.piv = (int32_t *)piv + oI;
    d.used = (int32_t *)used + oI;
    d.TB = (char *)TB + oB * fsize(ft);
    d.PB = lu ? (char *)PB + oPB * fsize(ft) : nullptr;
    if (!fused) {
      oP += size_t(d.n) * ELIM_NB;
      oT += size_t(ELIM_NB) * d.ld;
    }
    oI += size_t(d.n);
    oB += size_t(bw) * d.ld;
    if (lu) oPB += size_t(d.n) * bw;
  }
  ElimDesc *d_items;
  SP_TRY(upload(items, &d_items, false));
  const int nmax = items[0].n;
  auto nactive_at = [&](int k) {
    int na = 0;
    while (na < int(items.size()) && items[na].n > k) ++na;
    return na;
  };
  // elimination of block [k0, k0 + bw) in its own columns, then its
  // pivot rows of the other columns out to TB
  auto eliminate_block = [&](int k0) -> int {
    if (fused) {
      // one launch per 64-row size class (items are sorted by n, descending),
      // so that no workgroup carries waves without rows.  The class with
      // the most rows runs on the build stream, the others at the same time
      // on a second one (independent matrices): a class of a few large
      // matrices would otherwise hold the whole device for its long chain
      // of dependent steps.
      const int na = nactive_at(k0);
      std::vector<std::pair<int, int>> cls;
      for (int a = 0; a < na;) {
        int b = a + 1;
        while (b < na && cdiv(items[b].n, 64) == cdiv(items[a].n, 64)) ++b;
        cls.push_back({a, b});
        a = b;
      }
      if (cls.size() == 1 || one_stream) {
        for (const auto &c : cls)
          SP_TRY(launch_elim_block(ft, d_items + c.first, c.second - c.first, k0, mode,
                                   items[c.first].n, bw, d_flag, stream));
        return launch_elim_extract(ft, d_items, na, k0, bw, lu ? 1 : 0, stream);
      }
      size_t big = 0;
      for (size_t c = 1; c < cls.size(); ++c)
        if (int64_t(cls[c].second - cls[c].first) * items[cls[c].first].n >
            int64_t(cls[big].second - cls[big].first) * items[cls[big].first].n)
          big = c;
      if (!side2) SP_HIP(hipStreamCreateWithFlags(&side2, hipStreamNonBlocking));
      if (!cls_fork) SP_HIP(hipEventCreateWithFlags(&cls_fork, hipEventDisableTiming));
      if (!cls_join) SP_HIP(hipEventCreateWithFlags(&cls_join, hipEventDisableTiming));
      SP_HIP(hipEventRecord(cls_fork, stream));
      SP_HIP(hipStreamWaitEvent(side2, cls_fork, 0));
      int r = SPAND_OK;
      for (size_t c = 0; c < cls.size() && r == SPAND_OK; ++c)
        if (c != big)
          r = launch_elim_block(ft, d_items + cls[c].first, cls[c].second - cls[c].first, k0, mode,
                                items[cls[c].first].n, bw, d_flag, side2);
      if (r == SPAND_OK)
        r = launch_elim_block(ft, d_items + cls[big].first, cls[big].second - cls[big].first, k0,
                              mode, items[cls[big].first].n, bw, d_flag, stream);
      // joined even after a failed launch
      SP_HIP(hipEventRecord(cls_join, side2));
      SP_HIP(hipStreamWaitEvent(stream, cls_join, 0));
      SP_TRY(r);
    } else {
      for (int k = k0; k < std::min(nmax, k0 + ELIM_BLK); k += ELIM_NB) {
        const int nactive = nactive_at(k);
        const int max_tiles = int(cdiv(nmax, 64) * cdiv(ELIM_BLK, 64));   // the block's columns
        SP_TRY(launch_elim_step(ft, d_items, nactive, k, mode, max_tiles, d_flag, k0,
                                k0 + ELIM_BLK, stream));
        if (lu) SP_TRY(launch_elim_pb(ft, d_items, nactive, k, k0, stream));
      }
    }
    return launch_elim_extract(ft, d_items, nactive_at(k0), k0, bw, lu ? 1 : 0, stream);
  };
  // the first block runs while the products of all blocks are planned
  SP_TRY(eliminate_block(0));
  // trailing products of every block: columns [k0 + bw, ncols), and for
  // Gauss-Jordan also [0, k0).  In FP32 they run as strips of STRIP_TILES
  // tiles along N (one block of A staged once per strip).
  const size_t tsz = fsize(ft);
  constexpr int STRIP_TILES = 8;   // 256x256 p = 3 factorization: 2 tiles 395 ms, 4 386, 8 and 16 382
  const bool strip = ft == FType::F32;
  std::vector<GemmDesc> gd;
  std::vector<int32_t> ts(1, 0);
  std::vector<size_t> bstart;
  for (int k0 = 0; k0 < nmax; k0 += bw) {
    bstart.push_back(gd.size());
    for (auto &d : items) {
      if (d.n <= k0) break;
      const int wb = std::min(bw, d.n - k0);
      auto add = [&](int c_off, int width) {
        if (width <= 0) return;
        GemmDesc g{};
        g.A = lu ? d.PB : (char *)d.A + size_t(k0) * tsz;
        g.lda = lu ? bw : d.ld;
        g.B = (char *)d.TB + size_t(c_off) * tsz;
        g.C = (char *)d.A + size_t(c_off) * tsz;
        g.M = d.n;
        g.N = width;
        g.K = wb;
        g.ldb = g.ldc = d.ld;
        g.alpha = 1.0;
        g.beta = 1.0;
        gd.push_back(g);
        const int64_t ntn = cdiv(g.N, 64);
        ts.push_back(ts.back() + int32_t(cdiv(g.M, 64) * (strip ? cdiv(ntn, STRIP_TILES) : ntn)));
      };
      if (!lu) add(0, k0);
      add(k0 + bw, d.ncols - k0 - bw);
    }
  }
  bstart.push_back(gd.size());
  if (host_trace_on()) {
    double fl = 0.0, by = 0.0;
    for (const auto &d : gd) {
      fl += 2.0 * d.M * d.N * d.K;
      by += (double(d.M) * d.K + double(d.K) * d.N + 2.0 * d.M * d.N) * fsize(ft);
    }
    int nl = 0;
    for (size_t b = 0; b + 1 < bstart.size(); ++b) nl += bstart[b + 1] > bstart[b];
    std::fprintf(stderr, "[spand host] elim batch mode %d: %zu items nmax %d, %zu block products %.3f TFLOP %.3f GB, %d launches\n",
                 mode, items.size(), nmax, gd.size(), fl * 1e-12, by * 1e-9, nl);
  }
  // per block: uniform tile count, or the offset of its coarse index
  std::vector<int> buni(bstart.size(), 0);
  std::vector<size_t> boff(bstart.size(), 0);
  std::vector<int32_t> coarse;
  for (size_t b = 0; b + 1 < bstart.size(); ++b) {
    const size_t g0 = bstart[b], g1 = bstart[b + 1];
    if (g1 <= g0) continue;
    int uniform = ts[g0 + 1] - ts[g0];
    for (size_t q = g0; q < g1 && uniform > 0; ++q)
      if (ts[q + 1] - ts[q] != uniform) uniform = 0;
    buni[b] = uniform;
    boff[b] = coarse.size();
    if (!uniform) gemm_coarse(ts, g0, g1, coarse);
  }
  GemmDesc *d_gd;
  int32_t *d_ts, *d_coarse;
  SP_TRY(upload_parts({part(gd, &d_gd), part(ts, &d_ts), part(coarse, &d_coarse)}, false));
  for (int b = 0, k0 = 0; k0 < nmax; ++b, k0 += bw) {
    if (b > 0) SP_TRY(eliminate_block(k0));
    const size_t g0 = bstart[b], g1 = bstart[b + 1];
    if (g1 > g0) {   // this block's descriptors; their tile numbers start at ts[g0]
      double fl = 0.0, by = 0.0;
      gemm_work(gd.data() + g0, int(g1 - g0), fsize(ft), &fl, &by);
      SP_TRY(timed_launch(0, fl, by, [&]() {
        if (strip)
          return launch_gemm_strip(d_gd + g0, d_ts + g0, int(g1 - g0), ts[g1] - ts[g0], stream,
                                   ts[g0], buni[b], buni[b] ? nullptr : d_coarse + boff[b],
                                   STRIP_TILES);
        return launch_gemm(ft, d_gd + g0, d_ts + g0, int(g1 - g0), ts[g1] - ts[g0], stream, ts[g0],
                           0, buni[b], buni[b] ? nullptr : d_coarse + boff[b]);
      }));
    }
  }
  return SPAND_OK;
}

// Completion of the RRQR's orthogonal factors from their kept vectors, by
// Householder reconstruction (Ballard et al., IPDPS 2014), batched over the
// interfaces of a level.  With Q_c = [q_0 .. q_{k-1}] = [Q1; Q2] (Q1 k x k),
// V rows 0..k-1 holding the q_t:
//   M = Q1 - S, S = diag(s_j) chosen during the inversion (|pivot| >= 1);
//   G2' = Q2 M^-1 S, written to V rows k..m-1;
//   Q = [Q_c | E_c + Q_c G2'^T - [S G2'^T; 0]]   (E_c = columns k..m-1 of I;
//   S G2'^T = G2^T with G2 = Q2 M^-1, the rows of the reflector block).
// The right block is orthogonal to Q_c and completes it; with k = 0 Q = I.
int Factor::complete_q(int l, const LevelState &S, const std::vector<int> &ifs,
                       const std::vector<int32_t> &kg, const std::vector<void *> &Qm,
                       const std::vector<void *> &Vm) {
  const size_t tsz = fsize(ft);
  size_t nm = 0, ns = 0;
  for (size_t q = 0; q < ifs.size(); ++q) {
    const int m = S.size[ifs[q]], k = kg[q];
    if (k > 0 && k < m) {
      nm += size_t(k) * ld4(k);
      ns += size_t(k);
    }
  }
  void *Mb = nullptr, *Sg = nullptr;
  if (nm) {
    SP_TRY(dalloc(&Mb, nm * tsz, false));
    SP_TRY(dalloc(&Sg, ns * tsz, false));
  }
  std::vector<CopyDesc> c1, c2;
  std::vector<ElimDesc> gj;
  std::vector<ScaleDesc> sc, sc2;
  std::vector<GemmDesc> g1, g2;
  std::vector<EyeDesc> ey;
  size_t om = 0, os = 0;
  int maxe = 1;
  auto at = [&](void *p, size_t elems) { return (void *)((char *)p + elems * tsz); };
  for (size_t q = 0; q < ifs.size(); ++q) {
    const int s = ifs[q];
    const int m = S.size[s], k = kg[q];
    void *Qt = Vm[s], *Q = Qm[s];
    if (k < 0 || k > m) {
      set_error("RRQR returned %d kept vectors for an interface of size %d", k, m);
      return SPAND_EHIP;
    }
    if (k == 0) {
      ey.push_back(EyeDesc{Q, m, m});
      maxe = std::max(maxe, m);
      continue;
    }
    // Q(:, 0:k) = Q_c
    c2.push_back(CopyDesc{Qt, Q, m, k, m, m, 1, 0, 1.0});
    if (k == m) continue;
    const int ldm = ld4(k);
    void *M = at(Mb, om), *sg = at(Sg, os);
    om += size_t(k) * ldm;
    os += size_t(k);
    c1.push_back(CopyDesc{Qt, M, k, k, m, ldm, 1, 0, 1.0});     // M(i, c) = q_c[i]
    ElimDesc e{};
    e.A = M;
    e.n = e.ncols = k;
    e.ld = ldm;
    e.sg = sg;
    gj.push_back(e);
    sc.push_back(ScaleDesc{M, nullptr, sg, k, k, ldm, 0});     // M^-1 S
    GemmDesc a{};
    a.A = at(Qt, k);            // Q2(i, t) = q_t[k + i]
    a.transA = 1;
    a.lda = m;
    a.B = M;
    a.ldb = ldm;
    a.C = at(Qt, size_t(k) * m);
    a.ldc = m;
    a.M = m - k;
    a.N = k;
    a.K = k;
    a.alpha = 1.0;
    g1.push_back(a);
    // Q(0:k, k:m) = -S G2'^T ; Q(k:m, k:m) = I ; then Q(:, k:m) += Q_c G2'^T
    c2.push_back(CopyDesc{at(Qt, size_t(k) * m), at(Q, k), k, m - k, m, m, 1, 0, -1.0});
    sc2.push_back(ScaleDesc{at(Q, k), sg, nullptr, k, m - k, m, 0});
    ey.push_back(EyeDesc{at(Q, size_t(k) * m + k), m - k, m});
    maxe = std::max(maxe, m - k);
    GemmDesc b{};
    b.A = Qt;
    b.transA = 1;
    b.lda = m;
    b.B = at(Qt, size_t(k) * m);
    b.transB = 1;
    b.ldb = m;
    b.C = at(Q, k);
    b.ldc = m;
    b.M = m;
    b.N = m - k;
    b.K = k;
    b.alpha = 1.0;
    b.beta = 1.0;
    g2.push_back(b);
    acct(csys(l, s), 0.0, 2.0 * k * k * k + 2.0 * (m - k) * k * k + 2.0 * m * (m - k) * k);
  }
  SP_TRY(copy_batch(c1, 1));
  if (!gj.empty()) SP_TRY(elim_batch(gj, 3));
  if (!sc.empty()) {
    ScaleDesc *d_sc;
    SP_TRY(upload(sc, &d_sc, false));
    SP_TRY(launch_scale(ft, d_sc, int(sc.size()), stream));
  }
  SP_TRY(gemm_batch(g1));
  SP_TRY(copy_batch(c2, 1));
  if (!sc2.empty()) {
    ScaleDesc *d_sc;
    SP_TRY(upload(sc2, &d_sc, false));
    SP_TRY(launch_scale(ft, d_sc, int(sc2.size()), stream));
  }
  if (!ey.empty()) {
    EyeDesc *d_e;
    SP_TRY(upload(ey, &d_e, false));
    SP_TRY(launch_eye(ft, d_e, int(ey.size()), maxe, stream));
  }
  SP_TRY(gemm_batch(g2));
  return SPAND_OK;
}

// ------------------------------------------------------------------ timing
void Factor::mark(int phase) {
  const auto now = std::chrono::steady_clock::now();
  if (host_phase >= 0)
    ph_host_ms[host_phase] += std::chrono::duration<double, std::milli>(now - host_t).count();
  host_phase = phase;
  host_t = now;
  if (!timing) return;
  hipEvent_t e;
  if (event_get(&e) != SPAND_OK) return;
  (void)hipEventRecord(e, stream);
  events.push_back({phase, e});
}

void Factor::trace(const char *what, int l) {
  if (!host_trace_on()) return;
  const auto now = std::chrono::steady_clock::now();
  std::fprintf(stderr, "[spand host] L%-2d %-26s %8.2f ms\n", l, what,
               std::chrono::duration<double, std::milli>(now - trace_t).count());
  trace_t = now;
}

// ------------------------------------------------------------------ level 0
int Factor::level0(const NDResult &nd, LevelState &S) {
  const int b = bs;
  const auto &cl = nd.levels[0];
  const int ncl = int(cl.size());
  std::vector<int> ecl(K), epos(K);
  for (int c = 0; c < ncl; ++c)
    for (size_t q = 0; q < cl[c].elems.size(); ++q) {
      ecl[cl[c].elems[q]] = c;
      epos[cl[c].elems[q]] = int(q);
    }
  S.size.assign(ncl, 0);
  S.interior.assign(ncl, 0);
  for (int c = 0; c < ncl; ++c) {
    S.interior[c] = cl[c].interior;
    S.size[c] = int(cl[c].elems.size()) * b;
  }
  const size_t tsz = fsize(ft);
  const int64_t b2 = int64_t(b) * b;
  // ---- leaves: gather A_ss, invert
  std::vector<int> leaves;
  for (int c = 0; c < ncl; ++c)
    if (S.interior[c]) leaves.push_back(c);
  std::vector<void *> Ass(ncl, nullptr), Ainv(ncl, nullptr);
  {
    PlanArena pt, pk;
    std::vector<size_t> ot(ncl), ok(ncl);
    for (int s : leaves) {
      const int n = S.size[s];
      if (n > ELIM_MAXN || n > GEMV_MAXC) {
        set_error("leaf cluster of %d unknowns exceeds the kernel limit %d; use more levels", n,
                  ELIM_MAXN);
        return SPAND_EINVAL;
      }
      ot[s] = pt.add(size_t(n) * n * tsz);
      ok[s] = pk.add(size_t(n) * ld4(n) * tsz);
    }
    if (!leaves.empty()) {
      void *bt, *bk;
      SP_TRY(dalloc(&bt, pt.total, false));
      SP_TRY(dalloc(&bk, pk.total, true));
      SP_HIP(hipMemsetAsync(bt, 0, pt.total, stream));
      for (int s : leaves) {
        Ass[s] = (char *)bt + ot[s];
        Ainv[s] = (char *)bk + ok[s];
      }
    }
  }
  {
    // leaf blocks first: the leaf eliminations start while the interface
    // blocks are planned
    std::vector<GatherItem> gi;
    for (int s : leaves) {
      const int n = S.size[s];
      for (int e : cl[s].elems)
        for (int t = h_rowptr[e]; t < h_rowptr[e + 1]; ++t) {
          const int f = h_colind[t];
          if (ecl[f] == s)
            gi.push_back({(char *)Ass[s] + (size_t(epos[e]) * b * n + size_t(epos[f]) * b) * tsz,
                          blk_src(e, t), n, 0});
        }
    }
    mark(PH_GATHER);
    GatherItem *d_gi;
    SP_TRY(upload(gi, &d_gi, false));
    SP_TRY(launch_bsr_gather(ft, d_gi, int(gi.size()), b, stream));
    trace("leaf gather", 0);
  }
  mark(PH_LU);
  {
    std::vector<ElimDesc> items;
    for (int s : leaves) {
      ElimDesc d{};
      d.A = Ass[s];
      d.n = S.size[s];
      d.ncols = d.n;
      d.ld = d.n;
      d.pad = s;                 // owner leaf (elim_batch reorders the items)
      items.push_back(d);
    }
    SP_TRY(elim_batch(items, 0));
    trace("elim enqueue", 0);
    std::vector<RowGatherDesc> rg;
    for (auto &d : items) {
      // find the leaf whose A_ss this is
      RowGatherDesc g{};
      g.src = d.A;
      g.piv = d.piv;
      g.n = d.n;
      g.cols = d.n;
      g.lds = d.ld;
      g.ldd = d.n;
      g.colperm = 1;
      g.ldd = ld4(d.n);
      g.dst = Ainv[d.pad];
      rg.push_back(g);
    }
    RowGatherDesc *d_rg;
    SP_TRY(upload(rg, &d_rg, false));
    int mr = 0;
    for (auto &g : rg) mr = std::max(mr, g.n);
    SP_TRY(launch_row_gather(ft, d_rg, int(rg.size()), mr, stream));
  }
  // slot lists (the apply's sweeps), built while the leaves are eliminated
  S.slots.assign(ncl, {});
  for (int c = 0; c < ncl; ++c) {
    auto &sl = S.slots[c];
    sl.resize(size_t(S.size[c]));
    size_t o = 0;
    for (int e : cl[c].elems)
      for (int q = 0; q < b; ++q) sl[o++] = e * b + q;
  }
  SP_TRY(upload_level_slots(S));
  trace("L0 slots", 0);
  // ---- interface-pair blocks: adjacency among separator elements + fill
  // (cluster pairs as sorted unique keys ce * ncl + cf)
  std::vector<int64_t> pairs;
  std::vector<std::vector<int>> leaf_nbr(ncl);
  for (int e = 0; e < K; ++e) {
    for (int t = h_rowptr[e]; t < h_rowptr[e + 1]; ++t) {
      const int f = h_colind[t];
      const int ce = ecl[e], cf = ecl[f];
      if (!S.interior[ce] && !S.interior[cf]) pairs.push_back(int64_t(ce) * ncl + cf);
      if (S.interior[ce] && !S.interior[cf]) leaf_nbr[ce].push_back(cf);
      if (S.interior[ce] && S.interior[cf] && ce != cf) {
        set_error("block (%d,%d) couples two different leaves: the matrix pattern does not "
                  "match the element grid", e, f);
        return SPAND_EINVAL;
      }
    }
  }
  for (int s = 0; s < ncl; ++s) {
    auto &v = leaf_nbr[s];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    for (int n : v)
      for (int m : v) pairs.push_back(int64_t(n) * ncl + m);
  }
  for (int c = 0; c < ncl; ++c)
    if (!S.interior[c]) pairs.push_back(int64_t(c) * ncl + c);
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  trace("pair keys", 0);
  std::vector<Blk> pblk(pairs.size());
  {
    PlanArena pa;
    std::vector<size_t> offs;
    offs.reserve(pairs.size());
    for (int64_t key : pairs)
      offs.push_back(pa.add(size_t(S.size[key / ncl]) * S.size[key % ncl] * tsz));
    void *base;
    SP_TRY(dalloc(&base, pa.total, false));
    SP_HIP(hipMemsetAsync(base, 0, pa.total, stream));
    for (size_t q = 0; q < pairs.size(); ++q) {
      const int i = int(pairs[q] / ncl), j = int(pairs[q] % ncl);
      pblk[q] = Blk{(char *)base + offs[q], S.size[i], S.size[j]};
      S.blocks.emplace_hint(S.blocks.end(), std::make_pair(i, j), pblk[q]);
    }
  }
  trace("pair blocks", 0);
  auto pair_blk = [&](int i, int j) -> const Blk & {
    const int64_t key = int64_t(i) * ncl + j;
    return pblk[size_t(std::lower_bound(pairs.begin(), pairs.end(), key) - pairs.begin())];
  };
  {
    std::vector<GatherItem> gi;
    for (int e = 0; e < K; ++e) {
      const int ce = ecl[e];
      if (S.interior[ce]) continue;
      for (int t = h_rowptr[e]; t < h_rowptr[e + 1]; ++t) {
        const int f = h_colind[t];
        const int cf = ecl[f];
        if (S.interior[cf]) continue;
        const Blk &B = pair_blk(ce, cf);
        gi.push_back({(char *)B.p + (size_t(epos[e]) * b * B.cols + size_t(epos[f]) * b) * tsz,
                      blk_src(e, t), B.cols, 0});
      }
    }
    mark(PH_GATHER);
    GatherItem *d_gi;
    SP_TRY(upload(gi, &d_gi, false));
    SP_TRY(launch_bsr_gather(ft, d_gi, int(gi.size()), b, stream));
    trace("interface gather", 0);
  }
  mark(PH_SCHUR);
  // ---- couplings (separator element e, leaf element f) per leaf
  struct Coup {
    int e, f;
    int64_t t_ef, t_fe;
  };
  std::vector<std::vector<Coup>> coup(ncl);
  for (int f = 0; f < K; ++f) {
    const int cf = ecl[f];
    if (!S.interior[cf]) continue;
    for (int t = h_rowptr[f]; t < h_rowptr[f + 1]; ++t) {
      const int e = h_colind[t];
      if (S.interior[ecl[e]]) continue;
      // mirror block (e, f)
      int64_t tm = -1;
      for (int q = h_rowptr[e]; q < h_rowptr[e + 1]; ++q)
        if (h_colind[q] == f) tm = q;
      if (tm < 0) {
        set_error("block pattern is not structurally symmetric at (%d,%d)", e, f);
        return SPAND_EINVAL;
      }
      coup[cf].push_back({e, f, tm, t});
    }
  }
  // the coupling blocks in factor precision, leaf by leaf (A[e, f] then
  // A[f, e] for each coupling): operands of the Schur products below and
  // stored for the sweeps
  std::vector<size_t> cpl0(ncl, 0);
  void *cb = nullptr;
  size_t ncp = 0;
  {
    for (int s : leaves) {
      cpl0[s] = ncp;
      ncp += coup[s].size();
    }
    if (ncp) SP_TRY(dalloc(&cb, ncp * 2 * b2 * tsz, true));
    std::vector<GatherItem> cc;
    cc.reserve(2 * ncp);
    for (int s : leaves)
      for (size_t i = 0; i < coup[s].size(); ++i) {
        const auto &c = coup[s][i];
        const size_t q = cpl0[s] + i;
        cc.push_back({(char *)cb + (2 * q) * b2 * tsz, blk_src(c.e, c.t_ef), b, 0});
        cc.push_back({(char *)cb + (2 * q + 1) * b2 * tsz, blk_src(c.f, c.t_fe), b, 0});
      }
    if (!cc.empty()) {
      GatherItem *d_cc;
      SP_TRY(upload(cc, &d_cc, false));
      SP_TRY(launch_bsr_gather(ft, d_cc, int(cc.size()), b, stream));
    }
    trace("coupling copies", 0);
  }
  auto cpl_ns = [&](int s, size_t i) { return (void *)((char *)cb + (2 * (cpl0[s] + i)) * b2 * tsz); };
  auto cpl_sn = [&](int s, size_t i) { return (void *)((char *)cb + (2 * (cpl0[s] + i) + 1) * b2 * tsz); };
  {
    // Schur targets (e_a, e_c); the items of a target stay in (leaf, a, c)
    // order.  Targets get ids through short per-element lists, then a
    // counting sort places the items (no ordered map on this hot path).
    std::vector<std::vector<std::pair<int, int>>> tl(K);     // e_a -> (e_c, id)
    std::vector<std::pair<int, int>> tkey;                    // id -> (e_a, e_c)
    std::vector<int> cnt;
    size_t nitems = 0;
    for (int s : leaves) nitems += coup[s].size() * coup[s].size();
    std::vector<int> item_tid;
    item_tid.reserve(nitems);
    for (int s : leaves) {
      const auto &C = coup[s];
      for (const auto &ca : C) {
        auto &v = tl[ca.e];
        for (const auto &cc : C) {
          int id = -1;
          for (const auto &p : v)
            if (p.first == cc.e) { id = p.second; break; }
          if (id < 0) {
            id = int(tkey.size());
            v.push_back({cc.e, id});
            tkey.push_back({ca.e, cc.e});
            cnt.push_back(0);
          }
          ++cnt[id];
          item_tid.push_back(id);
        }
      }
    }
    trace("schur target ids", 0);
    std::vector<SchurGroup> groups(tkey.size());
    std::vector<SchurItem> items(nitems);
    {
      // consecutive targets come from one leaf's few neighbour clusters: a
      // small direct-mapped cache in front of the cluster-pair search
      struct PairHit {
        int64_t key;
        const Blk *blk;
      };
      std::vector<PairHit> hit(256, PairHit{-1, nullptr});
      int off = 0;
      for (size_t id = 0; id < tkey.size(); ++id) {
        const int ea = tkey[id].first, ec = tkey[id].second;
        const int64_t pk = int64_t(ecl[ea]) * ncl + ecl[ec];
        PairHit &h = hit[size_t(uint64_t(pk) * 0x9E3779B97F4A7C15ull >> 56)];
        if (h.key != pk) h = PairHit{pk, &pair_blk(ecl[ea], ecl[ec])};
        const Blk &B = *h.blk;
        SchurGroup &g = groups[id];
        g.target = (char *)B.p + (size_t(epos[ea]) * b * B.cols + size_t(epos[ec]) * b) * tsz;
        g.ldt = B.cols;
        g.item_begin = off;
        off += cnt[id];
        g.item_end = g.item_begin;      // advanced while filling
      }
    }
    trace("schur groups", 0);
    {
      size_t q = 0;
      for (int s : leaves) {
        const auto &C = coup[s];
        const int n = S.size[s];
        for (size_t ia = 0; ia < C.size(); ++ia)
          for (size_t ic = 0; ic < C.size(); ++ic) {
            const auto &ca = C[ia], &cc = C[ic];
            SchurItem it{};
            it.A1 = cpl_ns(s, ia);     // A[e_a, f_a]
            it.A2 = cpl_sn(s, ic);     // A[f_c, e_c]
            it.Y = (char *)Ainv[s] + (size_t(epos[ca.f]) * b * ld4(n) + size_t(epos[cc.f]) * b) * tsz;
            it.ldy = ld4(n);
            SchurGroup &g = groups[item_tid[q++]];
            items[g.item_end++] = it;
          }
      }
    }
    trace("schur items", 0);
    SchurGroup *d_g;
    SchurItem *d_i;
    SP_TRY(upload_parts({part(groups, &d_g), part(items, &d_i)}, false));
    {
      // per coupling pair: two b x b products; A1, Y, A2 read, plus every
      // target block read and written once
      const double fl = double(items.size()) * 4.0 * b * b * b;
      const double by = (double(items.size()) * 3.0 + 2.0 * double(groups.size())) * double(b) * b *
                        double(tsz);
      SP_TRY(timed_launch(1, fl, by, [&]() {
        return launch_schur_elem(ft, b, d_g, int(groups.size()), d_i, stream);
      }));
    }
    trace("schur plan+launch", 0);
    for (int s : leaves) acct(csys(0, s), 0.0, double(coup[s].size()) * coup[s].size() * 4.0 * b * b * b);
  }
  // ---- stored couplings and apply descriptors of level 0
  ApplyLevel &AL = lv[0];
  {
    // couplings indexed by separator element e and by leaf element f
    // (counting sort, stable: a key's couplings keep their (leaf, coupling)
    // order, which is the order the pull kernels accumulate them in)
    std::vector<int> off_e(size_t(K) + 1, 0), off_f(size_t(K) + 1, 0);
    for (int s : leaves)
      for (const auto &c : coup[s]) {
        ++off_e[size_t(c.e) + 1];
        ++off_f[size_t(c.f) + 1];
      }
    for (int e = 0; e < K; ++e) {
      off_e[size_t(e) + 1] += off_e[size_t(e)];
      off_f[size_t(e) + 1] += off_f[size_t(e)];
    }
    std::vector<std::pair<int, size_t>> by_e(ncp), by_f(ncp);   // (partner, coupling index)
    {
      std::vector<int> ce(off_e.begin(), off_e.end() - 1), cf(off_f.begin(), off_f.end() - 1);
      for (int s : leaves)
        for (size_t i = 0; i < coup[s].size(); ++i) {
          const auto &c = coup[s][i];
          by_e[size_t(ce[c.e]++)] = {c.f, cpl0[s] + i};
          by_f[size_t(cf[c.f]++)] = {c.e, cpl0[s] + i};
        }
    }
    // one pull group per key element; half = 0 takes A[e, f], 1 A[f, e]
    auto build = [&](const std::vector<int> &off, const std::vector<std::pair<int, size_t>> &lst,
                     int half, int trans, std::vector<PullGroup> &G, std::vector<PullItem> &I,
                     std::vector<int> &gs, bool all_leaf) {
      std::vector<int> keys;
      if (all_leaf) {
        for (int s : leaves)
          for (int f : cl[s].elems) keys.push_back(f);
        std::sort(keys.begin(), keys.end());
      } else {
        for (int e = 0; e < K; ++e)
          if (off[size_t(e) + 1] > off[size_t(e)]) keys.push_back(e);
      }
      G.reserve(keys.size());
      I.reserve(lst.size());
      gs.reserve(keys.size());
      for (int key : keys) {
        PullGroup g{};
        g.oslot = d_iota + int64_t(key) * b;
        g.rows = b;
        g.item_begin = int(I.size());
        for (int t = off[size_t(key)]; t < off[size_t(key) + 1]; ++t) {
          PullItem p{};
          p.B = (char *)cb + (2 * lst[size_t(t)].second + size_t(half)) * b2 * tsz;
          p.islot = d_iota + int64_t(lst[size_t(t)].first) * b;
          p.rows = p.cols = b;
          p.ldb = b;
          p.trans = trans;
          I.push_back(p);
        }
        g.item_end = int(I.size());
        G.push_back(g);
        gs.push_back(members.empty() ? 0 : esys[size_t(key)]);
      }
    };
    // each set is uploaded at the next rank read-back
    auto emit = [&](const std::vector<int> &off, const std::vector<std::pair<int, size_t>> &lst,
                    int half, int trans, bool all_leaf, PullSet ApplyLevel::*which) {
      std::vector<PullGroup> G;
      std::vector<PullItem> I;
      std::vector<int> gs;
      build(off, lst, half, trans, G, I, gs, all_leaf);
      defer([this, &AL, which, G = std::move(G), I = std::move(I), gs = std::move(gs)]() {
        SP_TRY((AL.*which).set(*this, G, I));
        return member_pull(0, which, G, I, gs);
      });
    };
    emit(off_e, by_e, 0, 0, false, &ApplyLevel::fw);    // x_n -= A_ns t_s
    emit(off_f, by_f, 1, 0, false, &ApplyLevel::bw);    // x_s -= A_sn x_n
    emit(off_e, by_e, 1, 1, false, &ApplyLevel::tfw);   // x_n -= A_sn^T x_s
    emit(off_f, by_f, 0, 1, true, &ApplyLevel::tbw);    // t_s = A_ns^T x_n
    trace("pull sets", 0);
    std::vector<GemvDesc> gv;
    std::vector<const std::vector<int32_t> *> os;
    std::vector<int> vs;
    for (int s : leaves) {
      GemvDesc d{};
      d.A = Ainv[s];
      d.islot = d.oslot = S.d_slots[s];
      d.rows = d.cols = S.size[s];
      d.lda = ld4(S.size[s]);
      gv.push_back(d);
      os.push_back(&S.slots[s]);
      vs.push_back(csys(0, s));
      acct(csys(0, s), double(S.size[s]) * S.size[s] * tsz * 2, 0.0);   // A_ss^-1: both sweeps
    }
    // band height of the sweep GEMVs: autotuned once per (precision, b)
    defer([this, &AL, gv, os, vs]() -> int {
      void *tin;
      SP_TRY(dalloc(&tin, size_t(N) * 8, false));
      SP_HIP(hipMemsetAsync(tin, 0, size_t(N) * 8, stream));
      auto build_set = [&](int R, GemvSet &g) { return g.set(*this, gv, os, 0, R); };
      SP_TRY(autotune_gemv(ft, bs, build_set, (double *)tin, d_tbuf, stream, &gemv_rows));
      SP_TRY(AL.inv.set(*this, gv, os, 0));
      SP_TRY(AL.invT.set(*this, gv, os, 1));
      SP_TRY(member_gemv(0, &ApplyLevel::inv, gv, os, vs, 0));
      return member_gemv(0, &ApplyLevel::invT, gv, os, vs, 1);
    });
    trace("inverse sweep sets", 0);
    for (int s : leaves)   // A_ns forward, A_sn backward; the inversion
      acct(csys(0, s), double(coup[s].size()) * 2 * b2 * tsz,
           2.0 * double(S.size[s]) * S.size[s] * S.size[s]);
  }
  for (int s : leaves) S.size[s] = 0;   // eliminated
  return SPAND_OK;
}

int PullSet::set(Factor &F, std::vector<PullGroup> G, const std::vector<PullItem> &I) {
  n = int(G.size());
  if (!n) return SPAND_OK;
  trans = -1;
  std::vector<PullChunk> ch;
  for (size_t gi = 0; gi < G.size(); ++gi) {
    PullGroup &g = G[gi];
    bool vec = true;
    for (int it = g.item_begin; it < g.item_end; ++it) {
      const PullItem &p = I[it];
      if (trans < 0) trans = p.trans;
      if (p.trans != trans) {
        set_error("a pull set mixes transposed and plain blocks");
        return SPAND_EINVAL;
      }
      if (p.cols > GEMV_MAXC) {
        set_error("coupling block with %d columns exceeds the sweep kernel limit %d", p.cols, GEMV_MAXC);
        return SPAND_EINVAL;
      }
      if (p.ldb % 4 != 0 || reinterpret_cast<uintptr_t>(p.B) % 16 != 0) vec = false;
    }
    g.pad = vec ? 1 : 0;
    for (int r0 = 0; r0 < g.rows; r0 += PULL_ROWS)
      ch.push_back(PullChunk{int32_t(gi), r0, std::min(PULL_ROWS, g.rows - r0), 0});
  }
  if (trans < 0) trans = 0;
  nchunks = int(ch.size());
  if (host_trace_on()) {
    double bytes = 0.0;
    int maxc = 0;
    for (const auto &p : I) {
      bytes += double(p.rows) * p.cols * fsize(F.ft);
      maxc = std::max(maxc, p.cols);
    }
    std::fprintf(stderr, "[spand host] pull set: %zu groups %d chunks %zu items %.3f GB, max cols %d, trans %d\n",
                 G.size(), nchunks, I.size(), bytes * 1e-9, maxc, trans);
  }
  SP_TRY(F.upload_parts({Factor::part(G, &d_groups), Factor::part(I, &d_items),
                         Factor::part(ch, &d_chunks)},
                        true));
  return SPAND_OK;
}

int GemvSet::set(Factor &F, std::vector<GemvDesc> items,
                 const std::vector<const std::vector<int32_t> *> &oslots, int trans, int rows) {
  n = int(items.size());
  if (!n) return SPAND_OK;
  int R = trans ? 256 : (rows > 0 ? rows : F.gemv_rows);
  if (!trans && rows <= 0) {
    // a set of fewer than 4096 bands (16 per CU: the upper levels) takes
    // shorter bands, down to one 16-row pass per workgroup: its launch is
    // bound by the passes' latency, not by bytes.  Each row's sum is the
    // same whatever the band.
    int64_t tot = 0;
    for (const auto &d : items) tot += d.rows;
    while (R > 16 && tot < int64_t(R) * 4096) R /= 2;
  }
  std::vector<GemvChunk> ch;
  std::vector<int32_t> sl;
  for (int i = 0; i < n; ++i) {
    items[i].trans = trans;
    for (int r0 = 0; r0 < items[i].rows; r0 += R)
      ch.push_back(GemvChunk{i, r0, std::min(R, items[i].rows - r0), 0});
    sl.insert(sl.end(), oslots[i]->begin(), oslots[i]->begin() + items[i].rows);
  }
  nchunks = int(ch.size());
  nslots = int64_t(sl.size());
  SP_TRY(F.upload_parts({Factor::part(items, &d_items), Factor::part(ch, &d_chunks),
                         Factor::part(sl, &d_slots)},
                        true));
  return SPAND_OK;
}

// ------------------------------------------------------------------ dense interior elimination (l >= 1)
int Factor::eliminate_dense(int l, LevelState &S) {
  const size_t tsz = fsize(ft);
  const int ncl = int(S.size.size());
  ApplyLevel &AL = lv[l];
  std::vector<int> ints;
  for (int c = 0; c < ncl; ++c)
    if (S.interior[c] && S.size[c] > 0) ints.push_back(c);
  if (ints.empty()) return SPAND_OK;
  std::vector<std::vector<int>> nb(ncl);
  for (auto &kv : S.blocks) {
    const int i = kv.first.first, j = kv.first.second;
    if (i != j && S.size[i] > 0 && S.size[j] > 0) nb[i].push_back(j);
  }
  for (auto &v : nb) std::sort(v.begin(), v.end());
  mark(PH_LU);
  std::vector<void *> Ainv(ncl, nullptr);
  std::vector<ElimDesc> items;
  for (int s : ints) {
    const int n = S.size[s];
    if (n > ELIM_MAXN || n > GEMV_MAXC) {
      set_error("interior cluster of %d unknowns at level %d exceeds the kernel limit %d; "
                "increase eps or the number of levels", n, l, ELIM_MAXN);
      return SPAND_EINVAL;
    }
    SP_TRY(dalloc(&Ainv[s], size_t(n) * ld4(n) * tsz, true));
    ElimDesc d{};
    d.A = S.blocks.at({s, s}).p;
    d.n = n;
    d.ncols = n;
    d.ld = n;
    d.pad = s;                   // owner cluster (elim_batch reorders the items)
    items.push_back(d);
    acct(csys(l, s), double(n) * n * tsz * 2, 2.0 * double(n) * n * n);   // A_ss^-1: both sweeps
  }
  SP_TRY(elim_batch(items, 0));
  trace("elim enqueue", l);
  {
    std::vector<RowGatherDesc> rg;
    int mr = 0;
    for (auto &d : items) {
      RowGatherDesc g{};
      g.src = d.A;
      g.piv = d.piv;
      g.n = g.cols = d.n;
      g.lds = d.n;
      g.ldd = ld4(d.n);
      g.colperm = 1;
      g.dst = Ainv[d.pad];
      rg.push_back(g);
      mr = std::max(mr, d.n);
    }
    RowGatherDesc *d_rg;
    SP_TRY(upload(rg, &d_rg, false));
    SP_TRY(launch_row_gather(ft, d_rg, int(rg.size()), mr, stream));
  }
  mark(PH_SCHUR);
  // X_sm = A_ss^-1 A_sm.  Per interior s, its neighbours' blocks and
  // products are kept in the order of nb[s] (map nodes do not move when
  // blocks are added later).
  std::vector<std::vector<void *>> X(ncl);
  std::vector<std::vector<const Blk *>> Bns(ncl), Bsn(ncl);   // A_ns, A_sn
  {
    std::vector<GemmDesc> gm;
    for (int s : ints) {
      const size_t nn = nb[s].size();
      X[s].resize(nn);
      Bns[s].resize(nn);
      Bsn[s].resize(nn);
      for (size_t i = 0; i < nn; ++i) {
        const int m = nb[s][i];
        const Blk &B = S.blocks.at({s, m});
        Bsn[s][i] = &B;
        Bns[s][i] = &S.blocks.at({m, s});
        void *x;
        SP_TRY(dalloc(&x, size_t(B.rows) * B.cols * tsz, false));
        X[s][i] = x;
        GemmDesc g{};
        g.A = Ainv[s];
        g.B = B.p;
        g.C = x;
        g.M = B.rows;
        g.N = B.cols;
        g.K = B.rows;
        g.lda = ld4(B.rows);
        g.ldb = B.cols;
        g.ldc = B.cols;
        g.alpha = 1.0;
        g.beta = 0.0;
        gm.push_back(g);
        acct(csys(l, s), 0.0, 2.0 * double(B.rows) * B.rows * B.cols);
      }
    }
    SP_TRY(gemm_batch(gm));
    trace("gemm", l);
  }
  // fill blocks and deterministic rounds of A_nm -= A_ns X_sm: the
  // contributions to a target (n, m) come in ascending order of s (round r
  // takes the r-th), targets in ascending (n, m)
  struct Contrib {
    int64_t key;          // n * ncl + m
    int s, in, im;        // interior, positions of n and m in nb[s]
  };
  std::vector<Contrib> contrib;
  for (int s : ints)
    for (int in = 0; in < int(nb[s].size()); ++in)
      for (int im = 0; im < int(nb[s].size()); ++im)
        contrib.push_back({int64_t(nb[s][in]) * ncl + nb[s][im], s, in, im});
  std::stable_sort(contrib.begin(), contrib.end(),
                   [](const Contrib &x, const Contrib &y) { return x.key < y.key; });
  std::vector<size_t> run;          // start of every target's contributions
  for (size_t q = 0; q < contrib.size(); ++q)
    if (q == 0 || contrib[q].key != contrib[q - 1].key) run.push_back(q);
  run.push_back(contrib.size());
  const size_t ntarget = run.size() - 1;
  {
    PlanArena pa;
    std::vector<std::pair<std::pair<int, int>, size_t>> offs;
    for (size_t t = 0; t < ntarget; ++t) {
      const int n = int(contrib[run[t]].key / ncl), m = int(contrib[run[t]].key % ncl);
      if (!S.blocks.count({n, m}))
        offs.push_back({{n, m}, pa.add(size_t(S.size[n]) * S.size[m] * tsz)});
    }
    if (!offs.empty()) {
      void *base;
      SP_TRY(dalloc(&base, pa.total, false));
      SP_HIP(hipMemsetAsync(base, 0, pa.total, stream));
      for (auto &o : offs)
        S.blocks[o.first] = Blk{(char *)base + o.second, S.size[o.first.first], S.size[o.first.second]};
    }
  }
  std::vector<const Blk *> tblk(ntarget);
  size_t rounds = 0;
  for (size_t t = 0; t < ntarget; ++t) {
    const int n = int(contrib[run[t]].key / ncl), m = int(contrib[run[t]].key % ncl);
    tblk[t] = &S.blocks.at({n, m});
    rounds = std::max(rounds, run[t + 1] - run[t]);
  }
  for (size_t r = 0; r < rounds; ++r) {
    std::vector<GemmDesc> gm;
    for (size_t t = 0; t < ntarget; ++t) {
      if (run[t + 1] - run[t] <= r) continue;
      const Contrib &c = contrib[run[t] + r];
      const Blk &Ans = *Bns[c.s][c.in];
      const Blk &T = *tblk[t];
      GemmDesc g{};
      g.A = Ans.p;
      g.B = X[c.s][c.im];
      g.C = T.p;
      g.M = T.rows;
      g.N = T.cols;
      g.K = Ans.cols;
      g.lda = Ans.cols;
      g.ldb = T.cols;
      g.ldc = T.cols;
      g.alpha = -1.0;
      g.beta = 1.0;
      gm.push_back(g);
      acct(csys(l, c.s), 0.0, 2.0 * double(T.rows) * T.cols * Ans.cols);
    }
    SP_TRY(gemm_batch(gm));
    trace("gemm", l);
  }
  // apply descriptors
  std::vector<GemvDesc> gv;
  std::vector<const std::vector<int32_t> *> os;
  std::vector<int> vs;
  for (int s : ints) {
    GemvDesc d{};
    d.A = Ainv[s];
    d.islot = d.oslot = S.d_slots[s];
    d.rows = d.cols = S.size[s];
    d.lda = ld4(S.size[s]);
    gv.push_back(d);
    os.push_back(&S.slots[s]);
    vs.push_back(csys(l, s));
  }
  defer([this, &AL, gv, os, vs, l]() {
    SP_TRY(AL.inv.set(*this, gv, os, 0));
    return member_gemv(l, &ApplyLevel::inv, gv, os, vs, 0);
  });
  defer([this, &AL, gv, os, vs, l]() {
    SP_TRY(AL.invT.set(*this, gv, os, 1));
    return member_gemv(l, &ApplyLevel::invT, gv, os, vs, 1);
  });
  std::vector<std::vector<PullItem>> fw(ncl), tfw(ncl);   // by neighbour n
  std::vector<PullGroup> G;
  std::vector<PullItem> I;
  std::vector<PullGroup> G2;
  std::vector<PullItem> I2;
  for (int s : ints)
    for (size_t i = 0; i < nb[s].size(); ++i) {
      const int n = nb[s][i];
      const Blk &Ans = *Bns[s][i];   // |n| x |s|
      const Blk &Asn = *Bsn[s][i];   // |s| x |n|
      PullItem p{};
      p.B = Ans.p;
      p.islot = S.d_slots[s];
      p.rows = S.size[n];
      p.cols = S.size[s];
      p.ldb = Ans.cols;
      p.trans = 0;
      fw[n].push_back(p);
      PullItem q{};
      q.B = Asn.p;
      q.islot = S.d_slots[s];
      q.rows = S.size[n];
      q.cols = S.size[s];
      q.ldb = Asn.cols;
      q.trans = 1;
      tfw[n].push_back(q);
      acct(csys(l, s), double(Ans.rows) * Ans.cols * tsz + double(Asn.rows) * Asn.cols * tsz, 0.0);
      if (S.size[n] > PULL_MAXR || S.size[s] > GEMV_MAXC) {
        set_error("coupling block %dx%d exceeds the sweep kernel limit", S.size[n], S.size[s]);
        return SPAND_EINVAL;
      }
    }
  std::vector<int> gs, gs2;
  for (int n = 0; n < ncl; ++n) {
    if (fw[n].empty()) continue;
    PullGroup g{};
    g.oslot = S.d_slots[n];
    g.rows = S.size[n];
    g.item_begin = int(I.size());
    I.insert(I.end(), fw[n].begin(), fw[n].end());
    g.item_end = int(I.size());
    G.push_back(g);
    gs.push_back(csys(l, n));
  }
  defer([this, &AL, G, I, gs, l]() {
    SP_TRY(AL.fw.set(*this, G, I));
    return member_pull(l, &ApplyLevel::fw, G, I, gs);
  });
  G.clear();
  I.clear();
  gs.clear();
  for (int n = 0; n < ncl; ++n) {
    if (tfw[n].empty()) continue;
    PullGroup g{};
    g.oslot = S.d_slots[n];
    g.rows = S.size[n];
    g.item_begin = int(I.size());
    I.insert(I.end(), tfw[n].begin(), tfw[n].end());
    g.item_end = int(I.size());
    G.push_back(g);
    gs.push_back(csys(l, n));
  }
  defer([this, &AL, G, I, gs, l]() {
    SP_TRY(AL.tfw.set(*this, G, I));
    return member_pull(l, &ApplyLevel::tfw, G, I, gs);
  });
  G.clear();
  I.clear();
  gs.clear();
  for (int s : ints) {
    PullGroup g{}, g2{};
    g.oslot = g2.oslot = S.d_slots[s];
    g.rows = g2.rows = S.size[s];
    g.item_begin = int(I.size());
    g2.item_begin = int(I2.size());
    for (size_t i = 0; i < nb[s].size(); ++i) {
      const int n = nb[s][i];
      const Blk &Asn = *Bsn[s][i];
      const Blk &Ans = *Bns[s][i];
      PullItem p{};
      p.B = Asn.p;
      p.islot = S.d_slots[n];
      p.rows = S.size[s];
      p.cols = S.size[n];
      p.ldb = Asn.cols;
      p.trans = 0;
      I.push_back(p);
      PullItem q{};
      q.B = Ans.p;
      q.islot = S.d_slots[n];
      q.rows = S.size[s];
      q.cols = S.size[n];
      q.ldb = Ans.cols;
      q.trans = 1;
      I2.push_back(q);
    }
    g.item_end = int(I.size());
    g2.item_end = int(I2.size());
    if (g.item_end > g.item_begin) {
      G.push_back(g);
      gs.push_back(csys(l, s));
    }
    G2.push_back(g2);
    gs2.push_back(csys(l, s));
  }
  defer([this, &AL, G, I, gs, l]() {
    SP_TRY(AL.bw.set(*this, G, I));
    return member_pull(l, &ApplyLevel::bw, G, I, gs);
  });
  trace("sweep sets", l);
  defer([this, &AL, G2, I2, gs2, l]() {
    SP_TRY(AL.tbw.set(*this, G2, I2));
    return member_pull(l, &ApplyLevel::tbw, G2, I2, gs2);
  });
  // eliminated clusters leave the trailing matrix
  for (int s : ints) {
    for (int n : nb[s]) {
      S.blocks.erase({s, n});
      S.blocks.erase({n, s});
    }
    S.blocks.erase({s, s});
    S.size[s] = 0;
  }
  return SPAND_OK;
}

// ------------------------------------------------------------------ interfaces (any level < top)
int Factor::sparsify(int l, const NDResult &nd, LevelState &S, LevelState &Nx) {
  const size_t tsz = fsize(ft);
  const int ncl = int(S.size.size());
  ApplyLevel &AL = lv[l];
  std::vector<int> ifs;
  for (int c = 0; c < ncl; ++c)
    if (!S.interior[c] && S.size[c] > 0) ifs.push_back(c);
  std::vector<std::vector<int>> nb(ncl);
  for (auto &kv : S.blocks) {
    const int i = kv.first.first, j = kv.first.second;
    if (i != j && S.size[i] > 0 && S.size[j] > 0) nb[i].push_back(j);
  }
  for (auto &v : nb) std::sort(v.begin(), v.end());
  for (int s : ifs) {
    const int m = S.size[s];
    if (m > QRCP_MAXM || m > ELIM_MAXN) {
      set_error("interface of %d unknowns at level %d exceeds the kernel limit %d; "
                "increase eps or the number of levels", m, l, QRCP_MAXM);
      return SPAND_EINVAL;
    }
  }
  // ---- scaling: [A_ss | I] -> U, L^-1 P^T ; U^-1 ; split diag(U)
  mark(PH_SCALE);
  std::vector<void *> Aug(ncl), Ust(ncl), Lh(ncl), Sv(ncl), Si(ncl);
  std::vector<ElimDesc> items;
  std::vector<CopyDesc> cps;
  std::vector<EyeDesc> eyes;
  int maxm = 0;
  for (int s : ifs) {
    const int m = S.size[s];
    maxm = std::max(maxm, m);
    SP_TRY(dalloc(&Aug[s], size_t(m) * 2 * m * tsz, false));
    SP_TRY(dalloc(&Ust[s], size_t(m) * m * tsz, false));
    SP_TRY(dalloc(&Lh[s], size_t(m) * m * tsz, false));
    SP_TRY(dalloc(&Sv[s], size_t(m) * tsz, false));
    SP_TRY(dalloc(&Si[s], size_t(m) * tsz, false));
    CopyDesc d{};
    d.src = S.blocks.at({s, s}).p;
    d.dst = Aug[s];
    d.rows = d.cols = m;
    d.lds = m;
    d.ldd = 2 * m;
    d.scale = 1.0;
    cps.push_back(d);
    EyeDesc e{};
    e.A = (char *)Aug[s] + size_t(m) * tsz;
    e.n = m;
    e.ld = 2 * m;
    eyes.push_back(e);
    ElimDesc el{};
    el.A = Aug[s];
    el.n = m;
    el.ncols = 2 * m;
    el.ld = 2 * m;
    el.pad = s;                  // owner interface (elim_batch reorders the items)
    items.push_back(el);
    acct(csys(l, s), 0.0, 4.0 * double(m) * m * m);
  }
  SP_TRY(copy_batch(cps, 1));
  {
    EyeDesc *d_e;
    SP_TRY(upload(eyes, &d_e, false));
    SP_TRY(launch_eye(ft, d_e, int(eyes.size()), maxm, stream));
  }
  SP_TRY(elim_batch(items, 1));
  trace("scale LU enqueue", l);
  {
    std::vector<RowGatherDesc> rg;
    for (auto &d : items) {
      const int s = d.pad;
      RowGatherDesc g{};
      g.src = d.A;
      g.piv = d.piv;
      g.n = g.cols = d.n;
      g.lds = d.ld;
      g.ldd = d.n;
      g.colperm = 0;
      g.col_off = 0;
      g.dst = Ust[s];
      rg.push_back(g);
      g.col_off = d.n;
      g.dst = Lh[s];
      rg.push_back(g);
    }
    RowGatherDesc *d_rg;
    SP_TRY(upload(rg, &d_rg, false));
    SP_TRY(launch_row_gather(ft, d_rg, int(rg.size()), maxm, stream));
    // diagonal split: Sv = sqrt|u_jj|, Si = 1/Sv
    std::vector<DiagDesc> dd;
    for (int s : ifs) dd.push_back(DiagDesc{Ust[s], Sv[s], Si[s], S.size[s], S.size[s]});
    DiagDesc *d_dd;
    SP_TRY(upload(dd, &d_dd, false));
    SP_TRY(launch_diag_split(ft, d_dd, int(dd.size()), stream));
    // U^-1 in place (Gauss-Jordan without pivoting; no permutation to undo)
    std::vector<ElimDesc> ui;
    for (int s : ifs) {
      ElimDesc el{};
      el.A = Ust[s];
      el.n = el.ncols = el.ld = S.size[s];
      ui.push_back(el);
      acct(csys(l, s), 0.0, 2.0 * double(S.size[s]) * S.size[s] * S.size[s]);
    }
    SP_TRY(elim_batch(ui, 2));
    // Lh^-1 P^T = S^-1 (L^-1 P^T) ; Uh^-1 = U^-1 S
    std::vector<ScaleDesc> sc;
    for (int s : ifs) {
      sc.push_back(ScaleDesc{Lh[s], Si[s], nullptr, S.size[s], S.size[s], S.size[s], 0});
      sc.push_back(ScaleDesc{Ust[s], nullptr, Sv[s], S.size[s], S.size[s], S.size[s], 0});
    }
    ScaleDesc *d_sc;
    SP_TRY(upload(sc, &d_sc, false));
    SP_TRY(launch_scale(ft, d_sc, int(sc.size()), stream));
    trace("scale done", l);
  }
  // scaled blocks A'_ij = Lh_i^-1 P_i^T A_ij Uh_j^-1 (i != j)
  {
    std::vector<GemmDesc> g1, g2;
    std::map<std::pair<int, int>, void *> tmp;
    for (auto &kv : S.blocks) {
      const int i = kv.first.first, j = kv.first.second;
      if (i == j || S.size[i] == 0 || S.size[j] == 0) continue;
      const Blk &B = kv.second;
      void *t;
      SP_TRY(dalloc(&t, size_t(B.rows) * B.cols * tsz, false));
      GemmDesc g{};
      g.A = Lh[i];
      g.B = B.p;
      g.C = t;
      g.M = B.rows;
      g.N = B.cols;
      g.K = B.rows;
      g.lda = B.rows;
      g.ldb = B.cols;
      g.ldc = B.cols;
      g.alpha = 1.0;
      g.beta = 0.0;
      g1.push_back(g);
      GemmDesc h{};
      h.A = t;
      h.B = Ust[j];
      h.C = B.p;
      h.M = B.rows;
      h.N = B.cols;
      h.K = B.cols;
      h.lda = B.cols;
      h.ldb = B.cols;
      h.ldc = B.cols;
      h.alpha = 1.0;
      h.beta = 0.0;
      h.tri = GEMM_TRI_B_UPPER;   // Uh_j^-1 is upper triangular
      g2.push_back(h);
      acct(csys(l, i), 0.0, 2.0 * double(B.rows) * B.cols * (B.rows + B.cols));
    }
    SP_TRY(gemm_batch(g1));
    SP_TRY(gemm_batch(g2));
    trace("gemm pair", l);
  }
  // ---- RRQR of W = [A'_sn ... | A'_ns^T ...]
  mark(PH_RRQR);
  std::vector<void *> Qm(ncl), Vm(ncl), Wm(ncl);
  std::vector<int> ncols(ncl, 0);
  std::vector<QrcpDesc> qd;
  void *kout, *kgs;
  SP_TRY(dalloc(&kout, std::max<size_t>(1, ifs.size()) * 4, false));
  SP_TRY(dalloc(&kgs, std::max<size_t>(1, ifs.size()) * 4, false));
  // Q is completed by batched launches (sign-shifted Gauss-Jordan on the
  // fused path, products on the matrix cores) for the interfaces that fit
  // the fused elimination, inside the QRCP kernel for the others.  Each
  // interface also takes its own candidate block width (the widest whose
  // LDS fits it), so that its arithmetic never depends on the other
  // interfaces of the launch.
  std::vector<char> cq_in(ncl, 0);
  for (int s : ifs) cq_in[s] = S.size[s] > elim_block_max_n(ft) ? 1 : 0;
  {
    // all W in one zeroed region (padding columns must read as zero)
    PlanArena pw;
    std::vector<size_t> wo(ncl, 0);
    for (int s : ifs) {
      int nc = 0;
      for (int n : nb[s]) nc += 2 * S.size[n];
      ncols[s] = nc;
      wo[s] = pw.add(size_t(S.size[s]) * ld4(std::max(nc, 1)) * tsz);
    }
    void *wbase = nullptr, *wbase2 = nullptr;
    if (!ifs.empty()) {
      SP_TRY(dalloc(&wbase, pw.total, false));
      SP_TRY(dalloc(&wbase2, pw.total, false));     // compaction target of the kernel
      // the copies below write every column but the padding up to ldw,
      // which must read as zero
      std::vector<ZeroDesc> zd;
      int64_t mz = 1;
      for (int s : ifs) {
        const int nc = ncols[s], ldw = ld4(std::max(nc, 1));
        if (ldw > nc) {
          zd.push_back(ZeroDesc{(char *)wbase + wo[s] + size_t(nc) * tsz, S.size[s], ldw - nc, ldw, 0});
          mz = std::max<int64_t>(mz, int64_t(S.size[s]) * (ldw - nc));
        }
      }
      if (!zd.empty()) {
        ZeroDesc *d_zd;
        SP_TRY(upload(zd, &d_zd, false));
        SP_TRY(launch_zero(ft, d_zd, int(zd.size()), mz, stream));
      }
    }
    // column groups of 16 bytes: 2 columns (FP64) or 4 (FP32)
    std::vector<int> grp(ncl, 1), bqs(ncl, 0);
    for (int s : ifs) {
      grp[s] = std::max(1, ld4(std::max(ncols[s], 1)) / (ft == FType::F64 ? 2 : 4));
      bqs[s] = qrcp_block_width(S.size[s], grp[s]);
      if (bqs[s] == 0) {
        set_error("RRQR problem too large for one workgroup (m=%d, %d column groups)", S.size[s],
                  grp[s]);
        return SPAND_EINVAL;
      }
    }
    std::vector<CopyDesc> wc;
    for (size_t q = 0; q < ifs.size(); ++q) {
      const int s = ifs[q];
      const int m = S.size[s];
      const int nc = ncols[s];
      const int ldw = ld4(std::max(nc, 1));
      Wm[s] = (char *)wbase + wo[s];
      SP_TRY(dalloc(&Qm[s], size_t(m) * m * tsz, false));
      SP_TRY(dalloc(&Vm[s], size_t(m) * m * tsz, false));
      void *tau, *vn1, *vn2, *sel, *hq;
      SP_TRY(dalloc(&hq, size_t(ldw) * bqs[s] * 8, false));
      SP_TRY(dalloc(&tau, size_t(m) * 8, false));
      SP_TRY(dalloc(&vn1, size_t(ldw) * 8, false));
      SP_TRY(dalloc(&vn2, size_t(ldw) * 8, false));
      SP_TRY(dalloc(&sel, size_t(ldw) * 4, false));
      int off = 0;
      for (int n : nb[s]) {
        const Blk &B = S.blocks.at({s, n});
        CopyDesc d{};
        d.src = B.p;
        d.dst = (char *)Wm[s] + size_t(off) * tsz;
        d.rows = m;
        d.cols = B.cols;
        d.lds = B.cols;
        d.ldd = ldw;
        d.scale = 1.0;
        wc.push_back(d);
        off += B.cols;
      }
      for (int n : nb[s]) {
        const Blk &B = S.blocks.at({n, s});   // |n| x m
        CopyDesc d{};
        d.src = B.p;
        d.dst = (char *)Wm[s] + size_t(off) * tsz;
        d.rows = m;
        d.cols = B.rows;
        d.lds = B.cols;
        d.ldd = ldw;
        d.trans = 1;
        d.scale = 1.0;
        wc.push_back(d);
        off += B.rows;
      }
      QrcpDesc Qd{};
      Qd.W = Wm[s];
      Qd.W2 = (char *)wbase2 + wo[s];
      Qd.Q = Qm[s];
      Qd.V = Vm[s];
      Qd.tau = (double *)tau;
      Qd.vn1 = (double *)vn1;
      Qd.vn2 = (double *)vn2;
      Qd.sel = (int32_t *)sel;
      Qd.H = (double *)hq;
      Qd.k_out = (int32_t *)kout + q;
      Qd.k_gs = (int32_t *)kgs + q;
      Qd.m = m;
      Qd.ncols = nc;
      Qd.ldw = ldw;
      qd.push_back(Qd);
      acct(csys(l, s), 0.0, 4.0 * double(m) * nc * std::min(m, nc));
    }
    SP_TRY(copy_batch(wc, 1));
    hipEvent_t qe0 = nullptr, qe1 = nullptr;
    if (timing) {
      if (event_get(&qe0) != SPAND_OK) qe0 = nullptr;
      if (event_get(&qe1) != SPAND_OK) qe1 = nullptr;
      if (qe0) (void)hipEventRecord(qe0, stream);
    }
    // one launch per (block width, completion) class; the LDS of a launch is
    // laid out for its largest m and its largest number of column groups,
    // which may come from different interfaces, so a class is cut into
    // several launches where the two together would not fit.  Within a
    // launch the interfaces go largest first (m times columns): workgroups
    // start in index order, so the small ones fill the last wave of the
    // grid instead of a large one starting last and running alone.
    std::vector<size_t> qord(ifs.size());
    for (size_t q = 0; q < ifs.size(); ++q) qord[q] = q;
    std::stable_sort(qord.begin(), qord.end(), [&](size_t a, size_t c) {
      return int64_t(S.size[ifs[a]]) * ncols[ifs[a]] > int64_t(S.size[ifs[c]]) * ncols[ifs[c]];
    });
    for (const int cq : {0, 1})
      for (const int bq : {8, 4, 2}) {
        std::vector<QrcpDesc> qc;
        int mq = 1, mg = 1;
        auto flush = [&]() -> int {
          if (qc.empty()) return SPAND_OK;
          QrcpDesc *d_q;
          SP_TRY(upload(qc, &d_q, false));
          SP_TRY(launch_qrcp(ft, d_q, int(qc.size()), eps, eps == 0.0 ? 1 : 0, mq, mg, bq, cq,
                             stream));
          qc.clear();
          mq = mg = 1;
          return SPAND_OK;
        };
        for (const size_t q : qord) {
          const int s = ifs[q];
          if (cq_in[s] != cq || bqs[s] != bq) continue;
          if (qrcp_lds_bytes(std::max(mq, S.size[s]), std::max(mg, grp[s]), bq) > QRCP_MAX_LDS)
            SP_TRY(flush());
          qc.push_back(qd[q]);
          mq = std::max(mq, S.size[s]);
          mg = std::max(mg, grp[s]);
        }
        SP_TRY(flush());
      }
    trace("qrcp plan+launch", l);
    if (timing) {
      if (qe1) (void)hipEventRecord(qe1, stream);
      qrcp_events.push_back({qe0, qe1});
    }
  }
  SP_TRY(flush_deferred());
  trace("deferred sets", l);
  std::vector<int32_t> ks(ifs.size(), 0), kg(ifs.size(), 0);
  if (!ifs.empty()) {
    SP_HIP(hipMemcpyAsync(ks.data(), kout, ifs.size() * 4, hipMemcpyDeviceToHost, stream));
    SP_HIP(hipMemcpyAsync(kg.data(), kgs, ifs.size() * 4, hipMemcpyDeviceToHost, stream));
  }
  SP_HIP(hipStreamSynchronize(stream));
  trace("sync", -1);
  release_retired();
  {
    std::vector<int> ib;
    std::vector<int32_t> kb;
    for (size_t q = 0; q < ifs.size(); ++q)
      if (!cq_in[ifs[q]]) {
        ib.push_back(ifs[q]);
        kb.push_back(kg[q]);
      }
    if (!ib.empty()) {
      SP_TRY(complete_q(l, S, ib, kb, Qm, Vm));
      trace("qrcp completion", l);
    }
  }
  std::vector<int> kk(ncl, 0);
  {
    RankStat rs;
    for (size_t q = 0; q < ifs.size(); ++q) {
      kk[ifs[q]] = ks[q];
      rs.add(S.size[ifs[q]], ks[q]);
      if (!members.empty()) {
        auto &mr = members[size_t(csys(l, ifs[q]))].ranks;
        if (size_t(l) < mr.size()) mr[size_t(l)].add(S.size[ifs[q]], ks[q]);
      }
      const double m = S.size[ifs[q]], c = ncols[ifs[q]], k = ks[q];
      qrcp_bytes += (m * c + m * m) * double(tsz);
      qrcp_flops += 4.0 * m * c * k - 2.0 * k * k * (m + c) + 4.0 * k * k * k / 3.0;
    }
    ranks.push_back(rs);
  }
  // ---- F_s = Q_s^T Lh_s^-1 P_s^T, B_s = Uh_s^-1 Q_s (stored) ; apply descriptors
  mark(PH_COMPRESS);
  {
    std::vector<GemmDesc> gm;
    std::vector<GemvDesc> gf, gb;
    std::vector<const std::vector<int32_t> *> os;
    std::vector<int> vs;
    for (int s : ifs) {
      const int m = S.size[s];
      void *Fp, *Bp;
      SP_TRY(dalloc(&Fp, size_t(m) * ld4(m) * tsz, true));
      SP_TRY(dalloc(&Bp, size_t(m) * ld4(m) * tsz, true));
      GemmDesc g{};
      g.A = Qm[s];
      g.transA = 1;
      g.B = Lh[s];
      g.C = Fp;
      g.M = g.N = g.K = m;
      g.lda = g.ldb = m;
      g.ldc = ld4(m);
      g.alpha = 1.0;
      gm.push_back(g);
      GemmDesc h{};
      h.A = Ust[s];
      h.B = Qm[s];
      h.C = Bp;
      h.M = h.N = h.K = m;
      h.lda = h.ldb = m;
      h.ldc = ld4(m);
      h.alpha = 1.0;
      h.tri = GEMM_TRI_A_UPPER;   // Uh^-1 is upper triangular
      gm.push_back(h);
      GemvDesc d{};
      d.islot = d.oslot = S.d_slots[s];
      d.rows = d.cols = m;
      d.lda = ld4(m);
      d.A = Fp;
      gf.push_back(d);
      d.A = Bp;
      gb.push_back(d);
      os.push_back(&S.slots[s]);
      vs.push_back(csys(l, s));
      acct(csys(l, s), 2.0 * double(m) * m * tsz, 4.0 * double(m) * m * m);   // F_s forward, B_s backward
    }
    SP_TRY(gemm_batch(gm));
    trace("gemm", l);
    defer([this, &AL, gf, gb, os, vs, l]() {
      SP_TRY(AL.F.set(*this, gf, os, 0));
      SP_TRY(AL.B.set(*this, gb, os, 0));
      SP_TRY(AL.FT.set(*this, gf, os, 1));
      SP_TRY(AL.BT.set(*this, gb, os, 1));
      SP_TRY(member_gemv(l, &ApplyLevel::F, gf, os, vs, 0));
      SP_TRY(member_gemv(l, &ApplyLevel::B, gb, os, vs, 0));
      SP_TRY(member_gemv(l, &ApplyLevel::FT, gf, os, vs, 1));
      return member_gemv(l, &ApplyLevel::BT, gb, os, vs, 1);
    });
    trace("compress F/B sets", l);
  }
  // ---- merge: next-level clusters from the coarse parts
  const auto &cl1 = nd.levels[l + 1];
  const auto &kids = nd.children[l + 1];
  const int ncl1 = int(cl1.size());
  std::vector<int> parent(ncl, -1), poff(ncl, 0);
  Nx.size.assign(ncl1, 0);
  Nx.interior.assign(ncl1, 0);
  Nx.slots.assign(ncl1, {});
  for (int I = 0; I < ncl1; ++I) {
    Nx.interior[I] = cl1[I].interior;
    int o = 0;
    for (int c : kids[I]) {
      parent[c] = I;
      poff[c] = o;
      o += kk[c];
      Nx.slots[I].insert(Nx.slots[I].end(), S.slots[c].begin(), S.slots[c].begin() + kk[c]);
    }
    Nx.size[I] = o;
  }
  // parent blocks (sorted unique keys parent_i * ncl1 + parent_j)
  std::vector<int64_t> pkeys;
  pkeys.reserve(S.blocks.size());
  for (auto &kv : S.blocks) {
    const int i = kv.first.first, j = kv.first.second;
    if (S.size[i] == 0 || S.size[j] == 0 || kk[i] == 0 || kk[j] == 0) continue;
    if (parent[i] < 0 || parent[j] < 0) continue;
    pkeys.push_back(int64_t(parent[i]) * ncl1 + parent[j]);
  }
  std::sort(pkeys.begin(), pkeys.end());
  pkeys.erase(std::unique(pkeys.begin(), pkeys.end()), pkeys.end());
  trace("parent keys", l);
  std::vector<Blk> pblk(pkeys.size());
  {
    PlanArena pk, pt;
    std::vector<std::pair<size_t, bool>> offs(pkeys.size());
    for (size_t q = 0; q < pkeys.size(); ++q) {
      const int i = int(pkeys[q] / ncl1), j = int(pkeys[q] % ncl1);
      const bool keep = Nx.interior[i] || Nx.interior[j];
      const size_t bytes = size_t(Nx.size[i]) * Nx.size[j] * tsz;
      offs[q] = {keep ? pk.add(bytes) : pt.add(bytes), keep};
    }
    void *bk = nullptr, *bt = nullptr;
    if (pk.total) {
      SP_TRY(dalloc(&bk, pk.total, true));
      SP_HIP(hipMemsetAsync(bk, 0, pk.total, stream));
    }
    if (pt.total) {
      SP_TRY(dalloc_next(&bt, pt.total));
      SP_HIP(hipMemsetAsync(bt, 0, pt.total, stream));
    }
    Nx.blocks.clear();
    for (size_t q = 0; q < pkeys.size(); ++q) {
      const int i = int(pkeys[q] / ncl1), j = int(pkeys[q] % ncl1);
      char *base = (char *)(offs[q].second ? bk : bt);
      pblk[q] = Blk{base + offs[q].first, Nx.size[i], Nx.size[j]};
      Nx.blocks.emplace_hint(Nx.blocks.end(), std::make_pair(i, j), pblk[q]);
    }
  }
  trace("parent blocks", l);
  auto parent_blk = [&](int i, int j) -> const Blk & {
    const int64_t key = int64_t(i) * ncl1 + j;
    return pblk[size_t(std::lower_bound(pkeys.begin(), pkeys.end(), key) - pkeys.begin())];
  };
  // compression A_ij <- Q_ic^T A'_ij Q_jc into the parent block; diagonals -> I_k
  {
    std::vector<GemmDesc> g1, g2;
    std::vector<EyeDesc> ey;
    int maxk = 0;
    for (auto &kv : S.blocks) {
      const int i = kv.first.first, j = kv.first.second;
      if (S.size[i] == 0 || S.size[j] == 0 || kk[i] == 0 || kk[j] == 0) continue;
      const Blk &P = parent_blk(parent[i], parent[j]);
      if (i == j) {
        EyeDesc e{};
        e.A = (char *)P.p + (size_t(poff[i]) * P.cols + poff[i]) * tsz;
        e.n = kk[i];
        e.ld = P.cols;
        ey.push_back(e);
        maxk = std::max(maxk, kk[i]);
        continue;
      }
      const Blk &B = kv.second;
      void *t;
      SP_TRY(dalloc(&t, size_t(kk[i]) * B.cols * tsz, false));
      GemmDesc g{};
      g.A = Qm[i];
      g.transA = 1;
      g.lda = S.size[i];
      g.B = B.p;
      g.ldb = B.cols;
      g.C = t;
      g.ldc = B.cols;
      g.M = kk[i];
      g.N = B.cols;
      g.K = S.size[i];
      g.alpha = 1.0;
      g1.push_back(g);
      GemmDesc h{};
      h.A = t;
      h.lda = B.cols;
      h.B = Qm[j];
      h.ldb = S.size[j];
      h.C = (char *)P.p + (size_t(poff[i]) * P.cols + poff[j]) * tsz;
      h.ldc = P.cols;
      h.M = kk[i];
      h.N = kk[j];
      h.K = B.cols;
      h.alpha = 1.0;
      g2.push_back(h);
      acct(csys(l, i), 0.0, 2.0 * double(kk[i]) * B.cols * (B.rows + kk[j]));
    }
    trace("pair descriptors", l);
    SP_TRY(gemm_batch(g1));
    SP_TRY(gemm_batch(g2));
    trace("gemm pair", l);
    EyeDesc *d_e;
    SP_TRY(upload(ey, &d_e, false));
    SP_TRY(launch_eye(ft, d_e, int(ey.size()), maxk, stream));
  }
  SP_TRY(upload_level_slots(Nx));
  trace("merge plan", l);
  // the sweep sets queued by this level (compression) are built while the
  // host next waits for the device, before the next level's rank read-back:
  // the device goes on to the next level's eliminations meanwhile (the
  // caller keeps S, whose slot lists they read, alive until then)
  return SPAND_OK;
}

// ------------------------------------------------------------------ driver
// Host copy of a BSR pattern, validated (rowptr monotone from 0 to nnzb,
// colind in range and strictly ascending in every row).
static int check_pattern(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int K,
                         int64_t nnzb, const char *who) {
  if (rp[0] != 0 || rp[size_t(K)] != nnzb) {
    set_error("%srowptr[0] must be 0 and rowptr[n_brows] must equal nnzb", who);
    return SPAND_EINVAL;
  }
  for (int e = 0; e < K; ++e) {
    if (rp[size_t(e) + 1] < rp[size_t(e)]) {
      set_error("%srowptr must be non-decreasing", who);
      return SPAND_EINVAL;
    }
    for (int t = rp[size_t(e)]; t < rp[size_t(e) + 1]; ++t) {
      if (ci[size_t(t)] < 0 || ci[size_t(t)] >= K || (t > rp[size_t(e)] && ci[size_t(t)] <= ci[size_t(t) - 1])) {
        set_error("%scolind must be in range and strictly ascending in every block row (row %d)",
                  who, e);
        return SPAND_EINVAL;
      }
    }
  }
  return SPAND_OK;
}

int Factor::build(const spand_bsr_t &A, const spand_grid_t &g, const spand_opts_t &o,
                  const Factor *sym) {
  build_t0 = std::chrono::steady_clock::now();
  trace_t = build_t0;
  build_drv0 = pool_driver_ms();
  bs = A.bs;
  K = A.n_brows;
  N = int64_t(K) * bs;
  if (N > INT_MAX) {     // the sweeps address unknowns with 32-bit slots
    set_error("%lld unknowns exceed the 32-bit indices of the factorization", (long long)N);
    return SPAND_EINVAL;
  }
  ft = o.factor_dtype == SPAND_F32 ? FType::F32 : FType::F64;
  eps = o.eps;
  L = o.nlevels > 0 ? o.nlevels : default_levels(K);
  grid = g;
  opts = o;
  d_val = A.d_val;
  if (sym) {
    // refactorization: the pattern (checked by the caller) and the ordering
    // of the earlier factorization; only the numeric phases run again
    h_rowptr = sym->h_rowptr;
    h_colind = sym->h_colind;
    nd_sym = sym->nd_sym;
    trace("symbolic phase reused", -1);
  } else {
    h_rowptr.resize(K + 1);
    h_colind.resize(A.nnzb);
    SP_HIP(hipMemcpyAsync(h_rowptr.data(), A.d_rowptr, (K + 1) * 4, hipMemcpyDeviceToHost, stream));
    SP_HIP(hipMemcpyAsync(h_colind.data(), A.d_colind, A.nnzb * 4, hipMemcpyDeviceToHost, stream));
    SP_HIP(hipStreamSynchronize(stream));
    trace("sync", -1);
    SP_TRY(check_pattern(h_rowptr, h_colind, K, A.nnzb, ""));
    trace("read pattern + validate", -1);
    nd_sym = std::make_shared<const NDResult>(
        nested_dissection(g.nx, g.ny, g.periodic_x != 0, g.periodic_y != 0, L));
    trace("nested dissection", -1);
  }
  return numeric();
}

int Factor::build_batch(const std::vector<BatchSystem> &sy, const spand_opts_t &o) {
  build_t0 = std::chrono::steady_clock::now();
  trace_t = build_t0;
  build_drv0 = pool_driver_ms();
  const int n = int(sy.size());
  bs = sy[0].A.bs;
  ft = o.factor_dtype == SPAND_F32 ? FType::F32 : FType::F64;
  eps = o.eps;
  opts = o;
  members.assign(size_t(n), Member{});
  int64_t eo = 0, no = 0;
  L = 0;
  for (int m = 0; m < n; ++m) {
    Member &M = members[size_t(m)];
    M.K = sy[size_t(m)].A.n_brows;
    M.L = sy[size_t(m)].L;
    M.elem_off = eo;
    M.nnz_off = no;
    M.dof_off = eo * bs;
    M.N = int64_t(M.K) * bs;
    M.d_val = sy[size_t(m)].A.d_val;
    M.ranks.assign(size_t(std::max(M.L - 1, 0)), RankStat{});
    eo += M.K;
    no += sy[size_t(m)].A.nnzb;
    L = std::max(L, M.L);
  }
  if (eo * bs > INT_MAX || no > INT_MAX) {
    set_error("batched factorization of %lld unknowns and %lld blocks exceeds the 32-bit indices",
              (long long)(eo * bs), (long long)no);
    return SPAND_EINVAL;
  }
  K = int(eo);
  N = eo * bs;
  // the systems' patterns: all copies queued, then one wait
  std::vector<std::vector<int32_t>> rps(static_cast<size_t>(n)), cis(static_cast<size_t>(n));
  for (int m = 0; m < n; ++m) {
    const spand_bsr_t &A = sy[size_t(m)].A;
    rps[size_t(m)].resize(size_t(A.n_brows) + 1);
    cis[size_t(m)].resize(size_t(A.nnzb));
    SP_HIP(hipMemcpyAsync(rps[size_t(m)].data(), A.d_rowptr, rps[size_t(m)].size() * 4,
                          hipMemcpyDeviceToHost, stream));
    SP_HIP(hipMemcpyAsync(cis[size_t(m)].data(), A.d_colind, cis[size_t(m)].size() * 4,
                          hipMemcpyDeviceToHost, stream));
  }
  SP_HIP(hipStreamSynchronize(stream));
  trace("sync", -1);
  h_rowptr.assign(size_t(K) + 1, 0);
  h_colind.resize(size_t(no));
  esys.resize(size_t(K));
  std::vector<NDResult> parts(static_cast<size_t>(n));
  std::vector<int64_t> eoffs(static_cast<size_t>(n));
  for (int m = 0; m < n; ++m) {
    const Member &M = members[size_t(m)];
    char who[32];
    std::snprintf(who, sizeof(who), "system %d: ", m);
    SP_TRY(check_pattern(rps[size_t(m)], cis[size_t(m)], M.K, int64_t(cis[size_t(m)].size()), who));
    for (int e = 0; e < M.K; ++e) {
      h_rowptr[size_t(M.elem_off + e)] = int32_t(M.nnz_off + rps[size_t(m)][size_t(e)]);
      esys[size_t(M.elem_off + e)] = m;
    }
    for (size_t t = 0; t < cis[size_t(m)].size(); ++t)
      h_colind[size_t(M.nnz_off) + t] = int32_t(cis[size_t(m)][t] + M.elem_off);
    const spand_grid_t &g = sy[size_t(m)].grid;
    parts[size_t(m)] = nested_dissection(g.nx, g.ny, g.periodic_x != 0, g.periodic_y != 0, M.L);
    eoffs[size_t(m)] = M.elem_off;
  }
  h_rowptr[size_t(K)] = int32_t(no);
  trace("read patterns + validate + nested dissections", -1);
  nd_sym = std::make_shared<const NDResult>(nd_union(parts, eoffs));
  for (auto &M : members) M.lv.assign(size_t(L), ApplyLevel{});
  trace("union ordering", -1);
  return numeric();
}

int Factor::numeric() {
  const NDResult &nd = *nd_sym;
  void *p;
  SP_TRY(dalloc(&p, size_t(N) * 4, true));
  d_iota = (int32_t *)p;
  SP_TRY(vec_iota(d_iota, N, stream));
  SP_TRY(dalloc(&p, size_t(N) * 8, true));
  d_tbuf = (double *)p;
  SP_TRY(dalloc(&p, size_t(N) * 8, true));
  d_xg = (double *)p;
  use_graphs = (opts.flags & SPAND_FLAG_NO_GRAPH) == 0 && !std::getenv("SPAND_NO_GRAPH");
  {
    const int tr = tuned_gemv_rows(ft, bs);
    if (tr > 0) gemv_rows = tr;
  }
  SP_TRY(dalloc(&p, 64, true));
  d_flag = (int *)p;
  SP_HIP(hipMemsetAsync(d_flag, 0, 64, stream));
  lv.assign(L, ApplyLevel{});
  auto t1 = std::chrono::steady_clock::now();
  t_host_ms += std::chrono::duration<double, std::milli>(t1 - build_t0).count();
  mark(PH_GATHER);
  LevelState S, prev;   // prev: the level before, read by sweep sets not yet built
  SP_TRY(level0(nd, S));
  for (int l = 0; l < L; ++l) {
    if (l >= 1) SP_TRY(eliminate_dense(l, S));
    // a system whose top level this is keeps what its top clusters hold
    for (size_t m = 0; m < members.size(); ++m)
      if (members[m].L - 1 == l)
        for (int c = 0; c < int(S.size.size()); ++c)
          if (csys(l, c) == int(m)) members[m].top_size += S.size[c];
    if (l == L - 1) break;
    LevelState Nx;
    SP_TRY(sparsify(l, nd, S, Nx));
    free_temp();
    // every set that read the level before was built in this sparsify (at
    // its rank read-back); the sets of this level's compression read S
    prev = std::move(S);
    S = std::move(Nx);
  }
  int tops = 0;
  if (members.empty())
    for (int c = 0; c < int(S.size.size()); ++c) tops += S.size[c];
  else
    for (const auto &M : members) tops += M.top_size;
  top_size = tops;
  SP_TRY(flush_deferred());
  mark(PH_END);
  SP_HIP(hipStreamSynchronize(stream));
  trace("sync", -1);
  temp.release();
  next_temp.release();
  retired.release();
  alloc_ms = pool_driver_ms() - build_drv0;
  int flag = 0;
  SP_HIP(hipMemcpy(&flag, d_flag, 4, hipMemcpyDeviceToHost));
  trace("release + flag", -1);
  collect_events();
  trace("timing events", -1);
  if (flag) {
    set_error("zero pivot met during the factorization");
    return SPAND_ESINGULAR;
  }
  return SPAND_OK;
}

// ------------------------------------------------------------------ apply
// y = M^-1 r:  forward over levels applies L' (interiors: x_n -= A_ns A_ss^-1 x_s)
// and F_s (interfaces); backward applies B_s and R' (x_s = A_ss^-1 (x_s - A_sn x_n)).
// y = M^-T r:  forward applies R'^T and B_s^T, backward F_s^T and L'^T.
int Factor::sweeps(const std::vector<ApplyLevel> &lv, double *x, int transpose, hipStream_t st) {
  const int L = int(lv.size());
  auto inplace = [&](const GemvSet &g) -> int {
    if (!g.n) return SPAND_OK;
    SP_TRY(launch_gemv(ft, g.d_items, g.d_chunks, g.nchunks, x, d_tbuf, 1.0, 0.0, st));
    return launch_slot_copy(g.d_slots, g.nslots, d_tbuf, x, st);
  };
  if (!transpose) {
    for (int l = 0; l < L; ++l) {
      const ApplyLevel &A = lv[l];
      if (A.fw.n) {
        SP_TRY(launch_gemv(ft, A.inv.d_items, A.inv.d_chunks, A.inv.nchunks, x, d_tbuf, 1.0, 0.0, st));
        SP_TRY(launch_pull2(ft, A.fw.d_groups, A.fw.d_items, A.fw.d_chunks, A.fw.nchunks, A.fw.trans, d_tbuf, x, -1.0, 1.0, st));
      }
      SP_TRY(inplace(A.F));
    }
    for (int l = L - 1; l >= 0; --l) {
      const ApplyLevel &A = lv[l];
      SP_TRY(inplace(A.B));
      if (A.bw.n) SP_TRY(launch_pull2(ft, A.bw.d_groups, A.bw.d_items, A.bw.d_chunks, A.bw.nchunks, A.bw.trans, x, x, -1.0, 1.0, st));
      SP_TRY(inplace(A.inv));
    }
  } else {
    for (int l = 0; l < L; ++l) {
      const ApplyLevel &A = lv[l];
      SP_TRY(inplace(A.invT));
      if (A.tfw.n) SP_TRY(launch_pull2(ft, A.tfw.d_groups, A.tfw.d_items, A.tfw.d_chunks, A.tfw.nchunks, A.tfw.trans, x, x, -1.0, 1.0, st));
      SP_TRY(inplace(A.BT));
    }
    for (int l = L - 1; l >= 0; --l) {
      const ApplyLevel &A = lv[l];
      SP_TRY(inplace(A.FT));
      if (A.tbw.n && A.invT.n) {
        SP_TRY(launch_pull2(ft, A.tbw.d_groups, A.tbw.d_items, A.tbw.d_chunks, A.tbw.nchunks, A.tbw.trans, x, d_tbuf, 1.0, 0.0, st));
        SP_TRY(launch_gemv(ft, A.invT.d_items, A.invT.d_chunks, A.invT.nchunks, d_tbuf, x, -1.0, 1.0, st));
      }
    }
  }
  return SPAND_OK;
}

// Capture the sweeps on the fixed vector d_xg once; replays need one launch.
// member >= 0: the sweeps of that system of a batch (its share of d_xg).
int Factor::capture(int member, int transpose) {
  const std::vector<ApplyLevel> &plan = member < 0 ? lv : members[size_t(member)].lv;
  hipGraphExec_t *ge = member < 0 ? gexec : members[size_t(member)].gexec;
  hipStream_t cs;
  SP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int r = SPAND_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("hipStreamBeginCapture failed");
    r = SPAND_EHIP;
  }
  if (r == SPAND_OK) {
    const int rs = sweeps(plan, d_xg, transpose, cs);
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rs != SPAND_OK) r = rs;
    else if (e != hipSuccess || !g) {
      set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
      r = SPAND_EHIP;
    }
  }
  if (r == SPAND_OK && hipGraphInstantiate(&ge[transpose], g, nullptr, nullptr, 0) != hipSuccess) {
    set_error("hipGraphInstantiate failed");
    ge[transpose] = nullptr;
    r = SPAND_EHIP;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  return r;
}

// Sweeps are captured once, by a thread of the caller and with no worker
// thread of this library alive: a capture never overlaps another thread's
// hipMalloc/hipFree/stream creation issued from here.  The M^-1 sweep right
// after the factorization, the M^-T sweep at the first public call that needs
// it (batched factorizations capture both at once).  The mutex keeps
// captures of concurrent host callers apart.  `which`: bit 0 M^-1, bit 1 M^-T.
static std::mutex g_capture_mu;

int Factor::capture_graphs(int which, int member) {
  if (!use_graphs) return SPAND_OK;
  std::lock_guard<std::mutex> lk(g_capture_mu);
  const hipGraphExec_t *ge = member < 0 ? gexec : members[size_t(member)].gexec;
  for (int t = 0; t < 2; ++t)
    if ((which >> t & 1) && !ge[t]) SP_TRY(capture(member, t));
  return SPAND_OK;
}

int Factor::apply(const double *in, double *out, int transpose, hipStream_t st, int member) {
  if (member >= 0) {
    // one system of a batch: its vector goes through its share of d_xg (the
    // sweeps address the unknowns of the whole batch)
    const Member &M = members[size_t(member)];
    double *seg = d_xg + M.dof_off;
    SP_HIP(hipMemcpyAsync(seg, in, size_t(M.N) * 8, hipMemcpyDeviceToDevice, st));
    if (use_graphs && M.gexec[transpose]) SP_HIP(hipGraphLaunch(M.gexec[transpose], st));
    else SP_TRY(sweeps(M.lv, d_xg, transpose, st));
    SP_HIP(hipMemcpyAsync(out, seg, size_t(M.N) * 8, hipMemcpyDeviceToDevice, st));
    return SPAND_OK;
  }
  if (!use_graphs || !gexec[transpose]) {
    if (out != in) SP_HIP(hipMemcpyAsync(out, in, size_t(N) * 8, hipMemcpyDeviceToDevice, st));
    return sweeps(lv, out, transpose, st);
  }
  SP_HIP(hipMemcpyAsync(d_xg, in, size_t(N) * 8, hipMemcpyDeviceToDevice, st));
  SP_HIP(hipGraphLaunch(gexec[transpose], st));
  SP_HIP(hipMemcpyAsync(out, d_xg, size_t(N) * 8, hipMemcpyDeviceToDevice, st));
  return SPAND_OK;
}

int Factor::apply_batch(const std::vector<const double *> &in, const std::vector<double *> &out,
                        int transpose, hipStream_t st) {
  for (size_t m = 0; m < members.size(); ++m)
    SP_HIP(hipMemcpyAsync(d_xg + members[m].dof_off, in[m], size_t(members[m].N) * 8,
                          hipMemcpyDeviceToDevice, st));
  if (use_graphs && gexec[transpose]) SP_HIP(hipGraphLaunch(gexec[transpose], st));
  else SP_TRY(sweeps(lv, d_xg, transpose, st));
  for (size_t m = 0; m < members.size(); ++m)
    SP_HIP(hipMemcpyAsync(out[m], d_xg + members[m].dof_off, size_t(members[m].N) * 8,
                          hipMemcpyDeviceToDevice, st));
  return SPAND_OK;
}

void Factor::fill_stats(spand_factor_stats_t *st, int member) const {
  std::memset(st, 0, sizeof(*st));
  const Member *M = member >= 0 ? &members[size_t(member)] : nullptr;
  const std::vector<RankStat> &ranks = M ? M->ranks : this->ranks;
  st->nlevels = M ? M->L : L;
  st->batch_systems = members.empty() ? 1 : int32_t(members.size());
  for (size_t l = 0; l < ranks.size() && l < SPAND_MAX_LEVELS; ++l) {
    const RankStat &r = ranks[l];
    st->n_clusters[l] = r.n;
    st->rank_min[l] = r.n ? r.kmin : 0;
    st->rank_max[l] = r.kmax;
    st->rank_avg[l] = r.n ? double(r.ksum) / r.n : 0.0;
    st->size_before[l] = r.msum;
    st->size_after[l] = r.ksum;
  }
  st->top_size = M ? M->top_size : top_size;
  st->factor_bytes = int64_t(M ? M->apply_bytes : apply_bytes);
  st->factor_flops = M ? M->flops : flops;
  st->t_host_ms = t_host_ms;
  st->t_device_ms = ph_ms[PH_GATHER] + ph_ms[PH_LU] + ph_ms[PH_SCHUR] + ph_ms[PH_SCALE] +
                    ph_ms[PH_RRQR] + ph_ms[PH_COMPRESS];
  st->t_lu_ms = ph_ms[PH_LU];
  st->t_schur_ms = ph_ms[PH_SCHUR];
  st->t_scale_ms = ph_ms[PH_SCALE];
  st->t_rrqr_ms = ph_ms[PH_RRQR];
  st->t_compress_ms = ph_ms[PH_COMPRESS];
  st->t_qrcp_ms = qrcp_ms;
  st->n_qrcp = n_qrcp;
  st->qrcp_bytes = qrcp_bytes;
  st->qrcp_flops = qrcp_flops;
  st->t_alloc_ms = alloc_ms;
  for (int p = 0; p < 6; ++p) st->t_plan_ms[p] = ph_host_ms[p];
  st->resident_bytes = int64_t(keep.bytes);
  st->t_gemm_ms = kt_ms[0];
  st->gemm_flops = kt_flops[0];
  st->gemm_bytes = kt_bytes[0];
  st->n_gemm = kt_n[0];
  st->t_schur_elem_ms = kt_ms[1];
  st->schur_elem_flops = kt_flops[1];
  st->schur_elem_bytes = kt_bytes[1];
  st->n_schur_elem = kt_n[1];
}

void Factor::collect_events() {
  for (size_t i = 0; i + 1 < events.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, events[i].second, events[i + 1].second) == hipSuccess)
      ph_ms[events[i].first] += ms;
  }
  for (auto &e : events) event_put(e.second);
  events.clear();
  for (auto &e : qrcp_events) {
    float ms = 0.f;
    if (e.first && e.second && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess)
      qrcp_ms += ms;
    event_put(e.first);
    event_put(e.second);
  }
  n_qrcp += int(qrcp_events.size());
  qrcp_events.clear();
  for (auto &e : kevents) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) kt_ms[e.kind] += ms;
    kt_flops[e.kind] += e.flops;
    kt_bytes[e.kind] += e.bytes;
    ++kt_n[e.kind];
    event_put(e.a);
    event_put(e.b);
  }
  kevents.clear();
}

}  // namespace spand
