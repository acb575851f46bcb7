// s-step GMRES (paper Algorithm 2 and its CAGMRES section), right
// preconditioned with the spaND factor.  Host driver; every vector
// operation is a kernel (kernels_vec / kernels_krylov), all in float64.
//
// Per cycle: r = b - A x, q0 = r/||r||.  The first cycle starts with s
// classical GMRES steps (MGS) whose Hessenberg matrix gives the Ritz values;
// they become Newton shifts in Leja order (real arithmetic: a complex pair
// a +- ib is applied as (A - a)^2 + b^2 over two steps).  Then blocks of s
// vectors: w_k = (A M^-1 - theta_k) w_{k-1}, two passes of block classical
// Gram-Schmidt + Cholesky QR, Hessenberg columns recovered from the
// change-of-basis matrix, Givens rotations and the residual estimate after
// every column.  The solution update is x += M^-1 (Q y).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "factor.h"

namespace spand {

// ------------------------------------------------------------------ host: eigenvalues
// Eigenvalues of a small real upper Hessenberg matrix by the implicit
// double-shift (Francis) QR iteration with deflation (Golub & Van Loan,
// Matrix Computations, Sec. 7.5).  Active block [lo, hi] only.
static void house3(const double *x, int n, double *v, double &beta) {
  double nrm = 0.0;
  for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
  nrm = std::sqrt(nrm);
  for (int i = 0; i < n; ++i) v[i] = x[i];
  if (nrm == 0.0) {
    beta = 0.0;
    return;
  }
  v[0] += (x[0] >= 0.0 ? nrm : -nrm);
  double vv = 0.0;
  for (int i = 0; i < n; ++i) vv += v[i] * v[i];
  beta = 2.0 / vv;
}

static void eig2(double a, double b, double c, double d, std::complex<double> &l1,
                 std::complex<double> &l2) {
  const double m = 0.5 * (a + d);
  const double disc = 0.25 * (a - d) * (a - d) + b * c;
  if (disc >= 0.0) {
    const double r = std::sqrt(disc);
    const double big = m + (m >= 0 ? r : -r);
    const double det = a * d - b * c;
    const double small = big != 0.0 ? det / big : m - r;
    l1 = big;
    l2 = small;
  } else {
    const double r = std::sqrt(-disc);
    l1 = std::complex<double>(m, r);
    l2 = std::complex<double>(m, -r);
  }
}

static bool hessenberg_eigs(std::vector<double> H, int n, std::vector<std::complex<double>> &ev) {
  auto h = [&](int i, int j) -> double & { return H[size_t(i) * n + j]; };
  ev.assign(n, 0.0);
  for (double v : H)
    if (!std::isfinite(v)) return false;
  int hi = n - 1, iter = 0;
  const double eps = 2.220446049250313e-16;
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = h(0, 0);
      --hi;
      continue;
    }
    int l = hi;
    while (l > 0) {
      double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (s == 0.0) s = 1.0;
      if (std::fabs(h(l, l - 1)) <= eps * s) break;
      --l;
    }
    if (l > 0) h(l, l - 1) = 0.0;
    if (l == hi) {
      ev[hi] = h(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      eig2(h(hi - 1, hi - 1), h(hi - 1, hi), h(hi, hi - 1), h(hi, hi), ev[hi - 1], ev[hi]);
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++iter > 200) return false;
    // double shift from the trailing 2x2 (exceptional shift every 11 sweeps)
    double s = h(hi - 1, hi - 1) + h(hi, hi);
    double t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    if (iter % 11 == 0) {
      const double w = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * w;
      t = w * w;
    }
    double x = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
    double y = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
    double z = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l - 1; k <= hi - 3; ++k) {
      double xv[3] = {x, y, z}, v[3], beta;
      house3(xv, 3, v, beta);
      const int q = std::max(l, k);
      for (int j = q; j <= hi; ++j) {
        const double dd = beta * (v[0] * h(k + 1, j) + v[1] * h(k + 2, j) + v[2] * h(k + 3, j));
        h(k + 1, j) -= dd * v[0];
        h(k + 2, j) -= dd * v[1];
        h(k + 3, j) -= dd * v[2];
      }
      const int r = std::min(k + 4, hi);
      for (int i = l; i <= r; ++i) {
        const double dd = beta * (h(i, k + 1) * v[0] + h(i, k + 2) * v[1] + h(i, k + 3) * v[2]);
        h(i, k + 1) -= dd * v[0];
        h(i, k + 2) -= dd * v[1];
        h(i, k + 3) -= dd * v[2];
      }
      x = h(k + 2, k + 1);
      y = h(k + 3, k + 1);
      if (k < hi - 3) z = h(k + 4, k + 1);
    }
    double xv[2] = {x, y}, v[2], beta;
    house3(xv, 2, v, beta);
    for (int j = hi - 2; j <= hi; ++j) {
      const double dd = beta * (v[0] * h(hi - 1, j) + v[1] * h(hi, j));
      h(hi - 1, j) -= dd * v[0];
      h(hi, j) -= dd * v[1];
    }
    for (int i = l; i <= hi; ++i) {
      const double dd = beta * (h(i, hi - 1) * v[0] + h(i, hi) * v[1]);
      h(i, hi - 1) -= dd * v[0];
      h(i, hi) -= dd * v[1];
    }
  }
  return true;
}

// Leja order for real arithmetic: largest modulus first, then the value
// maximising the sum of log distances to those already chosen; ties ->
// larger real part, then larger imaginary part; Im > 0 followed by its
// conjugate; a pair that would not fit in the last slot uses its real part.
struct Slot {
  int kind;        // 0 real, 1 first of pair, 2 second of pair
  double a, b;
};

static std::vector<Slot> leja_slots(std::vector<std::complex<double>> vals, int s) {
  std::vector<std::complex<double>> chosen;
  auto tie_better = [](std::complex<double> z, std::complex<double> w) {
    return z.real() != w.real() ? z.real() > w.real() : z.imag() > w.imag();
  };
  while (!vals.empty() && int(chosen.size()) < s) {
    int best = -1;
    double bs = 0.0;
    for (int i = 0; i < int(vals.size()); ++i) {
      double sc;
      if (chosen.empty()) {
        sc = std::abs(vals[i]);
      } else {
        sc = 0.0;
        bool zero = false;
        for (auto &c : chosen) {
          const double d = std::abs(vals[i] - c);
          if (d == 0.0) zero = true;
          sc += std::log(d > 0 ? d : 1.0);
        }
        if (zero) sc = -INFINITY;
      }
      bool take = false;
      if (best < 0) take = true;
      else {
        const double tol = 1e-12 * std::max(1.0, std::fabs(bs));
        if (sc > bs + tol) take = true;
        else if (sc >= bs - tol && tie_better(vals[i], vals[best])) take = true;
      }
      if (take) {
        best = i;
        bs = sc;
      }
    }
    const std::complex<double> z = vals[best];
    if (z.imag() != 0.0) {
      const std::complex<double> zp(z.real(), std::fabs(z.imag())), zm = std::conj(zp);
      for (auto target : {zp, zm}) {
        int bi = 0;
        if (vals.empty()) break;
        for (int i = 1; i < int(vals.size()); ++i)
          if (std::abs(vals[i] - target) < std::abs(vals[bi] - target)) bi = i;
        vals.erase(vals.begin() + bi);
      }
      chosen.push_back(zp);
      chosen.push_back(zm);
    } else {
      vals.erase(vals.begin() + best);
      chosen.push_back(z);
    }
  }
  if (int(chosen.size()) > s) chosen.resize(s);
  std::vector<Slot> out;
  for (int i = 0; i < int(chosen.size());) {
    const auto z = chosen[i];
    if (z.imag() > 0.0 && i + 1 < int(chosen.size())) {
      out.push_back({1, z.real(), z.imag()});
      out.push_back({2, z.real(), z.imag()});
      i += 2;
    } else {
      out.push_back({0, z.real(), 0.0});
      i += 1;
    }
  }
  return out;
}

// ------------------------------------------------------------------ timers
struct PhaseTimer {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<std::pair<int, hipEvent_t>> ev;
  void mark(int ph) {
    if (!on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, st);
    ev.push_back({ph, e});
  }
  void collect(double *ms) {
    for (size_t i = 0; i + 1 < ev.size(); ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[i].second, ev[i + 1].second) == hipSuccess) ms[ev[i].first] += t;
    }
    for (auto &e : ev) (void)hipEventDestroy(e.second);
    ev.clear();
  }
};
enum { T_SPMV = 0, T_APPLY, T_ORTH, T_OTHER, T_N };

// ------------------------------------------------------------------ solver
// Single-reduce schedule: a pending block whose one-pass residual estimate is
// within this factor of the tolerance gets its second pass at once instead of
// starting the next block's operator applications (which would be wasted if
// the block converges).  Only the work changes; the results are the same.
constexpr double kEagerFinish = 4.0;

// Device workspace of one solve, in allocation order (each piece rounded
// up to 256 bytes): the Krylov basis Q (N x (m+1)), Z and R (N), the small
// Krylov state, the partial sums of the reductions, the basis Gram matrix
// of the orthogonality record, and the mirror flag of a transposed solve.
static size_t ws_round(size_t b) { return (b + 255) & ~size_t(255); }
size_t sstep_workspace_bytes(int64_t N, const sstep_opts_t &o) {
  const int s = o.s, m = o.restart;
  const bool lagged = (o.flags & SSTEP_FLAG_LAGGED) != 0 && (o.flags & SSTEP_FLAG_CLASSICAL) == 0;
  size_t t = 0;
  t += ws_round(size_t(N) * (m + 1) * 8) + 2 * ws_round(size_t(N) * 8) + ws_round(sizeof(KrylovDev));
  const int64_t nchunk = std::max<int64_t>(cdiv(N, TS_CHUNK), cdiv(N, 4096));
  int64_t npart = nchunk * TS_MAXA * TS_MAXS;
  if (lagged) npart = std::max(npart, gram_wide_part_elems(N, m + 1, 2 * s));
  t += ws_round(size_t(npart) * 8);
  if (o.flags & SSTEP_FLAG_ORTH_LOSS) t += ws_round(size_t(m + 1) * (m + 1) * 8);
  if (o.transpose) t += ws_round(64);
  return t;
}

int sstep_solve(const spand_bsr_t &A0, Factor *M, int member, const double *b, double *x,
                const sstep_opts_t &o, sstep_stats_t *st, hipStream_t stream,
                const SolveWorkspace *ws) {
  const int64_t N = int64_t(A0.n_brows) * A0.bs;
  const int s = o.s, m = o.restart;
  const double rtol = o.rtol;
  const int maxit = o.maxit;
  const int tr = o.transpose != 0;
  // stability-study variants (Sec. CAGMRES, Fig. 6): monomial basis, one
  // orthogonalisation pass, loss of orthogonality after every block
  const bool monomial = (o.flags & SSTEP_FLAG_MONOMIAL) != 0;
  const int passes = (o.flags & SSTEP_FLAG_ONE_PASS) ? 1 : 2;
  const bool orth_log = (o.flags & SSTEP_FLAG_ORTH_LOSS) != 0;
  // classical GMRES (Algorithm 1): every column by the Arnoldi step with
  // modified Gram-Schmidt, no blocks
  const bool classical = (o.flags & SSTEP_FLAG_CLASSICAL) != 0;
  // single-reduce schedule (Algorithm 2): the second pass of a block lagged
  // into the one Gram matrix of the next block
  const bool lagged = (o.flags & SSTEP_FLAG_LAGGED) != 0 && !classical;
  if (lagged && passes == 1) {
    set_error("the single-reduce schedule needs two passes");
    return SPAND_EINVAL;
  }
  std::vector<double> orth_loss;
  std::vector<int> orth_cols;
  std::vector<std::pair<void *, size_t>> allocs;
  size_t ws_used = 0;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(stream);     // nothing queued may still use them
    for (auto &a : allocs) pool_release(a.first, a.second);
  };
  // from the device block cache, or carved from the caller's workspace
  auto alloc = [&](void **p, size_t bytes) -> int {
    if (ws) {
      const size_t need = ws_round(bytes);
      if (ws_used + need > ws->bytes) {
        set_error("solve workspace exceeds %zu bytes", ws->bytes);
        return SPAND_EINVAL;
      }
      *p = (char *)ws->base + ws_used;
      ws_used += need;
      return SPAND_OK;
    }
    size_t got = 0;
    SP_TRY(pool_alloc(p, bytes, &got));
    allocs.push_back({*p, got});
    return SPAND_OK;
  };
#define GTRY(e)            \
  do {                     \
    int r__ = (e);         \
    if (r__ < 0) {         \
      cleanup();           \
      return r__;          \
    }                      \
  } while (0)
  const spand_bsr_t &A = A0;
  void *pQ, *pZ, *pR, *pK, *pPart;
  GTRY(alloc(&pQ, size_t(N) * (m + 1) * 8));
  GTRY(alloc(&pZ, size_t(N) * 8));
  GTRY(alloc(&pR, size_t(N) * 8));
  GTRY(alloc(&pK, sizeof(KrylovDev)));
  const int64_t nchunk = std::max<int64_t>(cdiv(N, TS_CHUNK), cdiv(N, 4096));
  int64_t npart = nchunk * TS_MAXA * TS_MAXS;
  if (lagged) npart = std::max(npart, gram_wide_part_elems(N, m + 1, 2 * s));
  GTRY(alloc(&pPart, size_t(npart) * 8));
  double *Q = (double *)pQ, *Z = (double *)pZ, *Rv = (double *)pR, *part = (double *)pPart;
  double *Gq = nullptr;      // Gram matrix of the basis (diagnostic)
  if (orth_log) {
    void *pG;
    GTRY(alloc(&pG, size_t(m + 1) * (m + 1) * 8));
    Gq = (double *)pG;
  }
  if (tr) {
    // A^T products read the mirror blocks of A in place (no transposed
    // copy); the block pattern must be structurally symmetric
    void *fl;
    GTRY(alloc(&fl, 64));
    if (hipMemsetAsync(fl, 0, 64, stream) != hipSuccess) GTRY(SPAND_EHIP);
    GTRY(launch_spmv_t_check(A, (int *)fl, stream));
    int flag = 0;
    if (hipMemcpyAsync(&flag, fl, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      GTRY(SPAND_EHIP);
    if (flag) {
      set_error("transpose solve needs a structurally symmetric block pattern");
      cleanup();
      return SPAND_EINVAL;
    }
  }
  // ||Q^T Q - I||_F of the first nc basis vectors: Gram matrix in column
  // chunks of the block kernels' width, then on the host
  auto record_orth = [&](int nc) -> int {
    for (int c0 = 0; c0 < nc; c0 += TS_MAXS)
      SP_TRY(launch_gram(N, Q, N, nc, Q + int64_t(c0) * N, N, std::min(TS_MAXS, nc - c0), part,
                         Gq + c0, nc, stream));
    std::vector<double> G(size_t(nc) * nc);
    SP_HIP(hipMemcpyAsync(G.data(), Gq, G.size() * 8, hipMemcpyDeviceToHost, stream));
    SP_HIP(hipStreamSynchronize(stream));
    double f = 0.0;
    for (int r = 0; r < nc; ++r)
      for (int c = 0; c < nc; ++c) {
        const double d = G[size_t(r) * nc + c] - (r == c ? 1.0 : 0.0);
        f += d * d;
      }
    orth_loss.push_back(std::sqrt(f));
    orth_cols.push_back(nc);
    return SPAND_OK;
  };
  if (hipMemsetAsync(Z, 0, size_t(N) * 8, stream) != hipSuccess) GTRY(SPAND_EHIP);
  // lanes per row, once per block size (a caller's workspace means a call
  // that must not allocate or time: it keeps the tuned or default lanes)
  if (!ws) GTRY(autotune_spmv(A, Z, Rv, stream));
  KrylovDev *Kd = (KrylovDev *)pK;
  const int ld = KRY_MMAX;
  PhaseTimer tm;
  tm.on = st != nullptr && !ws;
  tm.st = stream;
  double ph[T_N] = {0, 0, 0, 0};
  hipEvent_t e0, e1;
  if (tm.on) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, stream);
  }
  int n_spmv = 0, n_apply = 0, n_reduce = 0;   // n_reduce: inner-product reductions
  auto Minv = [&](const double *in, double *out) -> int {
    ++n_apply;
    if (M) return M->apply(in, out, tr, stream, member);
    if (in != out)
      SP_HIP(hipMemcpyAsync(out, in, size_t(N) * 8, hipMemcpyDeviceToDevice, stream));
    return SPAND_OK;
  };
  // out = A M^-1 v + ca*w1 + cb*w2
  auto Ahat = [&](const double *v, double *out, const double *w1, double c1, const double *w2,
                  double c2) -> int {
    tm.mark(T_APPLY);
    SP_TRY(Minv(v, Z));
    tm.mark(T_SPMV);
    ++n_spmv;
    SP_TRY(launch_spmv(A, tr, 1.0, Z, 0.0, out, w1, c1, w2, c2, stream));
    tm.mark(T_OTHER);
    return SPAND_OK;
  };
  auto d2h = [&](void *dst, const void *src, size_t bytes) -> int {
    SP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
    SP_HIP(hipStreamSynchronize(stream));
    return SPAND_OK;
  };
  std::vector<double> hist;
  int iters = 0, restarts = 0, converged = 0, breakdown = 0;
  double relres = 0.0;
  std::vector<Slot> slots;
  tm.mark(T_OTHER);
  // ||b||
  ++n_reduce;
  GTRY(launch_dot(N, b, b, part, Kd->scal + 1, 1, stream));
  double bnorm = 0.0;
  GTRY(d2h(&bnorm, Kd->scal + 1, 8));
  if (!(bnorm > 0.0)) {
    if (hipMemsetAsync(x, 0, size_t(N) * 8, stream) != hipSuccess) GTRY(SPAND_EHIP);
    converged = 1;
    relres = 0.0;
  }
  const double tol = rtol * bnorm;
  while (!converged) {
    // r = b - A x, beta = ||r||
    if (hipMemcpyAsync(Rv, b, size_t(N) * 8, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      GTRY(SPAND_EHIP);
    tm.mark(T_SPMV);
    ++n_spmv;
    GTRY(launch_spmv(A, tr, -1.0, x, 1.0, Rv, nullptr, 0.0, nullptr, 0.0, stream));
    tm.mark(T_OTHER);
    ++n_reduce;
    GTRY(launch_dot(N, Rv, Rv, part, Kd->scal, 1, stream));
    double beta = 0.0;
    GTRY(d2h(&beta, Kd->scal, 8));
    relres = beta / bnorm;
    if (beta <= tol) {
      converged = 1;
      break;
    }
    if (iters >= maxit || breakdown) break;
    GTRY(vec_axpby(N, Rv, Q, 1.0, Kd->scal, 1, 0.0, stream));
    GTRY(kry_init_cycle(Kd, m, stream));
    int k = 0, j = 0;
    bool done = false;
    if (slots.empty() && monomial && !classical) {
      // all shifts zero: W = [A q, A^2 q, ...] from the first column on
      slots.assign(size_t(s), Slot{0, 0.0, 0.0});
      std::vector<double> Bb(size_t(s + 1) * s, 0.0);
      for (int q = 1; q <= s; ++q) Bb[size_t(q) * s + q - 1] = 1.0;
      if (hipMemcpyAsync(Kd->Bb, Bb.data(), Bb.size() * 8, hipMemcpyHostToDevice, stream) !=
          hipSuccess)
        GTRY(SPAND_EHIP);
      if (hipStreamSynchronize(stream) != hipSuccess) GTRY(SPAND_EHIP);
    }
    if (slots.empty()) {
      const int nsteps = classical ? m : s;
      for (int jj = 0; jj < nsteps; ++jj) {
        double *w = Q + (jj + 1) * N;
        GTRY(Ahat(Q + jj * N, w, nullptr, 0.0, nullptr, 0.0));
        tm.mark(T_ORTH);
        for (int i = 0; i <= jj; ++i) {
          double *hij = Kd->H + i * ld + jj;
          ++n_reduce;
    GTRY(launch_dot(N, w, Q + i * N, part, hij, 0, stream));
          GTRY(vec_axpby(N, Q + i * N, w, -1.0, hij, 0, 1.0, stream));
        }
        double *hn = Kd->H + (jj + 1) * ld + jj;
        ++n_reduce;
    GTRY(launch_dot(N, w, w, part, hn, 1, stream));
        GTRY(vec_axpby(N, w, w, 1.0, hn, 1, 0.0, stream));
        GTRY(kry_givens_col(Kd, jj, stream));
        tm.mark(T_OTHER);
        double hv[2];
        GTRY(d2h(&hv[0], Kd->est + jj, 8));
        GTRY(d2h(&hv[1], hn, 8));
        ++iters;
        hist.push_back(hv[0]);
        k = jj + 1;
        if (hv[1] == 0.0 || hv[0] <= tol || iters >= maxit) {
          done = true;
          break;
        }
      }
      // Shifts are fixed here even when the cycle already ended inside these
      // steps (then all zero, a monomial basis): a later cycle whose true
      // residual is still above the tolerance goes straight to the blocks.
      if (classical) {
        done = true;            // the cycle's m columns are all Arnoldi steps
      } else {
        std::vector<std::complex<double>> ev(s, 0.0);
        if (!done) {
          std::vector<double> Hh(size_t(s) * s);
          for (int i = 0; i < s; ++i) GTRY(d2h(&Hh[size_t(i) * s], Kd->H + i * ld, size_t(s) * 8));
          if (!hessenberg_eigs(Hh, s, ev)) ev.assign(s, 0.0);
        }
        for (auto &z : ev)
          if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) z = 0.0;
        slots = leja_slots(ev, s);
        while (int(slots.size()) < s) slots.push_back({0, 0.0, 0.0});
        std::vector<double> Bb(size_t(s + 1) * s, 0.0);
        for (int q = 1; q <= s; ++q) {
          const Slot &sl = slots[q - 1];
          if (sl.kind == 2) {
            Bb[size_t(q - 2) * s + q - 1] = -sl.b * sl.b;
          }
          Bb[size_t(q - 1) * s + q - 1] = sl.a;
          Bb[size_t(q) * s + q - 1] = 1.0;
        }
        if (hipMemcpyAsync(Kd->Bb, Bb.data(), Bb.size() * 8, hipMemcpyHostToDevice, stream) !=
            hipSuccess)
          GTRY(SPAND_EHIP);
        if (hipStreamSynchronize(stream) != hipSuccess) GTRY(SPAND_EHIP);
      }
      j = s;
    }
    // Single-reduce schedule.  j: last basis column (start of the next
    // operator applications); with a pending block P = Q[:, j-s+1:j+1] (one
    // pass, Hessenberg columns j0..j0+s-1 not yet assembled).  Each step: s
    // applications from q_j, one Gram matrix, the dense step, one pass over
    // the rows.  The last block of a cycle is finished by a step with no new
    // block; so is a block whose one-pass residual estimate already meets the
    // tolerance (then no applications are spent past convergence).
    bool pend = false, finish_now = false;
    int j0 = 0;
    while (lagged && !done) {
      const int sw = (j < m && !(pend && finish_now)) ? s : 0;
      if (!pend && sw == 0) break;
      for (int q = 1; q <= sw; ++q) {
        const Slot &sl = slots[q - 1];
        double *prev = Q + (j + q - 1) * N;
        double *out = Q + (j + q) * N;
        if (sl.kind == 2)
          GTRY(Ahat(prev, out, prev, -sl.a, Q + (j + q - 2) * N, sl.b * sl.b));
        else
          GTRY(Ahat(prev, out, prev, -sl.a, nullptr, 0.0));
      }
      tm.mark(T_ORTH);
      const int sp = pend ? s : 0, a = j + 1 - sp;
      ++n_reduce;
      GTRY(launch_gram_wide(N, Q, N, a + sp + sw, Q + int64_t(a) * N, N, sp + sw, part, Kd->LG,
                            sp + sw, stream));
      GTRY(kry_lag_block(Kd, a, sp, sw, s, stream));
      GTRY(launch_ts_lag_update(N, Q, N, a, sp, sw, s, Kd, stream));
      tm.mark(T_OTHER);
      int bad = 0;
      GTRY(d2h(&bad, &Kd->bad, 4));
      if (sp) {
        if (bad == 1) {
          breakdown = 1;
          k = j0;      // keep the columns before the pending block
          break;
        }
        if (orth_log) GTRY(record_orth(j0 + s + 1));
        std::vector<double> est(s);
        GTRY(d2h(est.data(), Kd->est + j0, size_t(s) * 8));
        for (int c = j0; c < j0 + s; ++c) {
          ++iters;
          hist.push_back(est[c - j0]);
          k = c + 1;
          if (est[c - j0] <= tol || iters >= maxit) {
            done = true;
            break;
          }
        }
      }
      if (done || !sw) {
        pend = false;
        continue;
      }
      if (bad == 2) {
        breakdown = 1;
        break;
      }
      std::vector<double> et(s);
      GTRY(d2h(et.data(), Kd->est_t, size_t(s) * 8));
      pend = true;
      j0 = j;
      j += s;
      const double emin = *std::min_element(et.begin(), et.end());
      finish_now = emin <= kEagerFinish * tol || j >= m || iters + s >= maxit;
    }
    while (!lagged && !done && j < m) {
      for (int q = 1; q <= s; ++q) {
        const Slot &sl = slots[q - 1];
        double *prev = Q + (j + q - 1) * N;
        double *out = Q + (j + q) * N;
        if (sl.kind == 2)
          GTRY(Ahat(prev, out, prev, -sl.a, Q + (j + q - 2) * N, sl.b * sl.b));
        else
          GTRY(Ahat(prev, out, prev, -sl.a, nullptr, 0.0));
      }
      tm.mark(T_ORTH);
      double *W = Q + (j + 1) * N;
      const int a = j + 1;
      double *Rp[2] = {Kd->R1, Kd->R2};
      double *Tp[2] = {Kd->T1, Kd->T2};
      for (int pass = 0; pass < passes; ++pass) {
        ++n_reduce;
        GTRY(launch_gram(N, Q, N, a, W, N, s, part, Rp[pass], s, stream));
        GTRY(launch_ts_update(N, Q, N, a, Rp[pass], s, W, N, s, stream));
        ++n_reduce;
        GTRY(launch_gram(N, W, N, s, W, N, s, part, Kd->G, s, stream));
        GTRY(kry_chol(Kd, s, Kd->G, Tp[pass], stream));
        GTRY(launch_ts_trsm(N, W, N, s, Tp[pass], &Kd->bad, stream));
      }
      GTRY(kry_block_finish(Kd, j, s, passes, stream));
      tm.mark(T_OTHER);
      if (orth_log) GTRY(record_orth(j + s + 1));
      std::vector<double> est(s);
      int bad = 0;
      GTRY(d2h(est.data(), Kd->est + j, size_t(s) * 8));
      GTRY(d2h(&bad, &Kd->bad, 4));
      if (bad) {
        breakdown = 1;
        done = true;
        k = j;      // keep the columns before this block
        break;
      }
      for (int c = j; c < j + s; ++c) {
        ++iters;
        hist.push_back(est[c - j]);
        k = c + 1;
        if (est[c - j] <= tol || iters >= maxit) {
          done = true;
          break;
        }
      }
      j += s;
    }
    if (k > 0) {
      GTRY(kry_lsq(Kd, k, stream));
      GTRY(launch_ts_gemv(N, Q, N, k, Kd->y, Rv, stream));
      tm.mark(T_APPLY);
      GTRY(Minv(Rv, Z));
      tm.mark(T_OTHER);
      GTRY(vec_axpby(N, Z, x, 1.0, nullptr, 0, 1.0, stream));
    }
    ++restarts;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) GTRY(SPAND_EHIP);
  if (st) {
    if (tm.on) {
      (void)hipEventRecord(e1, stream);
      (void)hipEventSynchronize(e1);
      float tt = 0.f;
      (void)hipEventElapsedTime(&tt, e0, e1);
      tm.mark(T_OTHER);
      tm.collect(ph);
      st->t_total_ms = tt;
      st->t_spmv_ms = ph[T_SPMV];
      st->t_apply_ms = ph[T_APPLY];
      st->t_orth_ms = ph[T_ORTH];
      st->t_other_ms = ph[T_OTHER];
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    st->n_spmv = n_spmv;
    st->n_apply = n_apply;
    st->iters = iters;
    st->restarts = restarts;
    st->converged = converged;
    st->relres = relres;
    st->n_hist = int(std::min<size_t>(hist.size(), SSTEP_MAX_HIST));
    for (int i = 0; i < st->n_hist; ++i) st->hist[i] = hist[i];
    st->n_reduce = n_reduce;
    st->n_orth = int(std::min<size_t>(orth_loss.size(), SSTEP_MAX_HIST));
    for (int i = 0; i < st->n_orth; ++i) {
      st->orth_loss[i] = orth_loss[i];
      st->orth_cols[i] = orth_cols[i];
    }
    st->n_shifts = int(std::min<size_t>(slots.size(), 8));
    for (int i = 0; i < st->n_shifts; ++i) {
      st->shift_re[i] = slots[i].a;
      st->shift_im[i] = slots[i].kind == 0 ? 0.0 : (slots[i].kind == 1 ? slots[i].b : -slots[i].b);
    }
  }
  cleanup();
#undef GTRY
  if (converged) return SPAND_OK;
  if (breakdown) {
    set_error("Cholesky QR met a Gram matrix that is not positive definite");
    return SPAND_EBREAKDOWN;
  }
  set_error("maximum number of iterations reached (relres %.3e)", relres);
  return SPAND_ENOTCONV;
}

}  // namespace spand
