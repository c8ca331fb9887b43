// Batched Krylov solvers for A x = b on the plan's operator.
//
// GMRES(m) (named with Bi-CGStab as a suitable unpreconditioned iteration in
// the Introduction and Discussion) with classical Gram-Schmidt and selective
// re-orthogonalisation, Givens rotations and the small least-squares solve on
// the host in FP64.  A classical pass loses orthogonality roughly like
// eps (||r_0|| / ||r_j||)^2, so a second pass is made once the cycle's residual
// estimate has dropped below 1e-6 ||r_0||, or when the first pass cancels all
// but 1e-4 of ||w||^2.  FP32 inner cycles of the mixed solver stop above that
// level and run single-pass.  Bi-CGStab is the solver of Section 5.
//
// Mixed precision: the outer loop recomputes the true residual
// r = b - A x with the FP64 apply and solves A d = r with the FP32 apply
// (Krylov vectors, Arnoldi and least squares stay FP64), x += d, until
// ||r|| / ||b|| <= tol.  Plain FP64 runs the same loop with the FP64 apply.
//
// Right-hand sides are advanced together in fused launches, but every
// decision (re-orthogonalisation, convergence, stagnation, inner cycle
// length, budget) is taken per right-hand side, every launch touches a slot
// only with that slot's own coefficients, and every reduction has a fixed
// order, so a right-hand side gets bitwise the same answer alone or in a
// batch.  Slots that have stopped are skipped by the launches (device flags
// per slot).
//
// Stagnation: a slot whose true residual has not fallen below 0.9 times its
// value of kStallMatvecs (or 3 restart cycles, if longer) matvecs earlier
// stops with VIE_W_NOCONV.  A slot that stops without reaching its target
// (stagnation, budget, a non-finite residual) returns the iterate with the
// smallest true residual it had.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <limits>
#include <vector>

#include "apply_kernels.hpp"
#include "plan.hpp"
#include "pointwise.hpp"

namespace vie {

namespace {

using cd = std::complex<double>;

inline size_t zu(long v) { return static_cast<size_t>(v); }

// VIE_TRACE=1: one line per GMRES iteration and right-hand side on stderr
bool trace_on() {
  static const bool on = [] {
    const char* v = std::getenv("VIE_TRACE");
    return v && *v && *v != '0';
  }();
  return on;
}

struct RhsState {
  double bnorm = 0, rnorm = 0;
  bool done = false, conv = false;
  int iters = 0, mv32 = 0, mv64 = 0, refine = 0;
  double best = 0;            // smallest true residual so far (its iterate is in xbest)
  double ref = 0;             // stagnation reference: true residual at matvec count ref_mv
  int ref_mv = 0;
  int matvecs() const { return mv32 + mv64; }
};

constexpr int kStallMatvecs = 300;

// Work vectors for batches of `cap` right-hand sides and bases of m + 1 vectors.
int ensure_krylov(vie_plan* pl, int cap, int m, hipStream_t s) {
  if (pl->kr_cap >= cap && pl->kr_m >= m) return VIE_OK;
  // pending copies may still read the old staging buffers
  HIPCHK(pl, hipStreamSynchronize(s));
  if (pl->gstream) HIPCHK(pl, hipStreamSynchronize(pl->gstream));
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  cap = std::max(cap, pl->kr_cap);
  m = std::max(m, pl->kr_m);
  dev_free(pl, pl->V);
  dev_free(pl, pl->xw);
  dev_free(pl, pl->bw);
  dev_free(pl, pl->rw);
  dev_free(pl, pl->ww);
  dev_free(pl, pl->xbest);
  dev_free(pl, pl->partials);
  dev_free(pl, pl->red);
  dev_free(pl, pl->stage_dev);
  dev_free(pl, pl->actd);
  pl->V = pl->xw = pl->bw = pl->rw = pl->ww = pl->xbest = pl->partials = pl->red = nullptr;
  pl->stage_dev = nullptr;
  pl->actd = nullptr;
  pl->act_last.clear();
  host_free(pl, pl->red_host);
  host_free(pl, pl->stage_host);
  pl->red_host = nullptr;
  pl->stage_host = nullptr;
  pl->kr_cap = pl->kr_m = 0;
  const size_t L = zu(pl->C) * zu(pl->box.np);  // vectors hold the support rows of the box
  const size_t nblk = zu(krylov_blocks(long(L)));
  const size_t vec = sizeof(c128) * L * zu(cap);
  int rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->V), vec * zu(m + 1));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->xw), vec);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->bw), vec);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->rw), vec);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->ww), vec);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->xbest), vec);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->partials), sizeof(c128) * zu(cap) * nblk * zu(m + 2));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->red), sizeof(c128) * zu(cap) * zu(m + 2));
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  pl->stage_off_count = sizeof(double) * zu(cap);
  pl->stage_off_coef = up(pl->stage_off_count + sizeof(int) * zu(cap));
  pl->stage_bytes = up(pl->stage_off_coef + sizeof(c128) * zu(cap) * zu(m + 2));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->stage_dev), 2 * pl->stage_bytes);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->actd), sizeof(int) * zu(cap));
  if (rc) return rc;
  rc = host_alloc(pl, reinterpret_cast<void**>(&pl->red_host), sizeof(c128) * zu(cap) * zu(m + 2));
  if (!rc) rc = host_alloc(pl, reinterpret_cast<void**>(&pl->stage_host), 2 * pl->stage_bytes);
  if (rc) return rc;
  pl->stage_epoch[0] = pl->stage_epoch[1] = -1;
  pl->kr_cap = cap;
  pl->kr_m = m;
  return VIE_OK;
}

// Context of one batch: nb right-hand sides in slots 0..nb-1 of the work vectors.
struct Batch {
  vie_plan* pl;
  hipStream_t s;
  int nb;
  long L;      // vector length C bx by bz (the support box)
  long vs;     // basis vector stride (cap * L)
  int nblk;
};

// Device flags of the right-hand sides that take part in the next launches
// (kernels skip the others entirely), or null when all do or the batch is
// too large to flag; *nact = how many take part.
const int* set_active(const Batch& b, const std::vector<bool>& active, int* nact, int* rc) {
  vie_plan* pl = b.pl;
  *rc = VIE_OK;
  int n = 0;
  for (int r = 0; r < b.nb; ++r) n += active[zu(r)] ? 1 : 0;
  *nact = n;
  if (n == b.nb || b.nb > kMaxFlagged) {
    *nact = b.nb;
    return nullptr;
  }
  std::vector<int> want(static_cast<size_t>(b.nb));
  unsigned long long words[4] = {0, 0, 0, 0};
  for (int r = 0; r < b.nb; ++r) {
    want[zu(r)] = active[zu(r)] ? 1 : 0;
    if (active[zu(r)]) words[r >> 6] |= 1ull << (r & 63);
  }
  if (want != pl->act_last) {
    const hipError_t e = launch_set_flags(words, b.nb, pl->actd, b.s);
    if (e != hipSuccess) {
      *rc = hip_fail(pl, e, "launch_set_flags");
      return nullptr;
    }
    pl->act_last = want;
  }
  return pl->actd;
}

// red[r][0..nv] <- (conj(V_i) . w_r, ||w_r||^2), copied to the host (slots
// flagged off in act are skipped and their entries are meaningless)
template <typename TV, typename TW>
int dots_host(const Batch& b, const TV* V, const TW* w, int nv, const int* act = nullptr, int nact = -1) {
  vie_plan* pl = b.pl;
  const double nrun = act && nact >= 0 ? nact : b.nb;
  int tok = prof_begin(pl, b.s);
  HIPCHK(pl, launch_dots(V, b.vs, b.L, w, b.L, nv, b.nb, b.nblk, pl->partials, b.s, act));
  prof_end(pl, FAM_DOTS, tok, b.s, (double(nv) * sizeof(TV) + sizeof(TW)) * nrun * double(b.L),
           (8.0 * nv + 4.0) * nrun * double(b.L));
  tok = prof_begin(pl, b.s);
  HIPCHK(pl, launch_reduce(pl->partials, b.nb, b.nblk, nv + 1, pl->red, b.s, act));
  prof_end(pl, FAM_REDUCE, tok, b.s, double(b.nb) * (b.nblk + 1) * (nv + 1) * sizeof(c128));
  HIPCHK(pl, hipMemcpyAsync(pl->red_host, pl->red, sizeof(c128) * zu(b.nb) * zu(nv + 1),
                            hipMemcpyDeviceToHost, b.s));
  HIPCHK(pl, hipStreamSynchronize(b.s));
  pl->sync_count++;
  return VIE_OK;
}

cd red_at(const Batch& b, int r, int i, int nv1) {
  const c128 v = b.pl->red_host[zu(r) * zu(nv1) + zu(i)];
  return {v.re, v.im};
}

// out_r = (w_r - sum_{i<nv} V_i c[r][i]) * scale[r], coefficients from host arrays
// counts (optional): right-hand side r uses its first counts[r] coefficients
// and is skipped (out left as it was) when counts[r] < 0
template <typename TV, typename TW, typename TO>
int combine_host(const Batch& b, const TV* V, const TW* w, TO* out, int nv, const std::vector<cd>& coef,
                 const std::vector<double>& scale, const std::vector<int>* counts = nullptr) {
  vie_plan* pl = b.pl;
  if (b.L <= 0) return VIE_OK;  // no unknowns (H = 0 everywhere): nothing to combine
  const int stride = std::max(nv, 1);
  // vectors read per right-hand side (for the byte counts)
  double nvec = 0.0, nrun = 0.0;
  for (int r = 0; r < b.nb; ++r) {
    const int k = counts ? std::min((*counts)[zu(r)], nv) : nv;
    if (k >= 0) {
      nvec += k;
      nrun += 1.0;
    }
  }
  const double bytes = (nvec * sizeof(TV) + nrun * (sizeof(TW) + sizeof(TO))) * double(b.L);
  const double flops = (8.0 * nvec + 2.0 * nrun) * double(b.L);
  if (b.nb <= kArgRhs && b.nb * stride <= kArgCoef) {
    // small batches: the coefficients travel as kernel arguments
    CombineArgs a;
    for (int r = 0; r < b.nb; ++r) {
      a.scale[r] = scale[zu(r)];
      a.count[r] = counts ? std::min((*counts)[zu(r)], nv) : nv;
      for (int i = 0; i < stride; ++i) {
        const cd c = i < nv ? coef[zu(r) * zu(nv) + zu(i)] : cd(0.0, 0.0);
        a.coef[r * stride + i] = {c.real(), c.imag()};
      }
    }
    const int tok = prof_begin(pl, b.s);
    HIPCHK(pl, launch_combine_args(V, b.vs, b.L, w, out, b.L, nv, a, b.nb, b.s));
    prof_end(pl, FAM_COMBINE, tok, b.s, bytes, flops);
    return VIE_OK;
  }
  // two staging slots used alternately; a slot is rewritten only after the
  // stream has been synchronised since its copies were queued
  const int slot = pl->stage_next;
  pl->stage_next ^= 1;
  if (pl->stage_epoch[slot] == pl->sync_count) {
    HIPCHK(pl, hipStreamSynchronize(b.s));
    pl->sync_count++;
  }
  pl->stage_epoch[slot] = pl->sync_count;
  unsigned char* hb = pl->stage_host + zu(slot) * pl->stage_bytes;
  unsigned char* db = pl->stage_dev + zu(slot) * pl->stage_bytes;
  double* sh = reinterpret_cast<double*>(hb);
  int* nh = reinterpret_cast<int*>(hb + pl->stage_off_count);
  c128* ch = reinterpret_cast<c128*>(hb + pl->stage_off_coef);
  const double* sdv = reinterpret_cast<const double*>(db);
  const int* ndv = reinterpret_cast<const int*>(db + pl->stage_off_count);
  const c128* cdv = reinterpret_cast<const c128*>(db + pl->stage_off_coef);
  for (int r = 0; r < b.nb; ++r) {
    for (int i = 0; i < stride; ++i) {
      const cd c = i < nv ? coef[zu(r) * zu(nv) + zu(i)] : cd(0.0, 0.0);
      ch[zu(r) * zu(stride) + zu(i)] = {c.real(), c.imag()};
    }
    sh[r] = scale[zu(r)];
  }
  for (int r = 0; r < b.nb; ++r)
    if (counts) nh[r] = std::min((*counts)[zu(r)], nv);
  // one copy: scales, counts and the used coefficients
  const size_t used = pl->stage_off_coef + sizeof(c128) * zu(b.nb) * zu(stride);
  HIPCHK(pl, hipMemcpyAsync(db, hb, used, hipMemcpyHostToDevice, b.s));
  const int tok = prof_begin(pl, b.s);
  HIPCHK(pl, launch_combine(V, b.vs, b.L, w, out, b.L, nv, cdv, sdv, b.nb, b.s, counts ? ndv : nullptr));
  prof_end(pl, FAM_COMBINE, tok, b.s, bytes, flops);
  return VIE_OK;
}

// counts of combine_host: nv for the flagged right-hand sides, -1 (skip) for the others
std::vector<int> counts_of(const std::vector<bool>& active, int nv) {
  std::vector<int> c(active.size());
  for (size_t r = 0; r < active.size(); ++r) c[r] = active[r] ? nv : -1;
  return c;
}

// ||v_r|| for every slot (for the flagged ones only when act is given; the
// others' entries are then meaningless)
int norms(const Batch& b, const c128* v, std::vector<double>& out, const int* act = nullptr, int nact = -1) {
  int rc = dots_host(b, static_cast<const c128*>(nullptr), v, 0, act, nact);
  if (rc) return rc;
  out.resize(zu(b.nb));
  for (int r = 0; r < b.nb; ++r) {
    // a NaN sum stays NaN (std::max would turn it into 0, i.e. "b = 0")
    const double v = red_at(b, r, 0, 1).real();
    out[zu(r)] = std::isnan(v) ? v : std::sqrt(std::max(0.0, v));
  }
  return VIE_OK;
}

// One GMRES(m) cycle on A d = r (r in rw, x += d in xw).  target[r]: absolute
// residual at which slot r stops; active[r]: slot takes part; budget[r]:
// matvecs it may still spend.  A slot's update x += V y is made in the
// iteration where it stops (target, breakdown, budget or the cycle's last),
// in place of the basis vector it would not use, so the basis is read once
// less per cycle.
// The basis stays complex128 in the FP32 inner cycles too: rounding it to
// complex64 acts as a unit roundoff of 6e-8 in the classical Gram-Schmidt
// bound above, and orthogonality is gone once the residual has dropped by
// about 1e-4, before the inner target of 1e-5.
int gmres_cycle(const Batch& b, bool fp64, int m, const std::vector<double>& rnorm, const std::vector<double>& target,
                std::vector<RhsState>& st, const std::vector<bool>& active_in, const std::vector<int>& budget) {
  vie_plan* pl = b.pl;
  c128* basis = pl->V;
  c128* wv = pl->ww;
  // FP32 inner cycles: w = A v_j holds FP32 values and is stored as complex64
  // (half the traffic of its write, of the multi-dot and of the combine)
  c64* wv32 = reinterpret_cast<c64*>(pl->ww);
  const bool w32 = !fp64;
  const int nb = b.nb;
  std::vector<bool> active = active_in;
  std::vector<double> scale(static_cast<size_t>(nb));
  std::vector<cd> none;
  // V_0 = r / ||r||
  for (int r = 0; r < nb; ++r) scale[zu(r)] = (active[zu(r)] && rnorm[zu(r)] > 0) ? 1.0 / rnorm[zu(r)] : 0.0;
  for (int r = 0; r < nb; ++r)
    if (!(rnorm[zu(r)] > 0)) active[zu(r)] = false;
  // Slots that are not active are skipped by every launch below (applies,
  // dots, combines): their basis vectors keep whatever they held, and the
  // final update reads only the vectors each slot wrote in this cycle.
  std::vector<int> cnt = counts_of(active, 0);
  int rc = combine_host(b, static_cast<const c128*>(nullptr), pl->rw, basis, 0, none, scale, &cnt);
  if (rc) return rc;
  // Hessenberg (column-major, (m+1) x m), rotations, rhs g
  std::vector<std::vector<cd>> Hs(static_cast<size_t>(nb), std::vector<cd>(zu((m + 1) * m)));
  std::vector<std::vector<double>> cs(static_cast<size_t>(nb), std::vector<double>(zu(m)));
  std::vector<std::vector<cd>> sn(static_cast<size_t>(nb), std::vector<cd>(zu(m)));
  std::vector<std::vector<cd>> g(static_cast<size_t>(nb), std::vector<cd>(zu(m + 1)));
  for (int r = 0; r < nb; ++r) g[zu(r)][0] = rnorm[zu(r)];
  const double eta2 = 1e-4;   // re-orthogonalise when ||w'||^2 < 1e-4 ||w||^2 ...
  const double deep = 1e-6;   // ... or once |g_j| < 1e-6 ||r_0||
  std::vector<cd> h1(zu(nb) * zu(m + 1)), h2(zu(nb) * zu(m + 1));
  std::vector<double> w2(static_cast<size_t>(nb)), wp2(zu(nb));
  std::vector<bool> reorth(static_cast<size_t>(nb));
  int j = 0;
  for (j = 0; j < m; ++j) {
    bool any = false;
    for (int r = 0; r < nb; ++r) any = any || active[zu(r)];
    if (!any) break;
    const c128* Vj = basis + long(j) * b.vs;
    c128* Vn = basis + long(j + 1) * b.vs;
    int nact = 0;
    const int* act = set_active(b, active, &nact, &rc);
    if (rc) return rc;
    rc = w32 ? apply_graph(pl, pl->box, Vj, wv32, nb, b.s, act, nact)
             : apply_graph(pl, pl->box, fp64, Vj, Vj, nullptr, wv, nb, MODE_MATVEC, b.s, act, nact);
    if (rc) return rc;
    const int nv = j + 1;
    rc = w32 ? dots_host(b, basis, wv32, nv, act, nact) : dots_host(b, basis, wv, nv, act, nact);
    if (rc) return rc;
    bool any_reorth = false;
    for (int r = 0; r < nb; ++r) {
      double p = 0;
      for (int i = 0; i < nv; ++i) {
        const cd v = red_at(b, r, i, nv + 1);
        h1[zu(r) * zu(nv) + zu(i)] = v;
        p += std::norm(v);
      }
      w2[zu(r)] = red_at(b, r, nv, nv + 1).real();
      wp2[zu(r)] = w2[zu(r)] - p;
      const bool converged_far = std::abs(g[zu(r)][zu(j)]) < deep * rnorm[zu(r)];
      reorth[zu(r)] = active[zu(r)] && (wp2[zu(r)] < eta2 * w2[zu(r)] || converged_far);
      any_reorth = any_reorth || reorth[zu(r)];
    }
    std::vector<cd> hcol(zu(nb) * zu(nv + 1));
    std::vector<cd> coef2(zu(nb) * zu(nv), cd(0, 0));
    for (int r = 0; r < nb; ++r)
      for (int i = 0; i < nv; ++i) hcol[zu(r) * zu(nv + 1) + zu(i)] = h1[zu(r) * zu(nv) + zu(i)];
    if (any_reorth) {
      std::vector<double> one(static_cast<size_t>(nb), 1.0);
      // w <- w - V h1 for the slots that re-orthogonalise only (the others
      // form V_{j+1} from their own w and h1 below, exactly as alone)
      std::vector<int> cnt_re(static_cast<size_t>(nb), -1);
      for (int r = 0; r < nb; ++r)
        if (reorth[zu(r)]) cnt_re[zu(r)] = nv;
      rc = w32 ? combine_host(b, basis, wv32, wv32, nv, h1, one, &cnt_re)
               : combine_host(b, basis, wv, wv, nv, h1, one, &cnt_re);
      if (rc) return rc;
      rc = w32 ? dots_host(b, basis, wv32, nv, act, nact) : dots_host(b, basis, wv, nv, act, nact);
      if (rc) return rc;
      for (int r = 0; r < nb; ++r) {
        double beta2;
        if (reorth[zu(r)]) {
          double p = 0;
          for (int i = 0; i < nv; ++i) {
            const cd v = red_at(b, r, i, nv + 1);
            coef2[zu(r) * zu(nv) + zu(i)] = v;
            hcol[zu(r) * zu(nv + 1) + zu(i)] += v;
            p += std::norm(v);
          }
          beta2 = red_at(b, r, nv, nv + 1).real() - p;
        } else {
          beta2 = wp2[zu(r)];
        }
        const double beta = std::sqrt(std::max(beta2, 0.0));
        hcol[zu(r) * zu(nv + 1) + zu(nv)] = beta;
        scale[zu(r)] = (active[zu(r)] && beta > 1e-300) ? 1.0 / beta : 0.0;
      }
    } else {
      for (int r = 0; r < nb; ++r) {
        const double beta = std::sqrt(std::max(wp2[zu(r)], 0.0));
        hcol[zu(r) * zu(nv + 1) + zu(nv)] = beta;
        scale[zu(r)] = (active[zu(r)] && beta > 1e-300) ? 1.0 / beta : 0.0;
      }
    }
    // Givens update per active slot: it needs only the new Hessenberg column,
    // so whether the slot stops here is known before V_{j+1} is formed
    std::vector<bool> finish(static_cast<size_t>(nb), false);
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      RhsState& S = st[zu(r)];
      S.iters++;
      if (fp64)
        S.mv64++;
      else
        S.mv32++;
      std::vector<cd>& H = Hs[zu(r)];
      for (int i = 0; i <= nv; ++i) H[zu(j) * zu(m + 1) + zu(i)] = hcol[zu(r) * zu(nv + 1) + zu(i)];
      cd* col = &H[zu(j) * zu(m + 1)];
      for (int i = 0; i < j; ++i) {
        const cd t = cs[zu(r)][zu(i)] * col[i] + sn[zu(r)][zu(i)] * col[i + 1];
        col[i + 1] = -std::conj(sn[zu(r)][zu(i)]) * col[i] + cs[zu(r)][zu(i)] * col[i + 1];
        col[i] = t;
      }
      const cd a = col[j], bb = col[j + 1];
      const double rho = std::sqrt(std::norm(a) + std::norm(bb));
      double c;
      cd sgn;
      if (std::abs(a) == 0.0) {
        c = 0.0;
        sgn = 1.0;
        col[j] = bb;
      } else {
        c = std::abs(a) / rho;
        const cd ph = a / std::abs(a);
        sgn = ph * std::conj(bb) / rho;
        col[j] = ph * rho;
      }
      col[j + 1] = 0.0;
      cs[zu(r)][zu(j)] = c;
      sn[zu(r)][zu(j)] = sgn;
      cd& gj = g[zu(r)][zu(j)];
      cd& gj1 = g[zu(r)][zu(j + 1)];
      gj1 = -std::conj(sgn) * gj;
      gj = c * gj;
      const double est = std::abs(gj1);
      const bool breakdown = !(hcol[zu(r) * zu(nv + 1) + zu(nv)].real() > 1e-300);
      if (trace_on())
        std::fprintf(stderr, "[vie] gmres%s rhs %d j %d est/r0 %.3e beta %.3e wp2/w2 %.3e reorth %d\n",
                     fp64 ? "64" : "32", r, j, est / rnorm[zu(r)], hcol[zu(r) * zu(nv + 1) + zu(nv)].real(),
                     wp2[zu(r)] / w2[zu(r)], int(reorth[zu(r)]));
      // a slot stops on its target, a breakdown or its budget, and the cycle
      // ends for all at its last iteration
      finish[zu(r)] = est <= target[zu(r)] || breakdown || S.mv32 + S.mv64 >= budget[zu(r)] || j == m - 1;
    }
    // continuing slots: V_{j+1} = (w - V h) / beta
    std::vector<int> cnt_next(static_cast<size_t>(nb), -1), cnt_x(zu(nb), -1);
    bool any_next = false, any_x = false;
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      if (finish[zu(r)]) {
        cnt_x[zu(r)] = nv;
        any_x = true;
      } else {
        cnt_next[zu(r)] = nv;
        any_next = true;
      }
    }
    if (any_next) {
      // per slot: the second-pass coefficients on the re-orthogonalised w,
      // else the first-pass ones on the original w
      std::vector<cd> vc(h1);
      for (int r = 0; r < nb; ++r)
        if (reorth[zu(r)])
          for (int i = 0; i < nv; ++i) vc[zu(r) * zu(nv) + zu(i)] = coef2[zu(r) * zu(nv) + zu(i)];
      rc = w32 ? combine_host(b, basis, wv32, Vn, nv, vc, scale, &cnt_next)
               : combine_host(b, basis, wv, Vn, nv, vc, scale, &cnt_next);
      if (rc) return rc;
    }
    // finishing slots: x += V y over their j + 1 basis vectors (instead of a
    // V_{j+1} they will not use), y from the triangular system R y = g
    if (any_x) {
      std::vector<cd> coef(zu(nb) * zu(nv), cd(0, 0));
      for (int r = 0; r < nb; ++r) {
        if (cnt_x[zu(r)] < 0) continue;
        const int k = nv;
        std::vector<cd> y(static_cast<size_t>(k));
        const std::vector<cd>& H = Hs[zu(r)];
        for (int i = k - 1; i >= 0; --i) {
          cd acc = g[zu(r)][zu(i)];
          for (int q = i + 1; q < k; ++q) acc -= H[zu(q) * zu(m + 1) + zu(i)] * y[zu(q)];
          const cd d = H[zu(i) * zu(m + 1) + zu(i)];
          y[zu(i)] = std::abs(d) > 0 ? acc / d : cd(0, 0);
        }
        for (int i = 0; i < k; ++i) coef[zu(r) * zu(nv) + zu(i)] = -y[zu(i)];
        active[zu(r)] = false;
      }
      std::vector<double> one(static_cast<size_t>(nb), 1.0);
      rc = combine_host(b, static_cast<const c128*>(basis), pl->xw, pl->xw, nv, coef, one, &cnt_x);
      if (rc) return rc;
    }
  }
  return VIE_OK;
}

// Bi-CGStab on A d = r (r in rw, d accumulated into xw).  Work vectors in the
// basis slots: 0 rhat, 1 v, 2 p, 3 s, 4 t.
int bicgstab_run(const Batch& b, bool fp64, const std::vector<double>& rnorm0, const std::vector<double>& target,
                 std::vector<RhsState>& st, const std::vector<bool>& active_in, const std::vector<int>& budget) {
  vie_plan* pl = b.pl;
  const int nb = b.nb;
  std::vector<bool> active = active_in;
  c128* rhat = pl->V;
  c128* v = pl->V + b.vs;
  c128* p = pl->V + 2 * b.vs;  // v, p consecutive: one two-vector combine forms p
  c128* sv = pl->V + 3 * b.vs; // p, s consecutive: one two-vector combine updates x
  c128* t = pl->V + 4 * b.vs;
  for (int r = 0; r < nb; ++r)
    if (!(rnorm0[zu(r)] > 0)) active[zu(r)] = false;
  // Slots that are not active are skipped by every launch (as in gmres_cycle).
  std::vector<cd> none;
  std::vector<double> one(static_cast<size_t>(nb), 1.0), zero(zu(nb), 0.0);
  const c128* nov = nullptr;
  std::vector<int> c0 = counts_of(active, 0), c1 = counts_of(active, 1), c2 = counts_of(active, 2);
  int rc = combine_host(b, nov, pl->rw, rhat, 0, none, one, &c0);    // rhat = r
  if (!rc) rc = combine_host(b, nov, pl->rw, p, 0, none, zero, &c0);  // p = 0
  if (!rc) rc = combine_host(b, nov, pl->rw, v, 0, none, zero, &c0);  // v = 0
  if (rc) return rc;
  std::vector<cd> rho(static_cast<size_t>(nb), 1.0), alpha(zu(nb), 1.0), omg(zu(nb), 1.0);
  const int max_steps = 100000;
  for (int it = 0; it < max_steps; ++it) {
    bool any = false;
    for (int r = 0; r < nb; ++r) any = any || active[zu(r)];
    if (!any) break;
    int nact = 0;
    const int* act = set_active(b, active, &nact, &rc);
    if (rc) return rc;
    c1 = counts_of(active, 1);
    c2 = counts_of(active, 2);
    // rho_new = (rhat, r)
    rc = dots_host(b, rhat, pl->rw, 1, act, nact);
    if (rc) return rc;
    std::vector<cd> cP(zu(nb) * 2, cd(0, 0));
    std::vector<cd> rho_new(static_cast<size_t>(nb));
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      rho_new[zu(r)] = red_at(b, r, 0, 2);
      const cd beta = (rho_new[zu(r)] / rho[zu(r)]) * (alpha[zu(r)] / omg[zu(r)]);
      // p = r + beta (p - omega v) = r - (v (beta omega) + p (-beta))
      cP[zu(r) * 2 + 0] = beta * omg[zu(r)];
      cP[zu(r) * 2 + 1] = -beta;
    }
    rc = combine_host(b, v, pl->rw, p, 2, cP, one, &c2);
    if (rc) return rc;
    rc = apply_graph(pl, pl->box, fp64, p, p, nullptr, v, nb, MODE_MATVEC, b.s, act, nact);
    if (rc) return rc;
    rc = dots_host(b, rhat, v, 1, act, nact);
    if (rc) return rc;
    std::vector<cd> cS(static_cast<size_t>(nb), cd(0, 0));
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      const cd den = red_at(b, r, 0, 2);
      alpha[zu(r)] = std::abs(den) > 0 ? rho_new[zu(r)] / den : cd(0, 0);
      cS[zu(r)] = alpha[zu(r)];
    }
    rc = combine_host(b, v, pl->rw, sv, 1, cS, one, &c1);  // s = r - alpha v
    if (rc) return rc;
    rc = apply_graph(pl, pl->box, fp64, sv, sv, nullptr, t, nb, MODE_MATVEC, b.s, act, nact);
    if (rc) return rc;
    rc = dots_host(b, sv, t, 1, act, nact);  // conj(s).t and ||t||^2
    if (rc) return rc;
    std::vector<cd> cX(zu(nb) * 2, cd(0, 0)), cR(zu(nb), cd(0, 0));
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      const cd st_ = std::conj(red_at(b, r, 0, 2));  // (t, s) = sum conj(t) s
      const double tt = red_at(b, r, 1, 2).real();
      omg[zu(r)] = tt > 0 ? st_ / tt : cd(0, 0);
      cX[zu(r) * 2 + 0] = -alpha[zu(r)];
      cX[zu(r) * 2 + 1] = -omg[zu(r)];
      cR[zu(r)] = omg[zu(r)];
      rho[zu(r)] = rho_new[zu(r)];
      st[zu(r)].iters++;
      if (fp64)
        st[zu(r)].mv64 += 2;
      else
        st[zu(r)].mv32 += 2;
    }
    rc = combine_host(b, p, pl->xw, pl->xw, 2, cX, one, &c2);  // x += alpha p + omega s
    if (rc) return rc;
    rc = combine_host(b, t, sv, pl->rw, 1, cR, one, &c1);  // r = s - omega t
    if (rc) return rc;
    std::vector<double> nr;
    rc = norms(b, pl->rw, nr, act, nact);
    if (rc) return rc;
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      RhsState& S = st[zu(r)];
      if (nr[zu(r)] <= target[zu(r)] || S.mv32 + S.mv64 >= budget[zu(r)] || !std::isfinite(nr[zu(r)]))
        active[zu(r)] = false;
    }
  }
  return VIE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Solver sessions: a batch of `cap` slots on the plan's Krylov workspace.
// Right-hand sides join free slots at any cycle boundary (session_add), every
// step advances all slots still iterating by one outer cycle (an inner GMRES
// cycle or Bi-CGStab run and the FP64 true residual), and finished slots are
// read out and freed (session_take) while the others continue.  vie_solve is
// a session filled with one chunk of right-hand sides at a time; the
// continuous-batching calls (vie_batch_*) expose it.  Each slot's arithmetic
// does not depend on the others, on its position, or on when it joined.
// ---------------------------------------------------------------------------
struct SolveSession {
  vie_solve_opts o{};
  bool mixed = false;
  bool user = false;  // opened through vie_batch_open
  int m = 0, cap = 0;
  long L = 0;
  std::vector<RhsState> st;
  std::vector<char> used;  // the slot holds a right-hand side not yet taken
  std::vector<std::chrono::steady_clock::time_point> t_add, t_done;
};

namespace {

// The launches of a session cover slots 0 .. hw - 1, hw = one past the
// highest slot in use (slots are filled lowest first), not the whole
// capacity: a batch holding a few right-hand sides launches for those only.
int high_water(const SolveSession& S) {
  int hw = 0;
  for (int r = 0; r < S.cap; ++r)
    if (S.used[size_t(r)]) hw = r + 1;
  return hw;
}

Batch batch_of(vie_plan* pl, const SolveSession& S, hipStream_t s, int nb) {
  return Batch{pl, s, nb, S.L, long(pl->kr_cap) * S.L, krylov_blocks(S.L)};
}

bool ends(const RhsState& S) { return S.done; }

}  // namespace

void close_session(vie_plan* pl) {
  delete pl->session;
  pl->session = nullptr;
}

int open_session(vie_plan* pl, int cap, const vie_solve_opts& o, bool user, hipStream_t s) {
  if (pl->session) return fail(pl, VIE_E_STATE, "a batch is already open on this plan");
  if (cap < 1 || cap > kMaxFlagged) return fail(pl, VIE_E_ARG, "batch capacity must be in [1, 256]");
  const bool mixed = pl->precision == VIE_PREC_MIXED && !(o.flags & VIE_SOLVE_FP64);
  const int m = o.solver == VIE_SOLVER_BICGSTAB ? 5 : std::max(1, o.restart);
  int rc = ensure_krylov(pl, cap, std::max(m, 5), s);
  if (rc) return rc;
  SolveSession* S = new (std::nothrow) SolveSession();
  if (!S) return fail(pl, VIE_E_NOMEM, "session");
  S->o = o;
  S->mixed = mixed;
  S->user = user;
  S->m = m;
  S->cap = cap;
  // Outside supp(H) the equation gives J = 0 exactly, so the unknowns are
  // the points of supp(H): per (z, y) row of its bounding box, the x-interval
  // from the first to the last support point.  U is needed only there too.
  S->L = long(pl->C) * pl->box.np;
  S->st.assign(zu(cap), RhsState{});
  for (auto& x : S->st) x.done = true;
  S->used.assign(zu(cap), 0);
  S->t_add.resize(zu(cap));
  S->t_done.resize(zu(cap));
  pl->session = S;
  return VIE_OK;
}

// Right-hand sides k of inc (whole-grid layout [k][C][n^3]) into free slots
// (written to slots[0..k-1]); x0: optional initial densities of the same layout.
int session_add(vie_plan* pl, const c128* inc, const c128* x0, int k, int* slots, hipStream_t s) {
  SolveSession* S = pl->session;
  const long L = S->L;
  const long Lg = long(pl->C) * pl->n3;
  const Box box = box_of(pl->box, pl->n);
  std::vector<int> sl;
  for (int r = 0; r < S->cap && int(sl.size()) < k; ++r)
    if (!S->used[zu(r)]) sl.push_back(r);
  if (int(sl.size()) < k) return fail(pl, VIE_E_ARG, "not enough free slots in the batch");
  const int hw = std::max(high_water(*S), sl.back() + 1);
  Batch b = batch_of(pl, *S, s, hw);
  std::vector<bool> fresh(zu(hw), false);
  for (int i = 0; i < k; ++i) {
    const int r = sl[zu(i)];
    fresh[zu(r)] = true;
    // b = 2 H g
    HIPCHK(pl, launch_rhs(pl->H64, pl->Hmu64, inc + long(i) * Lg, pl->bw + long(r) * L, 1, pl->C, box, s));
    if (x0) {
      HIPCHK(pl, launch_gather(x0 + long(i) * Lg, pl->xw + long(r) * L, pl->C, box, s));
    } else {
      HIPCHK(pl, launch_fill(pl->xw + long(r) * L, L, c128{0.0, 0.0}, s));
      HIPCHK(pl, launch_copy(pl->bw + long(r) * L, pl->rw + long(r) * L, L, s));
    }
  }
  int rc = VIE_OK, nact = 0;
  const int* act = set_active(b, fresh, &nact, &rc);
  if (rc) return rc;
  std::vector<double> bnorm, rnorm;
  rc = norms(b, pl->bw, bnorm, act, nact);
  if (rc) return rc;
  if (x0) {
    rc = apply_any(pl, pl->box, true, pl->xw, pl->xw, pl->bw, pl->rw, hw, MODE_RESIDUAL, s, act, nact);
    if (rc) return rc;
  }
  rc = norms(b, pl->rw, rnorm, act, nact);
  if (rc) return rc;
  const auto now = std::chrono::steady_clock::now();
  std::vector<int> c0(zu(hw), -1);
  for (int i = 0; i < k; ++i) {
    const int r = sl[zu(i)];
    RhsState& T = S->st[zu(r)];
    T = RhsState{};
    T.bnorm = bnorm[zu(r)];
    T.rnorm = T.best = T.ref = rnorm[zu(r)];
    if (x0) T.mv64++;
    if (!std::isfinite(T.bnorm) || !std::isfinite(T.rnorm)) {
      // a non-finite incident field (or initial guess): nothing to iterate on
      T.done = true;
    } else if (!(T.bnorm > 0)) {
      // b = 0: x = 0 is exact
      T.done = T.conv = true;
      T.rnorm = 0;
    } else if (T.rnorm <= S->o.tol * T.bnorm) {
      T.done = T.conv = true;
    }
    S->used[zu(r)] = 1;
    S->t_add[zu(r)] = S->t_done[zu(r)] = now;
    c0[zu(r)] = 0;
    if (slots) slots[i] = r;
  }
  // the best iterate so far of every new slot: its initial one
  std::vector<double> one(zu(hw), 1.0);
  std::vector<cd> none;
  const c128* nov = nullptr;
  return combine_host(b, nov, pl->xw, pl->xbest, 0, none, one, &c0);
}

// One outer cycle for every slot still iterating; *nactive = slots still
// iterating afterwards.
int session_step(vie_plan* pl, hipStream_t s, int* nactive) {
  SolveSession* Sx = pl->session;
  const vie_solve_opts& o = Sx->o;
  const int nb = high_water(*Sx), m = Sx->m;
  std::vector<RhsState>& st = Sx->st;
  Batch b = batch_of(pl, *Sx, s, nb);
  int rc = VIE_OK;
  std::vector<double> target(zu(nb)), rnorm(zu(nb));
  std::vector<bool> active(zu(nb));
  std::vector<int> budget(zu(nb));
  bool any = false;
  for (int r = 0; r < nb; ++r) {
    const RhsState& S = st[zu(r)];
    active[zu(r)] = Sx->used[zu(r)] && !ends(S);
    any = any || active[zu(r)];
    const double inner = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    target[zu(r)] = Sx->mixed ? std::max(inner * S.rnorm, 0.3 * o.tol * S.bnorm) : 0.5 * o.tol * S.bnorm;
    budget[zu(r)] = std::max(1, o.max_iters - 1);
    rnorm[zu(r)] = active[zu(r)] ? S.rnorm : 0.0;
  }
  if (any) {
    if (o.solver == VIE_SOLVER_BICGSTAB)
      rc = bicgstab_run(b, !Sx->mixed, rnorm, target, st, active, budget);
    else
      rc = gmres_cycle(b, !Sx->mixed, m, rnorm, target, st, active, budget);
    if (rc) return rc;
    // true residual with the FP64 operator, for the slots that iterated
    int nlive = 0;
    const int* act = set_active(b, active, &nlive, &rc);
    if (rc) return rc;
    rc = apply_graph(pl, pl->box, true, pl->xw, pl->xw, pl->bw, pl->rw, nb, MODE_RESIDUAL, s, act, nlive);
    if (rc) return rc;
    rc = norms(b, pl->rw, rnorm, act, nlive);
    if (rc) return rc;
    const int stall_mv = std::max(kStallMatvecs, 3 * m);
    std::vector<int> keep(zu(nb), -1), restore(zu(nb), -1);
    bool any_keep = false, any_restore = false;
    const auto now = std::chrono::steady_clock::now();
    for (int r = 0; r < nb; ++r) {
      if (!active[zu(r)]) continue;
      RhsState& S = st[zu(r)];
      S.mv64++;
      S.refine++;
      S.rnorm = rnorm[zu(r)];
      const bool finite = std::isfinite(S.rnorm);
      if (finite && S.rnorm < S.best) {
        S.best = S.rnorm;
        keep[zu(r)] = 0;
        any_keep = true;
      }
      if (finite && S.rnorm <= 0.9 * S.ref) {
        S.ref = S.rnorm;
        S.ref_mv = S.matvecs();
      }
      if (finite && S.rnorm <= o.tol * S.bnorm) {
        S.done = S.conv = true;
      } else if (!finite || S.matvecs() >= o.max_iters || S.matvecs() - S.ref_mv >= stall_mv) {
        // budget spent, stagnation or a non-finite residual: the best iterate
        S.done = true;
        if (!(S.rnorm <= S.best)) {
          restore[zu(r)] = 0;
          any_restore = true;
          S.rnorm = S.best;
        }
      }
      if (S.done) Sx->t_done[zu(r)] = now;
    }
    std::vector<double> one(zu(nb), 1.0);
    std::vector<cd> none;
    const c128* nov = nullptr;
    if (any_keep) {
      rc = combine_host(b, nov, pl->xw, pl->xbest, 0, none, one, &keep);
      if (rc) return rc;
    }
    if (any_restore) {
      rc = combine_host(b, nov, pl->xbest, pl->xw, 0, none, one, &restore);
      if (rc) return rc;
    }
  }
  int left = 0;
  for (int r = 0; r < Sx->cap; ++r) left += (Sx->used[zu(r)] && !ends(st[zu(r)])) ? 1 : 0;
  if (nactive) *nactive = left;
  return VIE_OK;
}

void fill_stats(const RhsState& S, double secs, vie_solve_stats* x) {
  x->status = S.conv ? VIE_OK : VIE_W_NOCONV;
  x->iters = S.iters;
  x->matvecs_fp32 = S.mv32;
  x->matvecs_fp64 = S.mv64;
  x->refinements = S.refine;
  x->rel_residual = !std::isfinite(S.bnorm) ? std::numeric_limits<double>::quiet_NaN()
                                            : (S.bnorm > 0 ? S.rnorm / S.bnorm : 0.0);
  x->seconds = secs;
}

int solve_batch(vie_plan* pl, const c128* inc, c128* density, c128* field, int nrhs, const vie_solve_opts& o,
                vie_solve_stats* stats, hipStream_t s) {
  if (pl->session) return fail(pl, VIE_E_STATE, "vie_solve: a continuous batch is open on this plan");
  const long Lg = long(pl->C) * pl->n3;
  const Box box = box_of(pl->box, pl->n);
  const int cap = std::max(1, std::min(nrhs, pl->max_rhs));
  int rc = open_session(pl, cap, o, false, s);
  if (rc) return rc;
  SolveSession* S = pl->session;
  int status = VIE_OK;
  for (int r0 = 0; r0 < nrhs && !rc; r0 += cap) {
    const auto t0 = std::chrono::steady_clock::now();
    const int nb = std::min(cap, nrhs - r0);
    const long off = long(r0) * Lg;
    std::vector<int> slots(zu(nb));
    rc = session_add(pl, inc + off, (o.flags & VIE_SOLVE_X0) ? density + off : nullptr, nb, slots.data(), s);
    int left = 1;
    while (!rc && left > 0) rc = session_step(pl, s, &left);
    if (rc) break;
    // slots 0..nb-1 (the session was empty): one launch for the chunk
    hipError_t e = launch_scatter(pl->xw, density + off, long(nb) * pl->C, box, s);
    if (e != hipSuccess) {
      rc = hip_fail(pl, e, "launch_scatter");
      break;
    }
    if (field) {
      rc = apply_any(pl, pl->grid, true, density + off, inc + off, nullptr, field + off, nb, MODE_FIELD, s);
      if (rc) break;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = hip_fail(pl, e, "hipStreamSynchronize");
      break;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nb; ++r) {
      const RhsState& T = S->st[zu(r)];
      if (!T.conv) status = VIE_W_NOCONV;
      if (stats) fill_stats(T, secs, &stats[r0 + r]);
      S->used[zu(r)] = 0;
    }
  }
  close_session(pl);
  return rc ? rc : status;
}

}  // namespace vie

using vie::SolveSession;

extern "C" int vie_batch_open(vie_plan* pl, int capacity, const vie_solve_opts* opts, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  vie_solve_opts o{1e-10, 2000, 40, 0.0, VIE_SOLVER_GMRES, 0u};
  if (opts) o = *opts;
  if (!(o.tol > 0) || o.max_iters < 1 || o.restart < 1 || o.restart > 1000 ||
      (o.solver != VIE_SOLVER_GMRES && o.solver != VIE_SOLVER_BICGSTAB))
    return vie::fail(pl, VIE_E_ARG, "vie_batch_open: invalid options");
  const vie::StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  return vie::open_session(pl, capacity, o, true, static_cast<hipStream_t>(hip_stream));
}

extern "C" int vie_batch_add(vie_plan* pl, const double* inc, const double* x0, int nrhs, int* slots,
                             void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!pl->session || !pl->session->user) return vie::fail(pl, VIE_E_STATE, "vie_batch_add: no open batch");
  if (!inc || nrhs < 1) return vie::fail(pl, VIE_E_ARG, "vie_batch_add: null pointer or nrhs < 1");
  const vie::StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  return vie::session_add(pl, reinterpret_cast<const vie::c128*>(inc), reinterpret_cast<const vie::c128*>(x0),
                          nrhs, slots, static_cast<hipStream_t>(hip_stream));
}

extern "C" int vie_batch_step(vie_plan* pl, int* nactive, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!pl->session || !pl->session->user) return vie::fail(pl, VIE_E_STATE, "vie_batch_step: no open batch");
  const vie::StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  return vie::session_step(pl, static_cast<hipStream_t>(hip_stream), nactive);
}

extern "C" int vie_batch_done(vie_plan* pl, int* slots, int max_slots, int* ndone, int* nfree) {
  if (!pl) return VIE_E_ARG;
  if (!pl->session || !pl->session->user) return vie::fail(pl, VIE_E_STATE, "vie_batch_done: no open batch");
  SolveSession* S = pl->session;
  int d = 0, f = 0;
  for (int r = 0; r < S->cap; ++r) {
    if (!S->used[size_t(r)]) {
      ++f;
    } else if (S->st[size_t(r)].done) {
      if (slots && d < max_slots) slots[d] = r;
      ++d;
    }
  }
  if (ndone) *ndone = d;
  if (nfree) *nfree = f;
  return VIE_OK;
}

extern "C" int vie_batch_take(vie_plan* pl, int slot, double* density, double* field, const double* inc,
                              vie_solve_stats* stats, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!pl->session || !pl->session->user) return vie::fail(pl, VIE_E_STATE, "vie_batch_take: no open batch");
  SolveSession* S = pl->session;
  if (slot < 0 || slot >= S->cap || !S->used[size_t(slot)] || !S->st[size_t(slot)].done)
    return vie::fail(pl, VIE_E_ARG, "vie_batch_take: the slot holds no finished right-hand side");
  if (!density || (field && !inc)) return vie::fail(pl, VIE_E_ARG, "vie_batch_take: null density (or inc with field)");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const vie::StreamUse use(pl, s);
  auto* d = reinterpret_cast<vie::c128*>(density);
  HIPCHK(pl, vie::launch_scatter(pl->xw + long(slot) * S->L, d, pl->C, vie::box_of(pl->box, pl->n), s));
  if (field) {
    const int rc = vie::apply_any(pl, pl->grid, true, d, reinterpret_cast<const vie::c128*>(inc), nullptr,
                                  reinterpret_cast<vie::c128*>(field), 1, vie::MODE_FIELD, s);
    if (rc) return rc;
  }
  const vie::RhsState& T = S->st[size_t(slot)];
  if (stats)
    vie::fill_stats(T, std::chrono::duration<double>(S->t_done[size_t(slot)] - S->t_add[size_t(slot)]).count(), stats);
  S->used[size_t(slot)] = 0;
  return T.conv ? VIE_OK : VIE_W_NOCONV;
}

extern "C" int vie_batch_close(vie_plan* pl) {
  if (!pl) return VIE_E_ARG;
  if (!pl->session || !pl->session->user) return vie::fail(pl, VIE_E_STATE, "vie_batch_close: no open batch");
  vie::close_session(pl);
  return VIE_OK;
}

extern "C" int vie_solve(vie_plan* pl, const double* inc, double* density, double* field, int nrhs,
                         const vie_solve_opts* opts, vie_solve_stats* stats, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!inc || !density || nrhs < 1) return vie::fail(pl, VIE_E_ARG, "vie_solve: null pointer or nrhs < 1");
  const vie::StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  vie_solve_opts o{1e-10, 2000, 40, 0.0, VIE_SOLVER_GMRES, 0u};
  if (opts) o = *opts;
  if (!(o.tol > 0) || o.max_iters < 1 || o.restart < 1 || o.restart > 1000 ||
      (o.solver != VIE_SOLVER_GMRES && o.solver != VIE_SOLVER_BICGSTAB))
    return vie::fail(pl, VIE_E_ARG, "vie_solve: invalid options");
  return vie::solve_batch(pl, reinterpret_cast<const vie::c128*>(inc), reinterpret_cast<vie::c128*>(density),
                          reinterpret_cast<vie::c128*>(field), nrhs, o, stats, static_cast<hipStream_t>(hip_stream));
}
