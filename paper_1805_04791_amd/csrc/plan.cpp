// Plan creation (contrast + kernel-table precompute), the batched FFT apply,
// autotuning of the pencil tiles, and the C entry points other than vie_solve.
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "lens.hpp"
#include "pointwise.hpp"
#include "postprocess.hpp"

using namespace vie;

// Workspace of vie_apply_noalloc: device memory the library owns from load
// time, so that the call allocates nothing.  Each device holds its own copy at
// its own address (looked up once per device when the first plan is created
// there); host code never passes the array's name to a kernel.
static __device__ __align__(256) unsigned char scratch[size_t(VIE_NOALLOC_SCRATCH_MIB) << 20];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};  // under hip_mutex()
}  // namespace

namespace vie {

template <typename R>
LenOps<R>* len_table() {
  static LenOps<R> t[(kMaxLen + 1) * kMaxSplits];
  return t;
}
template LenOps<float>* len_table<float>();
template LenOps<double>* len_table<double>();

std::string& last_create_error() {
  static thread_local std::string m;
  return m;
}

int fail(vie_plan* pl, int code, const std::string& msg) {
  if (pl) pl->err = msg;
  return code;
}

int hip_fail(vie_plan* pl, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (pl) pl->err = m;
  return e == hipErrorOutOfMemory ? VIE_E_NOMEM : VIE_E_DEVICE;
}

std::recursive_mutex& hip_mutex() {
  static std::recursive_mutex m;
  return m;
}

// Device blocks released by plans are kept for reuse by later allocations of
// about the same size: a hipFree waits for the whole device, which would
// serialise plans created and destroyed while others compute (a serving
// loop).  A block enters the cache only after the work queued on the
// releasing plan's streams has completed.  All of this under hip_mutex().
namespace {
struct FreeBlock {
  void* p;
  size_t bytes;
  int device;
};
std::vector<FreeBlock>& free_blocks() {
  static std::vector<FreeBlock> v;
  return v;
}
size_t g_cached_bytes = 0;
constexpr size_t kCacheLimit = size_t(96) << 30;  // bytes kept for reuse at most
constexpr size_t kCacheFloor = size_t(32) << 30;  // device memory left free for other allocators
std::vector<std::pair<void*, size_t>>& free_host_blocks() {
  static std::vector<std::pair<void*, size_t>> v;
  return v;
}
size_t g_cached_host_bytes = 0;
constexpr size_t kHostCacheLimit = size_t(256) << 20;

// Block sizes: multiples of 64 KiB below 64 MiB; above, size classes 2^(k/4)
// apart (rounded to 2 MiB), so that the plans of a serving stream, whose
// grids and batch sizes differ, release blocks that later plans can take
// (within the 1.25x the cache accepts) instead of allocating and freeing
// anew: a hipMalloc or hipFree of gigabytes holds every other thread's HIP
// calls for tens to hundreds of milliseconds.  At most 19% of a large block
// goes unused.
size_t round_block(size_t b) {
  if (b < (size_t(64) << 20)) {
    const size_t g = size_t(64) << 10;
    return (b + g - 1) / g * g;
  }
  const double k = std::ceil(4.0 * std::log2(double(b)) - 1e-9);
  size_t c = size_t(std::ceil(std::exp2(k / 4.0)));
  if (c < b) c = b;
  const size_t g = size_t(2) << 20;
  return (c + g - 1) / g * g;
}

}  // namespace

size_t cached_bytes() { return g_cached_bytes; }

void release_all_cached() {
  release_cached(-1);
  for (auto& b : free_host_blocks()) (void)hipHostFree(b.first);
  free_host_blocks().clear();
  g_cached_host_bytes = 0;
}

int host_alloc(vie_plan* pl, void** p, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  *p = nullptr;
  bytes = (std::max<size_t>(bytes, 1) + 4095) / 4096 * 4096;
  auto& v = free_host_blocks();
  long best = -1;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].second >= bytes && v[i].second - bytes <= bytes / 4 &&
        (best < 0 || v[i].second < v[size_t(best)].second))
      best = long(i);
  if (best >= 0) {
    *p = v[size_t(best)].first;
    bytes = v[size_t(best)].second;
    g_cached_host_bytes -= bytes;
    v.erase(v.begin() + best);
  } else {
    const hipError_t e = hipHostMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(pl, VIE_E_NOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  pl->host_allocs.push_back({*p, bytes});
  return VIE_OK;
}

// a pinned block no queued work uses any more: cached, or freed beyond the limit
void give_host_block(void* p, size_t bytes) {
  if (g_cached_host_bytes + bytes > kHostCacheLimit) {
    (void)hipHostFree(p);
    return;
  }
  free_host_blocks().push_back({p, bytes});
  g_cached_host_bytes += bytes;
}

void host_free(vie_plan* pl, void* p) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  for (size_t i = 0; i < pl->host_allocs.size(); ++i) {
    if (pl->host_allocs[i].first == p) {
      const size_t bytes = pl->host_allocs[i].second;
      pl->host_allocs.erase(pl->host_allocs.begin() + long(i));
      quiesce(pl);
      give_host_block(p, bytes);
      return;
    }
  }
}

// frees the cached blocks of `device` (all devices when device < 0)
void release_cached(int device) {
  auto& v = free_blocks();
  for (size_t i = 0; i < v.size();) {
    if (device < 0 || v[i].device == device) {
      int cur = -1;
      (void)hipGetDevice(&cur);
      if (cur != v[i].device) (void)hipSetDevice(v[i].device);
      (void)hipFree(v[i].p);
      if (cur >= 0 && cur != v[i].device) (void)hipSetDevice(cur);
      g_cached_bytes -= v[i].bytes;
      v.erase(v.begin() + long(i));
    } else {
      ++i;
    }
  }
}

// a block no queued work uses any more: cached, or freed beyond the limit or
// when the device would keep less than kCacheFloor free for other allocators
void give_block(void* p, size_t bytes, int device) {
  bool keep = g_cached_bytes + bytes <= kCacheLimit;
  if (keep) {
    size_t free_b = 0, total_b = 0;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) keep = free_b >= kCacheFloor;
    if (cur != device && cur >= 0) (void)hipSetDevice(cur);
  }
  if (!keep) {
    (void)hipFree(p);
    return;
  }
  free_blocks().push_back({p, bytes, device});
  g_cached_bytes += bytes;
}

// waits for the work the plan has queued (its latest stream and its graph stream)
void quiesce(vie_plan* pl) {
  (void)hipStreamSynchronize(pl->last_stream);
  if (pl->gstream) (void)hipStreamSynchronize(pl->gstream);
}

StreamUse::~StreamUse() {
  if (!pl->done_ev) return;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) {
    pl->done_valid = false;
    return;
  }
  pl->done_valid = hipEventRecord(pl->done_ev, s) == hipSuccess;
}

int dev_alloc(vie_plan* pl, void** p, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  bytes = round_block(bytes);
  // the smallest cached block of this device that is at most 1.25x the request
  auto& v = free_blocks();
  long best = -1;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].device == pl->device && v[i].bytes >= bytes && v[i].bytes - bytes <= bytes / 4 &&
        (best < 0 || v[i].bytes < v[size_t(best)].bytes))
      best = long(i);
  if (best >= 0) {
    *p = v[size_t(best)].p;
    bytes = v[size_t(best)].bytes;
    g_cached_bytes -= bytes;
    v.erase(v.begin() + best);
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      // give the cached blocks back and try once more
      (void)hipGetLastError();
      release_cached(pl->device);
      e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(pl, VIE_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  pl->allocs.push_back({*p, bytes});
  pl->dev_bytes += bytes;
  return VIE_OK;
}

void dev_free(vie_plan* pl, void* p) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  for (size_t i = 0; i < pl->allocs.size(); ++i) {
    if (pl->allocs[i].first == p) {
      const size_t bytes = pl->allocs[i].second;
      pl->dev_bytes -= bytes;
      pl->allocs.erase(pl->allocs.begin() + long(i));
      quiesce(pl);
      give_block(p, bytes, pl->device);
      return;
    }
  }
}

static hipEvent_t take_event(vie_plan* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int prof_begin(vie_plan* pl, hipStream_t s) {
  if (!pl->prof_on) return -1;
  hipEvent_t a = take_event(pl), b = take_event(pl);
  if (!a || !b) return -1;
  (void)hipEventRecord(a, s);
  pl->prof.push_back({-1, a, b, 0.0, 0.0});
  return int(pl->prof.size()) - 1;
}

void prof_end(vie_plan* pl, int fam, int token, hipStream_t s, double bytes, double flops) {
  if (token < 0 || !pl->prof_on) return;
  pl->prof[size_t(token)].fam = fam;
  pl->prof[size_t(token)].bytes = bytes;
  pl->prof[size_t(token)].flops = flops;
  (void)hipEventRecord(pl->prof[size_t(token)].b, s);
}

// fold recorded pairs into the per-family totals
static void prof_collect(vie_plan* pl) {
  for (auto& r : pl->prof) {
    if (r.fam >= 0) {
      (void)hipEventSynchronize(r.b);
      float ms = 0;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        pl->prof_ms[r.fam] += ms;
        pl->prof_cnt[r.fam] += 1;
        pl->prof_bytes[r.fam] += r.bytes;
        pl->prof_flops[r.fam] += r.flops;
      }
    }
    pl->ev_pool.push_back(r.a);
    pl->ev_pool.push_back(r.b);
  }
  pl->prof.clear();
}

}  // namespace vie

namespace {

// exp(-2 pi i j / L) with exact quadrant reduction
void twiddle_host(long j, long L, double* re, double* im) {
  j %= L;
  if (j < 0) j += L;
  const long q = (4 * j) / L;
  const long r = 4 * j - q * L;
  double c, s;
  if (2 * r <= L) {
    const double phi = (M_PI / 2.0) * double(r) / double(L);
    c = std::cos(phi);
    s = std::sin(phi);
  } else {
    const double psi = (M_PI / 2.0) * double(L - r) / double(L);
    c = std::sin(psi);
    s = std::cos(psi);
  }
  double cc, ss;
  switch (q & 3) {
    case 0: cc = c; ss = s; break;
    case 1: cc = -s; ss = c; break;
    case 2: cc = -c; ss = -s; break;
    default: cc = s; ss = -c; break;
  }
  *re = cc;
  *im = -ss;
}

template <typename R>
int upload_twiddles(vie_plan* pl, int L, cx<R>** out, hipStream_t s) {
  std::vector<cx<R>> h(static_cast<size_t>(L));
  for (int j = 0; j < L; ++j) {
    double re, im;
    twiddle_host(j, L, &re, &im);
    h[size_t(j)] = {R(re), R(im)};
  }
  int rc = dev_alloc(pl, reinterpret_cast<void**>(out), sizeof(cx<R>) * size_t(L));
  if (rc) return rc;
  HIPCHK(pl, hipMemcpyAsync(*out, h.data(), sizeof(cx<R>) * size_t(L), hipMemcpyHostToDevice, s));
  HIPCHK(pl, hipStreamSynchronize(s));
  return VIE_OK;
}

constexpr int kTileChoices[] = {2, 4, 8, 12, 16, 24, 32};

template <typename R, bool CONTIG>
size_t lds_need(int P1, int P2, int T) {
  const size_t per = size_t(std::max(P2 * (P1 + 1), P1 * (P2 + 1)));  // both layouts pad one slot per row
  return sizeof(cx<R>) * (size_t(P1 * P2) + size_t(T) * per);
}

// T columns per block must divide `cols` (the column count of a strided
// pass, or the transform length for contiguous passes)
// Strided passes read and write runs of T consecutive complex values per row;
// a run shorter than a 128-byte cache line makes neighbouring tiles, which
// run on different XCDs, fetch the same line twice, so T * sizeof >= 128 B
// whenever the column count allows it.
// ragged: the last tile of columns may be partial (the fused z pass masks
// columns beyond cols)
template <typename R>
bool tile_ok(const vie_plan* pl, int P1, int P2, int T, bool contig, long cols, int maxthreads,
             bool full_lines = true, bool ragged = false) {
  const int J = std::max(P1, P2);
  if (T * J > maxthreads || T * J < 16) return false;
  if (cols > 0 && !ragged && cols % T != 0) return false;
  const int full = int(128 / sizeof(cx<R>));
  if (full_lines && !contig && T < full && (cols <= 0 || cols >= full)) return false;
  const size_t need = contig ? lds_need<R, true>(P1, P2, T) : lds_need<R, false>(P1, P2, T);
  return need <= pl->max_lds;
}

template <typename R>
int default_tile(const vie_plan* pl, int P1, int P2, bool contig, int maxthreads, long cols, bool ragged = false) {
  const int J = std::max(P1, P2);
  for (int strict = 1; strict >= 0; --strict) {
    int best = 0;
    for (int T : kTileChoices) {
      if (!tile_ok<R>(pl, P1, P2, T, contig, cols, maxthreads, strict != 0, ragged)) continue;
      // prefer ~256 threads per block
      if (best == 0 || std::abs(T * J - 256) < std::abs(best * J - 256)) best = T;
    }
    if (best) return best;
  }
  return 0;
}

int bucket_of(int nb) {
  int b = 1;
  while (b < nb) b <<= 1;
  return b;
}

bool env_flag(const char* name, bool dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return !(v[0] == '0' || v[0] == 'n' || v[0] == 'N' || v[0] == 'f' || v[0] == 'F');
}

// ---------------------------------------------------------------------------
// the five passes of one batched apply
// ---------------------------------------------------------------------------
// the spectral multiply applied on a geometry
int geom_mul(const vie_plan* pl, const Geom& g) {
  if (g.mul >= 0) return g.mul;
  return pl->full ? MUL_MAX6 : MUL_SYM3;
}

template <typename R>
struct ApplyCall {
  vie_plan* pl;
  const LenOps<R>* ops;   // length Pxy: x and y passes
  const cx<R>* tw;
  const LenOps<R>* opsz;  // length Pz: the fused z pass
  const cx<R>* twz;
  cx<R>* A;
  cx<R>* B;
  int nb;
  Geom g;
  const int* act = nullptr;  // optional device flags per right-hand side: 0 = skip it
};

// x forward: rows (rhs, c, z, y) of the box, bx samples -> P; TV is the
// storage of the input vectors (complex128, or complex64 in FP32 applies)
template <typename R, typename TV>
hipError_t pass_xfwd(const ApplyCall<R>& c, const LenOps<R>* ops, const TV* in, int T, hipStream_t s) {
  const vie_plan* pl = c.pl;
  const long nr = long(c.g.bz) * c.g.by;
  const long rows = long(c.nb) * pl->C * nr;
  const int P = c.g.sp->Pxy;
  Geo g{T, int((rows + T - 1) / T), rows, c.g.bx, P, c.act, long(pl->C) * nr};
  MemStore<cx<R>> dst{c.A, 0, pitch_x(P), 1, 1.0, 0};
  if constexpr (std::is_same<TV, c128>::value) {
    if (c.g.rows) return ops->contig_fwd_rows(RowLoad<c128>{in, c.g.rows, nr, c.g.np}, dst, g, 1, c.tw, s);
    return ops->contig_fwd(MemLoad<c128>{in, 0, c.g.bx, 1}, dst, g, 1, c.tw, s);
  } else {
    if (c.g.rows) return hipErrorInvalidValue;
    return ops->contig_fwd_v32(MemLoad<c64>{in, 0, c.g.bx, 1}, dst, g, 1, c.tw, s);
  }
}

// y forward: A [rhs][c][bz][by][Wx] -> B [rhs][c][bz][P][Wy], rows of
// Wx = pitch_x(P) and Wy = pitch_y(P) elements of which the first P are used
template <typename R>
hipError_t pass_yfwd(const ApplyCall<R>& c, const LenOps<R>* ops, int T, hipStream_t s) {
  const vie_plan* pl = c.pl;
  const long P = c.g.sp->Pxy, by = c.g.by, Wx = pitch_x(P), Wy = pitch_y(P);
  Geo g{T, int(P / T), P, int(by), int(P), c.act, long(pl->C) * c.g.bz * P};
  MemLoad<cx<R>> src{c.A, by * Wx, 1, Wx};
  MemStore<cx<R>> dst{c.B, P * Wy, 1, Wy, 1.0, 0};
  return ops->strided(false, src, dst, g, long(c.nb) * pl->C * c.g.bz, c.tw, s);
}

// order 1: mirror groups (the four slices reading the same folded table rows
// back to back on one XCD); order 0: slices (ky, tile), mirrored ky slices
// paired when the slice count allows it
template <typename R>
hipError_t pass_z(const ApplyCall<R>& c, const LenOps<R>* opsz, const cx<R>* tab, int T, int order, hipStream_t s) {
  const vie_plan* pl = c.pl;
  const long Pz = c.g.sp->Pz, Q = c.g.sp->Pxy, bz = c.g.bz, W = pitch_y(Q);
  const long ntiles = (Q + T - 1) / T;  // the last tile may be partial
  ZArgs a{T,      int(ntiles), int(Pz / 2),           int(Pz), c.g.sp->nxp, c.g.sp->ne, bz * Q * W,
          long(pl->C) * bz * Q * W, c.nb, int(bz), int(Q), pl->omega, c.act};
  a.pitch = W;
  long nblocks;
  if (order == 1) {
    a.quad = 1;
    a.ntx = int((Q / 2 + T - 1) / T);
    a.ngroups = (Q / 2) * a.ntx;
    nblocks = (a.ngroups + 7) / 8 * 8 * 4 * c.nb;
  } else {
    if (ntiles * Q % 8 != 0) return hipErrorInvalidValue;  // XCD block order: slices in groups of 8
    a.pair_ky = (Q % 2 == 0 && (Q / 2) * ntiles % 8 == 0) ? 1 : 0;
    nblocks = ntiles * Q * c.nb;
  }
  return opsz->zpass(geom_mul(pl, c.g), c.B, tab, a, nblocks, c.twz, s);
}

// y inverse: B -> A, outputs y < by
template <typename R>
hipError_t pass_yinv(const ApplyCall<R>& c, const LenOps<R>* ops, int T, hipStream_t s) {
  const vie_plan* pl = c.pl;
  const long P = c.g.sp->Pxy, by = c.g.by, Wx = pitch_x(P), Wy = pitch_y(P);
  Geo g{T, int(P / T), P, int(P), int(by), c.act, long(pl->C) * c.g.bz * P};
  MemLoad<cx<R>> src{c.B, P * Wy, 1, Wy};
  MemStore<cx<R>> dst{c.A, by * Wx, 1, Wx, 1.0, 0};
  return ops->strided(true, src, dst, g, long(c.nb) * pl->C * c.g.bz, c.tw, s);
}

// TV: storage of J (the input), TO: of the output (complex64 output from
// complex128 input: the FP32 matvec of the mixed solver)
template <typename R, typename TV, typename TO = TV>
hipError_t pass_xinv(const ApplyCall<R>& c, const LenOps<R>* ops, const TV* addv, const c128* bvec, TO* out,
                     int mode, int T, hipStream_t s) {
  const vie_plan* pl = c.pl;
  const long NN = long(c.g.bz) * c.g.by;
  const int xcd = 1;  // tiles of all right-hand sides that share H run back to back on one XCD
  XArgs a{T,      long(c.nb) * NN, pl->n,  pl->n3, c.nb,   xcd,  c.g.bx,
          c.g.by, c.g.bz,          c.g.x0, c.g.y0, c.g.z0, c.g.np, c.g.rows, c.act};
  a.pitch = pitch_x(c.g.sp->Pxy);
  const cx<R>* H;
  const cx<R>* Hmu;
  if constexpr (std::is_same<R, float>::value) {
    H = pl->H32;
    Hmu = pl->Hmu32;
  } else {
    H = pl->H64;
    Hmu = pl->Hmu64;
  }
  if constexpr (std::is_same<TV, c128>::value && std::is_same<TO, c128>::value) {
    return ops->xinv(pl->C, mode, c.A, a, addv, bvec, H, Hmu, out, c.tw, s);
  } else if constexpr (std::is_same<TV, c128>::value) {
    if (mode != MODE_MATVEC || !ops->xinv_w32) return hipErrorInvalidValue;
    return ops->xinv_w32(pl->C, c.A, a, addv, H, Hmu, out, c.tw, s);
  } else {
    if (mode != MODE_MATVEC || !ops->xinv_v32) return hipErrorInvalidValue;
    return ops->xinv_v32(pl->C, c.A, a, addv, H, Hmu, out, c.tw, s);
  }
}

template <typename R>
int ensure_workspace(vie_plan* pl, int nb) {
  const int idx = std::is_same<R, double>::value ? 1 : 0;
  if (pl->ws_cap[idx] >= nb) return VIE_OK;
  clear_graphs(pl);  // captured applies hold the old workspace pointers
  dev_free(pl, pl->wsA[idx]);
  dev_free(pl, pl->wsB[idx]);
  pl->wsA[idx] = pl->wsB[idx] = nullptr;
  pl->ws_cap[idx] = 0;
  // every transform length is at most P = 2n, and the pitches grow with it
  const size_t N = size_t(pl->n), P = size_t(pl->P), C = size_t(pl->C);
  const size_t Wx = size_t(pitch_x(pl->P)), Wy = size_t(pitch_y(pl->P));
  int rc = dev_alloc(pl, &pl->wsA[idx], sizeof(cx<R>) * size_t(nb) * C * N * N * Wx);
  if (rc) return rc;
  rc = dev_alloc(pl, &pl->wsB[idx], sizeof(cx<R>) * size_t(nb) * C * N * P * Wy);
  if (rc) return rc;
  pl->ws_cap[idx] = nb;
  return VIE_OK;
}

// time one pass for each tile candidate and keep the fastest
// best_ms (optional): the time of the chosen tile (3 launches); skip_unrunnable:
// candidates whose launch is refused (an order that does not fit the tile
// count) are skipped instead of failing the choice
template <typename R, typename F>
int pick_tile(vie_plan* pl, int P1, int P2, bool contig, int maxthreads, int cols, F&& run, hipStream_t s, int* out,
              bool ragged = false, float* best_out = nullptr, bool skip_unrunnable = false) {
  hipEvent_t e0, e1;
  HIPCHK(pl, hipEventCreate(&e0));
  HIPCHK(pl, hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best = 0;
  bool any_full = false;
  for (int T : kTileChoices)
    any_full = any_full || tile_ok<R>(pl, P1, P2, T, contig, cols, maxthreads, true, ragged);
  for (int T : kTileChoices) {
    if (!tile_ok<R>(pl, P1, P2, T, contig, cols, maxthreads, any_full, ragged)) continue;
    if (skip_unrunnable) {
      const hipError_t e = run(T);  // warm-up; a refused launch shape is skipped
      if (e == hipErrorInvalidValue) {
        (void)hipGetLastError();
        continue;
      }
      HIPCHK(pl, e);
    } else {
      HIPCHK(pl, run(T));  // warm-up
    }
    HIPCHK(pl, hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) HIPCHK(pl, run(T));
    HIPCHK(pl, hipEventRecord(e1, s));
    HIPCHK(pl, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(pl, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = T;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best == 0) {
    if (skip_unrunnable) {
      *out = 0;
      return VIE_OK;
    }
    return fail(pl, VIE_E_SIZE, "no tile shape fits the LDS limit");
  }
  *out = best;
  if (best_out) *best_out = best_ms;
  return VIE_OK;
}

int tune_key(int nb, const Geom& g) { return bucket_of(nb) + (g.id << 20) + ((g.mul + 1) << 24); }

// Tile choices measured by any plan of the process, so that later plans of
// the same shape (a serving stream's requests on one grid, whatever their
// media) do not measure again: keyed by precision, transform lengths,
// components, multiply, batch bucket and whether the data are support rows.
// The extent of the support box is left out: it sets the number of pencils
// of the x and y passes and the z length of the data, not which launch shape
// is fastest, and boxes of one transform length differ by a few planes.
using SharedTuneKey = std::tuple<int, int, int, int, int, int, int>;
std::map<SharedTuneKey, Tune>& shared_tunes() {
  static std::map<SharedTuneKey, Tune> m;
  return m;
}
std::mutex& shared_tunes_mutex() {
  static std::mutex m;
  return m;
}
SharedTuneKey shared_key(const vie_plan* pl, int rsize, int nb, const Geom& g) {
  return SharedTuneKey{rsize, g.sp->Pxy, g.sp->Pz, pl->C, g.mul < 0 ? (pl->full ? MUL_MAX6 : MUL_SYM3) : g.mul,
                       bucket_of(nb), g.rows ? 1 : 0};
}
// The split of every pass, per shape without the batch bucket: the split
// sets the rounding of the transforms, so it is measured once per shape and
// precision and kept for every batch size, and a right-hand side gets
// bitwise the same applies alone or in any batch of the process (tiles and
// the z block order leave the arithmetic as it is and are measured per bucket).
std::map<SharedTuneKey, std::array<int, 5>>& shared_splits() {
  static std::map<SharedTuneKey, std::array<int, 5>> m;
  return m;
}

// tiles chosen without measuring: about 256 threads per block, whole 128-byte
// lines where the column count allows
template <typename R>
int default_tune(vie_plan* pl, const ApplyCall<R>& c, Tune* d) {
  const int P1 = c.ops->P1, P2 = c.ops->P2, Z1 = c.opsz->P1, Z2 = c.opsz->P2;
  const int P = P1 * P2;  // the x and y transform length; the z pass runs over P x P columns
  d->tx_fwd = default_tile<R>(pl, P1, P2, true, kPassMaxThreads, P);
  const int fmax = pl->C == 6 ? fused_max_threads<R, 6>() : fused_max_threads<R, 3>();
  d->tx_inv = default_tile<R>(pl, P1, P2, true, fmax, P);
  d->ty_fwd = d->ty_inv = default_tile<R>(pl, P1, P2, false, kPassMaxThreads, P);
  d->tz = default_tile<R>(pl, Z1, Z2, false, fmax, P, true);
  if (d->tx_fwd == 0 || d->tz == 0 || d->tx_inv == 0 || d->ty_fwd == 0)
    return fail(pl, VIE_E_SIZE, "no tile shape fits the LDS limit");
  return VIE_OK;
}

// the tiles measured earlier for this batch size and geometry, else the
// defaults; measures nothing and records nothing (the allocation-free apply)
template <typename R>
int fixed_tune(vie_plan* pl, const ApplyCall<R>& c, Tune* t) {
  const int idx = std::is_same<R, double>::value ? 1 : 0;
  auto it = pl->tune[idx].find(tune_key(c.nb, c.g));
  if (it != pl->tune[idx].end()) {
    *t = it->second;
    return VIE_OK;
  }
  return default_tune<R>(pl, c, t);
}

// the split variant v of the x/y length (Pxy) and of the z length usable for
// vectors TV and outputs TO, or null
template <typename R, typename TV, typename TO>
const LenOps<R>* xy_ops(int P, int v) {
  const LenOps<R>* o = len_ops<R>(P, v);
  if (!o || !o->strided || !o->contig_fwd || !o->xinv) return nullptr;
  if (!std::is_same<TV, c128>::value && (!o->contig_fwd_v32 || !o->xinv_v32)) return nullptr;
  if (!std::is_same<TO, TV>::value && !o->xinv_w32) return nullptr;
  return o;
}
template <typename R>
const LenOps<R>* z_ops(int P, int v) {
  const LenOps<R>* o = len_ops<R>(P, v);
  return (o && o->zpass) ? o : nullptr;
}

template <typename R, typename TV, typename TO = TV>
int get_tune(vie_plan* pl, const ApplyCall<R>& c, const TV* in, TO* out, hipStream_t s, Tune* t) {
  const int idx = std::is_same<R, double>::value ? 1 : 0;
  const int key = tune_key(c.nb, c.g);
  auto it = pl->tune[idx].find(key);
  if (it != pl->tune[idx].end()) {
    *t = it->second;
    return VIE_OK;
  }
  const SharedTuneKey skey = shared_key(pl, int(sizeof(R)), c.nb, c.g);
  // VIE_TILES="xfwd,yfwd,z,yinv,xinv[,zorder]" pins the tiles (and the z
  // pass's block order, 0 paired by default, 1 mirror groups) of this precision, and
  // VIE_SPLITS="xfwd,yfwd,z,yinv,xinv" the split variant of each pass (where
  // the length has it) with default tiles (profiling runs that must repeat a
  // measured launch shape, and tests of every split); pinned choices are not
  // shared with other plans
  const char* pin = std::getenv(sizeof(R) == 8 ? "VIE_TILES_FP64" : "VIE_TILES");
  const char* spin = std::getenv("VIE_SPLITS");
  auto from_shared = [&]() {
    if (pin || spin) return false;
    std::lock_guard<std::mutex> lk(shared_tunes_mutex());
    auto sit = shared_tunes().find(skey);
    if (sit == shared_tunes().end()) return false;
    pl->tune[idx][key] = sit->second;
    *t = sit->second;
    return true;
  };
  if (from_shared()) return VIE_OK;
  const int Pxy = c.g.sp->Pxy, Pz = c.g.sp->Pz;
  const int fmax = pl->C == 6 ? fused_max_threads<R, 6>() : fused_max_threads<R, 3>();
  Tune d;
  int rc = default_tune<R>(pl, c, &d);
  if (rc) return rc;
  int sv[5] = {0, 0, 0, 0, 0};
  const int nsv = spin ? std::sscanf(spin, "%d,%d,%d,%d,%d", &sv[0], &sv[1], &sv[2], &sv[3], &sv[4]) : 0;
  if (nsv == 5) {
    // a pinned variant that a length does not have falls back to its split 0
    for (int i = 0; i < 5; ++i) {
      const bool has = i == 2 ? z_ops<R>(Pz, sv[i]) != nullptr : xy_ops<R, TV, TO>(Pxy, sv[i]) != nullptr;
      if (!has) sv[i] = 0;
    }
    const LenOps<R>* o[5] = {xy_ops<R, TV, TO>(Pxy, sv[0]), xy_ops<R, TV, TO>(Pxy, sv[1]), z_ops<R>(Pz, sv[2]),
                             xy_ops<R, TV, TO>(Pxy, sv[3]), xy_ops<R, TV, TO>(Pxy, sv[4])};
    d.vx_fwd = sv[0];
    d.vy_fwd = sv[1];
    d.vz = sv[2];
    d.vy_inv = sv[3];
    d.vx_inv = sv[4];
    d.tx_fwd = default_tile<R>(pl, o[0]->P1, o[0]->P2, true, kPassMaxThreads, Pxy);
    d.ty_fwd = default_tile<R>(pl, o[1]->P1, o[1]->P2, false, kPassMaxThreads, Pxy);
    d.tz = default_tile<R>(pl, o[2]->P1, o[2]->P2, false, fmax, Pxy, true);
    d.ty_inv = default_tile<R>(pl, o[3]->P1, o[3]->P2, false, kPassMaxThreads, Pxy);
    d.tx_inv = default_tile<R>(pl, o[4]->P1, o[4]->P2, true, fmax, Pxy);
    if (!d.tx_fwd || !d.ty_fwd || !d.tz || !d.ty_inv || !d.tx_inv)
      return fail(pl, VIE_E_SIZE, "no tile shape fits the LDS limit");
  }
  int pt[6] = {0, 0, 0, 0, 0, 0};
  const int npin = pin ? std::sscanf(pin, "%d,%d,%d,%d,%d,%d", &pt[0], &pt[1], &pt[2], &pt[3], &pt[4], &pt[5]) : 0;
  if (npin >= 5) {
    const LenOps<R>* o[5] = {xy_ops<R, TV, TO>(Pxy, d.vx_fwd), xy_ops<R, TV, TO>(Pxy, d.vy_fwd), z_ops<R>(Pz, d.vz),
                             xy_ops<R, TV, TO>(Pxy, d.vy_inv), xy_ops<R, TV, TO>(Pxy, d.vx_inv)};
    const bool ok = tile_ok<R>(pl, o[0]->P1, o[0]->P2, pt[0], true, Pxy, kPassMaxThreads, false) &&
                    tile_ok<R>(pl, o[1]->P1, o[1]->P2, pt[1], false, Pxy, kPassMaxThreads, false) &&
                    tile_ok<R>(pl, o[2]->P1, o[2]->P2, pt[2], false, Pxy, fmax, false, true) &&
                    tile_ok<R>(pl, o[3]->P1, o[3]->P2, pt[3], false, Pxy, kPassMaxThreads, false) &&
                    tile_ok<R>(pl, o[4]->P1, o[4]->P2, pt[4], true, Pxy, fmax, false);
    if (!ok) return fail(pl, VIE_E_ARG, std::string("tiles pinned by the environment do not fit: ") + pin);
    d.tx_fwd = pt[0];
    d.ty_fwd = pt[1];
    d.tz = pt[2];
    d.ty_inv = pt[3];
    d.tx_inv = pt[4];
    d.zorder = pt[5] != 0 ? 1 : 0;
  } else if (nsv != 5 && pl->n >= 48 && env_flag("VIE_AUTOTUNE", true)) {
    // measure only where it pays: large grids, unless switched off.  Every
    // pass reads and writes its data in natural order, so each may use its
    // own split; per pass the fastest (split, tile) over the compiled splits,
    // or over the tiles of the split this shape already has.  Plans on other
    // threads may measure at the same time (serving workers: their timings
    // then share the device); the first splits stored for a shape win.
    //
    // A batch bucket within a factor of 4 of one that this shape has already
    // measured takes that one's choices instead of measuring: a serving
    // stream meets every batch size from 1 to 16 on every grid, and a
    // measurement costs more than a small solve.
    if (!pin && !spin) {
      std::lock_guard<std::mutex> lk(shared_tunes_mutex());
      const int b0 = bucket_of(c.nb);
      for (const int b : {b0 / 2, b0 * 2, b0 / 4, b0 * 4}) {
        if (b < 1) continue;
        SharedTuneKey near = skey;
        std::get<5>(near) = b;
        const auto it = shared_tunes().find(near);
        if (it == shared_tunes().end()) continue;
        // kept by this plan only: the process-wide map holds measured choices
        pl->tune[idx][key] = it->second;
        *t = it->second;
        return VIE_OK;
      }
    }
    const SharedTuneKey split_key = shared_key(pl, int(sizeof(R)), 0, c.g);
    std::array<int, 5> only{-1, -1, -1, -1, -1};
    bool have_splits = false;
    {
      std::lock_guard<std::mutex> lk(shared_tunes_mutex());
      auto sit = shared_splits().find(split_key);
      if (sit != shared_splits().end() && !pin && !spin) {
        only = sit->second;
        have_splits = true;
      }
    }
    const cx<R>* tab;
    if constexpr (std::is_same<R, float>::value)
      tab = c.g.sp->tab32;
    else
      tab = c.g.sp->tab64;
    const bool dbg = env_flag("VIE_DEBUG", false);
    // (variant, tile) with the smallest time of run(ops, T) over the splits
    auto best_of = [&](const char* name, int pass, bool contig, int maxthreads, int* vout, int* tout,
                       auto&& run) -> int {
      float best = 1e30f;
      const bool z = pass == 2;
      for (int v = 0; v < kMaxSplits; ++v) {
        if (only[size_t(pass)] >= 0 && v != only[size_t(pass)]) continue;
        const LenOps<R>* o = z ? z_ops<R>(Pz, v) : xy_ops<R, TV, TO>(Pxy, v);
        if (!o) continue;
        int tv = 0;
        float ms = 0;
        const int r = pick_tile<R>(pl, o->P1, o->P2, contig, maxthreads, Pxy, [&](int T) { return run(o, T); }, s,
                                   &tv, z, &ms, true);
        if (r) return r;
        if (dbg && tv)
          std::fprintf(stderr, "[vie] %s P=%d split %dx%d fp%d nb=%d: T=%d %.3f ms\n", name, o->P, o->P1, o->P2,
                       int(8 * sizeof(R)), c.nb, tv, double(ms));
        if (tv && ms < best) {
          best = ms;
          *vout = v;
          *tout = tv;
        }
      }
      return best < 1e30f ? VIE_OK : fail(pl, VIE_E_SIZE, std::string("no launch shape for the ") + name);
    };
    for (int attempt = 0; attempt < 2; ++attempt) {
      rc = best_of("x fwd", 0, true, kPassMaxThreads, &d.vx_fwd, &d.tx_fwd,
                   [&](const LenOps<R>* o, int T) { return pass_xfwd<R, TV>(c, o, in, T, s); });
      if (rc) return rc;
      rc = best_of("y fwd", 1, false, kPassMaxThreads, &d.vy_fwd, &d.ty_fwd,
                   [&](const LenOps<R>* o, int T) { return pass_yfwd<R>(c, o, T, s); });
      if (rc) return rc;
      // the z pass: split, tile width and block order (the paired order needs
      // the slices in groups of 8: tiles that do not allow it are refused at
      // launch and skipped)
      {
        int vq = 0, tq = 0, vp = 0, tp = 0;
        rc = best_of("z (mirror groups)", 2, false, fmax, &vq, &tq,
                     [&](const LenOps<R>* o, int T) { return pass_z<R>(c, o, tab, T, 1, s); });
        if (rc) return rc;
        float mq = 0, mp = 1e30f;
        rc = pick_tile<R>(pl, z_ops<R>(Pz, vq)->P1, z_ops<R>(Pz, vq)->P2, false, fmax, Pxy,
                          [&](int T) { return pass_z<R>(c, z_ops<R>(Pz, vq), tab, T, 1, s); }, s, &tq, true, &mq, true);
        if (rc) return rc;
        const int rp = best_of("z (paired)", 2, false, fmax, &vp, &tp,
                               [&](const LenOps<R>* o, int T) { return pass_z<R>(c, o, tab, T, 0, s); });
        if (rp == VIE_OK && tp) {
          rc = pick_tile<R>(pl, z_ops<R>(Pz, vp)->P1, z_ops<R>(Pz, vp)->P2, false, fmax, Pxy,
                            [&](int T) { return pass_z<R>(c, z_ops<R>(Pz, vp), tab, T, 0, s); }, s, &tp, true, &mp,
                            true);
          if (rc) return rc;
        }
        if (tp && mp < mq) {
          d.zorder = 0;
          d.vz = vp;
          d.tz = tp;
        } else {
          d.zorder = 1;
          d.vz = vq;
          d.tz = tq;
        }
      }
      rc = best_of("y inv", 3, false, kPassMaxThreads, &d.vy_inv, &d.ty_inv,
                   [&](const LenOps<R>* o, int T) { return pass_yinv<R>(c, o, T, s); });
      if (rc) return rc;
      // the raw convolution for complex128 vectors (any J), the matvec for complex64
      const int xmode = std::is_same<TV, c128>::value && std::is_same<TO, c128>::value ? MODE_CONV : MODE_MATVEC;
      rc = best_of("x inv", 4, true, fmax, &d.vx_inv, &d.tx_inv, [&](const LenOps<R>* o, int T) {
        return pass_xinv<R, TV, TO>(c, o, in, nullptr, out, xmode, T, s);
      });
      if (rc) return rc;
      if (have_splits || pin || spin) break;
      const std::array<int, 5> got{d.vx_fwd, d.vy_fwd, d.vz, d.vy_inv, d.vx_inv};
      std::lock_guard<std::mutex> lk(shared_tunes_mutex());
      const auto ins = shared_splits().emplace(split_key, got);
      if (ins.second || ins.first->second == got) break;
      // another plan of this shape stored different splits while this one
      // measured: take those, and measure their tiles
      only = ins.first->second;
      have_splits = true;
    }
  }
  d.tuned = true;
  if (env_flag("VIE_DEBUG", false))
    std::fprintf(stderr,
                 "[vie] tiles Pxy=%d Pz=%d fp%d nb=%d box %dx%dx%d: xfwd %d/%d yfwd %d/%d z %d/%d order %d "
                 "yinv %d/%d xinv %d/%d (split/tile)\n",
                 Pxy, Pz, int(8 * sizeof(R)), c.nb, c.g.bx, c.g.by, c.g.bz, d.vx_fwd, d.tx_fwd, d.vy_fwd, d.ty_fwd,
                 d.vz, d.tz, d.zorder, d.vy_inv, d.ty_inv, d.vx_inv, d.tx_inv);
  pl->tune[idx][key] = d;
  if (!pin && !spin) {
    std::lock_guard<std::mutex> lk(shared_tunes_mutex());
    shared_tunes()[skey] = d;
  }
  *t = d;
  return VIE_OK;
}

// act (device, optional): per right-hand side, 0 = skip it (its output is
// left as it was); nact = the number of non-zero flags, for the byte counts
// Caller-provided apply workspace (the allocation-free entry point): arrays A
// and B for `cap` right-hand sides; tiles are not measured and no kernel is
// timed.  Without it the plan's own workspace is used (grown on demand).
struct FixedWork {
  void* A;
  void* B;
  int cap;
};

template <typename R, typename TV, typename TO = TV>
int apply_typed(vie_plan* pl, const Geom& geom, const TV* in, const TV* addv, const c128* bvec, TO* out,
                int nrhs, int mode, hipStream_t s, const int* act = nullptr, int nact = -1,
                const FixedWork* fw = nullptr) {
  const Spec& sp = *geom.sp;
  const LenOps<R>* ops = len_ops<R>(sp.Pxy);
  const LenOps<R>* opsz = len_ops<R>(sp.Pz);
  if (!ops || !ops->contig_fwd || !ops->xinv || !opsz || !opsz->zpass)
    return fail(pl, VIE_E_SIZE, "no compiled FFT lengths " + std::to_string(sp.Pxy) + ", " + std::to_string(sp.Pz));
  if (!std::is_same<TV, c128>::value && (!ops->contig_fwd_v32 || !ops->xinv_v32))
    return fail(pl, VIE_E_STATE, "complex64 vectors need the FP32 apply");
  if (!std::is_same<TO, TV>::value && (!ops->xinv_w32 || mode != MODE_MATVEC))
    return fail(pl, VIE_E_STATE, "complex64 output needs the FP32 matvec");
  const int idx = std::is_same<R, double>::value ? 1 : 0;
  int chunk = std::max(1, std::min(nrhs, pl->max_rhs));
  cx<R>* wA;
  cx<R>* wB;
  if (fw) {
    chunk = std::max(1, std::min(chunk, fw->cap));
    wA = static_cast<cx<R>*>(fw->A);
    wB = static_cast<cx<R>*>(fw->B);
  } else {
    const int rc = ensure_workspace<R>(pl, chunk);
    if (rc) return rc;
    wA = static_cast<cx<R>*>(pl->wsA[idx]);
    wB = static_cast<cx<R>*>(pl->wsB[idx]);
  }
  int rc = VIE_OK;
  const cx<R>* tw;
  const cx<R>* twz;
  const cx<R>* tab;
  if constexpr (std::is_same<R, float>::value) {
    tw = sp.tw32;
    twz = sp.twz32;
    tab = sp.tab32;
  } else {
    tw = sp.tw64;
    twz = sp.twz64;
    tab = sp.tab64;
  }
  const long L = long(pl->C) * geom.np;
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int nb = std::min(chunk, nrhs - r0);
    ApplyCall<R> c{pl, ops, tw, opsz, twz, wA, wB, nb, geom};
    const long off = long(r0) * L;
    const TV* inr = in + off;
    TO* outr = out + off;
    Tune t;
    rc = fw ? fixed_tune<R>(pl, c, &t) : get_tune<R, TV, TO>(pl, c, inr, outr, s, &t);
    if (rc) return rc;
    c.act = act ? act + r0 : nullptr;
    const int nrun = (act && nact >= 0 && nrhs <= chunk) ? nact : nb;  // right-hand sides computed
    const int f0 = std::is_same<R, double>::value ? FAM_XFWD64 : FAM_XFWD32;
    // algorithmic bytes: every operand read or written once per launch
    const double cr = double(sizeof(cx<R>)), c16 = double(sizeof(TV)), co = double(sizeof(TO));
    const double vN3 = double(nrun) * pl->C * double(geom.np);
    // rows of the x-transformed array: every (z, y) row of the box, of which
    // the x inverse reads only those holding support points
    const double vN2P = double(nrun) * pl->C * geom.bz * geom.by * sp.Pxy, vNP2 = vN2P / geom.by * sp.Pxy;
    const double vN2Pw = geom.rows ? double(nrun) * pl->C * double(geom.rows_nz) * sp.Pxy : vN2P;
    const double hb = 9.0 * double(geom.np) * cr * (pl->full ? 2 : 1);
    const double xinv_b = vN2Pw * cr + hb * (mode == MODE_MATVEC || mode == MODE_RESIDUAL) +
                          vN3 * (co + c16 * (mode != MODE_CONV)) + vN3 * sizeof(c128) * (mode == MODE_RESIDUAL);
    // nominal flops: 5 P log2 P per transformed pencil of length P; 66 per
    // frequency point for the 3x3 multiply (216 for the 6x6 Maxwell block);
    // 72 per point and 3-component half for the combine
    const double P = sp.Pxy, fft_row = 5.0 * P * std::log2(P);
    const double Pz = sp.Pz, fft_row_z = 5.0 * Pz * std::log2(Pz);
    const double rows_x = vN2P / P, rows_y = vN2P / geom.by, rows_z = vNP2 / geom.bz;
    const double pts = double(nrun) * P * P * Pz;
    const int mul = geom_mul(pl, geom);
    const double mul_f = (mul == MUL_MAX6 ? 216.0 : (mul == MUL_SYM3 ? 66.0 : 24.0)) * pts;
    const double comb_f = (mode == MODE_CONV) ? 0.0 : 72.0 * vN3 / 3.0;
    // the allocation-free path records no events (creating one may allocate)
    const bool prof = !fw;
    // the split of each pass (tuned or pinned; variant 0 by default)
    const LenOps<R>* ox_f = xy_ops<R, TV, TO>(sp.Pxy, t.vx_fwd);
    const LenOps<R>* oy_f = xy_ops<R, TV, TO>(sp.Pxy, t.vy_fwd);
    const LenOps<R>* oz = z_ops<R>(sp.Pz, t.vz);
    const LenOps<R>* oy_i = xy_ops<R, TV, TO>(sp.Pxy, t.vy_inv);
    const LenOps<R>* ox_i = xy_ops<R, TV, TO>(sp.Pxy, t.vx_inv);
    if (!ox_f || !oy_f || !oz || !oy_i || !ox_i) return fail(pl, VIE_E_STATE, "tuned split not compiled");
    int tok = prof ? prof_begin(pl, s) : -1;
    HIPCHK(pl, (pass_xfwd<R, TV>(c, ox_f, inr, t.tx_fwd, s)));
    prof_end(pl, f0 + 0, tok, s, vN3 * c16 + vN2P * cr, rows_x * fft_row);
    tok = prof ? prof_begin(pl, s) : -1;
    HIPCHK(pl, pass_yfwd<R>(c, oy_f, t.ty_fwd, s));
    prof_end(pl, f0 + 1, tok, s, (vN2P + vNP2) * cr, rows_y * fft_row);
    tok = prof ? prof_begin(pl, s) : -1;
    HIPCHK(pl, pass_z<R>(c, oz, tab, t.tz, t.zorder, s));
    prof_end(pl, f0 + 2, tok, s, 2.0 * vNP2 * cr + double(sp.tab_elems) * cr, 2.0 * rows_z * fft_row_z + mul_f);
    tok = prof ? prof_begin(pl, s) : -1;
    HIPCHK(pl, pass_yinv<R>(c, oy_i, t.ty_inv, s));
    prof_end(pl, f0 + 3, tok, s, (vN2P + vNP2) * cr, rows_y * fft_row);
    tok = prof ? prof_begin(pl, s) : -1;
    HIPCHK(pl, (pass_xinv<R, TV, TO>(c, ox_i, addv ? addv + off : inr, bvec ? bvec + off : nullptr, outr, mode,
                                     t.tx_inv, s)));
    prof_end(pl, f0 + 4, tok, s, xinv_b, rows_x * fft_row + comb_f);
  }
  return VIE_OK;
}

// ---------------------------------------------------------------------------
// precompute of the kernel-transform tables (FP64)
// ---------------------------------------------------------------------------
// Tables of the periodic grid (Pz, Pxy, Pxy) <= 2n: the kernel windowed to
// |m_z| <= Pz/2 - 1, |m_x|, |m_y| <= Pxy/2 - 1 (the window of the whole grid
// when both are 2n), transformed on that grid.  The box convolution needs
// offsets |m_a| <= b_a - 1 < P_a/2 only, and its wrapped copies lie at
// |m_a| >= P_a - (b_a - 1) > P_a/2 - 1.
int build_tables(vie_plan* pl, Spec& sp, hipStream_t s) {
  const int Z = sp.Pz, Q = sp.Pxy, M = pl->M, NE = sp.ne;
  const LenOps<double>* opsM = len_ops<double>(M);
  const LenOps<double>* opsQ = len_ops<double>(Q);
  const LenOps<double>* opsZ = len_ops<double>(Z);
  if (!opsM || !opsM->symbol_inv || !opsM->strided)
    return fail(pl, VIE_E_SIZE, "no compiled oversampled FFT length " + std::to_string(M));
  if (!opsQ || !opsQ->contig_fwd || !opsQ->strided || !opsZ || !opsZ->strided)
    return fail(pl, VIE_E_SIZE, "no compiled FFT lengths " + std::to_string(Q) + ", " + std::to_string(Z));
  c128* twM = nullptr;
  int rc = upload_twiddles<double>(pl, M, &twM, s);
  if (rc) return rc;
  const long MM = long(M), QQ = long(Q), ZZ = long(Z);
  c128 *buf1 = nullptr, *buf2 = nullptr, *buf3 = nullptr;
  rc = dev_alloc(pl, reinterpret_cast<void**>(&buf1), sizeof(c128) * size_t(MM * MM * QQ));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&buf2), sizeof(c128) * size_t(MM * QQ * QQ));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&buf3), sizeof(c128) * size_t(NE) * size_t(ZZ * QQ * QQ));
  auto cleanup = [&]() {
    dev_free(pl, buf1);
    dev_free(pl, buf2);
    dev_free(pl, buf3);
    dev_free(pl, twM);
  };
  if (rc) {
    cleanup();
    return rc;
  }
  // strided passes run over Q (y) or Q^2 (z) columns
  const int TcM = default_tile<double>(pl, opsM->P1, opsM->P2, true, kPassMaxThreads, 0);
  const int TsM = default_tile<double>(pl, opsM->P1, opsM->P2, false, kPassMaxThreads, Q);
  const int TcQ = default_tile<double>(pl, opsQ->P1, opsQ->P2, true, kPassMaxThreads, 0);
  const int TsQ = default_tile<double>(pl, opsQ->P1, opsQ->P2, false, kPassMaxThreads, Q);
  const int TsZ = default_tile<double>(pl, opsZ->P1, opsZ->P2, false, kPassMaxThreads, Q);
  if (!TcM || !TsM || !TcQ || !TsQ || !TsZ) {
    cleanup();
    return fail(pl, VIE_E_SIZE, "no tile shape fits the LDS limit for the precompute");
  }
  hipError_t e = hipSuccess;
  for (int ent = 0; ent < NE && e == hipSuccess; ++ent) {
    // (a) symbol samples of entry `ent` -> inverse transform along x; keep
    //     outputs 0..Q-1 (displacements -Q/2..Q/2-1), zero displacement -Q/2
    {
      SymbolSrc src{M, sp.set, ent, Q / 2, Q / 2, Z / 2, pl->h, pl->omega, pl->R};
      const long rows = MM * MM;
      Geo g{TcM, int((rows + TcM - 1) / TcM), rows, M, Q};
      MemStore<c128> dst{buf1, 0, QQ, 1, 1.0 / double(M), 1};
      e = opsM->symbol_inv(src, dst, g, 1, twM, s);
    }
    // (b) inverse along y: buf1[kz][ky][nx] -> buf2[kz][ny][nx], ny < Q
    if (e == hipSuccess) {
      Geo g{TsM, int(QQ / TsM), QQ, M, Q};
      MemLoad<c128> src{buf1, MM * QQ, 1, QQ};
      MemStore<c128> dst{buf2, QQ * QQ, 1, QQ, 1.0 / double(M), 1};
      e = opsM->strided(true, src, dst, g, MM, twM, s);
    }
    // (c) inverse along z: buf2[kz][ny][nx] -> buf3[ent][nz][ny][nx], nz < Z
    if (e == hipSuccess) {
      const long cols = QQ * QQ;
      Geo g{TsM, int(cols / TsM), cols, M, Z};
      MemLoad<c128> src{buf2, 0, 1, QQ * QQ};
      MemStore<c128> dst{buf3 + long(ent) * ZZ * QQ * QQ, 0, 1, QQ * QQ, 1.0 / double(M), 1};
      e = opsM->strided(true, src, dst, g, 1, twM, s);
    }
  }
  // (d) forward transforms along x (Q), y (Q), z (Z) (in place, all entries)
  if (e == hipSuccess) {
    const long rows = long(NE) * ZZ * QQ;
    Geo g{TcQ, int((rows + TcQ - 1) / TcQ), rows, Q, Q};
    MemLoad<c128> src{buf3, 0, QQ, 1};
    MemStore<c128> dst{buf3, 0, QQ, 1, 1.0, 0};
    e = opsQ->contig_fwd(src, dst, g, 1, sp.tw64, s);
  }
  if (e == hipSuccess) {
    Geo g{TsQ, int(QQ / TsQ), QQ, Q, Q};
    MemLoad<c128> src{buf3, QQ * QQ, 1, QQ};
    MemStore<c128> dst{buf3, QQ * QQ, 1, QQ, 1.0, 0};
    e = opsQ->strided(false, src, dst, g, long(NE) * ZZ, sp.tw64, s);
  }
  if (e == hipSuccess) {
    const long cols = QQ * QQ;
    Geo g{TsZ, int(cols / TsZ), cols, Z, Z};
    MemLoad<c128> src{buf3, ZZ * QQ * QQ, 1, QQ * QQ};
    MemStore<c128> dst{buf3, ZZ * QQ * QQ, 1, QQ * QQ, 1.0, 0};
    e = opsZ->strided(false, src, dst, g, NE, sp.twz64, s);
  }
  // (e) shift by P_a/2 in every axis ((-1)^q), scale by 1/(Z Q^2), fold to the octant
  if (e == hipSuccess) e = launch_finalize_tables(buf3, sp.tab64, sp.tab32, Q, Z, sp.nxp, NE, pl->omega, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  return e == hipSuccess ? VIE_OK : hip_fail(pl, e, "table precompute");
}

}  // namespace

namespace vie {

int apply_any(vie_plan* pl, const Geom& g, bool fp64, const c128* in, const c128* addv, const c128* bvec,
              c128* out, int nrhs, int mode, hipStream_t s, const int* act, int nact) {
  if (g.sp == &pl->sg) {
    const int rc = ensure_grid_spec(pl, s);
    if (rc) return rc;
  }
  return fp64 ? apply_typed<double, c128>(pl, g, in, addv, bvec, out, nrhs, mode, s, act, nact)
              : apply_typed<float, c128>(pl, g, in, addv, bvec, out, nrhs, mode, s, act, nact);
}

int apply_any(vie_plan* pl, const Geom& g, const c64* in, c64* out, int nrhs, hipStream_t s) {
  if (g.sp == &pl->sg) {
    const int rc = ensure_grid_spec(pl, s);
    if (rc) return rc;
  }
  return apply_typed<float, c64>(pl, g, in, in, nullptr, out, nrhs, MODE_MATVEC, s);
}

int apply_any(vie_plan* pl, const Geom& g, const c128* in, c64* out, int nrhs, hipStream_t s, const int* act,
              int nact) {
  if (g.sp == &pl->sg) {
    const int rc = ensure_grid_spec(pl, s);
    if (rc) return rc;
  }
  return apply_typed<float, c128, c64>(pl, g, in, in, nullptr, out, nrhs, MODE_MATVEC, s, act, nact);
}

void clear_graphs(vie_plan* pl) {
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
  pl->graphs.clear();
}

namespace {

// Replays the apply `run(stream)` from a hipGraph captured at its first call
// with this key; eager when capture is off, while timing kernels, for chunked
// batches, or before the first apply of this batch size (tiling and
// workspace set up).
template <typename F>
int graph_or_eager(vie_plan* pl, const Geom& g, bool fp64, int nrhs, const vie_plan::GraphKey& key, hipStream_t s,
                   F&& run) {
  const int idx = fp64 ? 1 : 0;
  if (!pl->use_graphs || pl->prof_on || nrhs > pl->max_rhs || pl->ws_cap[idx] < nrhs ||
      pl->tune[idx].find(tune_key(nrhs, g)) == pl->tune[idx].end())
    return run(s);
  if (!pl->gstream) {
    HIPCHK(pl, hipStreamCreateWithFlags(&pl->gstream, hipStreamNonBlocking));
  }
  auto it = pl->graphs.find(key);
  if (it == pl->graphs.end()) {
    if (pl->graphs.size() >= 512) clear_graphs(pl);
    std::lock_guard<std::recursive_mutex> lk(hip_mutex());
    hipGraph_t graph = nullptr;
    HIPCHK(pl, hipStreamBeginCapture(pl->gstream, hipStreamCaptureModeRelaxed));
    const int rc = run(pl->gstream);
    const hipError_t ec = hipStreamEndCapture(pl->gstream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) return hip_fail(pl, ec, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(pl, ei, "hipGraphInstantiate");
    it = pl->graphs.emplace(key, ex).first;
  }
  // replayed on the caller's stream itself: captured on the plan's stream
  // (so that nothing else of the caller's stream is recorded), run in order
  // with the caller's work without an event hop per apply
  HIPCHK(pl, hipGraphLaunch(it->second, s));
  pl->graph_launches++;
  return VIE_OK;
}

}  // namespace

int apply_graph(vie_plan* pl, const Geom& g, bool fp64, const c128* in, const c128* addv, const c128* bvec,
                c128* out, int nrhs, int mode, hipStream_t s, const int* act, int nact) {
  const vie_plan::GraphKey key{fp64 ? 1 : 0, mode, nrhs, g.id, in, addv, bvec, out, act, 0};
  return graph_or_eager(pl, g, fp64, nrhs, key, s, [&](hipStream_t st) {
    return apply_any(pl, g, fp64, in, addv, bvec, out, nrhs, mode, st, act, nact);
  });
}

int apply_graph(vie_plan* pl, const Geom& g, const c128* in, c64* out, int nrhs, hipStream_t s, const int* act,
                int nact) {
  const vie_plan::GraphKey key{0, MODE_MATVEC, nrhs, g.id, in, in, nullptr, out, act, 1};
  return graph_or_eager(pl, g, false, nrhs, key, s, [&](hipStream_t st) {
    return apply_any(pl, g, in, out, nrhs, st, act, nact);
  });
}

}  // namespace vie

namespace {

const int kSupportedN[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 160};

bool n_supported(int n) {
  for (int v : kSupportedN)
    if (v == n) return true;
  return false;
}

void destroy_plan(vie_plan* pl) {
  if (!pl) return;
  // wait for the plan's own work before taking the library lock: the stream
  // may be another thread's, still busy with later work (the event marks the
  // end of the plan's last call), and the lock would stall every allocation
  // meanwhile
  if (pl->done_valid) {
    (void)hipEventSynchronize(pl->done_ev);
    if (pl->gstream) (void)hipStreamSynchronize(pl->gstream);
  } else {
    quiesce(pl);
  }
  std::lock_guard<std::recursive_mutex> lk(hip_mutex());
  if (pl->done_ev) (void)hipEventDestroy(pl->done_ev);
  pl->done_ev = nullptr;
  vie::close_session(pl);
  vie::clear_graphs(pl);
  if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
  pl->gstream = nullptr;
  for (auto& r : pl->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pl->ev_pool) (void)hipEventDestroy(e);
  for (auto& a : pl->allocs) give_block(a.first, a.second, pl->device);
  pl->allocs.clear();
  for (auto& a : pl->host_allocs) give_host_block(a.first, a.second);
  pl->host_allocs.clear();
  delete pl;
}

// twiddles and kernel-transform tables of the grid (Pz, Pxy, Pxy) for the
// symbol set `set` (ne entries)
int make_spec(vie_plan* pl, int Pz, int Pxy, int set, int ne, Spec& sp, hipStream_t s) {
  sp.set = set;
  sp.ne = ne;
  sp.Pz = Pz;
  sp.Pxy = Pxy;
  sp.nxp = ((Pz / 2 + 1 + 15) / 16) * 16;
  int rc = upload_twiddles<double>(pl, Pxy, &sp.tw64, s);
  if (!rc) rc = upload_twiddles<float>(pl, Pxy, &sp.tw32, s);
  if (!rc && Pz == Pxy) {
    sp.twz64 = sp.tw64;
    sp.twz32 = sp.tw32;
  } else {
    if (!rc) rc = upload_twiddles<double>(pl, Pz, &sp.twz64, s);
    if (!rc) rc = upload_twiddles<float>(pl, Pz, &sp.twz32, s);
  }
  if (rc) return rc;
  sp.tab_elems = long(Pz / 2 + 1) * (Pz / 2 + 1) * ne * sp.nxp;
  rc = dev_alloc(pl, reinterpret_cast<void**>(&sp.tab64), sizeof(c128) * size_t(sp.tab_elems));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&sp.tab32), sizeof(c64) * size_t(sp.tab_elems));
  if (rc) return rc;
  return build_tables(pl, sp, s);
}

}  // namespace

int vie::ensure_grid_spec(vie_plan* pl, hipStream_t s) {
  if (pl->sg.tab64) return VIE_OK;
  return make_spec(pl, pl->P, pl->P, pl->sym_set, pl->ne, pl->sg, s);
}

int vie::ensure_div_spec(vie_plan* pl, hipStream_t s) {
  if (pl->sdiv.tab64) return VIE_OK;
  return make_spec(pl, pl->P, pl->P, SYM_DIV, 3, pl->sdiv, s);
}

namespace {

// The shortest compiled transform length L <= 2n with L >= 2 max(bx, by)
// (so that the cyclic convolution of box data has no wrap-around along x and
// y) whose apply and precompute kernels exist (along z: z_length).
int box_length(const vie_plan* pl) {
  const int need = 2 * std::max(pl->box.bx, pl->box.by);
  for (int L = need + (need & 1); L < pl->P; L += 2) {
    const LenOps<float>* o32 = len_ops<float>(L);
    const LenOps<double>* o64 = len_ops<double>(L);
    if (L % 8 == 0 && o32 && o64 && o32->contig_fwd && o32->strided && o32->xinv && o64->contig_fwd &&
        o64->strided && o64->xinv)
      return L;
  }
  return pl->P;
}

// The z length of the box's transforms: at least 2 bz (no wrap-around along
// z), at least the x/y length (the table octant holds qx, qy <= Pxy/2 <=
// Pz/2) and at most 2n.  A length with a square split (64 = 8 x 8,
// 256 = 16 x 16) is taken when it fits: its fused z pass keeps every lane
// busy in all four DFT steps, in blocks of whole waves, where the other
// splits idle lanes (the 20 x 16 split of 320 ran at about half its issue
// rate); else 2n, as before.
int z_length(const vie_plan* pl, int pxy) {
  const int need = std::max(2 * pl->box.bz, pxy);
  for (const int L : {64, 256}) {
    if (L < need || L >= pl->P) continue;
    const LenOps<float>* o32 = len_ops<float>(L);
    const LenOps<double>* o64 = len_ops<double>(L);
    if (o32 && o64 && o32->zpass && o64->zpass && o64->strided) return L;
  }
  return pl->P;
}

// Support rows of the box: per (z, y) row the x-interval of the points where
// H (or H_mu) is non-zero; the solver's vectors hold only these points.
int build_rows(vie_plan* pl, hipStream_t s) {
  const long nr = long(pl->box.by) * pl->box.bz;
  int* xalen = nullptr;
  int rc = dev_alloc(pl, reinterpret_cast<void**>(&xalen), sizeof(int) * 2 * size_t(nr));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->rows_d), sizeof(int) * 3 * size_t(nr));
  if (rc) return rc;
  HIPCHK(pl, launch_row_support(pl->H64, pl->full ? pl->Hmu64 : nullptr, box_of(pl->box, pl->n), xalen, s));
  std::vector<int> h2(size_t(2 * nr)), h3(size_t(3 * nr));
  HIPCHK(pl, hipMemcpyAsync(h2.data(), xalen, sizeof(int) * h2.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(pl, hipStreamSynchronize(s));
  long off = 0;
  for (long r = 0; r < nr; ++r) {
    h3[size_t(3 * r)] = h2[size_t(2 * r)];
    h3[size_t(3 * r + 1)] = h2[size_t(2 * r + 1)];
    h3[size_t(3 * r + 2)] = int(off);
    off += h2[size_t(2 * r + 1)];
  }
  long nonempty = 0;
  for (long r = 0; r < nr; ++r) nonempty += h2[size_t(2 * r + 1)] > 0 ? 1 : 0;
  HIPCHK(pl, hipMemcpyAsync(pl->rows_d, h3.data(), sizeof(int) * h3.size(), hipMemcpyHostToDevice, s));
  HIPCHK(pl, hipStreamSynchronize(s));
  dev_free(pl, xalen);
  pl->box.rows = pl->rows_d;
  pl->box.np = off;
  pl->box.rows_nz = nonempty;
  return VIE_OK;
}

int create_impl(const vie_problem* p, hipStream_t s, vie_plan* pl) {
  if (p->kind < VIE_LAPLACE || p->kind > VIE_MAXWELL) return fail(pl, VIE_E_ARG, "unknown kind");
  if (!p->coef) return fail(pl, VIE_E_ARG, "coef is NULL");
  if (p->n <= 0 || !(p->h > 0.0) || !std::isfinite(p->h)) return fail(pl, VIE_E_ARG, "n and h must be positive");
  if (p->kind != VIE_LAPLACE && !(p->omega > 0.0 && std::isfinite(p->omega)))
    return fail(pl, VIE_E_ARG, "omega must be positive for Helmholtz and Maxwell");
  if (p->mu && p->kind != VIE_MAXWELL) return fail(pl, VIE_E_ARG, "mu is only used by Maxwell");
  if (p->precision != VIE_PREC_FP64 && p->precision != VIE_PREC_MIXED) return fail(pl, VIE_E_ARG, "bad precision");
  if (p->max_rhs < 1 || p->max_rhs > 4096) return fail(pl, VIE_E_ARG, "max_rhs out of range");
  if (!n_supported(p->n))
    return fail(pl, VIE_E_SIZE, "n = " + std::to_string(p->n) + " has no compiled FFT lengths (2n, 4n)");
  pl->kind = p->kind;
  pl->n = p->n;
  pl->h = p->h;
  for (int a = 0; a < 3; ++a) pl->origin[a] = p->origin[a];
  pl->omega = p->kind == VIE_LAPLACE ? 0.0 : p->omega;
  pl->full = p->mu != nullptr;
  pl->C = pl->full ? 6 : 3;
  pl->P = 2 * p->n;
  pl->M = 4 * p->n;
  pl->R = std::sqrt(3.0) * p->n * p->h;
  pl->sym_set = p->kind == VIE_MAXWELL ? SYM_MAXWELL : SYM_GRAD;
  pl->ne = pl->full ? 9 : 6;
  pl->precision = p->precision;
  pl->max_rhs = p->max_rhs;
  pl->flags = p->flags;
  pl->n3 = long(p->n) * p->n * p->n;
  pl->use_graphs = !(p->flags & VIE_NO_GRAPHS);
  const StreamUse use(pl, s);
  HIPCHK(pl, hipGetDevice(&pl->device));
  if (pl->device < 0 || pl->device >= kMaxDevices) return fail(pl, VIE_E_DEVICE, "device index out of range");
  HIPCHK(pl, hipEventCreateWithFlags(&pl->done_ev, hipEventDisableTiming));
  {
    // the device address of the scratch of vie_apply_noalloc, once per device
    std::lock_guard<std::recursive_mutex> lk(hip_mutex());
    if (!g_scratch_ptr[pl->device]) {
      void* sp = nullptr;
      HIPCHK(pl, hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
      g_scratch_ptr[pl->device] = sp;
    }
  }
  {
    hipDeviceProp_t prop;
    HIPCHK(pl, hipGetDeviceProperties(&prop, pl->device));
    pl->max_lds = std::min<size_t>(prop.sharedMemPerBlock, 65536);
  }
  const size_t tf = sizeof(c128) * 9 * size_t(pl->n3);
  // coefficient upload (device copy) -> contrast
  c128* coef_d = nullptr;
  int rc = dev_alloc(pl, reinterpret_cast<void**>(&coef_d), tf);
  if (rc) return rc;
  const hipMemcpyKind kind = (p->flags & VIE_PTR_HOST) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  HIPCHK(pl, hipMemcpyAsync(coef_d, p->coef, tf, kind, s));
  rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->H64), tf);
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->H32), tf / 2);
  if (rc) return rc;
  const int nblk = int(std::min<long>(4096, (pl->n3 + 255) / 256));
  double* bmax = nullptr;
  int* bbad = nullptr;
  int* bbox = nullptr;
  rc = dev_alloc(pl, reinterpret_cast<void**>(&bmax), sizeof(double) * size_t(nblk));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&bbad), sizeof(int) * size_t(nblk));
  if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&bbox), sizeof(int) * 6 * size_t(nblk));
  if (rc) return rc;
  std::vector<double> hmax(static_cast<size_t>(nblk));
  std::vector<int> hbad(static_cast<size_t>(nblk));
  std::vector<int> hbox(static_cast<size_t>(6 * nblk));
  double worst = 0.0;
  long bad = 0;
  int lo[3] = {p->n, p->n, p->n}, hi[3] = {-1, -1, -1};
  for (int pass = 0; pass < (pl->full ? 2 : 1); ++pass) {
    c128* H64 = pl->H64;
    c64* H32 = pl->H32;
    if (pass == 1) {
      HIPCHK(pl, hipMemcpyAsync(coef_d, p->mu, tf, kind, s));
      rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->Hmu64), tf);
      if (!rc) rc = dev_alloc(pl, reinterpret_cast<void**>(&pl->Hmu32), tf / 2);
      if (rc) return rc;
      H64 = pl->Hmu64;
      H32 = pl->Hmu32;
    }
    HIPCHK(pl, launch_contrast(coef_d, H64, H32, pl->n, bmax, bbad, bbox, nblk, s));
    HIPCHK(pl, hipMemcpyAsync(hmax.data(), bmax, sizeof(double) * size_t(nblk), hipMemcpyDeviceToHost, s));
    HIPCHK(pl, hipMemcpyAsync(hbad.data(), bbad, sizeof(int) * size_t(nblk), hipMemcpyDeviceToHost, s));
    HIPCHK(pl, hipMemcpyAsync(hbox.data(), bbox, sizeof(int) * 6 * size_t(nblk), hipMemcpyDeviceToHost, s));
    HIPCHK(pl, hipStreamSynchronize(s));
    for (int i = 0; i < nblk; ++i) {
      worst = std::max(worst, hmax[size_t(i)]);
      bad += hbad[size_t(i)];
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], hbox[size_t(6 * i + 2 * a)]);
        hi[a] = std::max(hi[a], hbox[size_t(6 * i + 2 * a + 1)]);
      }
    }
  }
  dev_free(pl, coef_d);
  dev_free(pl, bmax);
  dev_free(pl, bbad);
  dev_free(pl, bbox);
  // whole grid and the bounding box of supp(H) (a single point if H vanishes)
  pl->grid = Geom{&pl->sg, p->n, p->n, p->n, 0, 0, 0, 0, nullptr, pl->n3};
  if (hi[0] < 0) {
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = 0;
  }
  pl->box = Geom{&pl->sb, hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1, lo[0], lo[1], lo[2], 1, nullptr, 0};
  pl->box.np = long(pl->box.bx) * pl->box.by * pl->box.bz;
  pl->use_box = !(p->flags & VIE_WHOLE_GRID);
  if (!pl->use_box) {
    pl->box = pl->grid;
    pl->box.sp = &pl->sb;
  } else if (!(p->flags & VIE_DENSE_BOX)) {
    rc = build_rows(pl, s);
    if (rc) return rc;
  }
  pl->hmax = worst;
  if (bad > 0)
    return fail(pl, VIE_E_MEDIUM, std::to_string(bad) + " grid points where a + I is singular or not finite");
  if ((p->flags & VIE_STRICT_MEDIUM) && !(worst < 1.0))
    return fail(pl, VIE_E_MEDIUM, "max ||H(x)||_2 = " + std::to_string(worst) + " >= 1 (contrast not a contraction)");
  // twiddles and kernel tables: the whole grid's, and the box's when shorter
  // (the whole grid's are built at its first use when they differ: a solve
  // without field output never needs them)
  const bool shorter = pl->use_box && !(p->flags & VIE_FULL_LENGTH);
  const int pb = shorter ? box_length(pl) : pl->P;
  const int pz = shorter ? z_length(pl, pb) : pl->P;
  rc = make_spec(pl, pz, pb, pl->sym_set, pl->ne, pl->sb, s);
  if (rc) return rc;
  if (pb == pl->P && pz == pl->P) pl->sg = pl->sb;
  if (p->flags & VIE_GRID_TABLES) {
    rc = ensure_grid_spec(pl, s);
    if (rc) return rc;
  }
  return VIE_OK;
}

}  // namespace

namespace {

// the whole grid with the divergence tables and a multiply mode
vie::Geom div_geom(vie_plan* pl, int mul) {
  vie::Geom g = pl->grid;
  g.sp = &pl->sdiv;
  g.mul = mul;
  g.id = mul == vie::MUL_DIV ? 2 : 3;
  return g;
}

// grow-only device scratch of the post-processing calls
int ensure_post(vie_plan* pl, size_t bytes, hipStream_t s) {
  if (pl->post_bytes >= bytes) return VIE_OK;
  HIPCHK(pl, hipStreamSynchronize(s));  // earlier calls may still read it
  vie::dev_free(pl, pl->post_buf);
  pl->post_buf = nullptr;
  pl->post_bytes = 0;
  const int rc = vie::dev_alloc(pl, &pl->post_buf, bytes);
  if (rc) return rc;
  pl->post_bytes = bytes;
  return VIE_OK;
}

vie::PostGrid post_grid(const vie_plan* pl) {
  const vie::Geom& b = pl->box;
  return vie::PostGrid{pl->n, pl->h, pl->origin[0], pl->origin[1], pl->origin[2], b.x0, b.y0, b.z0, b.bx, b.by, b.bz};
}

}  // namespace

extern "C" {

int vie_plan_create(const vie_problem* p, void* hip_stream, vie_plan** out) {
  if (!out) return VIE_E_ARG;
  *out = nullptr;
  if (!p) return VIE_E_ARG;
  vie_plan* pl = new (std::nothrow) vie_plan();
  if (!pl) return VIE_E_NOMEM;
  const int rc = create_impl(p, static_cast<hipStream_t>(hip_stream), pl);
  if (rc != VIE_OK) {
    vie::last_create_error() = pl->err;
    destroy_plan(pl);
    return rc;
  }
  *out = pl;
  return VIE_OK;
}

int vie_destroy(vie_plan* pl) {
  if (!pl) return VIE_OK;
  destroy_plan(pl);  // synchronises the plan's latest stream first
  return VIE_OK;
}

long vie_release_cached_memory(void) {
  std::lock_guard<std::recursive_mutex> lk(vie::hip_mutex());
  const long bytes = long(vie::cached_bytes());
  vie::release_all_cached();
  return bytes;
}

int vie_apply(vie_plan* pl, const double* x, double* y, int nrhs, unsigned flags, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!x || !y || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_apply: null pointer or nrhs < 1");
  if ((flags & VIE_APPLY_FP64) && (flags & VIE_APPLY_FP32)) return fail(pl, VIE_E_ARG, "FP64 and FP32 both set");
  if (x == y) return fail(pl, VIE_E_ARG, "vie_apply: x and y must not overlap");
  const StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  bool fp64 = pl->precision == VIE_PREC_FP64;
  if (flags & VIE_APPLY_FP64) fp64 = true;
  if (flags & VIE_APPLY_FP32) fp64 = false;
  const int mode = (flags & VIE_APPLY_CONV) ? MODE_CONV : MODE_MATVEC;
  if (flags & VIE_APPLY_C64) {
    if (fp64 || mode != MODE_MATVEC)
      return fail(pl, VIE_E_ARG, "vie_apply: complex64 vectors need the FP32 matvec (no FP64, no CONV)");
    return apply_any(pl, pl->grid, reinterpret_cast<const c64*>(x), reinterpret_cast<c64*>(y), nrhs,
                     static_cast<hipStream_t>(hip_stream));
  }
  const c128* in = reinterpret_cast<const c128*>(x);
  return apply_any(pl, pl->grid, fp64, in, in, nullptr, reinterpret_cast<c128*>(y), nrhs, mode,
                   static_cast<hipStream_t>(hip_stream));
}

int vie_apply_noalloc(vie_plan* pl, const double* x, double* y, int nrhs, unsigned flags, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!x || !y || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_apply_noalloc: null pointer or nrhs < 1");
  if ((flags & VIE_APPLY_FP64) && (flags & VIE_APPLY_FP32)) return fail(pl, VIE_E_ARG, "FP64 and FP32 both set");
  if (x == y) return fail(pl, VIE_E_ARG, "vie_apply_noalloc: x and y must not overlap");
  if (!pl->sg.tab64)
    return fail(pl, VIE_E_STATE,
                "vie_apply_noalloc: the whole grid's kernel tables are not built (create the plan with "
                "VIE_GRID_TABLES, or call vie_apply once first)");
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[pl->device]);
  if (!base) return fail(pl, VIE_E_STATE, "vie_apply_noalloc: no scratch address for this device");
  bool fp64 = pl->precision == VIE_PREC_FP64;
  if (flags & VIE_APPLY_FP64) fp64 = true;
  if (flags & VIE_APPLY_FP32) fp64 = false;
  const int mode = (flags & VIE_APPLY_CONV) ? MODE_CONV : MODE_MATVEC;
  if ((flags & VIE_APPLY_C64) && (fp64 || mode != MODE_MATVEC))
    return fail(pl, VIE_E_ARG, "vie_apply_noalloc: complex64 vectors need the FP32 matvec (no FP64, no CONV)");
  // workspace of one right-hand side (the arrays A and B of the whole grid)
  const size_t N = size_t(pl->n), P = size_t(pl->P), C = size_t(pl->C);
  const size_t Wx = size_t(pitch_x(pl->P)), Wy = size_t(pitch_y(pl->P));
  const size_t el = fp64 ? sizeof(c128) : sizeof(c64);
  const size_t a1 = el * C * N * N * Wx, b1 = el * C * N * P * Wy;
  const size_t total = size_t(VIE_NOALLOC_SCRATCH_MIB) << 20;
  const size_t cap = (total - 256) / (a1 + b1);
  if (cap < 1)
    return fail(pl, VIE_E_SIZE, "vie_apply_noalloc: one right-hand side needs " + std::to_string(a1 + b1) +
                                    " bytes of workspace at n = " + std::to_string(pl->n) + ", more than the " +
                                    std::to_string(total) + "-byte scratch");
  const int ncap = int(std::min<size_t>(cap, 4096));
  const FixedWork fw{base, base + (a1 * size_t(ncap) + 255) / 256 * 256, ncap};
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const StreamUse use(pl, s);
  if (flags & VIE_APPLY_C64) {
    const c64* in = reinterpret_cast<const c64*>(x);
    return apply_typed<float, c64>(pl, pl->grid, in, in, nullptr, reinterpret_cast<c64*>(y), nrhs, MODE_MATVEC, s,
                                   nullptr, -1, &fw);
  }
  const c128* in = reinterpret_cast<const c128*>(x);
  c128* out = reinterpret_cast<c128*>(y);
  return fp64 ? apply_typed<double, c128>(pl, pl->grid, in, in, nullptr, out, nrhs, mode, s, nullptr, -1, &fw)
              : apply_typed<float, c128>(pl, pl->grid, in, in, nullptr, out, nrhs, mode, s, nullptr, -1, &fw);
}

int vie_rhs(vie_plan* pl, const double* inc, double* b, int nrhs, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!inc || !b || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_rhs: null pointer or nrhs < 1");
  const StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  hipError_t e = launch_rhs(pl->H64, pl->Hmu64, reinterpret_cast<const c128*>(inc), reinterpret_cast<c128*>(b),
                            nrhs, pl->C, box_of(pl->grid, pl->n), static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? VIE_OK : hip_fail(pl, e, "vie_rhs");
}

int vie_field(vie_plan* pl, const double* density, const double* inc, double* field, int nrhs, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!density || !inc || !field || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_field: null pointer or nrhs < 1");
  const StreamUse use(pl, static_cast<hipStream_t>(hip_stream));
  return apply_any(pl, pl->grid, true, reinterpret_cast<const c128*>(density),
                   reinterpret_cast<const c128*>(inc), nullptr, reinterpret_cast<c128*>(field), nrhs, MODE_FIELD,
                   static_cast<hipStream_t>(hip_stream));
}

int vie_potential(vie_plan* pl, const double* density, double* phi, int nrhs, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!density || !phi || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_potential: null pointer or nrhs < 1");
  if (pl->kind == VIE_MAXWELL) return fail(pl, VIE_E_STATE, "vie_potential: Laplace and Helmholtz plans only");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const StreamUse use(pl, s);
  int rc = ensure_div_spec(pl, s);
  if (rc) return rc;
  // (div V J, 0, 0) per right-hand side into the scratch, then its first component
  const int chunk = std::max(1, std::min(nrhs, pl->max_rhs));
  const long vec = 3 * pl->n3;
  rc = ensure_post(pl, sizeof(c128) * size_t(vec) * size_t(chunk), s);
  if (rc) return rc;
  c128* tmp = static_cast<c128*>(pl->post_buf);
  const c128* d = reinterpret_cast<const c128*>(density);
  c128* out = reinterpret_cast<c128*>(phi);
  const Geom g = div_geom(pl, MUL_DIV);
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int nb = std::min(chunk, nrhs - r0);
    rc = apply_any(pl, g, true, d + long(r0) * vec, d + long(r0) * vec, nullptr, tmp, nb, MODE_CONV, s);
    if (rc) return rc;
    for (int r = 0; r < nb; ++r) HIPCHK(pl, launch_copy(tmp + long(r) * vec, out + long(r0 + r) * pl->n3, pl->n3, s));
  }
  return VIE_OK;
}

int vie_field_h(vie_plan* pl, const double* density, const double* h_inc, double* h, int nrhs, void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!density || !h || nrhs < 1) return fail(pl, VIE_E_ARG, "vie_field_h: null pointer or nrhs < 1");
  if (pl->kind != VIE_MAXWELL || pl->full)
    return fail(pl, VIE_E_STATE, "vie_field_h: Maxwell plans with mu = I only (vie_field returns E and H otherwise)");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const StreamUse use(pl, s);
  const int rc = ensure_div_spec(pl, s);
  if (rc) return rc;
  const c128* d = reinterpret_cast<const c128*>(density);
  const c128* add = h_inc ? reinterpret_cast<const c128*>(h_inc) : d;
  return apply_any(pl, div_geom(pl, MUL_CURLH), true, d, add, nullptr, reinterpret_cast<c128*>(h), nrhs,
                   h_inc ? MODE_FIELD : MODE_CONV, s);
}

int vie_fields_at(vie_plan* pl, const double* density, int nrhs, const double* points, int npts, double* out,
                  void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!density || !points || !out || nrhs < 1 || npts < 1)
    return fail(pl, VIE_E_ARG, "vie_fields_at: null pointer, nrhs < 1 or npts < 1");
  if (npts > 65535 || nrhs > 65535) return fail(pl, VIE_E_ARG, "vie_fields_at: at most 65535 points and rhs");
  // the sums are accurate away from the density: outside the support box grown by 2h
  const Geom& b = pl->box;
  const double lo[3] = {pl->origin[0] + (b.x0 - 1.5) * pl->h, pl->origin[1] + (b.y0 - 1.5) * pl->h,
                        pl->origin[2] + (b.z0 - 1.5) * pl->h};
  const double hi[3] = {pl->origin[0] + (b.x0 + b.bx + 1.5) * pl->h, pl->origin[1] + (b.y0 + b.by + 1.5) * pl->h,
                        pl->origin[2] + (b.z0 + b.bz + 1.5) * pl->h};
  for (int p = 0; p < npts; ++p) {
    bool inside = true;
    for (int a = 0; a < 3; ++a) inside = inside && points[3 * p + a] > lo[a] && points[3 * p + a] < hi[a];
    if (inside || !std::isfinite(points[3 * p]) || !std::isfinite(points[3 * p + 1]) ||
        !std::isfinite(points[3 * p + 2]))
      return fail(pl, VIE_E_ARG, "vie_fields_at: point " + std::to_string(p) + " is within 2h of the support box");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const StreamUse use(pl, s);
  const bool mx = pl->kind == VIE_MAXWELL;
  const long part = points_partial_doubles(post_grid(pl), mx, npts, nrhs);
  int rc = ensure_post(pl, sizeof(double) * (size_t(3 * npts) + size_t(part)), s);
  if (rc) return rc;
  double* dpts = static_cast<double*>(pl->post_buf);
  HIPCHK(pl, hipMemcpyAsync(dpts, points, sizeof(double) * 3 * size_t(npts), hipMemcpyHostToDevice, s));
  HIPCHK(pl, launch_fields_at(reinterpret_cast<const c128*>(density), pl->C, mx, post_grid(pl), dpts, npts, nrhs,
                              pl->omega, dpts + 3 * npts, reinterpret_cast<c128*>(out), s));
  return VIE_OK;
}

int vie_far_field(vie_plan* pl, const double* density, int nrhs, const double* dirs, int ndirs, double* out,
                  void* hip_stream) {
  if (!pl) return VIE_E_ARG;
  if (!density || !dirs || !out || nrhs < 1 || ndirs < 1)
    return fail(pl, VIE_E_ARG, "vie_far_field: null pointer, nrhs < 1 or ndirs < 1");
  if (ndirs > 65535 || nrhs > 65535) return fail(pl, VIE_E_ARG, "vie_far_field: at most 65535 directions and rhs");
  if (!(pl->omega > 0.0)) return fail(pl, VIE_E_STATE, "vie_far_field: needs omega > 0 (Helmholtz, Maxwell)");
  for (int d = 0; d < ndirs; ++d) {
    const double nrm = std::sqrt(dirs[3 * d] * dirs[3 * d] + dirs[3 * d + 1] * dirs[3 * d + 1] +
                                 dirs[3 * d + 2] * dirs[3 * d + 2]);
    if (!(std::fabs(nrm - 1.0) < 1e-9))
      return fail(pl, VIE_E_ARG, "vie_far_field: direction " + std::to_string(d) + " is not a unit vector");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const StreamUse use(pl, s);
  const bool mx = pl->kind == VIE_MAXWELL;
  const long part = far_partial_doubles(post_grid(pl), pl->C, ndirs, nrhs);
  int rc = ensure_post(pl, sizeof(double) * (size_t(3 * ndirs) + size_t(part)), s);
  if (rc) return rc;
  double* ddirs = static_cast<double*>(pl->post_buf);
  HIPCHK(pl, hipMemcpyAsync(ddirs, dirs, sizeof(double) * 3 * size_t(ndirs), hipMemcpyHostToDevice, s));
  HIPCHK(pl, launch_far_field(reinterpret_cast<const c128*>(density), pl->C, mx, post_grid(pl), ddirs, ndirs, nrhs,
                              pl->omega, ddirs + 3 * ndirs, reinterpret_cast<c128*>(out), s));
  return VIE_OK;
}

int vie_plan_info(const vie_plan* pl, double* out, int nout) {
  if (!pl || !out) return VIE_E_ARG;
  const double v[20] = {double(pl->n),         double(pl->C),      double(pl->P),      double(pl->M),
                        pl->hmax,              double(pl->ne),     double(pl->dev_bytes),
                        double(pl->graph_launches), double(pl->box.x0), double(pl->box.y0), double(pl->box.z0),
                        double(pl->box.bx),    double(pl->box.by), double(pl->box.bz), double(pl->box.np),
                        double(pl->sb.Pxy),    double(pl->ws_cap[0]), double(pl->ws_cap[1]), double(pl->kr_cap),
                        double(pl->sb.Pz)};
  for (int i = 0; i < nout && i < 20; ++i) out[i] = v[i];
  return VIE_OK;
}

int vie_copy_tables(const vie_plan* cpl, double* host, long host_bytes, long* needed, int* nxp, int* ne) {
  if (!cpl) return VIE_E_ARG;
  // the tables of the whole grid are built at their first use
  vie_plan* pl = const_cast<vie_plan*>(cpl);
  const int rc = ensure_grid_spec(pl, pl->last_stream);
  if (rc) return rc;
  const long bytes = long(sizeof(c128)) * pl->sg.tab_elems;
  if (needed) *needed = bytes;
  if (nxp) *nxp = pl->sg.nxp;
  if (ne) *ne = pl->ne;
  if (!host) return VIE_OK;
  if (host_bytes < bytes) return VIE_E_ARG;
  hipError_t e = hipMemcpy(host, pl->sg.tab64, size_t(bytes), hipMemcpyDeviceToHost);
  return e == hipSuccess ? VIE_OK : VIE_E_DEVICE;
}

int vie_copy_contrast(const vie_plan* pl, double* host, long host_bytes) {
  if (!pl || !host) return VIE_E_ARG;
  const long one = long(sizeof(c128)) * 9 * pl->n3;
  const long bytes = pl->full ? 2 * one : one;
  if (host_bytes < bytes) return VIE_E_ARG;
  hipError_t e = hipMemcpy(host, pl->H64, size_t(one), hipMemcpyDeviceToHost);
  if (e == hipSuccess && pl->full) e = hipMemcpy(reinterpret_cast<char*>(host) + one, pl->Hmu64, size_t(one),
                                                 hipMemcpyDeviceToHost);
  return e == hipSuccess ? VIE_OK : VIE_E_DEVICE;
}

const char* vie_status_string(int status) {
  switch (status) {
    case VIE_OK: return "VIE_OK";
    case VIE_E_ARG: return "VIE_E_ARG: invalid argument";
    case VIE_E_SIZE: return "VIE_E_SIZE: unsupported grid size";
    case VIE_E_MEDIUM: return "VIE_E_MEDIUM: invalid medium";
    case VIE_E_NOMEM: return "VIE_E_NOMEM: device memory exhausted";
    case VIE_E_DEVICE: return "VIE_E_DEVICE: HIP error";
    case VIE_E_STATE: return "VIE_E_STATE: call not valid for this plan";
    case VIE_W_NOCONV: return "VIE_W_NOCONV: not converged";
    default: return "unknown status";
  }
}

const char* vie_last_error(const vie_plan* pl) { return pl ? pl->err.c_str() : vie::last_create_error().c_str(); }

int vie_supported_n(int n) { return n_supported(n) ? 1 : 0; }

long vie_footprint_bytes(int kind, int n, int full, int nrhs_batch, int restart) {
  if (n <= 0 || nrhs_batch < 1 || restart < 1) return -1;
  const double n3 = double(n) * n * n, P = 2.0 * n, M = 4.0 * n;
  const double C = full ? 6 : 3, ne = full ? 9 : 6;
  const double nxp = double(((n + 1 + 15) / 16) * 16);
  const double Wx = double(pitch_x(2L * n)), Wy = double(pitch_y(2L * n));  // row pitches of the workspaces
  (void)kind;
  double b = 0;
  b += (full ? 2 : 1) * 9 * n3 * (16 + 8);                       // H in FP64 and FP32
  b += 2 * double(n + 1) * (n + 1) * ne * nxp * (16 + 8);        // octant tables (grid and box lengths)
  const double precompute = (M * M * P + M * P * P + ne * P * P * P) * 16 + 9 * n3 * 16;
  const double nb = nrhs_batch;
  const double ws = nb * C * (double(n) * n * Wx + double(n) * P * Wy);  // apply workspace elements
  b += ws * (8 + 16);                                             // FP32 and FP64 workspaces
  const double L = C * n3;
  b += (double(restart) + 1 + 4) * nb * L * 16;                   // Krylov basis + x, b, r, w
  return long(std::max(b, precompute + b - ws * 24 - (double(restart) + 5) * nb * L * 16));
}

int vie_profile(vie_plan* pl, int enable) {
  if (!pl) return VIE_E_ARG;
  if (pl->prof_on) vie::prof_collect(pl);
  pl->prof_on = enable != 0;
  for (int i = 0; i < 16; ++i) {
    pl->prof_ms[i] = 0;
    pl->prof_cnt[i] = 0;
    pl->prof_bytes[i] = 0;
    pl->prof_flops[i] = 0;
  }
  return VIE_OK;
}

int vie_profile_read(vie_plan* pl, double* ms, long* counts, double* bytes, double* flops, int nfam) {
  if (!pl || !ms || !counts || !bytes) return VIE_E_ARG;
  vie::prof_collect(pl);
  for (int i = 0; i < nfam && i < vie::FAM_COUNT; ++i) {
    ms[i] = pl->prof_ms[i];
    counts[i] = pl->prof_cnt[i];
    bytes[i] = pl->prof_bytes[i];
    if (flops) flops[i] = pl->prof_flops[i];
  }
  return vie::FAM_COUNT;
}

const char* vie_profile_family(int fam) {
  static const char* names[] = {"fft_x_fwd_fp32", "fft_y_fwd_fp32", "fft_z_mul_fp32", "fft_y_inv_fp32",
                                "fft_x_inv_combine_fp32", "fft_x_fwd_fp64", "fft_y_fwd_fp64", "fft_z_mul_fp64",
                                "fft_y_inv_fp64", "fft_x_inv_combine_fp64", "krylov_dots", "krylov_reduce",
                                "krylov_combine"};
  return (fam >= 0 && fam < vie::FAM_COUNT) ? names[fam] : "";
}

}  // extern "C"
