// Plan object shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cx.hpp"
#include "pointwise.hpp"
#include "vie.h"

namespace vie {

struct SolveSession;  // an open batch of solver slots (solve.cpp)

// Extent of the data an apply works on: the whole grid, or the bounding box
// of the support of H (the Krylov vectors vanish outside it exactly).
// Spectral data of one periodic grid: transform length Pz along z and Pxy
// along x and y (Pxy <= Pz); the kernel-transform octant tables
// [qz][qy][entry][qx], qz, qy in [0, Pz/2], qx < nxp = (Pz/2 + 1) rounded up to
// 16 (entries with qy or qx > Pxy/2 are zero); twiddles of both lengths.
struct Spec {
  int set = 0, ne = 0;  // symbol set (SYM_*) and its table entries
  int Pz = 0, Pxy = 0, nxp = 0;
  long tab_elems = 0;
  c128* tab64 = nullptr;
  c64* tab32 = nullptr;
  c128* tw64 = nullptr;   // length Pxy
  c64* tw32 = nullptr;
  c128* twz64 = nullptr;  // length Pz
  c64* twz32 = nullptr;
};

struct Geom {
  const Spec* sp = nullptr;  // transform length and tables used on this geometry
  int bx = 0, by = 0, bz = 0;
  int x0 = 0, y0 = 0, z0 = 0;
  int id = 0;                // 0 whole grid, 1 solver geometry
  const int* rows = nullptr; // support rows (xa, len, off) per (z, y) row; null: dense box
  long np = 0;               // points per component of the vectors
  int mul = -1;              // spectral multiply (MUL_*); -1: the plan's operator
  long rows_nz = 0;          // with rows: (z, y) rows holding at least one support point
};
inline Box box_of(const Geom& g, int n) { return Box{n, g.bx, g.by, g.bz, g.x0, g.y0, g.z0, g.rows, g.np}; }

// tile choices of the five apply passes
struct Tune {
  int tx_fwd = 0, ty_fwd = 0, tz = 0, ty_inv = 0, tx_inv = 0;
  int vx_fwd = 0, vy_fwd = 0, vz = 0, vy_inv = 0, vx_inv = 0;  // split variant of each pass
  int zorder = 0;  // block order of the z pass: 0 paired ky slices (plain if not pairable), 1 mirror groups
  bool tuned = false;
};

struct DeviceArena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
};

}  // namespace vie

struct vie_plan {
  int kind = 0, n = 0, C = 3, P = 0, M = 0, ne = 6, sym_set = 0, precision = 0, max_rhs = 1;
  unsigned flags = 0;
  double h = 0, omega = 0, R = 0, hmax = 0;
  long n3 = 0;
  bool full = false;  // mu present (6 unknowns per point)
  vie::Geom grid, box;  // whole grid; the solver's: bounding box of supp(H) (and H_mu), support rows
  bool use_box = true;
  int* rows_d = nullptr;  // device (xa, len, off) per (z, y) row of the box
  hipStream_t last_stream = nullptr;  // stream of the latest call
  // recorded on last_stream after each call's work (vie_destroy waits for it,
  // not for later work of other callers on that stream); not valid when the
  // call's stream was being captured
  hipEvent_t done_ev = nullptr;
  bool done_valid = false;
  int device = 0;
  size_t max_lds = 65536;

  vie::c128 *H64 = nullptr, *Hmu64 = nullptr;
  vie::c64 *H32 = nullptr, *Hmu32 = nullptr;
  vie::Spec sg;  // P = 2n: the whole grid (vie_apply, vie_field)
  vie::Spec sb;  // the solver's box: Pz = 2n, Pxy the shortest compiled length >= 2 max(bx, by), <= 2n
  vie::Spec sdiv;  // the divergence / curl symbol i s G^ on the 2n grid (built at first use)
  double origin[3] = {0, 0, 0};
  void* post_buf = nullptr;  // device scratch of the point and far-field sums
  size_t post_bytes = 0;

  // apply workspaces [0] FP32, [1] FP64; capacity in right-hand sides
  void* wsA[2] = {nullptr, nullptr};
  void* wsB[2] = {nullptr, nullptr};
  int ws_cap[2] = {0, 0};
  std::map<int, vie::Tune> tune[2];  // keyed by batch size bucket

  // Krylov workspace (FP64)
  vie::c128* V = nullptr;  // [(m+1)][cap][L]
  int kr_cap = 0, kr_m = 0;
  vie::c128 *xw = nullptr, *bw = nullptr, *rw = nullptr, *ww = nullptr;
  vie::c128* xbest = nullptr;  // per slot: the iterate with the smallest true residual so far
  vie::c128* partials = nullptr;  // [cap][nblk][m+2]
  vie::c128* red = nullptr;       // [cap][m+2]
  vie::c128* red_host = nullptr;  // pinned
  // staging of the combine arguments, two slots used alternately (pinned on
  // the host, mirrored on the device); a slot holds scale [cap] doubles,
  // count [cap] ints and coefficients [cap][m + 2] complex, in that order, so
  // that one copy of its used prefix carries them all
  unsigned char* stage_host = nullptr;
  unsigned char* stage_dev = nullptr;
  size_t stage_bytes = 0, stage_off_count = 0, stage_off_coef = 0;
  int* actd = nullptr;            // [cap] flags of the right-hand sides still iterating (0 = skip)
  vie::SolveSession* session = nullptr;  // the open batch of slots (vie_solve, vie_batch_*)
  std::vector<int> act_last;      // the flags last written to actd

  size_t dev_bytes = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  std::vector<std::pair<void*, size_t>> host_allocs;  // pinned host blocks (host_alloc)
  std::string err;

  // captured applies: key (fp64, mode, nb, in, addv, bvec, out) -> graph
  struct GraphKey {
    int fp64, mode, nb, geom;
    const void *in, *addv, *bvec, *out, *act;
    int out64;  // 1: the output is stored as complex64
    bool operator<(const GraphKey& o) const {
      return std::tie(fp64, mode, nb, geom, in, addv, bvec, out, act, out64) <
             std::tie(o.fp64, o.mode, o.nb, o.geom, o.in, o.addv, o.bvec, o.out, o.act, o.out64);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t gstream = nullptr;
  bool use_graphs = true;
  long graph_launches = 0;

  // pinned staging slots of the basis coefficients (two, used alternately)
  long sync_count = 0;
  long stage_epoch[2] = {-1, -1};
  int stage_next = 0;

  // kernel timing with HIP events (vie_profile)
  struct ProfRec {
    int fam;
    hipEvent_t a, b;
    double bytes, flops;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[16] = {0};
  long prof_cnt[16] = {0};
  double prof_bytes[16] = {0};
  double prof_flops[16] = {0};
};

namespace vie {

#define HIPCHK(pl, expr)                                       \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return vie::hip_fail(pl, e_, #expr); \
  } while (0)

std::string& last_create_error();

// The stream of an entry point's work: sets the plan's last stream and, on
// leaving the call, records done_ev after the work the call enqueued.
struct StreamUse {
  vie_plan* pl;
  hipStream_t s;
  StreamUse(vie_plan* p, hipStream_t st) : pl(p), s(st) { pl->last_stream = st; }
  ~StreamUse();
  StreamUse(const StreamUse&) = delete;
  StreamUse& operator=(const StreamUse&) = delete;
};

// allocation helpers (record bytes on the plan)
int dev_alloc(vie_plan* pl, void** p, size_t bytes);
void dev_free(vie_plan* pl, void* p);
// the library's cache of released device blocks (callers hold hip_mutex())
void quiesce(vie_plan* pl);
void give_block(void* p, size_t bytes, int device);
void release_cached(int device);
void release_all_cached();
size_t cached_bytes();
// pinned host memory through a cache of the same kind (hipHostFree, too,
// waits for the device)
int host_alloc(vie_plan* pl, void** p, size_t bytes);
void host_free(vie_plan* pl, void* p);
void give_host_block(void* p, size_t bytes);
int fail(vie_plan* pl, int code, const std::string& msg);
int hip_fail(vie_plan* pl, hipError_t e, const char* what);

// apply: out = f(in) for nrhs vectors; mode MODE_*; addv: J for the
// combine (MODE_MATVEC/RESIDUAL: the input itself, MODE_FIELD: the incident
// field); bvec: b of MODE_RESIDUAL.
// Serialises the library's stream captures with its allocations, frees and
// synchronisations, which HIP forbids while any stream of the process is
// being captured.
std::recursive_mutex& hip_mutex();

// Vectors are laid out on geometry g ([rhs][C][bz][by][bx]).  act (device,
// optional): a flag per right-hand side of the call, 0 = skip it (nothing of
// it is read or written); nact = the count of non-zero flags (byte counts).
int apply_any(vie_plan* pl, const Geom& g, bool fp64, const c128* in, const c128* addv, const c128* bvec,
              c128* out, int nrhs, int mode, hipStream_t s, const int* act = nullptr, int nact = -1);
// the same through a captured hipGraph replayed on the plan's stream (solver
// calls with stable pointers); falls back to apply_any when capture is off
int apply_graph(vie_plan* pl, const Geom& g, bool fp64, const c128* in, const c128* addv, const c128* bvec,
                c128* out, int nrhs, int mode, hipStream_t s, const int* act = nullptr, int nact = -1);
// builds the whole grid's tables, or the divergence tables, at their first use
int ensure_grid_spec(vie_plan* pl, hipStream_t s);
int ensure_div_spec(vie_plan* pl, hipStream_t s);
// FP32 matvec y = A x with x, y stored as complex64
int apply_any(vie_plan* pl, const Geom& g, const c64* in, c64* out, int nrhs, hipStream_t s);
// FP32 matvec with x stored as complex128 and y as complex64 (the values are
// FP32 results either way), eager or from a captured graph
int apply_any(vie_plan* pl, const Geom& g, const c128* in, c64* out, int nrhs, hipStream_t s, const int* act,
              int nact);
int apply_graph(vie_plan* pl, const Geom& g, const c128* in, c64* out, int nrhs, hipStream_t s,
                const int* act = nullptr, int nact = -1);
void clear_graphs(vie_plan* pl);

// kernel families timed by vie_profile
enum {
  FAM_XFWD32 = 0, FAM_YFWD32, FAM_Z32, FAM_YINV32, FAM_XINV32,
  FAM_XFWD64, FAM_YFWD64, FAM_Z64, FAM_YINV64, FAM_XINV64,
  FAM_DOTS, FAM_REDUCE, FAM_COMBINE, FAM_COUNT
};
// record an event pair around the launches between prof_begin and prof_end
int prof_begin(vie_plan* pl, hipStream_t s);
// bytes: algorithmic HBM bytes of the launch (each operand read or written once)
void prof_end(vie_plan* pl, int fam, int token, hipStream_t s, double bytes, double flops = 0.0);

int solve_batch(vie_plan* pl, const c128* inc, c128* density, c128* field, int nrhs, const vie_solve_opts& o,
                vie_solve_stats* stats, hipStream_t s);
// frees the plan's open batch, if any
void close_session(vie_plan* pl);

}  // namespace vie
