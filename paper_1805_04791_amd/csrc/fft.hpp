// Pencil FFT building blocks for gfx950.
//
// A length-P transform (P = P1 * P2) of one pencil is split into two
// register-resident DFTs with one LDS exchange in between:
//
//   forward  X[k1 + P1 k2] = sum_n2 W_P2^{n2 k2} . W_P^{n2 k1} . sum_n1 x[P2 n1 + n2] W_P1^{n1 k1}
//            step A: thread (col, n2) loads P1 inputs, DFT_P1, twiddle, -> LDS
//            step B: thread (col, k1) reads P2 values from LDS, DFT_P2 -> X[k1 + P1 k2]
//   inverse  x[m1 + P2 m2] = sum_k1 W_P1^{-m2 k1} . W_P^{-m1 k1} . sum_k2 X[k1 + P1 k2] W_P2^{-m1 k2}
//            step C: thread (col, k1) holds X[k1 + P1 k2] (all k2), IDFT_P2, twiddle, -> LDS
//            step D: thread (col, m1) reads P1 values, IDFT_P1 -> x[m1 + P2 m2]
//
// The forward result of step B is laid out exactly as step C expects, so a
// fused forward-multiply-inverse pencil needs no exchange between the halves.
// Zero-padded inputs (n >= nin) are never read and cropped outputs
// (n >= nout) never written.
//
// Two thread layouts: "strided" pencils (y and z axes) put adjacent columns
// on adjacent lanes so every global access is a contiguous run of T complex
// values; "contiguous" pencils (x axis) put adjacent pencil indices on
// adjacent lanes.
#pragma once

#include "cx.hpp"
#include "dft.hpp"

namespace vie {

template <typename T>
struct scalar_of;
template <typename R>
struct scalar_of<cx<R>> {
  using type = R;
};

// The fused z / x-inverse passes in FP32 issue the loads of all components
// before the first transform (more bytes in flight for the same occupancy);
// the FP64 ones load one component at a time to stay within their registers.
template <typename R>
constexpr bool kUpfront = sizeof(R) == 4;

// Row pitch of an apply's intermediate arrays: A, the x-transformed rows
// [..][by][pitch_x(P)], and B, the y-transformed planes [..][P][pitch_y(P)].
// The rows of B start on 128-byte lines (P rounded up to 16 elements): a
// z-pass tile of 16 columns of a row is then one line (complex64) instead of
// straddling two, which the blocks of neighbouring tiles, on other XCDs,
// would each fetch whole.
constexpr long kRowAlign = 16;
__host__ __device__ constexpr long pitch_x(long P) { return P; }
__host__ __device__ constexpr long pitch_y(long P) { return (P + kRowAlign - 1) / kRowAlign * kRowAlign; }

// largest block of each kernel family (the tile choice keeps T*J within it)
constexpr int kPassMaxThreads = 512;
constexpr int kFusedMaxThreads = 512;
// The FP64 fused kernels hold three (or six) complex128 spectra per thread:
// at most one wave per SIMD per block, so that a wave may use the whole
// register file (VGPRs and AGPRs) instead of spilling to memory.
template <typename R, int C>
constexpr int fused_max_threads() {
  return sizeof(R) == 8 ? 256 : kFusedMaxThreads;
}

struct Geo {
  int T;          // columns (strided) or rows (contiguous) per block
  int ntiles;     // column tiles per pencil group
  long ncols;     // columns per group
  int nin;        // valid inputs along the transform axis
  int nout;       // outputs written along the transform axis
  // optional: pencil (g, c) belongs to right-hand side (g * ncols + c) /
  // per_rhs, and is skipped (nothing loaded or stored) when act[rhs] == 0
  const int* act = nullptr;
  long per_rhs = 1;
};

// Sources of a pass: column(g, c) binds pencil (g, c) once per thread; the
// bound column's load<R>(n) returns element n.
// element n of pencil (g, c) lives at p + g*gs + c*cs + n*as
template <typename T>
struct MemLoad {
  const T* p;
  long gs, cs, as;
  struct Col {
    const T* q;
    long as;
    template <typename R>
    __device__ __forceinline__ cx<R> load(int n) const {
      return cvt<R>(q[long(n) * as]);
    }
  };
  __device__ __forceinline__ Col column(long g, long c) const { return {p + g * gs + c * cs, as}; }
};

// Rows of a support-compressed vector: row c of the x pass is row r = c % nr
// (a (z, y) row of the box) of component v = c / nr; the row holds only its
// samples x in [xa, xa + len), stored at p + v * np + off + (x - xa).
// rows[3 r .. 3 r + 2] = (xa, len, off).
// (Row and component indices fit 32 bits: nrhs * C * rows < 2^31.)
template <typename T>
struct RowLoad {
  const T* p;
  const int* rows;
  long nr, np;
  struct Col {
    const T* q;  // the row's first kept sample (x = xa)
    int xa, len;
    template <typename R>
    __device__ __forceinline__ cx<R> load(int n) const {
      const int i = n - xa;
      return (i >= 0 && i < len) ? cvt<R>(q[i]) : czero<R>();
    }
  };
  __device__ __forceinline__ Col column(long, long c) const {
    const unsigned cu = unsigned(c), nru = unsigned(nr);
    const unsigned r = cu % nru, v = cu / nru;
    return {p + long(v) * np + rows[3 * r + 2], rows[3 * r], rows[3 * r + 1]};
  }
};

template <typename T>
struct MemStore {
  T* p;
  long gs, cs, as;
  double scale;       // multiplies every stored value
  int zero_first;     // store 0 at n == 0
  template <typename R>
  __device__ __forceinline__ void store(long g, long c, int n, cx<R> v) const {
    using S = typename scalar_of<T>::type;
    if (zero_first && n == 0) v = czero<R>();
    v = R(scale) * v;
    p[g * gs + c * cs + long(n) * as] = cvt<S>(v);
  }
};

template <bool CONTIG>
struct Layout;

// strided: (a * (Bd + 1) + b) * T + col.  The extra slot per a-row shifts the
// pencil groups a, a+1 of one half-wave by T elements so that their
// contiguous T-column runs fall into different LDS banks.
template <>
struct Layout<false> {
  __device__ __forceinline__ static int idx(int col, int a, int b, int Bd, int Ad, int T) {
    (void)Ad;
    return (a * (Bd + 1) + b) * T + col;
  }
  __device__ __forceinline__ static void lane(int tid, int T, int J, int& col, int& j) {
    (void)J;
    col = tid % T;
    j = tid / T;
  }
};

// contiguous: col * Ad * (Bd + 1) + a * (Bd + 1) + b
template <>
struct Layout<true> {
  __device__ __forceinline__ static int idx(int col, int a, int b, int Bd, int Ad, int T) {
    (void)T;
    return col * (Ad * (Bd + 1)) + a * (Bd + 1) + b;
  }
  __device__ __forceinline__ static void lane(int tid, int T, int J, int& col, int& j) {
    (void)T;
    col = tid / J;
    j = tid % J;
  }
};

template <int P1, int P2>
__host__ __device__ constexpr int lds_elems_per_col(bool contig) {
  (void)contig;
  return P2 * (P1 + 1) > P1 * (P2 + 1) ? P2 * (P1 + 1) : P1 * (P2 + 1);
}

// Twiddles W_P^{j i} of thread j, read from the LDS table when needed.  Step A
// multiplies by W_P^{n2 k1} (n2 = j, k1 < P1) and step C by W_P^{-m1 k1}
// (k1 = j, m1 < P2 <= P1); j i < P in both.
template <typename R, int P1, int P2>
struct ThreadTw {
  const cx<R>* t;
  int j;
  __device__ __forceinline__ void init(const cx<R>* tw, int jj) {
    t = tw;
    j = jj;
  }
  template <int I>
  __device__ __forceinline__ cx<R> get() const {
    return t[j * I];
  }
};

// Inputs of step A for thread j (< P2): u[n1] = x[P2 n1 + j], zero for n >= nin.
template <typename R, int P1, int P2, typename LoadF>
__device__ __forceinline__ void fft_load(LoadF&& load, int nin, int j, bool valid, cx<R> (&u)[P1]) {
  static_for<0, P1>([&](auto n1) {
    const int n = P2 * n1 + j;
    u[n1] = (valid && j < P2 && n < nin) ? load(n) : czero<R>();
  });
}

// Step A + B from preloaded inputs u (destroyed).  On return the threads with
// j < P1 hold X[j + P1 k2] in X[k2].  Two block barriers: every thread of the
// block must call it.
template <typename R, int P1, int P2, bool CONTIG, typename TW>
__device__ __forceinline__ void fft_fwd_core(cx<R> (&u)[P1], const TW& twr, cx<R>* lds, int col, int j, int T,
                                             cx<R> (&X)[P2]) {
  if (j < P2) {
    DFT<P1, false>::run(u);
    static_for<1, P1>([&](auto k1) { u[k1] = u[k1] * twr.template get<decltype(k1)::value>(); });
    static_for<0, P1>([&](auto k1) { lds[Layout<CONTIG>::idx(col, j, k1, P1, P2, T)] = u[k1]; });
  }
  __syncthreads();
  if (j < P1) {
    static_for<0, P2>([&](auto n2) { X[n2] = lds[Layout<CONTIG>::idx(col, n2, j, P1, P2, T)]; });
    DFT<P2, false>::run(X);
  }
  __syncthreads();
}

// Step A + B with the loads done here.
template <typename R, int P1, int P2, bool CONTIG, typename LoadF, typename TW>
__device__ __forceinline__ void fft_fwd_AB(LoadF&& load, int nin, cx<R>* lds, const TW& twr, int col, int j,
                                           int T, bool valid, cx<R> (&X)[P2]) {
  cx<R> u[P1];
  fft_load<R, P1, P2>(load, nin, j, valid, u);
  fft_fwd_core<R, P1, P2, CONTIG>(u, twr, lds, col, j, T, X);
}

// Step C + D.  Threads with j < P1 supply X[j + P1 k2] in X[k2] (destroyed).
// store(m2, n, v) is called for n = j + P2 m2 < nout only (m2 is a compile-time
// index), and only for m2 < M2MAX: the outputs of the last step beyond it are
// never formed (M2MAX = P1 / 2 covers nout <= P / 2).
template <typename R, int P1, int P2, bool CONTIG, int M2MAX = P1, typename StoreF, typename TW>
__device__ __forceinline__ void fft_inv_CD(cx<R> (&X)[P2], StoreF&& store, int nout, cx<R>* lds, const TW& twr,
                                           int col, int j, int T, bool valid) {
  if (j < P1) {
    DFT<P2, true>::run(X);
    static_for<1, P2>([&](auto m1) { X[m1] = cmulc(twr.template get<decltype(m1)::value>(), X[m1]); });
    static_for<0, P2>([&](auto m1) { lds[Layout<CONTIG>::idx(col, j, m1, P2, P1, T)] = X[m1]; });
  }
  __syncthreads();
  if (j < P2) {
    cx<R> u[P1];
    static_for<0, P1>([&](auto k1) { u[k1] = lds[Layout<CONTIG>::idx(col, k1, j, P2, P1, T)]; });
    DFT<P1, true>::run(u);
    static_for<0, M2MAX>([&](auto m2) {
      const int n = j + P2 * m2;
      if (valid && n < nout) store(m2, n, u[m2]);
    });
  }
  __syncthreads();
}

// stage the length-P twiddle table W_P^j into LDS
template <typename R, int P>
__device__ __forceinline__ void load_twiddles(cx<R>* tw, const cx<R>* __restrict__ twg) {
  for (int i = threadIdx.x; i < P; i += blockDim.x) tw[i] = twg[i];
}

// Minimum waves per SIMD the register allocation of k_pass must allow.  The
// FP32 strided inverse of length 216 needs 81 registers when left alone (5
// waves); held to 80 it runs 6 without spilling and is faster.  Longer
// lengths would spill, shorter ones already fit.
template <typename R, int P1, int P2, bool CONTIG, bool INV>
constexpr int pass_min_waves() {
  return (!CONTIG && INV && sizeof(R) == 4 && P1 * P2 <= 216) ? 6 : 1;
}

// One pass of a batched pencil FFT (forward or inverse, pruned).
template <typename R, int P1, int P2, bool CONTIG, bool INV, typename Src, typename Dst>
__global__ void __launch_bounds__(kPassMaxThreads)
__attribute__((amdgpu_waves_per_eu(pass_min_waves<R, P1, P2, CONTIG, INV>()))) k_pass(Src src, Dst dst, Geo geo, const cx<R>* __restrict__ twg) {
  constexpr int P = P1 * P2;
  constexpr int J = P1 > P2 ? P1 : P2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const long tile = long(blockIdx.x) % geo.ntiles;
  const long g = long(blockIdx.x) / geo.ntiles;
  if (geo.act) {
    // the whole block belongs to one inactive right-hand side
    const long first = g * geo.ncols + tile * geo.T;
    const long last = g * geo.ncols + (tile * geo.T + geo.T < geo.ncols ? tile * geo.T + geo.T : geo.ncols) - 1;
    if (first / geo.per_rhs == last / geo.per_rhs && !geo.act[first / geo.per_rhs]) return;
  }
  cx<R>* tw = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* lds = tw + P;
  load_twiddles<R, P>(tw, twg);
  int col, j;
  Layout<CONTIG>::lane(threadIdx.x, geo.T, J, col, j);
  const long c = tile * geo.T + col;
  const bool valid = c < geo.ncols && (!geo.act || geo.act[(g * geo.ncols + c) / geo.per_rhs]);
  cx<R> u[P1];
  const auto col_src = src.column(g, valid ? c : 0);
  if constexpr (!INV) fft_load<R, P1, P2>([&](int n) { return col_src.template load<R>(n); }, geo.nin, j, valid, u);
  __syncthreads();
  ThreadTw<R, P1, P2> twr;
  twr.init(tw, j);
  cx<R> X[P2];
  if constexpr (!INV) {
    fft_fwd_core<R, P1, P2, CONTIG>(u, twr, lds, col, j, geo.T, X);
    if (j < P1 && valid) {
      static_for<0, P2>([&](auto k2) {
        const int n = j + P1 * k2;
        if (n < geo.nout) dst.template store<R>(g, c, n, X[k2]);
      });
    }
  } else {
    if (j < P1) {
      static_for<0, P2>([&](auto k2) {
        const int n = j + P1 * k2;
        X[k2] = (valid && n < geo.nin) ? col_src.template load<R>(n) : czero<R>();
      });
    }
    // every inverse pass keeps at most the first half of its outputs (the
    // launchers check nout <= P / 2)
    fft_inv_CD<R, P1, P2, CONTIG, P1 / 2>(
        X, [&](auto, int n, cx<R> v) { dst.template store<R>(g, c, n, v); }, geo.nout, lds, twr, col, j, geo.T, valid);
  }
}

template <int P1, int P2>
struct Split {
  static constexpr int p1 = P1, p2 = P2, P = P1 * P2, J = (P1 > P2 ? P1 : P2);
};

}  // namespace vie
