// Kernels specific to the operator apply: the fused z pass (forward FFT,
// spectral kernel multiply, inverse FFT) and the last inverse x pass fused
// with the pointwise contrast combine.
//
// Spectral multiply (symbols of Sections 2-4, eqs. Todef, Vw, represent_Maxwell):
//   MUL_SYM3: U^ = K^ J^ with K^ complex symmetric 3x3 (grad div V or
//             (grad div + omega^2) V), 6 tables;
//   MUL_MAX6: [Z_J; Z_M] = [[D, c x], [-c x, D]] [J^; M^] with D the
//             (grad div + omega^2) V symbol and c = i omega (i s G^) the curl
//             symbol scaled by i omega, 9 tables; so that Z_J = U_J + i omega W_M and
//             Z_M = U_M - i omega W_J (eqs. intM and represent_Maxwell).
//   MUL_DIV:  phi^ = d . J^ into component 0 (components 1, 2 zero), d = i s G^,
//             3 tables: the potential div V J (Section 3's summary).
//   MUL_CURLH: H^ = -i omega d x J^, 3 tables: the H field of Maxwell with mu = I
//             (eq. represent_Maxwell_reduced).
// The tables hold one octant q in [0, n]^3 of the 2n-periodic transform; the
// other octants follow from the parity of each entry (odd in s_a for the
// off-diagonal entries ab and for curl component a).  Layout
// [qz][qy][qx < nxp][entry]: the entries of one frequency point are adjacent,
// so a thread reads them with a few wide loads (three 16-byte loads for the
// six FP32 entries of MUL_SYM3).
//
// Pointwise combine (eqs. intLap, contractionK with the derived sign,
// contraction_Maxwell_reduced, intM):
//   MODE_MATVEC:   y = J - H (J + 2 U)            (per 3-component half)
//   MODE_FIELD:    y = g + U                       (total field)
//   MODE_CONV:     y = U                           (raw convolution)
//   MODE_RESIDUAL: y = b - (J - H (J + 2 U))
#pragma once

#include "fft.hpp"

namespace vie {

enum { MUL_SYM3 = 0, MUL_MAX6 = 1, MUL_DIV = 2, MUL_CURLH = 3 };
// table entries each multiply reads
__host__ __device__ constexpr int mul_entries(int mul) { return mul == MUL_SYM3 ? 6 : (mul == MUL_MAX6 ? 9 : 3); }
enum { MODE_MATVEC = 0, MODE_FIELD = 1, MODE_CONV = 2, MODE_RESIDUAL = 3 };

struct ZArgs {
  int T;            // kx columns per block
  int ntiles;       // pxy / T
  int n;            // P / 2: the tables' octant is qz in [0, n], qy, qx in [0, n] (only <= pxy / 2 used)
  int P;            // z transform length
  int nxp;          // padded octant row length (n + 1 rounded up to 16)
  int ne;           // table entries (6 or 9)
  long comp_stride; // nz * pxy * pitch
  long rhs_stride;  // C * comp_stride
  int nb;           // right-hand sides in the launch
  int nz;           // z extent of the data (n, or the support box): inputs z < nz, outputs z < nz
  int pxy;          // x and y transform length (<= P): columns (ky, kx) in [0, pxy)^2
  double omega;     // MUL_CURLH: the factor -i omega
  const int* act = nullptr;  // optional: right-hand side r is skipped when act[r] == 0
  int pair_ky = 0;  // 1: slices ky and pxy - ky of a tile back to back on one XCD (needs (pxy/2) ntiles % 8 == 0)
  // mirror groups (quad = 1): the four slices that read the same folded table
  // rows run back to back on one XCD: ky and its mirror, each for the kx
  // tile kx = fx (fx in [t T, t T + T), fx < pxy/2) and the mirrored tile
  // kx = pxy - fx (fx in [t T + 1, t T + T], fx <= pxy/2).  ntx = tiles per
  // side (ceil(pxy / 2 / T)), ngroups = (pxy / 2) ntx groups, padded to a
  // multiple of 8 in the launch.
  int quad = 0;
  int ntx = 0;
  long ngroups = 0;
  long pitch = 0;   // elements from row ky to row ky + 1 of a plane (pitch_y(pxy))
};

// Minimum waves per SIMD the register allocation of k_zpass must allow: the
// FP64 three-component pass needs a little over 256 registers when left
// alone, which allows one wave; held to 256 (a few bytes of spill) it runs
// two and is faster.
template <typename R, int C>
constexpr int zpass_min_waves() {
  return (sizeof(R) == 8 && C == 3) ? 2 : 1;
}

// Block order: blocks are dealt round-robin to the 8 XCDs (block b runs on
// XCD b % 8).  The nb right-hand sides of one (ky, kx-tile) slice read the
// same table slice, so they are given consecutive launch slots on one XCD and
// the slice is re-read from that XCD's L2.  Requires (pxy / T) * pxy % 8 == 0.
// With pair_ky the slices (ky, tile) and (pxy - ky, tile), which read the
// same folded table rows, follow each other on one XCD (ky = 0 is paired
// with ky = pxy / 2): slice s of XCD-order is member s % 16 / 8 of pair
// (s / 16) * 8 + s % 8.
// TT > 0: the tile width a.T == TT is known at compile time, so every LDS
// offset of the exchanges is an instruction immediate.
template <typename R, int P1, int P2, int C, int MUL, int TT = 0>
__global__ void __launch_bounds__((fused_max_threads<R, C>()))
__attribute__((amdgpu_waves_per_eu(zpass_min_waves<R, C>()))) k_zpass(cx<R>* buf, const cx<R>* __restrict__ tab, ZArgs a,
                                                            const cx<R>* __restrict__ twg) {
  constexpr int P = P1 * P2;
  constexpr int J = P1 > P2 ? P1 : P2;
  constexpr int H1 = P1 / 2;  // z < n = P/2  <=>  n1 < P1/2 for z = P2 n1 + j
  static_assert(P1 % 2 == 0, "pruned z input assumes P1 even");
  static_assert(MUL != MUL_SYM3 || C == 3, "SYM3 multiply acts on 3 components");
  static_assert(MUL != MUL_MAX6 || C == 6, "MAX6 multiply acts on 6 components");
  static_assert((MUL != MUL_DIV && MUL != MUL_CURLH) || C == 3, "DIV and CURLH act on 3 components");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const unsigned xcd = blockIdx.x % 8u;
  const unsigned k = blockIdx.x / 8u;
  if (a.act && !a.act[k % unsigned(a.nb)]) return;  // an inactive right-hand side: the whole block
  cx<R>* tw = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* lds = tw + P;
  load_twiddles<R, P>(tw, twg);
  const int T = TT > 0 ? TT : a.T;
  int col, j;
  Layout<false>::lane(threadIdx.x, T, J, col, j);
  const long slice = long(k / unsigned(a.nb)) * 8 + xcd;
  const long rhs = long(k % unsigned(a.nb));
  int tile, ky;
  int kx0 = 0, kxdir = 1, fxmin = 0, fxmax = a.pxy;  // column col of the block: kx = kx0 + kxdir col
  if (a.quad) {
    const long q = long(k / unsigned(a.nb));
    const long grp = (q / 4) * 8 + xcd;
    if (grp >= a.ngroups) return;  // padding
    const int member = int(q % 4);
    const int pk = int(grp / a.ntx);
    const int t = int(grp % a.ntx);
    ky = (member & 1) == 0 ? pk : (pk == 0 ? a.pxy / 2 : a.pxy - pk);
    const int T0 = TT > 0 ? TT : a.T;
    if (member < 2) {
      kx0 = t * T0;          // fx = kx = t T + col < pxy / 2
      fxmin = 0;
      fxmax = a.pxy / 2 - 1;
    } else {
      kx0 = a.pxy - t * T0 - 1;  // fx = t T + col + 1 <= pxy / 2, kx = pxy - fx
      kxdir = -1;
      fxmin = 1;
      fxmax = a.pxy / 2;
    }
    tile = t;
  } else if (a.pair_ky) {
    const int within = int(slice % 16);
    const long pair = (slice / 16) * 8 + within % 8;
    const int pk = int(pair / a.ntiles);
    tile = int(pair % a.ntiles);
    ky = within < 8 ? pk : (pk == 0 ? a.pxy / 2 : a.pxy - pk);
  } else {
    tile = int(slice % a.ntiles);
    ky = int(slice / a.ntiles);
  }
  int kx;
  bool valid;
  if (a.quad) {
    kx = kx0 + kxdir * col;
    const int fx = kxdir > 0 ? kx : a.pxy - kx;
    valid = fx >= fxmin && fx <= fxmax;
  } else {
    kx = tile * T + col;
    valid = kx < a.pxy;
  }
  const long PP = long(a.pxy) * a.pitch;  // one z plane
  cx<R>* base = buf + rhs * a.rhs_stride + long(ky) * a.pitch + (valid ? kx : 0);

  // kUpfront: all inputs of the block in flight at once
  constexpr int CU = kUpfront<R> ? C : 1;
  cx<R> in[CU][H1];
  // z = P2 n1 + j: one 64-bit step of P2 planes per n1
  const long zstep = long(P2) * PP;
  auto load_comp = [&](int c, cx<R>(&dst)[H1]) {
    const cx<R>* src = base + c * a.comp_stride + long(j) * PP;
    static_for<0, H1>([&](auto n1) {
      const int z = P2 * n1 + j;
      dst[n1] = (valid && j < P2 && z < a.nz) ? src[decltype(n1)::value * zstep] : czero<R>();
    });
  };
  if constexpr (kUpfront<R>) static_for<0, C>([&](auto c) { load_comp(c, in[c]); });
  __syncthreads();
  ThreadTw<R, P1, P2> twr;
  twr.init(tw, j);

  cx<R> X[C][P2];
  static_for<0, C>([&](auto c) {
    if constexpr (!kUpfront<R>) load_comp(c, in[0]);
    cx<R> u[P1];
    static_for<0, P1>([&](auto n1) {
      if constexpr (decltype(n1)::value < H1)
        u[n1] = in[kUpfront<R> ? int(c) : 0][n1];
      else
        u[n1] = czero<R>();
    });
    fft_fwd_core<R, P1, P2, false>(u, twr, lds, col, j, T, X[c]);
  });

  if (j < P1 && valid) {
    // table geometry follows from P: octant [0, N]^3, (qz, qy) rows of NXP
    // (N + 1 padded to 16) points of NE adjacent entries
    constexpr int N = P / 2;
    constexpr int NXP = ((N + 1 + 15) / 16) * 16;
    constexpr int NE = mul_entries(MUL);
    constexpr int ROW = NE * NXP;
    static_assert(P2 % 2 == 0, "the z fold assumes P2 even");
    const int Nxy = a.pxy / 2;
    const int fy = ky <= Nxy ? ky : a.pxy - ky;
    const int fx = kx <= Nxy ? kx : a.pxy - kx;
    const R sy = ky > Nxy ? R(-1) : R(1);
    const R sx = kx > Nxy ? R(-1) : R(1);
    const R sxy = sx * sy;
    const cx<R>* tb = tab + (fy * ROW + fx * NE);  // offsets below 2^31 elements
    static_for<0, P2>([&](auto k2) {
      // kz = j + P1 k2 < N exactly when k2 < P2 / 2.  The entries odd in s_z
      // vanish on the plane kz = N, so taking the folded side there is exact.
      constexpr bool upper = 2 * decltype(k2)::value >= P2;
      constexpr R sz = upper ? R(-1) : R(1);
      const int kz = j + P1 * decltype(k2)::value;
      const int fz = upper ? P - kz : kz;
      const cx<R>* t = tb + fz * ((N + 1) * ROW);
      if constexpr (MUL == MUL_DIV || MUL == MUL_CURLH) {
        const cx<R> dx = sx * t[0], dy = sy * t[1], dz = sz * t[2];
        const cx<R> x0 = X[0][k2], x1 = X[1][k2], x2 = X[2][k2];
        if constexpr (MUL == MUL_DIV) {
          X[0][k2] = dx * x0 + dy * x1 + dz * x2;
          X[1][k2] = czero<R>();
          X[2][k2] = czero<R>();
        } else {
          const R w = R(a.omega);
          const cx<R> w0 = dy * x2 - dz * x1, w1 = dz * x0 - dx * x2, w2 = dx * x1 - dy * x0;
          X[0][k2] = {w * w0.im, -w * w0.re};  // -i omega w
          X[1][k2] = {w * w1.im, -w * w1.re};
          X[2][k2] = {w * w2.im, -w * w2.re};
        }
      } else {
        const cx<R> kxx = t[0], kyy = t[1], kzz = t[2];
        const cx<R> kxy = sxy * t[3];
        const cx<R> kxz = (sx * sz) * t[4];
        const cx<R> kyz = (sy * sz) * t[5];
        if constexpr (MUL == MUL_SYM3) {
          const cx<R> x0 = X[0][k2], x1 = X[1][k2], x2 = X[2][k2];
          X[0][k2] = kxx * x0 + kxy * x1 + kxz * x2;
          X[1][k2] = kxy * x0 + kyy * x1 + kyz * x2;
          X[2][k2] = kxz * x0 + kyz * x1 + kzz * x2;
        } else {
          const cx<R> cxv = sx * t[6], cyv = sy * t[7], czv = sz * t[8];
          const cx<R> j0 = X[0][k2], j1 = X[1][k2], j2 = X[2][k2];
          const cx<R> m0 = X[3][k2], m1 = X[4][k2], m2 = X[5][k2];
          if constexpr (sizeof(R) == 4) {
            // Z_J = D j + c x m and Z_M = D m - c x j as chains of fused
            // multiply-adds ((c x m)_0 = c_y m_2 - c_z m_1, and cyclically):
            // 9% fewer instructions than products summed, and no spills at
            // two waves per SIMD.  (The 3x3 multiply keeps its sums: its
            // chains needed more registers than three waves allow.)
            X[0][k2] = cmsb(czv, m1, cmad(cyv, m2, cmad(kxz, j2, cmad(kxy, j1, kxx * j0))));
            X[1][k2] = cmsb(cxv, m2, cmad(czv, m0, cmad(kyz, j2, cmad(kyy, j1, kxy * j0))));
            X[2][k2] = cmsb(cyv, m0, cmad(cxv, m1, cmad(kzz, j2, cmad(kyz, j1, kxz * j0))));
            X[3][k2] = cmad(czv, j1, cmsb(cyv, j2, cmad(kxz, m2, cmad(kxy, m1, kxx * m0))));
            X[4][k2] = cmad(cxv, j2, cmsb(czv, j0, cmad(kyz, m2, cmad(kyy, m1, kxy * m0))));
            X[5][k2] = cmad(cyv, j0, cmsb(cxv, j1, cmad(kzz, m2, cmad(kyz, m1, kxz * m0))));
          } else {
            // FP64: the cross products formed first keep fewer values live
            // at the register limit
            const cx<R> cm0 = cyv * m2 - czv * m1, cm1 = czv * m0 - cxv * m2, cm2 = cxv * m1 - cyv * m0;
            const cx<R> cj0 = cyv * j2 - czv * j1, cj1 = czv * j0 - cxv * j2, cj2 = cxv * j1 - cyv * j0;
            X[0][k2] = kxx * j0 + kxy * j1 + kxz * j2 + cm0;
            X[1][k2] = kxy * j0 + kyy * j1 + kyz * j2 + cm1;
            X[2][k2] = kxz * j0 + kyz * j1 + kzz * j2 + cm2;
            X[3][k2] = kxx * m0 + kxy * m1 + kxz * m2 - cj0;
            X[4][k2] = kxy * m0 + kyy * m1 + kyz * m2 - cj1;
            X[5][k2] = kxz * m0 + kyz * m1 + kzz * m2 - cj2;
          }
        }
      }
    });
  }

  // outputs z < nz <= N: only m2 < P1 / 2 of the last step are ever stored
  static_for<0, C>([&](auto c) {
    cx<R>* dst = base + c * a.comp_stride + long(j) * PP;  // z = j + P2 m2
    fft_inv_CD<R, P1, P2, false, P1 / 2>(
        X[c], [&](auto m2, int, cx<R> v) { dst[decltype(m2)::value * zstep] = v; }, a.nz, lds, twr, col, j, T,
        valid);
  });
}

struct XArgs {
  int T;            // rows per block
  long nrows;       // nrhs * bz * by
  int n;            // grid points per axis (layout of H)
  long n3;          // n^3
  int nb;           // right-hand sides in the launch
  int xcd_order;    // 1: row tiles of all right-hand sides back-to-back per XCD
  int bx, by, bz;   // extent of the data box (n, n, n for the whole grid)
  int x0, y0, z0;   // its corner in the grid
  long np;          // points per component of the vectors
  const int* rows;  // support rows (xa, len, off) per (z, y) row, or null: dense box
  const int* act = nullptr;  // optional: rows of right-hand side r are skipped when act[r] == 0
  long pitch = 0;   // elements from one spectral row of A to the next (pitch_x(P))
};

// Blocks of a k_xinv launch.  With xcd_order the ceil(bz by / T) row tiles of
// each right-hand side are padded to a multiple of 8 (the padding blocks
// exit at once), so that tile t of every right-hand side lands on XCD t % 8.
__host__ __device__ inline long xinv_blocks(const XArgs& a) {
  const long NN = long(a.bz) * a.by;
  if (!a.xcd_order) return (a.nrows + a.T - 1) / a.T;
  const long nt = (NN + a.T - 1) / a.T;
  return (nt + 7) / 8 * 8 * a.nb;
}

// Rows (rhs, z, y) of the data box: inverse x transform of every component,
// then the pointwise combine.  Vectors J, B, out are [rhs][C][np]: the dense
// box [bz][by][bx], or only the support samples of each row (a.rows),
// J and out stored as TV (complex128, or complex64 for the FP32 Krylov basis
// of the mixed solver), B as complex128; H, Hmu [9][n^3] on the whole grid.
// TO: storage of out (TV by default; complex64 for the FP32 apply's output
// in the mixed solver, which carries FP32 values only).
template <typename R, int P1, int P2, int C, int MODE, typename TV = c128, typename TO = TV>
__global__ void __launch_bounds__((fused_max_threads<R, C>())) k_xinv(const cx<R>* __restrict__ A, XArgs a, const TV* __restrict__ Jv,
                                               const c128* __restrict__ Bv, const cx<R>* __restrict__ H,
                                               const cx<R>* __restrict__ Hmu, TO* __restrict__ out,
                                               const cx<R>* __restrict__ twg) {
  using S = decltype(TO::re);
  constexpr int P = P1 * P2;
  constexpr int J = P1 > P2 ? P1 : P2;
  static_assert(P1 % 2 == 0, "the cropped inverse assumes bx <= P/2 with P1 even");
  constexpr int NV = P1 / 2;  // outputs per thread per component: x = j + P2 m2 < bx <= P/2
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int N = a.n;
  const long NN = long(a.bz) * a.by;  // rows per right-hand side
  // xcd_order: block b runs on XCD b % 8; the nb right-hand sides of one
  // (z, y) row tile share H, so they take consecutive slots on one XCD
  // rows [row0, row1) of the flattened (rhs, z, y) rows
  long row0, row1;
  if (a.xcd_order) {
    const unsigned xcd = blockIdx.x % 8u, k = blockIdx.x / 8u;
    const long slice = long(k / unsigned(a.nb)) * 8 + xcd;
    const long r = long(k % unsigned(a.nb));
    if (slice * a.T >= NN) return;  // padding block
    row0 = r * NN + slice * a.T;
    row1 = r * NN + (slice * a.T + a.T < NN ? slice * a.T + a.T : NN);
  } else {
    row0 = long(blockIdx.x) * a.T;
    row1 = row0 + a.T < a.nrows ? row0 + a.T : a.nrows;
  }
  if (a.act && (row0 / NN == (row1 - 1) / NN) && !a.act[row0 / NN]) return;  // one inactive right-hand side
  cx<R>* tw = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* lds = tw + P;
  load_twiddles<R, P>(tw, twg);
  int col, j;
  Layout<true>::lane(threadIdx.x, a.T, J, col, j);
  const long row = row0 + col;
  const bool valid = row < row1 && (!a.act || a.act[row / NN]);
  const long rhs = valid ? row / NN : 0;
  const long zy = valid ? row % NN : 0;
  const long hrow = (long(a.z0) + zy / a.by) * N + (a.y0 + zy % a.by);  // (z, y) in the grid
  // a row without support samples has no output: its spectrum is not read
  const bool need = valid && (!a.rows || a.rows[3 * zy + 1] > 0);

  // kUpfront: all spectral inputs of the row in flight at once
  constexpr int CU = kUpfront<R> ? C : 1;
  cx<R> X[CU][P2];
  auto load_comp = [&](int c, cx<R>(&dst)[P2]) {
    const cx<R>* src = A + ((rhs * C + c) * NN + zy) * a.pitch;
    static_for<0, P2>([&](auto k2) { dst[k2] = (need && j < P1) ? src[j + P1 * k2] : czero<R>(); });
  };
  if constexpr (kUpfront<R>) static_for<0, C>([&](auto c) { load_comp(c, X[c]); });
  __syncthreads();
  ThreadTw<R, P1, P2> twr;
  twr.init(tw, j);

  cx<R> U[C][NV];
  static_for<0, C>([&](auto c) {
    if constexpr (!kUpfront<R>) load_comp(c, X[0]);
    fft_inv_CD<R, P1, P2, true, NV>(
        X[kUpfront<R> ? int(c) : 0],
        [&](auto m2, int, cx<R> v) {
          if constexpr (decltype(m2)::value < NV) U[c][decltype(m2)::value] = v;
        },
        a.bx, lds, twr, col, j, a.T, valid);
  });

  if (!valid || j >= P2) return;
  const long vs = a.np;
  // samples x of this row kept in the vectors: [xa, xa + len) at p0 + x
  int xa = 0, xe = a.bx;
  long p0 = zy * a.bx;
  if (a.rows) {
    xa = a.rows[3 * zy];
    xe = xa + a.rows[3 * zy + 1];
    p0 = long(a.rows[3 * zy + 2]) - xa;
  }
  static_for<0, NV>([&](auto m2) {
    const int x = j + P2 * m2;
    if (x >= a.bx || x < xa || x >= xe) return;
    const long p = p0 + x;                    // point in the vectors' layout
    const long ph = hrow * N + (a.x0 + x);    // the same point in the grid (H)
    static_for<0, C / 3>([&](auto half) {
      constexpr int c0 = 3 * decltype(half)::value;
      const long vb = (rhs * C + c0) * vs + p;
      if constexpr (MODE == MODE_CONV) {
        static_for<0, 3>([&](auto c) { out[vb + c * vs] = cvt<S>(U[c0 + c][m2]); });
      } else if constexpr (MODE == MODE_FIELD) {
        static_for<0, 3>([&](auto c) {
          out[vb + c * vs] = cvt<S>(cvt<R>(Jv[vb + c * vs]) + U[c0 + c][m2]);
        });
      } else {
        const cx<R>* Hh = (c0 == 0) ? H : Hmu;
        cx<R> jv[3], v[3];
        static_for<0, 3>([&](auto c) {
          jv[c] = cvt<R>(Jv[vb + c * vs]);
          v[c] = jv[c] + R(2) * U[c0 + c][m2];
        });
        static_for<0, 3>([&](auto r) {
          cx<R> acc = jv[r];
          static_for<0, 3>([&](auto s) { acc = acc - Hh[(3 * r + s) * a.n3 + ph] * v[s]; });
          if constexpr (MODE == MODE_RESIDUAL) {
            out[vb + r * vs] = cvt<S>(Bv[vb + r * vs] - cvt<double>(acc));
          } else {
            out[vb + r * vs] = cvt<S>(acc);
          }
        });
      }
    });
  });
}

}  // namespace vie
