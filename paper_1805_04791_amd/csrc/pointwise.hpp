// Launchers of the pointwise and Krylov kernels (pointwise.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "cx.hpp"

namespace vie {

// A box of the n^3 grid: extent (bx, by, bz), corner (x0, y0, z0).  Box
// vectors are laid out [bz][by][bx] per component, or, when rows is set,
// hold only the samples [xa, xa + len) of each (z, y) row r = z * by + y,
// at offset off (rows[3 r .. 3 r + 2] = xa, len, off; np points in all).
struct Box {
  int n;
  int bx, by, bz;
  int x0, y0, z0;
  const int* rows;
  long np;
};

// Support rows of a box: for each (z, y) row, the first x and the count of
// samples from the first to the last point where H (or H_mu, if given) has a
// non-zero entry (0, 0 for a row without such points).  xalen[2 r], xalen[2 r + 1].
hipError_t launch_row_support(const c128* H, const c128* Hmu, const Box& g, int* xalen, hipStream_t s);

// H = (a + I)^{-1} (a - I) = I - 2 (a + I)^{-1} at every point (eq. rhodef).
// Writes H in FP64 and FP32, and per block: max ||H||_2 (blk_max), the count
// of singular or non-finite points (blk_bad) and the bounding box of the
// points where H != 0 (blk_box[6 b ..] = xmin, xmax, ymin, ymax, zmin, zmax;
// min = n, max = -1 for a block without such points).
hipError_t launch_contrast(const c128* coef, c128* H64, c64* H32, int n, double* blk_max, int* blk_bad,
                           int* blk_box, int nblocks, hipStream_t s);

// b = 2 H g per 3-component half (H for the first half, Hmu for the second),
// at the points of box g: inc on the whole grid [nrhs][C][n^3], b in box layout
// (dense or support rows).
hipError_t launch_rhs(const c128* H, const c128* Hmu, const c128* inc, c128* b, int nrhs, int C, const Box& g,
                      hipStream_t s);
// box[v] <- full[v] restricted to the box, v < nv components
hipError_t launch_gather(const c128* full, c128* box, long nv, const Box& g, hipStream_t s);
// full[v] <- box[v] at the points the box vectors hold, 0 elsewhere, v < nv components
hipError_t launch_scatter(const c128* box, c128* full, long nv, const Box& g, hipStream_t s);

// Partial sums, per right-hand side r and block: conj(V_i) . w_r for i < nv and
// ||w_r||^2 (slot nv).  V_i of rhs r at V + i * vstride + r * rstride.
// Products and sums in FP64 (vectors complex128; the kernel also reads other
// storage types, instantiated where used).  act (optional): right-hand sides
// with act[r] == 0 are skipped (their partial sums are not written).
template <typename TV, typename TW>
hipError_t launch_dots(const TV* V, long vstride, long rstride, const TW* w, long L, int nv, int nrhs, int nblk,
                       c128* partials, hipStream_t s, const int* act = nullptr);
// out[r][i] = sum over blocks of partials[r][blk][i], fixed order.
hipError_t launch_reduce(const c128* partials, int nrhs, int nblk, int nv1, c128* out, hipStream_t s,
                         const int* act = nullptr);
// out_r = (w_r - sum_{i < count_r} V_i c[r][i]) * s[r]   (out may alias w), in
// FP64, rounded to the storage of out (instantiated for complex128); count_r =
// count[r] (capped at nv), or nv without count; out_r untouched when count[r] < 0.
template <typename TV, typename TW, typename TO>
hipError_t launch_combine(const TV* V, long vstride, long rstride, const TW* w, TO* out, long L, int nv,
                          const c128* coef, const double* scale, int nrhs, hipStream_t s,
                          const int* count = nullptr);
// The same combine with its coefficients, scales and counts passed as kernel
// arguments (no staging copy before the launch), for up to kArgRhs right-hand
// sides and kArgCoef coefficients in all ([rhs][stride], stride = max(nv, 1)).
constexpr int kArgRhs = 8;
constexpr int kArgCoef = 160;
struct CombineArgs {
  double scale[kArgRhs];
  int count[kArgRhs];  // < 0: skip the right-hand side
  c128 coef[kArgCoef];
};
template <typename TV, typename TW, typename TO>
hipError_t launch_combine_args(const TV* V, long vstride, long rstride, const TW* w, TO* out, long L, int nv,
                               const CombineArgs& a, int nrhs, hipStream_t s);
// out[r] = bit r of words[0..3] (r < nb <= kMaxFlagged), as 0 / 1
constexpr int kMaxFlagged = 256;
hipError_t launch_set_flags(const unsigned long long (&words)[4], int nb, int* out, hipStream_t s);
hipError_t launch_fill(c128* p, long n, c128 v, hipStream_t s);
hipError_t launch_copy(const c128* src, c128* dst, long n, hipStream_t s);
// FP32 tables from FP64
hipError_t launch_demote(const c128* src, c64* dst, long n, hipStream_t s);

// Octant tables from the (Z, Q, Q) transforms of the windowed kernel
// buf[e][qz][qy][qx]: tab[((qz (Z/2+1) + qy) ne + e) nxp + qx] =
// (-1)^(qx+qy+qz) * scale_e * buf[e][qz][qy][qx] for qz, qy in [0, Z/2], qx < nxp,
// zero where qx or qy > Q/2; scale_e = 1/(Z Q^2), times i*omega for the curl
// entries e >= 6.
hipError_t launch_finalize_tables(const c128* buf, c128* tab64, c64* tab32, int Q, int Z, int nxp, int ne,
                                  double omega, hipStream_t s);

int krylov_blocks(long L);

}  // namespace vie
