// Fields after the solve, evaluated away from the support: at user points and
// as far-field patterns.  Direct sums over the grid points y (trapezoidal rule,
// weights h^3) of the free-space kernel G(r) = e^{i w r} / (4 pi r) applied to
// the density (the representations of Sections 3 and 4, eqs. Vw and
// represent_Maxwell), in FP64, over the support box of the plan (the density
// vanishes outside it).  Each launch splits the box into chunks; partial sums
// are reduced in a fixed order by a second kernel.
#include "postprocess.hpp"

#include <cmath>

namespace vie {

namespace {

constexpr int kB = 256;
constexpr double kInv4Pi = 0.079577471545947667884441881686257181;  // 1 / (4 pi)

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sums acc[0..K) over the block; thread 0 writes them to out
template <int K>
__device__ __forceinline__ void block_sum(double (&acc)[K], double* out) {
  __shared__ double red[kB / 64][K];
  const int w = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const double v = wave_sum(acc[i]);
    if ((threadIdx.x & 63) == 0) red[w][i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double s = 0.0;
      for (int k = 0; k < kB / 64; ++k) s += red[k][i];
      out[i] = s;
    }
  }
}

// Per point and group of RB right-hand sides: Laplace / Helmholtz (phi,
// grad phi), or Maxwell (E, H).  The kernel factors depend on the point pair
// only and are formed once for the group.  With r = x - y, rh = r / |r|:
//   grad G = G' rh,  (grad grad G) v = (G'' - G'/r) rh (rh . v) + (G'/r) v,
//   G' = (i w r - 1) e / r^2,  G'' = (2 - 2 i w r - w^2 r^2) e / r^3,  e = e^{i w r} / (4 pi).
// Grid: (point, rhs group, chunk of the support box's points).
template <bool MAXWELL, int RB>
__global__ void __launch_bounds__(kB) k_points(const c128* __restrict__ dens, int C, PostGrid g,
                                               const double* __restrict__ pts, int nrhs, double w, int chunk,
                                               double* __restrict__ part) {
  constexpr int NO = MAXWELL ? 6 : 4;
  constexpr int K = RB * 2 * NO;
  const int p = blockIdx.x, rg = blockIdx.y, k = blockIdx.z;
  const int ngroups = gridDim.y, nchunk = gridDim.z;
  const int r0 = rg * RB, nr = nrhs - r0 < RB ? nrhs - r0 : RB;
  const long n3 = long(g.n) * g.n * g.n;
  const int nb = g.bx * g.by * g.bz;
  const int lo = k * chunk, hi = lo + chunk < nb ? lo + chunk : nb;
  const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
  const c128* Jg = dens + long(r0) * C * n3;
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0.0;
  for (int t = lo + int(threadIdx.x); t < hi; t += kB) {
    const int ix = t % g.bx, iyz = t / g.bx;
    const int iy = iyz % g.by, iz = iyz / g.by;
    const long q = (long(g.z0 + iz) * g.n + (g.y0 + iy)) * g.n + (g.x0 + ix);
    const double d[3] = {px - (g.ox + (g.x0 + ix + 0.5) * g.h), py - (g.oy + (g.y0 + iy + 0.5) * g.h),
                         pz - (g.oz + (g.z0 + iz + 0.5) * g.h)};
    const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double ir = 1.0 / rr;
    const double rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
    double sn, cs;
    sincos(w * rr, &sn, &cs);
    const c128 e = {cs * kInv4Pi, sn * kInv4Pi};
    const c128 G = ir * e;
    const c128 G1 = (ir * ir) * (c128{-1.0, w * rr} * e);
    const c128 G2 = (ir * ir * ir) * (c128{2.0 - w * w * rr * rr, -2.0 * w * rr} * e);
    const c128 A = G2 - ir * G1;  // (grad grad G) v = A rh (rh . v) + (G'/r) v
    const c128 Bq = ir * G1;
    const c128 w2G = (w * w) * G;
    const c128 gr[3] = {rh[0] * G1, rh[1] * G1, rh[2] * G1};  // grad G
    auto hess = [&](const c128 (&v)[3], c128 (&out)[3]) {
      const c128 Ar = A * (rh[0] * v[0] + rh[1] * v[1] + rh[2] * v[2]);
      for (int a = 0; a < 3; ++a) out[a] = rh[a] * Ar + Bq * v[a];
    };
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      if (j < nr) {
        const c128* Jr = Jg + long(j) * C * n3;
        c128 J[3], M[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          J[c] = Jr[c * n3 + q];
          M[c] = (MAXWELL && C == 6) ? Jr[(3 + c) * n3 + q] : c128{0.0, 0.0};
        }
        double* a = acc + j * 2 * NO;
        if constexpr (!MAXWELL) {
          const c128 phi = G1 * (rh[0] * J[0] + rh[1] * J[1] + rh[2] * J[2]);
          c128 gp[3];
          hess(J, gp);
          a[0] += phi.re;
          a[1] += phi.im;
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            a[2 + 2 * b] += gp[b].re;
            a[3 + 2 * b] += gp[b].im;
          }
        } else {
          c128 HJ[3], HM[3];
          hess(J, HJ);
          hess(M, HM);
          const c128 cJ[3] = {gr[1] * J[2] - gr[2] * J[1], gr[2] * J[0] - gr[0] * J[2], gr[0] * J[1] - gr[1] * J[0]};
          const c128 cM[3] = {gr[1] * M[2] - gr[2] * M[1], gr[2] * M[0] - gr[0] * M[2], gr[0] * M[1] - gr[1] * M[0]};
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const c128 E = HJ[b] + w2G * J[b] + w * times_i(cM[b]);
            const c128 H = HM[b] + w2G * M[b] - w * times_i(cJ[b]);
            a[2 * b] += E.re;
            a[2 * b + 1] += E.im;
            a[6 + 2 * b] += H.re;
            a[7 + 2 * b] += H.im;
          }
        }
      }
    }
  }
  block_sum(acc, part + ((long(p) * ngroups + rg) * nchunk + k) * K);
}

// Fourier sums J^_c(xh) = sum_y e^{-i w xh . y} J_c(y) for a group of DB
// directions.  On the grid the phase factors: e^{-i w xh . y} =
// px(x) pyz(y, z), so each thread keeps one x of the support box, adds
// pyz (staged in LDS per row) times J over its rows and multiplies by px(x)
// at the end.  Grid: (direction group, rhs, chunk of the box's (z, y) rows).
constexpr int kRowsStaged = 32;

template <int C, int DB>
__global__ void __launch_bounds__(kB) k_far(const c128* __restrict__ dens, PostGrid g,
                                            const double* __restrict__ dirs, int ndirs, double w, int rows_per_chunk,
                                            double* __restrict__ part) {
  constexpr int K = DB * 2 * C;
  __shared__ double u[DB][3];
  __shared__ c128 pyz[kRowsStaged][DB];
  const int gi = blockIdx.x, r = blockIdx.y, k = blockIdx.z;
  const int nrhs = gridDim.y, nchunk = gridDim.z;
  const long n3 = long(g.n) * g.n * g.n;
  const int rows = g.by * g.bz;
  const int row_lo = k * rows_per_chunk;
  const int row_hi = row_lo + rows_per_chunk < rows ? row_lo + rows_per_chunk : rows;
  if (threadIdx.x < DB * 3) {
    const int j = threadIdx.x / 3, d = gi * DB + j;
    u[j][threadIdx.x % 3] = d < ndirs ? dirs[3 * d + threadIdx.x % 3] : 0.0;
  }
  __syncthreads();
  const int rpi = kB / g.bx;  // rows per pass of the block
  const int ix = int(threadIdx.x) % g.bx, sub = int(threadIdx.x) / g.bx;
  const c128* Jr = dens + long(r) * C * n3;
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0.0;
  for (int base = row_lo; base < row_hi; base += kRowsStaged) {
    __syncthreads();
    for (int t = threadIdx.x; t < kRowsStaged * DB; t += kB) {
      const int rr = t / DB, j = t % DB, row = base + rr;
      const double yy = g.oy + (g.y0 + row % g.by + 0.5) * g.h;
      const double yz = g.oz + (g.z0 + row / g.by + 0.5) * g.h;
      double sn, cs;
      sincos(-w * (u[j][1] * yy + u[j][2] * yz), &sn, &cs);
      pyz[rr][j] = {cs, sn};
    }
    __syncthreads();
    const int nrow = row_hi - base < kRowsStaged ? row_hi - base : kRowsStaged;
    if (sub < rpi) {
      for (int rr = sub; rr < nrow; rr += rpi) {
        const int row = base + rr;
        const long q = (long(g.z0 + row / g.by) * g.n + (g.y0 + row % g.by)) * g.n + (g.x0 + ix);
        c128 J[C];
#pragma unroll
        for (int c = 0; c < C; ++c) J[c] = Jr[c * n3 + q];
#pragma unroll
        for (int j = 0; j < DB; ++j) {
          const c128 ph = pyz[rr][j];
#pragma unroll
          for (int c = 0; c < C; ++c) {
            acc[2 * (j * C + c)] += ph.re * J[c].re - ph.im * J[c].im;
            acc[2 * (j * C + c) + 1] += ph.re * J[c].im + ph.im * J[c].re;
          }
        }
      }
    }
  }
  if (sub < rpi) {
    const double yx = g.ox + (g.x0 + ix + 0.5) * g.h;
#pragma unroll
    for (int j = 0; j < DB; ++j) {
      double sn, cs;
      sincos(-w * u[j][0] * yx, &sn, &cs);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double re = acc[2 * (j * C + c)], im = acc[2 * (j * C + c) + 1];
        acc[2 * (j * C + c)] = cs * re - sn * im;
        acc[2 * (j * C + c) + 1] = cs * im + sn * re;
      }
    }
  }
  block_sum(acc, part + ((long(gi) * nrhs + r) * nchunk + k) * K);
}

// out[r][p][o] = h^3 sum_k part[p][r / RB][k][r % RB][o]
__global__ void __launch_bounds__(kB) k_points_reduce(const double* __restrict__ part, int npts, int nrhs, int rb,
                                                      int nchunk, int no, double h3, c128* __restrict__ out) {
  const long total = long(npts) * nrhs * no;
  const int ngroups = (nrhs + rb - 1) / rb;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int o = int(t % no);
    const long pr = t / no;
    const int r = int(pr % nrhs), p = int(pr / nrhs);
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nchunk; ++k) {
      const double* s = part + ((long(p) * ngroups + r / rb) * nchunk + k) * rb * 2 * no + ((r % rb) * no + o) * 2;
      re += s[0];
      im += s[1];
    }
    out[(long(r) * npts + p) * no + o] = {h3 * re, h3 * im};
  }
}

// far-field patterns from the Fourier sums: Helmholtz phi_inf = (i w / 4 pi) xh . J^;
// Maxwell E_inf = (w^2 / 4 pi) [(I - xh xh^T) J^ - xh x M^],
//         H_inf = (w^2 / 4 pi) [(I - xh xh^T) M^ + xh x J^]
__global__ void __launch_bounds__(kB) k_far_reduce(const double* __restrict__ part, const double* __restrict__ dirs,
                                                   int ndirs, int nrhs, int db, int nchunk, int C, int maxwell,
                                                   double w, double h3, c128* __restrict__ out) {
  const long total = long(ndirs) * nrhs;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int r = int(t % nrhs), d = int(t / nrhs);
    c128 S[6] = {};
    for (int k = 0; k < nchunk; ++k) {
      const double* s = part + ((long(d / db) * nrhs + r) * nchunk + k) * db * 2 * C + (d % db) * 2 * C;
      for (int c = 0; c < C; ++c) S[c] = S[c] + c128{s[2 * c], s[2 * c + 1]};
    }
    for (int c = 0; c < C; ++c) S[c] = h3 * S[c];
    const double u[3] = {dirs[3 * d], dirs[3 * d + 1], dirs[3 * d + 2]};
    if (!maxwell) {
      const c128 uj = u[0] * S[0] + u[1] * S[1] + u[2] * S[2];
      out[long(r) * ndirs + d] = (w * kInv4Pi) * times_i(uj);
      continue;
    }
    const c128* Jh = S;
    const c128 Mh[3] = {C == 6 ? S[3] : c128{0.0, 0.0}, C == 6 ? S[4] : c128{0.0, 0.0},
                        C == 6 ? S[5] : c128{0.0, 0.0}};
    const c128 uJ = u[0] * Jh[0] + u[1] * Jh[1] + u[2] * Jh[2];
    const c128 uM = u[0] * Mh[0] + u[1] * Mh[1] + u[2] * Mh[2];
    const c128 xM[3] = {u[1] * Mh[2] - u[2] * Mh[1], u[2] * Mh[0] - u[0] * Mh[2], u[0] * Mh[1] - u[1] * Mh[0]};
    const c128 xJ[3] = {u[1] * Jh[2] - u[2] * Jh[1], u[2] * Jh[0] - u[0] * Jh[2], u[0] * Jh[1] - u[1] * Jh[0]};
    const double f = w * w * kInv4Pi;
    c128* o = out + (long(r) * ndirs + d) * 6;
    for (int a = 0; a < 3; ++a) {
      o[a] = f * (Jh[a] - u[a] * uJ - xM[a]);
      o[3 + a] = f * (Mh[a] - u[a] * uM + xJ[a]);
    }
  }
}

// right-hand sides per block of k_points, directions per block of k_far
constexpr int rhs_per_block(bool maxwell) { return maxwell ? 4 : 8; }
// (8 directions for C = 3 measured faster than 16: 176 against 256 VGPRs)
constexpr int dirs_per_block(int C) { return C == 6 ? 4 : 8; }

// chunks so that a launch has about 2048 blocks, each with at least `unit` items
int chunks_for(long items, long blocks_without, long unit) {
  long k = (2048 + blocks_without - 1) / blocks_without;
  const long most = (items + unit - 1) / unit;
  if (k > most) k = most;
  if (k > 1024) k = 1024;
  if (k < 1) k = 1;
  return int(k);
}

struct PointsLaunch {
  int rb, ngroups, nchunk, chunk, no;
};
PointsLaunch points_launch(const PostGrid& g, bool maxwell, int npts, int nrhs) {
  PointsLaunch L;
  L.rb = rhs_per_block(maxwell);
  L.ngroups = (nrhs + L.rb - 1) / L.rb;
  const long nb = long(g.bx) * g.by * g.bz;
  L.nchunk = chunks_for(nb, long(npts) * L.ngroups, kB);
  L.chunk = int((nb + L.nchunk - 1) / L.nchunk);
  L.no = maxwell ? 6 : 4;
  return L;
}

struct FarLaunch {
  int db, ngroups, nchunk, rows_per_chunk;
};
FarLaunch far_launch(const PostGrid& g, int C, int ndirs, int nrhs) {
  FarLaunch L;
  L.db = dirs_per_block(C);
  L.ngroups = (ndirs + L.db - 1) / L.db;
  const long rows = long(g.by) * g.bz;
  L.nchunk = chunks_for(rows, long(L.ngroups) * nrhs, kRowsStaged);
  L.rows_per_chunk = int((rows + L.nchunk - 1) / L.nchunk);
  return L;
}

}  // namespace

long points_partial_doubles(const PostGrid& g, bool maxwell, int npts, int nrhs) {
  const PointsLaunch L = points_launch(g, maxwell, npts, nrhs);
  return long(npts) * L.ngroups * L.nchunk * L.rb * 2 * L.no;
}

long far_partial_doubles(const PostGrid& g, int C, int ndirs, int nrhs) {
  const FarLaunch L = far_launch(g, C, ndirs, nrhs);
  return long(L.ngroups) * nrhs * L.nchunk * L.db * 2 * C;
}

hipError_t launch_fields_at(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* pts, int npts,
                            int nrhs, double w, double* part, c128* out, hipStream_t s) {
  const PointsLaunch L = points_launch(g, maxwell, npts, nrhs);
  const dim3 grid{unsigned(npts), unsigned(L.ngroups), unsigned(L.nchunk)};
  if (maxwell)
    k_points<true, rhs_per_block(true)><<<grid, kB, 0, s>>>(dens, C, g, pts, nrhs, w, L.chunk, part);
  else
    k_points<false, rhs_per_block(false)><<<grid, kB, 0, s>>>(dens, C, g, pts, nrhs, w, L.chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double h3 = g.h * g.h * g.h;
  k_points_reduce<<<unsigned((long(npts) * nrhs * L.no + kB - 1) / kB), kB, 0, s>>>(part, npts, nrhs, L.rb,
                                                                                   L.nchunk, L.no, h3, out);
  return hipGetLastError();
}

hipError_t launch_far_field(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* dirs, int ndirs,
                            int nrhs, double w, double* part, c128* out, hipStream_t s) {
  if (g.bx < 1 || g.bx > kB) return hipErrorInvalidValue;
  const FarLaunch L = far_launch(g, C, ndirs, nrhs);
  const dim3 grid{unsigned(L.ngroups), unsigned(nrhs), unsigned(L.nchunk)};
  if (C == 6)
    k_far<6, dirs_per_block(6)><<<grid, kB, 0, s>>>(dens, g, dirs, ndirs, w, L.rows_per_chunk, part);
  else
    k_far<3, dirs_per_block(3)><<<grid, kB, 0, s>>>(dens, g, dirs, ndirs, w, L.rows_per_chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double h3 = g.h * g.h * g.h;
  k_far_reduce<<<unsigned((long(ndirs) * nrhs + kB - 1) / kB), kB, 0, s>>>(part, dirs, ndirs, nrhs, L.db, L.nchunk,
                                                                           C, maxwell ? 1 : 0, w, h3, out);
  return hipGetLastError();
}

}  // namespace vie
