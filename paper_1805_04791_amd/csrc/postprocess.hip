// Fields after the solve, evaluated away from the support: at user points and
// as far-field patterns.  Direct sums over the grid points y (trapezoidal rule,
// weights h^3) of the free-space kernel G(r) = e^{i w r} / (4 pi r) applied to
// the density (the representations of Sections 3 and 4, eqs. Vw and
// represent_Maxwell), in FP64.  Each launch splits the grid into chunks;
// partial sums are reduced in a fixed order by a second kernel.
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

__device__ __forceinline__ void grid_point(long q, const PostGrid& g, double& x, double& y, double& z) {
  const long n = g.n;
  x = g.ox + (double(q % n) + 0.5) * g.h;
  y = g.oy + (double((q / n) % n) + 0.5) * g.h;
  z = g.oz + (double(q / (n * n)) + 0.5) * g.h;
}

// Per point and right-hand side: Laplace / Helmholtz (phi, grad phi), or
// Maxwell (E, H).  With r = x - y, rh = r / |r|:
//   grad G = G' rh,  (grad grad G) v = (G'' - G'/r) rh (rh . v) + (G'/r) v,
//   G' = (i w r - 1) e / r^2,  G'' = (2 - 2 i w r - w^2 r^2) e / r^3,  e = e^{i w r} / (4 pi).
template <bool MAXWELL>
__global__ void __launch_bounds__(kB) k_points(const c128* __restrict__ dens, int C, PostGrid g,
                                               const double* __restrict__ pts, double w, long chunk,
                                               double* __restrict__ part) {
  constexpr int NO = MAXWELL ? 6 : 4;
  const int p = blockIdx.x, r = blockIdx.y, k = blockIdx.z;
  const int nrhs = gridDim.y, nchunk = gridDim.z;
  const long n3 = long(g.n) * g.n * g.n;
  const long lo = long(k) * chunk, hi = lo + chunk < n3 ? lo + chunk : n3;
  const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
  const c128* Jr = dens + long(r) * C * n3;
  double acc[2 * NO];
#pragma unroll
  for (int i = 0; i < 2 * NO; ++i) acc[i] = 0.0;
  for (long q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    c128 J[3], M[3];
    bool nz = false;
    for (int c = 0; c < 3; ++c) {
      J[c] = Jr[c * n3 + q];
      M[c] = (MAXWELL && C == 6) ? Jr[(3 + c) * n3 + q] : c128{0.0, 0.0};
      nz = nz || J[c].re != 0.0 || J[c].im != 0.0 || M[c].re != 0.0 || M[c].im != 0.0;
    }
    if (!nz) continue;
    double yx, yy, yz;
    grid_point(q, g, yx, yy, yz);
    const double d[3] = {px - yx, py - yy, pz - yz};
    const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double rh[3] = {d[0] / rr, d[1] / rr, d[2] / rr};
    double sn, cs;
    sincos(w * rr, &sn, &cs);
    const c128 e = {cs * kInv4Pi, sn * kInv4Pi};
    const c128 G = (1.0 / rr) * e;
    const c128 G1 = (1.0 / (rr * rr)) * (c128{-1.0, w * rr} * e);
    const c128 G2 = (1.0 / (rr * rr * rr)) * (c128{2.0 - w * w * rr * rr, -2.0 * w * rr} * e);
    const c128 A = G2 - (1.0 / rr) * G1;  // (grad grad G) v = A rh (rh . v) + (G'/r) v
    const c128 Bq = (1.0 / rr) * G1;
    auto hess = [&](const c128 (&v)[3], c128 (&out)[3]) {
      const c128 rv = rh[0] * v[0] + rh[1] * v[1] + rh[2] * v[2];
      const c128 Ar = A * rv;
      for (int a = 0; a < 3; ++a) out[a] = rh[a] * Ar + Bq * v[a];
    };
    if constexpr (!MAXWELL) {
      const c128 rv = rh[0] * J[0] + rh[1] * J[1] + rh[2] * J[2];
      const c128 phi = G1 * rv;
      c128 gp[3];
      hess(J, gp);
      acc[0] += phi.re;
      acc[1] += phi.im;
      for (int a = 0; a < 3; ++a) {
        acc[2 + 2 * a] += gp[a].re;
        acc[3 + 2 * a] += gp[a].im;
      }
    } else {
      c128 HJ[3], HM[3];
      hess(J, HJ);
      hess(M, HM);
      const c128 gr[3] = {rh[0] * G1, rh[1] * G1, rh[2] * G1};  // grad G
      const c128 cJ[3] = {gr[1] * J[2] - gr[2] * J[1], gr[2] * J[0] - gr[0] * J[2], gr[0] * J[1] - gr[1] * J[0]};
      const c128 cM[3] = {gr[1] * M[2] - gr[2] * M[1], gr[2] * M[0] - gr[0] * M[2], gr[0] * M[1] - gr[1] * M[0]};
      const c128 w2G = (w * w) * G;
      for (int a = 0; a < 3; ++a) {
        const c128 E = HJ[a] + w2G * J[a] + w * times_i(cM[a]);
        const c128 H = HM[a] + w2G * M[a] - w * times_i(cJ[a]);
        acc[2 * a] += E.re;
        acc[2 * a + 1] += E.im;
        acc[6 + 2 * a] += H.re;
        acc[7 + 2 * a] += H.im;
      }
    }
  }
  block_sum(acc, part + ((long(p) * nrhs + r) * nchunk + k) * 2 * NO);
}

// Fourier sums J^(xh) = sum_y e^{-i w xh . y} J(y) per direction and rhs (C components)
template <int C>
__global__ void __launch_bounds__(kB) k_far(const c128* __restrict__ dens, PostGrid g,
                                            const double* __restrict__ dirs, double w, long chunk,
                                            double* __restrict__ part) {
  const int d = blockIdx.x, r = blockIdx.y, k = blockIdx.z;
  const int nrhs = gridDim.y, nchunk = gridDim.z;
  const long n3 = long(g.n) * g.n * g.n;
  const long lo = long(k) * chunk, hi = lo + chunk < n3 ? lo + chunk : n3;
  const double ux = dirs[3 * d], uy = dirs[3 * d + 1], uz = dirs[3 * d + 2];
  const c128* Jr = dens + long(r) * C * n3;
  double acc[2 * C];
#pragma unroll
  for (int i = 0; i < 2 * C; ++i) acc[i] = 0.0;
  for (long q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    double yx, yy, yz;
    grid_point(q, g, yx, yy, yz);
    double sn, cs;
    sincos(-w * (ux * yx + uy * yy + uz * yz), &sn, &cs);
    const c128 ph = {cs, sn};
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const c128 v = ph * Jr[c * n3 + q];
      acc[2 * c] += v.re;
      acc[2 * c + 1] += v.im;
    }
  }
  block_sum(acc, part + ((long(d) * nrhs + r) * nchunk + k) * 2 * C);
}

// out[r][p][o] = h^3 sum_k part[p][r][k][o]
__global__ void __launch_bounds__(kB) k_points_reduce(const double* __restrict__ part, int npts, int nrhs, int nchunk,
                                                      int no, double h3, c128* __restrict__ out) {
  const long total = long(npts) * nrhs * no;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int o = int(t % no);
    const long pr = t / no;
    const int r = int(pr % nrhs), p = int(pr / nrhs);
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nchunk; ++k) {
      const double* s = part + ((long(p) * nrhs + r) * nchunk + k) * 2 * no + 2 * o;
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
                                                   int ndirs, int nrhs, int nchunk, int C, int maxwell, double w,
                                                   double h3, c128* __restrict__ out) {
  const long total = long(ndirs) * nrhs;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const int r = int(t % nrhs), d = int(t / nrhs);
    c128 S[6] = {};
    for (int k = 0; k < nchunk; ++k) {
      const double* s = part + ((long(d) * nrhs + r) * nchunk + k) * 2 * C;
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

int nchunks_for(long n3, long items) {
  long k = (2048 + items - 1) / items;
  const long most = (n3 + kB - 1) / kB;
  if (k > most) k = most;
  if (k > 1024) k = 1024;
  if (k < 1) k = 1;
  return int(k);
}

}  // namespace

long post_partial_doubles(long n3, int nitems, int nrhs, int nout) {
  return long(nitems) * nrhs * nchunks_for(n3, long(nitems) * nrhs) * 2 * nout;
}

hipError_t launch_fields_at(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* pts, int npts,
                            int nrhs, double w, double* part, c128* out, hipStream_t s) {
  const long n3 = long(g.n) * g.n * g.n;
  const int nchunk = nchunks_for(n3, long(npts) * nrhs);
  const long chunk = (n3 + nchunk - 1) / nchunk;
  const dim3 grid{unsigned(npts), unsigned(nrhs), unsigned(nchunk)};
  const int no = maxwell ? 6 : 4;
  if (maxwell)
    k_points<true><<<grid, kB, 0, s>>>(dens, C, g, pts, w, chunk, part);
  else
    k_points<false><<<grid, kB, 0, s>>>(dens, C, g, pts, w, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double h3 = g.h * g.h * g.h;
  k_points_reduce<<<unsigned((long(npts) * nrhs * no + kB - 1) / kB), kB, 0, s>>>(part, npts, nrhs, nchunk, no, h3,
                                                                                out);
  return hipGetLastError();
}

hipError_t launch_far_field(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* dirs, int ndirs,
                            int nrhs, double w, double* part, c128* out, hipStream_t s) {
  const long n3 = long(g.n) * g.n * g.n;
  const int nchunk = nchunks_for(n3, long(ndirs) * nrhs);
  const long chunk = (n3 + nchunk - 1) / nchunk;
  const dim3 grid{unsigned(ndirs), unsigned(nrhs), unsigned(nchunk)};
  if (C == 6)
    k_far<6><<<grid, kB, 0, s>>>(dens, g, dirs, w, chunk, part);
  else
    k_far<3><<<grid, kB, 0, s>>>(dens, g, dirs, w, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double h3 = g.h * g.h * g.h;
  k_far_reduce<<<unsigned((long(ndirs) * nrhs + kB - 1) / kB), kB, 0, s>>>(part, dirs, ndirs, nrhs, nchunk, C,
                                                                           maxwell ? 1 : 0, w, h3, out);
  return hipGetLastError();
}

}  // namespace vie
