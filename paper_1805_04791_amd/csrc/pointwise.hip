// Pointwise kernels: contrast, right-hand side, table finalisation and the
// FP64 Krylov vector operations (multi-dot, fixed-order reductions, basis
// combinations).  Every reduction is two-phase with a block count that depends
// only on the vector length, so results are bitwise independent of how many
// right-hand sides share a launch.
#include "pointwise.hpp"

#include <algorithm>
#include <cmath>

namespace vie {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_imin(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_imax(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// spectral norm of a 3x3 complex matrix: sqrt(largest eigenvalue of H^H H)
__device__ double spec_norm3(const c128 h[9]) {
  // M = H^H H
  c128 m[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      c128 acc = {0.0, 0.0};
      for (int k = 0; k < 3; ++k) acc = acc + cmulc(h[3 * k + a], h[3 * k + b]);
      m[a][b] = acc;
    }
  const double m00 = m[0][0].re, m11 = m[1][1].re, m22 = m[2][2].re;
  const double q = (m00 + m11 + m22) / 3.0;
  const double p1 = norm2(m[0][1]) + norm2(m[0][2]) + norm2(m[1][2]);
  const double p2 = (m00 - q) * (m00 - q) + (m11 - q) * (m11 - q) + (m22 - q) * (m22 - q) + 2.0 * p1;
  if (!(p2 > 1e-300)) return sqrt(fmax(q, 0.0));
  const double p = sqrt(p2 / 6.0);
  const double b00 = (m00 - q) / p, b11 = (m11 - q) / p, b22 = (m22 - q) / p;
  const c128 b01 = (1.0 / p) * m[0][1], b02 = (1.0 / p) * m[0][2], b12 = (1.0 / p) * m[1][2];
  const c128 t = b01 * b12;
  const double re_t = t.re * b02.re + t.im * b02.im;  // Re(b01 b12 conj(b02))
  const double det = b00 * b11 * b22 + 2.0 * re_t - b00 * norm2(b12) - b11 * norm2(b02) - b22 * norm2(b01);
  const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
  const double phi = acos(r) / 3.0;
  return sqrt(fmax(q + 2.0 * p * cos(phi), 0.0));
}

// H = I - 2 (a + I)^{-1}, the block maximum of ||H(x)||_2, the count of
// singular points and the bounding box (x, y, z min/max) of the points where
// H has a non-zero entry.
__global__ void __launch_bounds__(kBlock) k_contrast(const c128* __restrict__ coef, c128* __restrict__ H64,
                                                     c64* __restrict__ H32, int n, double* __restrict__ blk_max,
                                                     int* __restrict__ blk_bad, int* __restrict__ blk_box) {
  __shared__ double smax[kBlock / 64];
  __shared__ double sbad[kBlock / 64];
  __shared__ int sbox[kBlock / 64][6];
  const long n3 = long(n) * n * n;
  double vmax = 0.0;
  double bad = 0.0;
  int lo[3] = {n, n, n}, hi[3] = {-1, -1, -1};
  for (long p = long(blockIdx.x) * blockDim.x + threadIdx.x; p < n3; p += long(gridDim.x) * blockDim.x) {
    c128 b[9];
    for (int e = 0; e < 9; ++e) b[e] = coef[e * n3 + p];
    b[0].re += 1.0;
    b[4].re += 1.0;
    b[8].re += 1.0;
    // adjugate of B = a + I
    c128 adj[9];
    adj[0] = b[4] * b[8] - b[5] * b[7];
    adj[1] = b[2] * b[7] - b[1] * b[8];
    adj[2] = b[1] * b[5] - b[2] * b[4];
    adj[3] = b[5] * b[6] - b[3] * b[8];
    adj[4] = b[0] * b[8] - b[2] * b[6];
    adj[5] = b[2] * b[3] - b[0] * b[5];
    adj[6] = b[3] * b[7] - b[4] * b[6];
    adj[7] = b[1] * b[6] - b[0] * b[7];
    adj[8] = b[0] * b[4] - b[1] * b[3];
    const c128 det = b[0] * adj[0] + b[1] * adj[3] + b[2] * adj[6];
    const double dn = norm2(det);
    double scale_b = 0.0;
    for (int e = 0; e < 9; ++e) scale_b = fmax(scale_b, norm2(b[e]));
    const bool singular = !(dn > 1e-28 * scale_b * scale_b * scale_b) || !isfinite(dn);
    c128 h[9];
    if (singular) {
      bad += 1.0;
      for (int e = 0; e < 9; ++e) h[e] = {0.0, 0.0};
    } else {
      const c128 inv_det = {det.re / dn, -det.im / dn};
      for (int e = 0; e < 9; ++e) {
        const c128 v = adj[e] * inv_det;
        h[e] = {-2.0 * v.re, -2.0 * v.im};
      }
      h[0].re += 1.0;
      h[4].re += 1.0;
      h[8].re += 1.0;
      const double nrm = spec_norm3(h);
      if (!isfinite(nrm)) bad += 1.0;
      vmax = fmax(vmax, nrm);
    }
    bool nz = false;
    for (int e = 0; e < 9; ++e) {
      H64[e * n3 + p] = h[e];
      H32[e * n3 + p] = cvt<float>(h[e]);
      nz = nz || h[e].re != 0.0 || h[e].im != 0.0;
    }
    if (nz) {
      const int q[3] = {int(p % n), int((p / n) % n), int(p / (long(n) * n))};
      for (int a = 0; a < 3; ++a) {
        lo[a] = min(lo[a], q[a]);
        hi[a] = max(hi[a], q[a]);
      }
    }
  }
  vmax = wave_max(vmax);
  bad = wave_sum(bad);
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_imin(lo[a]);
    hi[a] = wave_imax(hi[a]);
  }
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    smax[w] = vmax;
    sbad[w] = bad;
    for (int a = 0; a < 3; ++a) {
      sbox[w][2 * a] = lo[a];
      sbox[w][2 * a + 1] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0, c = 0.0;
    int b[6] = {n, -1, n, -1, n, -1};
    for (int i = 0; i < kBlock / 64; ++i) {
      m = fmax(m, smax[i]);
      c += sbad[i];
      for (int a = 0; a < 3; ++a) {
        b[2 * a] = min(b[2 * a], sbox[i][2 * a]);
        b[2 * a + 1] = max(b[2 * a + 1], sbox[i][2 * a + 1]);
      }
    }
    blk_max[blockIdx.x] = m;
    blk_bad[blockIdx.x] = int(c);
    for (int i = 0; i < 6; ++i) blk_box[6 * blockIdx.x + i] = b[i];
  }
}

// grid index of box point q (dense box order [bz][by][bx])
__device__ __forceinline__ long box_to_grid(long q, const Box& g) {
  const long x = q % g.bx, y = (q / g.bx) % g.by, z = q / (long(g.bx) * g.by);
  return ((z + g.z0) * g.n + (y + g.y0)) * g.n + (x + g.x0);
}

// index of box point q in the box vectors, or -1 if they do not hold it
__device__ __forceinline__ long box_to_vec(long q, const Box& g) {
  if (!g.rows) return q;
  const long r = q / g.bx;
  const int i = int(q % g.bx) - g.rows[3 * r];
  return (i >= 0 && i < g.rows[3 * r + 1]) ? long(g.rows[3 * r + 2]) + i : -1;
}

__global__ void __launch_bounds__(kBlock) k_row_support(const c128* __restrict__ H, const c128* __restrict__ Hmu,
                                                        Box g, int* __restrict__ xalen) {
  const long n3 = long(g.n) * g.n * g.n;
  const long nr = long(g.by) * g.bz;
  for (long r = long(blockIdx.x) * blockDim.x + threadIdx.x; r < nr; r += long(gridDim.x) * blockDim.x) {
    const long base = box_to_grid(r * g.bx, g);
    int lo = -1, hi = -1;
    for (int x = 0; x < g.bx; ++x) {
      bool nz = false;
      for (int e = 0; e < 9; ++e) {
        const c128 h = H[e * n3 + base + x];
        nz = nz || h.re != 0.0 || h.im != 0.0;
        if (Hmu) {
          const c128 m = Hmu[e * n3 + base + x];
          nz = nz || m.re != 0.0 || m.im != 0.0;
        }
      }
      if (nz) {
        if (lo < 0) lo = x;
        hi = x;
      }
    }
    xalen[2 * r] = lo < 0 ? 0 : lo;
    xalen[2 * r + 1] = lo < 0 ? 0 : hi - lo + 1;
  }
}

// b = 2 H g on the box; g on the whole grid [rhs][C][n^3], b in box vector layout
__global__ void __launch_bounds__(kBlock) k_rhs(const c128* __restrict__ H, const c128* __restrict__ Hmu,
                                                const c128* __restrict__ inc, c128* __restrict__ b, int nrhs,
                                                int C, Box g) {
  const long vn3 = long(g.bx) * g.by * g.bz;
  const long n3 = long(g.n) * g.n * g.n;
  const long total = long(nrhs) * (C / 3) * vn3;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long q = t % vn3;
    const long rh = t / vn3;  // rhs * (C/3) + half
    const long p = box_to_vec(q, g);
    if (p < 0) continue;
    const int half = int(rh % (C / 3));
    const c128* Hh = half == 0 ? H : Hmu;
    const long ph = box_to_grid(q, g);
    const long vb = rh * 3 * g.np + p;
    const long gb = rh * 3 * n3 + ph;
    c128 v[3];
    for (int c = 0; c < 3; ++c) v[c] = inc[gb + c * n3];
    for (int r = 0; r < 3; ++r) {
      c128 acc = {0.0, 0.0};
      for (int c = 0; c < 3; ++c) acc = acc + Hh[(3 * r + c) * n3 + ph] * v[c];
      b[vb + r * g.np] = 2.0 * acc;
    }
  }
}

// box <- grid (gather) for nv = nrhs * C components
__global__ void __launch_bounds__(kBlock) k_gather(const c128* __restrict__ full, c128* __restrict__ box, long nv,
                                                   Box g) {
  const long vn3 = long(g.bx) * g.by * g.bz;
  const long n3 = long(g.n) * g.n * g.n;
  const long total = nv * vn3;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long q = t % vn3, c = t / vn3;
    const long p = box_to_vec(q, g);
    if (p >= 0) box[c * g.np + p] = full[c * n3 + box_to_grid(q, g)];
  }
}

// grid <- box with zeros outside the box (scatter), over the whole grid
__global__ void __launch_bounds__(kBlock) k_scatter(const c128* __restrict__ box, c128* __restrict__ full, long nv,
                                                    Box g) {
  const long n3 = long(g.n) * g.n * g.n;
  const long total = nv * n3;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    const long ph = t % n3, c = t / n3;
    const int x = int(ph % g.n) - g.x0, y = int((ph / g.n) % g.n) - g.y0, z = int(ph / (long(g.n) * g.n)) - g.z0;
    c128 v = {0.0, 0.0};
    if (x >= 0 && x < g.bx && y >= 0 && y < g.by && z >= 0 && z < g.bz) {
      const long p = box_to_vec((long(z) * g.by + y) * g.bx + x, g);
      if (p >= 0) v = box[c * g.np + p];
    }
    full[t] = v;
  }
}

constexpr int kGroup = 8;  // basis vectors per accumulation sweep

// TV, TW: storage of the basis and of w (complex128 or complex64); the
// products are formed and summed in FP64.  Block (blk, rhs, z) forms the
// partial sums over chunk blk of the groups z, z + gridDim.z, ... of kGroup
// vectors: the partial of (blk, vector) is the same sum in the same order
// whatever gridDim.z is (small launches spread the groups over blocks).
template <typename TV, typename TW>
__global__ void __launch_bounds__(kBlock) k_dots(const TV* __restrict__ V, long vstride, long rstride,
                                                 const TW* __restrict__ w, long L, int nv, long chunk,
                                                 c128* __restrict__ partials, const int* __restrict__ act) {
  __shared__ double red[kBlock / 64][2 * kGroup];
  const int rhs = blockIdx.y;
  if (act && !act[rhs]) return;
  const int blk = blockIdx.x;
  const int nblk = gridDim.x;
  const long lo = long(blk) * chunk;
  const long hi = lo + chunk < L ? lo + chunk : L;
  const TW* wr = w + rhs * rstride;
  const TV* Vr = V + rhs * rstride;
  const int nv1 = nv + 1;
  c128* out = partials + (long(rhs) * nblk + blk) * nv1;
  for (int g0 = int(blockIdx.z) * kGroup; g0 < nv1; g0 += int(gridDim.z) * kGroup) {
    double ar[kGroup], ai[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q) ar[q] = ai[q] = 0.0;
    for (long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
      const c128 we = cvt<double>(wr[e]);
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
        const int i = g0 + q;
        if (i < nv) {
          const c128 v = cvt<double>(Vr[long(i) * vstride + e]);
          ar[q] += v.re * we.re + v.im * we.im;
          ai[q] += v.re * we.im - v.im * we.re;
        } else if (i == nv) {
          ar[q] += we.re * we.re + we.im * we.im;
        }
      }
    }
    const int wv = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      const double sr = wave_sum(ar[q]);
      const double si = wave_sum(ai[q]);
      if ((threadIdx.x & 63) == 0) {
        red[wv][2 * q] = sr;
        red[wv][2 * q + 1] = si;
      }
    }
    __syncthreads();
    if (threadIdx.x < kGroup && g0 + int(threadIdx.x) < nv1) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < kBlock / 64; ++k) {
        sr += red[k][2 * threadIdx.x];
        si += red[k][2 * threadIdx.x + 1];
      }
      out[g0 + threadIdx.x] = {sr, si};
    }
    __syncthreads();
  }
}

// Block (rhs, i) sums the nblk partials of coefficient i.
__global__ void __launch_bounds__(kBlock) k_reduce(const c128* __restrict__ partials, int nblk, int nv1,
                                                   c128* __restrict__ out, const int* __restrict__ act) {
  __shared__ double red[kBlock / 64][2];
  const int rhs = blockIdx.x;
  if (act && !act[rhs]) return;
  const int i = blockIdx.y;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const c128 v = partials[(long(rhs) * nblk + b) * nv1 + i];
    sr += v.re;
    si += v.im;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x / 64][0] = sr;
    red[threadIdx.x / 64][1] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) {
      a += red[k][0];
      c += red[k][1];
    }
    out[long(rhs) * nv1 + i] = {a, c};
  }
}

// TV, TW, TO: storage of the basis, of w and of out; arithmetic in FP64.
// count (optional): right-hand side r uses its first count[r] <= nv
// coefficients, and is skipped (out left as it was) when count[r] < 0.
template <typename TV, typename TW, typename TO>
__global__ void __launch_bounds__(kBlock) k_combine(const TV* __restrict__ V, long vstride, long rstride,
                                                    const TW* w, TO* out, long L, int nv,
                                                    const c128* __restrict__ coef, const double* __restrict__ scale,
                                                    const int* __restrict__ count) {
  const int rhs = blockIdx.y;
  const int nvr = count ? (count[rhs] < nv ? count[rhs] : nv) : nv;
  if (nvr < 0) return;
  const TW* wr = w + rhs * rstride;
  TO* outr = out + rhs * rstride;
  const TV* Vr = V + rhs * rstride;
  const c128* cr = coef + long(rhs) * (nv > 0 ? nv : 1);
  const double sc = scale[rhs];
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < L; e += long(gridDim.x) * blockDim.x) {
    c128 acc = cvt<double>(wr[e]);
    for (int i = 0; i < nvr; ++i) acc = acc - cvt<double>(Vr[long(i) * vstride + e]) * cr[i];
    outr[e] = cvt<decltype(TO::re)>(sc * acc);
  }
}

template <typename TV, typename TW, typename TO>
__global__ void __launch_bounds__(kBlock) k_combine_args(const TV* __restrict__ V, long vstride, long rstride,
                                                         const TW* w, TO* out, long L, int nv, CombineArgs a) {
  const int rhs = blockIdx.y;
  const int nvr = a.count[rhs] < nv ? a.count[rhs] : nv;
  if (nvr < 0) return;
  const TW* wr = w + rhs * rstride;
  TO* outr = out + rhs * rstride;
  const TV* Vr = V + rhs * rstride;
  const c128* cr = a.coef + rhs * (nv > 0 ? nv : 1);
  const double sc = a.scale[rhs];
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < L; e += long(gridDim.x) * blockDim.x) {
    c128 acc = cvt<double>(wr[e]);
    for (int i = 0; i < nvr; ++i) acc = acc - cvt<double>(Vr[long(i) * vstride + e]) * cr[i];
    outr[e] = cvt<decltype(TO::re)>(sc * acc);
  }
}

struct FlagWords {
  unsigned long long w[4];
};

__global__ void __launch_bounds__(kBlock) k_set_flags(FlagWords f, int nb, int* out) {
  for (int r = threadIdx.x; r < nb; r += blockDim.x) out[r] = int((f.w[r >> 6] >> (r & 63)) & 1ull);
}

__global__ void __launch_bounds__(kBlock) k_fill(c128* p, long n, c128 v) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) p[e] = v;
}

__global__ void __launch_bounds__(kBlock) k_copy(const c128* __restrict__ s, c128* __restrict__ d, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) d[e] = s[e];
}

__global__ void __launch_bounds__(kBlock) k_demote(const c128* __restrict__ s, c64* __restrict__ d, long n) {
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x)
    d[e] = cvt<float>(s[e]);
}

__global__ void __launch_bounds__(kBlock) k_finalize(const c128* __restrict__ buf, c128* __restrict__ tab64,
                                                     c64* __restrict__ tab32, int Q, int Z, int nxp, int ne,
                                                     double omega) {
  const long n1 = Z / 2 + 1;
  const long total = n1 * n1 * ne * nxp;
  const double sc = 1.0 / (double(Q) * double(Q) * double(Z));
  const long V = long(Z) * Q * Q;
  for (long t = long(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += long(gridDim.x) * blockDim.x) {
    // layout [qz][qy][qx < nxp][e]: the entries of one frequency point adjacent
    const int e = int(t % ne);
    long r = t / ne;
    const int qx = int(r % nxp);
    r /= nxp;
    const int qy = int(r % n1);
    const int qz = int(r / n1);
    c128 v = {0.0, 0.0};
    if (qx <= Q / 2 && qy <= Q / 2) {
      v = buf[e * V + (long(qz) * Q + qy) * Q + qx];
      double f = ((qx + qy + qz) & 1) ? -sc : sc;
      v = f * v;
      if (e >= 6) v = omega * times_i(v);
    }
    tab64[t] = v;
    tab32[t] = cvt<float>(v);
  }
}

int grid_for(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return int(b);
}

}  // namespace

// Chunks of the two-phase reductions over vectors of length L: about 8
// elements per thread, at least 64 chunks (of at least one element per
// thread) for short vectors so that a single right-hand side still spreads
// over the device, at most 1024.  A function of L alone, so that a
// right-hand side's sums do not depend on the batch it is in.
int krylov_blocks(long L) {
  long b = (L + 8 * kBlock - 1) / (8 * kBlock);
  const long lo = std::min<long>(64, (L + kBlock - 1) / kBlock);
  if (b < lo) b = lo;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return int(b);
}

hipError_t launch_contrast(const c128* coef, c128* H64, c64* H32, int n, double* blk_max, int* blk_bad,
                           int* blk_box, int nblocks, hipStream_t s) {
  k_contrast<<<nblocks, kBlock, 0, s>>>(coef, H64, H32, n, blk_max, blk_bad, blk_box);
  return hipGetLastError();
}

hipError_t launch_rhs(const c128* H, const c128* Hmu, const c128* inc, c128* b, int nrhs, int C, const Box& g,
                      hipStream_t s) {
  k_rhs<<<grid_for(long(nrhs) * (C / 3) * g.bx * g.by * g.bz), kBlock, 0, s>>>(H, Hmu, inc, b, nrhs, C, g);
  return hipGetLastError();
}

hipError_t launch_row_support(const c128* H, const c128* Hmu, const Box& g, int* xalen, hipStream_t s) {
  k_row_support<<<grid_for(long(g.by) * g.bz), kBlock, 0, s>>>(H, Hmu, g, xalen);
  return hipGetLastError();
}

hipError_t launch_gather(const c128* full, c128* box, long nv, const Box& g, hipStream_t s) {
  k_gather<<<grid_for(nv * g.bx * g.by * g.bz), kBlock, 0, s>>>(full, box, nv, g);
  return hipGetLastError();
}

hipError_t launch_scatter(const c128* box, c128* full, long nv, const Box& g, hipStream_t s) {
  k_scatter<<<grid_for(nv * g.n * g.n * g.n), kBlock, 0, s>>>(box, full, nv, g);
  return hipGetLastError();
}

template <typename TV, typename TW>
hipError_t launch_dots(const TV* V, long vstride, long rstride, const TW* w, long L, int nv, int nrhs, int nblk,
                       c128* partials, hipStream_t s, const int* act) {
  const long chunk = (L + nblk - 1) / nblk;
  // groups of kGroup vectors over blocks while the launch is short of ~4
  // blocks per compute unit
  const int ngroups = (nv + 1 + kGroup - 1) / kGroup;
  int gz = 1;
  while (gz < ngroups && long(nblk) * nrhs * gz < 1024) ++gz;
  k_dots<TV, TW><<<dim3(nblk, nrhs, gz), kBlock, 0, s>>>(V, vstride, rstride, w, L, nv, chunk, partials, act);
  return hipGetLastError();
}
template hipError_t launch_dots<c128, c128>(const c128*, long, long, const c128*, long, int, int, int, c128*,
                                            hipStream_t, const int*);
template hipError_t launch_dots<c128, c64>(const c128*, long, long, const c64*, long, int, int, int, c128*,
                                           hipStream_t, const int*);


hipError_t launch_reduce(const c128* partials, int nrhs, int nblk, int nv1, c128* out, hipStream_t s,
                         const int* act) {
  k_reduce<<<dim3(nrhs, nv1), kBlock, 0, s>>>(partials, nblk, nv1, out, act);
  return hipGetLastError();
}

template <typename TV, typename TW, typename TO>
hipError_t launch_combine(const TV* V, long vstride, long rstride, const TW* w, TO* out, long L, int nv,
                          const c128* coef, const double* scale, int nrhs, hipStream_t s, const int* count) {
  long bx = (L + kBlock - 1) / kBlock;
  if (bx > 2048) bx = 2048;
  k_combine<TV, TW, TO>
      <<<dim3(unsigned(bx), nrhs), kBlock, 0, s>>>(V, vstride, rstride, w, out, L, nv, coef, scale, count);
  return hipGetLastError();
}
#define VIE_COMBINE_INST(TV, TW, TO)                                                                        \
  template hipError_t launch_combine<TV, TW, TO>(const TV*, long, long, const TW*, TO*, long, int, const c128*, \
                                                 const double*, int, hipStream_t, const int*);
VIE_COMBINE_INST(c128, c128, c128)
VIE_COMBINE_INST(c128, c64, c128)
VIE_COMBINE_INST(c128, c64, c64)
#undef VIE_COMBINE_INST

template <typename TV, typename TW, typename TO>
hipError_t launch_combine_args(const TV* V, long vstride, long rstride, const TW* w, TO* out, long L, int nv,
                               const CombineArgs& a, int nrhs, hipStream_t s) {
  if (nrhs < 1 || nrhs > kArgRhs || nrhs * (nv > 0 ? nv : 1) > kArgCoef) return hipErrorInvalidValue;
  long bx = (L + kBlock - 1) / kBlock;
  if (bx > 2048) bx = 2048;
  k_combine_args<TV, TW, TO><<<dim3(unsigned(bx), nrhs), kBlock, 0, s>>>(V, vstride, rstride, w, out, L, nv, a);
  return hipGetLastError();
}
#define VIE_COMBINE_ARGS_INST(TV, TW, TO)                                                                       \
  template hipError_t launch_combine_args<TV, TW, TO>(const TV*, long, long, const TW*, TO*, long, int,        \
                                                      const CombineArgs&, int, hipStream_t);
VIE_COMBINE_ARGS_INST(c128, c128, c128)
VIE_COMBINE_ARGS_INST(c128, c64, c128)
VIE_COMBINE_ARGS_INST(c128, c64, c64)
#undef VIE_COMBINE_ARGS_INST

hipError_t launch_set_flags(const unsigned long long (&words)[4], int nb, int* out, hipStream_t s) {
  if (nb < 1 || nb > kMaxFlagged) return hipErrorInvalidValue;
  FlagWords f{{words[0], words[1], words[2], words[3]}};
  k_set_flags<<<1, kBlock, 0, s>>>(f, nb, out);
  return hipGetLastError();
}

hipError_t launch_fill(c128* p, long n, c128 v, hipStream_t s) {
  k_fill<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_copy(const c128* src, c128* dst, long n, hipStream_t s) {
  k_copy<<<grid_for(n), kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_demote(const c128* src, c64* dst, long n, hipStream_t s) {
  k_demote<<<grid_for(n), kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_finalize_tables(const c128* buf, c128* tab64, c64* tab32, int Q, int Z, int nxp, int ne,
                                  double omega, hipStream_t s) {
  const long total = long(Z / 2 + 1) * (Z / 2 + 1) * ne * nxp;
  k_finalize<<<grid_for(total), kBlock, 0, s>>>(buf, tab64, tab32, Q, Z, nxp, ne, omega);
  return hipGetLastError();
}

}  // namespace vie
