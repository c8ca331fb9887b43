// Per-length kernel registry.  Each supported FFT length P = P1 * P2 is
// compiled in its own translation unit (len_<P>.hip) which registers launch
// functions for every kernel of that length at library load.
#pragma once

#include <hip/hip_runtime.h>

#include "apply_kernels.hpp"
#include "fft.hpp"
#include "symbol.hpp"

namespace vie {

// Source functor of the first precompute pass: symbol samples on the M^3
// frequency grid, odd entries zeroed on their Nyquist planes, modulated by
// exp(-2 pi i (ix shx + iy shy + iz shz) / M) so that the inverse
// transform's first P_a outputs along axis a are the displacements
// -P_a / 2 .. P_a / 2 - 1 (sh_a = P_a / 2).
struct SymbolSrc {
  int M;
  int set;      // SYM_GRAD or SYM_MAXWELL
  int entry0;   // table entry of group 0
  int shx, shy, shz;  // P_x / 2, P_y / 2, P_z / 2
  double h, w, R;
  struct Col {
    const SymbolSrc* s;
    long g, c;
    template <typename Rt>
    __device__ __forceinline__ cx<Rt> load(int n) const {
      return s->template load<Rt>(g, c, n);
    }
  };
  __device__ __forceinline__ Col column(long g, long c) const { return {this, g, c}; }
  // g = table entry - entry0, c = row index iz * M + iy, n = ix
  template <typename Rt>
  __device__ __forceinline__ cx<Rt> load(long g, long c, int n) const {
    const int e = entry0 + int(g);
    const int ix = n, iy = int(c % M), iz = int(c / M);
    const int half = M / 2;
    if ((ix == half && symbol_odd_in_set(set, e, 0)) || (iy == half && symbol_odd_in_set(set, e, 1)) ||
        (iz == half && symbol_odd_in_set(set, e, 2)))
      return czero<Rt>();
    const double ds = 2.0 * kPi / (double(M) * h);
    const double sx = ds * double(ix < half ? ix : ix - M);
    const double sy = ds * double(iy < half ? iy : iy - M);
    const double sz = ds * double(iz < half ? iz : iz - M);
    c128 v = symbol_entry(set, e, sx, sy, sz, w, R);
    // phase -2 pi q / M
    const long q = (long(ix) * shx + long(iy) * shy + long(iz) * shz) % M;
    if ((4 * q) % M == 0) {
      switch (int(4 * q / M)) {
        case 1: v = times_mi(v); break;
        case 2: v = -v; break;
        case 3: v = times_i(v); break;
        default: break;
      }
    } else {
      double sn, cs;
      sincospi(-2.0 * double(q) / double(M), &sn, &cs);
      v = c128{v.re * cs - v.im * sn, v.re * sn + v.im * cs};
    }
    return cvt<Rt>(v);
  }
};

template <typename R>
struct LenOps {
  int P = 0, P1 = 0, P2 = 0;
  // x-axis forward pass reading complex128 input
  hipError_t (*contig_fwd)(MemLoad<c128>, MemStore<cx<R>>, Geo, long ngroups, const cx<R>*, hipStream_t) = nullptr;
  // y/z-axis pass, forward or inverse
  hipError_t (*strided)(bool inv, MemLoad<cx<R>>, MemStore<cx<R>>, Geo, long ngroups, const cx<R>*,
                        hipStream_t) = nullptr;
  // fused z pass, mul = MUL_SYM3 or MUL_MAX6
  hipError_t (*zpass)(int mul, cx<R>*, const cx<R>*, ZArgs, long nblocks, const cx<R>*, hipStream_t) = nullptr;
  // last inverse x pass with combine, C in {3, 6}, mode MODE_*
  hipError_t (*xinv)(int C, int mode, const cx<R>*, XArgs, const c128*, const c128*, const cx<R>*, const cx<R>*,
                     c128*, const cx<R>*, hipStream_t) = nullptr;
  // x-axis forward pass reading the support rows of complex128 vectors
  hipError_t (*contig_fwd_rows)(RowLoad<c128>, MemStore<cx<R>>, Geo, long ngroups, const cx<R>*, hipStream_t) = nullptr;
  // the same two passes with the vectors stored as complex64 (the FP32 Krylov
  // basis of the mixed solver; float only, MODE_MATVEC only)
  hipError_t (*contig_fwd_v32)(MemLoad<c64>, MemStore<cx<R>>, Geo, long ngroups, const cx<R>*, hipStream_t) = nullptr;
  hipError_t (*xinv_v32)(int C, const cx<R>*, XArgs, const c64*, const cx<R>*, const cx<R>*, c64*, const cx<R>*,
                         hipStream_t) = nullptr;
  // the FP32 matvec reading complex128 vectors and writing complex64 (float only, MODE_MATVEC)
  hipError_t (*xinv_w32)(int C, const cx<R>*, XArgs, const c128*, const cx<R>*, const cx<R>*, c64*, const cx<R>*,
                         hipStream_t) = nullptr;
  // precompute: inverse x pass of length M fed by the symbol (double only)
  hipError_t (*symbol_inv)(SymbolSrc, MemStore<c128>, Geo, long ngroups, const c128*, hipStream_t) = nullptr;
};

// Each length may be compiled with more than one split P = P1 x P2 (variant
// 0: the one of the precompute; variant 1: an alternative the autotuner may
// pick per pass).
constexpr int kMaxLen = 640;
constexpr int kMaxSplits = 2;
template <typename R>
LenOps<R>* len_table();  // [kMaxLen + 1][kMaxSplits]

template <typename R>
inline const LenOps<R>* len_ops(int P, int variant = 0) {
  if (P < 0 || P > kMaxLen || variant < 0 || variant >= kMaxSplits) return nullptr;
  const LenOps<R>* o = &len_table<R>()[P * kMaxSplits + variant];
  return o->P == P ? o : nullptr;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <typename R, int P1, int P2, bool CONTIG>
inline size_t pass_lds_bytes(int T) {
  return sizeof(cx<R>) * (size_t(P1 * P2) + size_t(T) * lds_elems_per_col<P1, P2>(CONTIG));
}

template <typename R, int P1, int P2>
struct LenImpl {
  static constexpr int P = P1 * P2;
  static constexpr int J = P1 > P2 ? P1 : P2;

  static hipError_t contig_fwd(MemLoad<c128> src, MemStore<cx<R>> dst, Geo geo, long ngroups, const cx<R>* tw,
                               hipStream_t s) {
    const long blocks = long(geo.ntiles) * ngroups;
    k_pass<R, P1, P2, true, false, MemLoad<c128>, MemStore<cx<R>>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<R, P1, P2, true>(geo.T), s>>>(src, dst, geo, tw);
    return hipGetLastError();
  }
  static hipError_t contig_fwd_rows(RowLoad<c128> src, MemStore<cx<R>> dst, Geo geo, long ngroups,
                                    const cx<R>* tw, hipStream_t s) {
    const long blocks = long(geo.ntiles) * ngroups;
    k_pass<R, P1, P2, true, false, RowLoad<c128>, MemStore<cx<R>>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<R, P1, P2, true>(geo.T), s>>>(src, dst, geo, tw);
    return hipGetLastError();
  }
  static hipError_t contig_fwd_v32(MemLoad<c64> src, MemStore<cx<R>> dst, Geo geo, long ngroups, const cx<R>* tw,
                                   hipStream_t s) {
    const long blocks = long(geo.ntiles) * ngroups;
    k_pass<R, P1, P2, true, false, MemLoad<c64>, MemStore<cx<R>>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<R, P1, P2, true>(geo.T), s>>>(src, dst, geo, tw);
    return hipGetLastError();
  }
  static hipError_t xinv_v32(int C, const cx<R>* A, XArgs a, const c64* J_, const cx<R>* H, const cx<R>* Hmu,
                             c64* out, const cx<R>* tw, hipStream_t s) {
    const long blocks = xinv_blocks(a);
    if (C == 3)
      k_xinv<R, P1, P2, 3, MODE_MATVEC, c64><<<dim3(unsigned(blocks)), dim3(a.T * J), pass_lds_bytes<R, P1, P2, true>(a.T), s>>>(A, a, J_, nullptr, H, Hmu, out, tw);
    else if (C == 6)
      k_xinv<R, P1, P2, 6, MODE_MATVEC, c64><<<dim3(unsigned(blocks)), dim3(a.T * J), pass_lds_bytes<R, P1, P2, true>(a.T), s>>>(A, a, J_, nullptr, H, Hmu, out, tw);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  static hipError_t xinv_w32(int C, const cx<R>* A, XArgs a, const c128* J_, const cx<R>* H, const cx<R>* Hmu,
                             c64* out, const cx<R>* tw, hipStream_t s) {
    const long blocks = xinv_blocks(a);
    if (C == 3)
      k_xinv<R, P1, P2, 3, MODE_MATVEC, c128, c64><<<dim3(unsigned(blocks)), dim3(a.T * J), pass_lds_bytes<R, P1, P2, true>(a.T), s>>>(A, a, J_, nullptr, H, Hmu, out, tw);
    else if (C == 6)
      k_xinv<R, P1, P2, 6, MODE_MATVEC, c128, c64><<<dim3(unsigned(blocks)), dim3(a.T * J), pass_lds_bytes<R, P1, P2, true>(a.T), s>>>(A, a, J_, nullptr, H, Hmu, out, tw);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  static hipError_t strided(bool inv, MemLoad<cx<R>> src, MemStore<cx<R>> dst, Geo geo, long ngroups,
                            const cx<R>* tw, hipStream_t s) {
    const long blocks = long(geo.ntiles) * ngroups;
    if (inv && 2 * geo.nout > P) return hipErrorInvalidValue;  // inverse passes keep outputs < P / 2
    if (inv)
      k_pass<R, P1, P2, false, true, MemLoad<cx<R>>, MemStore<cx<R>>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<R, P1, P2, false>(geo.T), s>>>(src, dst, geo, tw);
    else
      k_pass<R, P1, P2, false, false, MemLoad<cx<R>>, MemStore<cx<R>>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<R, P1, P2, false>(geo.T), s>>>(src, dst, geo, tw);
    return hipGetLastError();
  }
  static hipError_t zpass(int mul, cx<R>* buf, const cx<R>* tab, ZArgs a, long nblocks, const cx<R>* tw,
                          hipStream_t s) {
    // the z fold needs P1 and P2 even
    if constexpr (P1 % 2 != 0 || P2 % 2 != 0) {
      (void)mul; (void)buf; (void)tab; (void)a; (void)nblocks; (void)tw; (void)s;
      return hipErrorInvalidValue;
    } else {
    // the kernel takes the table geometry from P
    if (2 * a.n != P || a.nxp != ((a.n + 1 + 15) / 16) * 16 || a.ne != mul_entries(mul) || 2 * a.nz > P ||
        a.pxy > P || a.pxy % 2 != 0)
      return hipErrorInvalidValue;
    if (a.quad) {
      if (a.ntx != (a.pxy / 2 + a.T - 1) / a.T || a.ngroups != long(a.pxy / 2) * a.ntx ||
          nblocks != (a.ngroups + 7) / 8 * 8 * 4 * a.nb)
        return hipErrorInvalidValue;
    } else if (a.ntiles != (a.pxy + a.T - 1) / a.T || nblocks != long(a.ntiles) * a.pxy * a.nb ||
               (long(a.ntiles) * a.pxy) % 8 != 0) {
      return hipErrorInvalidValue;
    }
    const size_t lds = pass_lds_bytes<R, P1, P2, false>(a.T);
    // the solver's usual tile width has its own compiled kernel
    constexpr int TC = std::is_same<R, float>::value ? 16 : 8;
    const dim3 grid{unsigned(nblocks)}, block{unsigned(a.T * J)};
    if (mul == MUL_SYM3) {
      if (a.T == TC)
        k_zpass<R, P1, P2, 3, MUL_SYM3, TC><<<grid, block, lds, s>>>(buf, tab, a, tw);
      else
        k_zpass<R, P1, P2, 3, MUL_SYM3><<<grid, block, lds, s>>>(buf, tab, a, tw);
    } else if (mul == MUL_MAX6) {
      if (a.T == TC)
        k_zpass<R, P1, P2, 6, MUL_MAX6, TC><<<grid, block, lds, s>>>(buf, tab, a, tw);
      else
        k_zpass<R, P1, P2, 6, MUL_MAX6><<<grid, block, lds, s>>>(buf, tab, a, tw);
    } else {
      // potentials and the reduced Maxwell H field: FP64 only
      if constexpr (std::is_same<R, double>::value) {
        if (mul == MUL_DIV)
          k_zpass<R, P1, P2, 3, MUL_DIV><<<dim3(unsigned(nblocks)), dim3(a.T * J), lds, s>>>(buf, tab, a, tw);
        else if (mul == MUL_CURLH)
          k_zpass<R, P1, P2, 3, MUL_CURLH><<<dim3(unsigned(nblocks)), dim3(a.T * J), lds, s>>>(buf, tab, a, tw);
        else
          return hipErrorInvalidValue;
      } else {
        return hipErrorInvalidValue;
      }
    }
    return hipGetLastError();
    }
  }
  template <int C, int MODE>
  static void xinv_launch(const cx<R>* A, XArgs a, const c128* J_, const c128* B, const cx<R>* H, const cx<R>* Hmu,
                          c128* out, const cx<R>* tw, hipStream_t s) {
    const long blocks = xinv_blocks(a);
    k_xinv<R, P1, P2, C, MODE><<<dim3(unsigned(blocks)), dim3(a.T * J), pass_lds_bytes<R, P1, P2, true>(a.T), s>>>(A, a, J_, B, H, Hmu, out, tw);
  }
  static hipError_t xinv(int C, int mode, const cx<R>* A, XArgs a, const c128* J_, const c128* B, const cx<R>* H,
                         const cx<R>* Hmu, c128* out, const cx<R>* tw, hipStream_t s) {
#define VIE_XINV_CASE(CC, MM) \
  if (C == CC && mode == MM) { xinv_launch<CC, MM>(A, a, J_, B, H, Hmu, out, tw, s); return hipGetLastError(); }
    VIE_XINV_CASE(3, MODE_MATVEC)
    VIE_XINV_CASE(3, MODE_FIELD)
    VIE_XINV_CASE(3, MODE_CONV)
    VIE_XINV_CASE(3, MODE_RESIDUAL)
    VIE_XINV_CASE(6, MODE_MATVEC)
    VIE_XINV_CASE(6, MODE_FIELD)
    VIE_XINV_CASE(6, MODE_CONV)
    VIE_XINV_CASE(6, MODE_RESIDUAL)
#undef VIE_XINV_CASE
    return hipErrorInvalidValue;
  }
  static hipError_t symbol_inv(SymbolSrc src, MemStore<c128> dst, Geo geo, long ngroups, const c128* tw,
                               hipStream_t s) {
    const long blocks = long(geo.ntiles) * ngroups;
    if (2 * geo.nout > P) return hipErrorInvalidValue;
    k_pass<double, P1, P2, true, true, SymbolSrc, MemStore<c128>><<<dim3(unsigned(blocks)), dim3(geo.T * J), pass_lds_bytes<double, P1, P2, true>(geo.T), s>>>(src, dst, geo, tw);
    return hipGetLastError();
  }

  // register the apply kernels and, for double, the precompute passes
  template <bool APPLY, bool SYMBOL>
  static void register_all(int variant = 0) {
    LenOps<R>& o = len_table<R>()[P * kMaxSplits + variant];
    o.P = P;
    o.P1 = P1;
    o.P2 = P2;
    o.strided = &strided;
    if constexpr (APPLY) {
      o.contig_fwd = &contig_fwd;
      o.contig_fwd_rows = &contig_fwd_rows;
      o.zpass = &zpass;
      o.xinv = &xinv;
      if constexpr (std::is_same<R, float>::value) {
        o.contig_fwd_v32 = &contig_fwd_v32;
        o.xinv_v32 = &xinv_v32;
        o.xinv_w32 = &xinv_w32;
      }
    }
    if constexpr (SYMBOL && std::is_same<R, double>::value) o.symbol_inv = &symbol_inv;
  }
};

// Registers length P1*P2.  APPLY: apply kernels in FP32 and FP64 (and the FP64
// forward passes of the precompute).  SYMBOL: the FP64 symbol pass and
// strided inverse used as the oversampled length M.
#define VIE_REGISTER_LEN(P1_, P2_, APPLY_, SYMBOL_)                                  \
  namespace {                                                                        \
  struct RegLen##P1_##x##P2_ {                                                       \
    RegLen##P1_##x##P2_() {                                                          \
      if constexpr (APPLY_) vie::LenImpl<float, P1_, P2_>::register_all<true, false>(); \
      vie::LenImpl<double, P1_, P2_>::register_all<APPLY_, SYMBOL_>();                 \
    }                                                                                \
  } reg_len_##P1_##x##P2_;                                                           \
  }

// Registers the split P1 x P2 of a length already registered with another
// split, as variant 1 (apply kernels in FP32 and FP64 only).
#define VIE_REGISTER_SPLIT(P1_, P2_)                                                  \
  namespace {                                                                        \
  struct RegSplit##P1_##x##P2_ {                                                     \
    RegSplit##P1_##x##P2_() {                                                        \
      vie::LenImpl<float, P1_, P2_>::register_all<true, false>(1);                   \
      vie::LenImpl<double, P1_, P2_>::register_all<true, false>(1);                  \
    }                                                                                \
  } reg_split_##P1_##x##P2_;                                                         \
  }

}  // namespace vie
