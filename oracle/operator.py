"""Contrast, discrete convolution and the matvec of the volume integral equations.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Equations followed:

* contrast (eq. rhodef):            H(x) = (a(x) + I)^{-1} (a(x) - I), with
  a = eps (Laplace, eq. intLap), a = eps^{-1} (Helmholtz, eq. intH),
  a = eps and a = mu (Maxwell, eq. intM / contraction_Maxwell_reduced);
* Laplace / Helmholtz (eqs. intLap, contractionK):
      J - 2 H T J = 2 H grad phi_inc,   T J = J/2 + grad div V J,
  i.e.  A J = J - H (J + 2 U),  U = grad div V J.  For Helmholtz the printed
  summary eq. intH carries a "+" in front of the operator; the derivation
  just before it (multiplying by -2 (eps^{-1} + I)^{-1}) gives "-", which is
  the sign used here (it also reduces to the Laplace equation as omega -> 0);
* reduced Maxwell, mu = I (eq. contraction_Maxwell_reduced):
      A J = J - H (J + 2 U),  U = (grad div + omega^2) V J;
* full Maxwell (eq. intM):
      y_J = J - H_eps (J + 2 U_J + 2 i omega W_M),
      y_M = M - H_mu  (M + 2 U_M - 2 i omega W_J),
  with U = (grad div + omega^2) V and W = curl V;
* right-hand side 2 H g (g = grad phi_inc, or E_inc / H_inc);
* total field (eqs. represent_Maxwell, represent_Maxwell_reduced and
  grad phi = grad phi_inc + grad div V J):
      c = 3:  g + U;      full Maxwell:  E_inc + U_J + i omega W_M,  H_inc + U_M - i omega W_J.

Densities are arrays [c][n][n][n] (components x, y, z; axes z, y, x).
"""

from __future__ import annotations

import math

import numpy as np

from . import tables as tb
from .symbol import SYM_ENTRIES

KIND_LAPLACE, KIND_HELMHOLTZ, KIND_MAXWELL = 0, 1, 2


# ----------------------------------------------------------------------------
# contrast
# ----------------------------------------------------------------------------

def contrast(coef: np.ndarray) -> np.ndarray:
    """H = (a + I)^{-1}(a - I) at every grid point; coef and result are [9][n][n][n]."""
    n = coef.shape[-1]
    a = np.moveaxis(coef.reshape(3, 3, -1), -1, 0)          # (pts, 3, 3)
    eye = np.eye(3)[None]
    H = np.linalg.solve(a + eye, a - eye)
    return np.ascontiguousarray(np.moveaxis(H, 0, -1).reshape(9, n, n, n))


def contrast_norm_max(H: np.ndarray) -> float:
    """max over grid points of the spectral norm ||H(x)||_2 (Lemma 1 asks for < 1)."""
    h = np.moveaxis(H.reshape(3, 3, -1), -1, 0)
    return float(np.max(np.linalg.norm(h, ord=2, axis=(1, 2))))


def pointwise(H: np.ndarray, v: np.ndarray) -> np.ndarray:
    """(H v)_a = sum_b H_ab v_b at every point."""
    Hm = H.reshape(3, 3, *H.shape[1:])
    return np.einsum("ab...,b...->a...", Hm, v)


# ----------------------------------------------------------------------------
# scalar convolutions U(i) = sum_j K_{i-j} f(j)
# ----------------------------------------------------------------------------

def conv_direct(K: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Direct sum over the non-zero source points of f; K is the window table."""
    n = f.shape[-1]
    out = np.zeros(f.shape, dtype=np.complex128)
    for (jz, jy, jx) in np.argwhere(f != 0):
        out += K[n - 1 - jz:2 * n - 1 - jz, n - 1 - jy:2 * n - 1 - jy,
                 n - 1 - jx:2 * n - 1 - jx] * f[jz, jy, jx]
    return out


def conv_direct_at(K: np.ndarray, f: np.ndarray, point) -> complex:
    """U at one output point i: sum over all j of K[i - j] f[j]."""
    n = f.shape[-1]
    iz, iy, ix = point
    Kr = K[iz:iz + n, iy:iy + n, ix:ix + n][::-1, ::-1, ::-1]
    return complex(np.sum(Kr * f))


def window_transform(K: np.ndarray) -> np.ndarray:
    """FFT of the window placed (wrapped) on the 2n grid, zero at offset n."""
    n = (K.shape[-1] + 1) // 2
    P = 2 * n
    idx = np.arange(-(n - 1), n) % P
    Kp = np.zeros((P, P, P), dtype=np.complex128)
    Kp[np.ix_(idx, idx, idx)] = K
    return tb.fftn(Kp)


def conv_fft_window_hat(Khat: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Circular convolution on the 2n grid with a transformed window, cropped to n."""
    n = f.shape[-1]
    P = 2 * n
    fp = np.zeros((P, P, P), dtype=np.complex128)
    fp[:n, :n, :n] = f
    return tb.ifftn(Khat * tb.fftn(fp))[:n, :n, :n]


def conv_fft_window(K: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Same sum with the window placed (wrapped) on a 2n grid and FFTs; zero at offset n."""
    return conv_fft_window_hat(window_transform(K), f)


def conv_fft_mgrid(F: np.ndarray, f: np.ndarray) -> np.ndarray:
    """crop_n IFFT_M[F . FFT_M(pad_M f)] with F the sampled symbol on the M grid."""
    n = f.shape[-1]
    M = F.shape[0]
    fp = np.zeros((M, M, M), dtype=np.complex128)
    fp[:n, :n, :n] = f
    return tb.ifftn(F * tb.fftn(fp))[:n, :n, :n]


# ----------------------------------------------------------------------------
# vector operators built from the tables
# ----------------------------------------------------------------------------

def _sym_index(a: int, b: int) -> int:
    for e, (p, q) in enumerate(SYM_ENTRIES):
        if (p, q) == (a, b) or (q, p) == (a, b):
            return e
    raise KeyError


LEVI = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}


class Convolver:
    """Applies the symmetric (grad/D) and curl operators with a chosen route.

    route 'direct': direct sum (tiny grids, or sparse sources);
    route 'window': FFT of the window on the 2n grid;
    route 'mgrid' : FFT on the oversampled M grid with the sampled symbol.
    """

    def __init__(self, kind_sym: str, n: int, h: float, omega: float, route: str = "window",
                 with_curl: bool = False, R: float = None, M: int = None):
        self.n, self.h, self.omega, self.route = n, h, omega, route
        self.kind_sym = kind_sym
        self.with_curl = with_curl
        if route == "mgrid":
            self.sym = tb.sampled_symbol(kind_sym, n, h, omega, R, M)
            self.curl = tb.sampled_symbol("curl", n, h, omega, R, M) if with_curl else None
        else:
            self.sym = tb.kernel_tables(kind_sym, n, h, omega, R, M)
            self.curl = tb.kernel_tables("curl", n, h, omega, R, M) if with_curl else None
        if route == "window":
            # transform each window once; the convolution then needs 2 FFTs
            self.sym = [window_transform(K) for K in self.sym]
            self.curl = [window_transform(K) for K in self.curl] if with_curl else None
        self._conv = {"direct": conv_direct, "window": conv_fft_window_hat, "mgrid": conv_fft_mgrid}[route]

    def spectra(self, J: np.ndarray):
        """Window route: the transform of each zero-padded component on the 2n grid."""
        n, P = self.n, 2 * self.n
        out = []
        for b in range(J.shape[0]):
            fp = np.zeros((P, P, P), dtype=np.complex128)
            fp[:n, :n, :n] = J[b]
            out.append(tb.fftn(fp))
        return out

    def _crop_inverse(self, spec: np.ndarray) -> np.ndarray:
        n = self.n
        return tb.ifftn(spec)[:n, :n, :n]

    def sym_apply(self, J: np.ndarray, Jh=None) -> np.ndarray:
        """U_a = sum_b K^{ab} * J_b.  Window route: by the convolution theorem,
        U_a = crop IFFT(sum_b K^_ab J^_b) with J^_b = FFT(pad J_b) (Jh: these
        transforms, when already computed)."""
        U = np.zeros(J.shape, dtype=np.complex128)
        if self.route == "window":
            Jh = self.spectra(J) if Jh is None else Jh
            for a in range(3):
                acc = self.sym[_sym_index(a, 0)] * Jh[0]
                for b in (1, 2):
                    acc += self.sym[_sym_index(a, b)] * Jh[b]
                U[a] = self._crop_inverse(acc)
            return U
        for a in range(3):
            for b in range(3):
                U[a] += self._conv(self.sym[_sym_index(a, b)], J[b])
        return U

    def curl_apply(self, J: np.ndarray, Jh=None) -> np.ndarray:
        """W_a = sum_bc eps_abc C_b * J_c (window route: one inverse transform per a)."""
        W = np.zeros(J.shape, dtype=np.complex128)
        if self.route == "window":
            Jh = self.spectra(J) if Jh is None else Jh
            for a in range(3):
                acc = np.zeros_like(Jh[0])
                for (p, b, c), sgn in LEVI.items():
                    if p == a:
                        acc += sgn * (self.curl[b] * Jh[c])
                W[a] = self._crop_inverse(acc)
            return W
        for (a, b, c), sgn in LEVI.items():
            W[a] += sgn * self._conv(self.curl[b], J[c])
        return W


def symbol_kind(kind: int) -> str:
    return "D" if kind == KIND_MAXWELL else "grad"


class Operator:
    """The discrete operator A of the integral equation and its field map."""

    def __init__(self, kind: int, coef: np.ndarray, omega: float, mu: np.ndarray = None,
                 h: float = None, route: str = "window", R: float = None, M: int = None):
        self.kind = kind
        self.n = coef.shape[-1]
        self.h = 2.0 / self.n if h is None else h
        self.omega = 0.0 if kind == KIND_LAPLACE else float(omega)
        self.full = mu is not None
        if self.full and kind != KIND_MAXWELL:
            raise ValueError("mu is only meaningful for Maxwell")
        self.H = contrast(coef)
        self.Hmu = contrast(mu) if self.full else None
        self.conv = Convolver(symbol_kind(kind), self.n, self.h, self.omega, route,
                              with_curl=self.full, R=R, M=M)

    @property
    def ncomp(self) -> int:
        return 6 if self.full else 3

    def _spectra(self, v):
        return self.conv.spectra(v) if self.conv.route == "window" else None

    def apply(self, x: np.ndarray) -> np.ndarray:
        if not self.full:
            U = self.conv.sym_apply(x)
            return x - pointwise(self.H, x + 2.0 * U)
        w = self.omega
        J, M = x[:3], x[3:]
        Jh, Mh = self._spectra(J), self._spectra(M)
        UJ, UM = self.conv.sym_apply(J, Jh), self.conv.sym_apply(M, Mh)
        WJ, WM = self.conv.curl_apply(J, Jh), self.conv.curl_apply(M, Mh)
        yJ = J - pointwise(self.H, J + 2.0 * UJ + 2j * w * WM)
        yM = M - pointwise(self.Hmu, M + 2.0 * UM - 2j * w * WJ)
        return np.concatenate([yJ, yM])

    def rhs(self, inc: np.ndarray) -> np.ndarray:
        if not self.full:
            return 2.0 * pointwise(self.H, inc)
        return np.concatenate([2.0 * pointwise(self.H, inc[:3]), 2.0 * pointwise(self.Hmu, inc[3:])])

    def field(self, x: np.ndarray, inc: np.ndarray) -> np.ndarray:
        if not self.full:
            return inc + self.conv.sym_apply(x)
        w = self.omega
        J, M = x[:3], x[3:]
        Jh, Mh = self._spectra(J), self._spectra(M)
        E = inc[:3] + self.conv.sym_apply(J, Jh) + 1j * w * self.conv.curl_apply(M, Mh)
        Hf = inc[3:] + self.conv.sym_apply(M, Mh) - 1j * w * self.conv.curl_apply(J, Jh)
        return np.concatenate([E, Hf])
