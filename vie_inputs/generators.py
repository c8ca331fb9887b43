"""Seeded synthetic media, incident fields and densities.

Every array uses the solver's layout: components first, then z, y, x with x
the fastest axis, complex128.  A tensor field is stored as ``[9][n][n][n]``
with entry (a, b) of the 3x3 matrix at index ``3*a + b``.

Grid: the box [-1, 1]^3 is sampled cell-centred, x_i = origin + (i + 1/2) h
with origin = -1 and h = 2/n (the grid placement is a reading of the paper's
"uniform n x n x n mesh", Section 5).

Seeds: ``numpy.random.SeedSequence([180504791, config_id, item])``.  Item 0
of a configuration draws the medium, item 1 + j draws right-hand side j.
The draw order inside each helper is written in its docstring and never
changes, so that every consumer sees identical inputs.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_ROOT = 180504791

# configuration ids used in the seed sequence
CONFIG_IDS = {
    "laplace32": 1,      # anisotropic Laplace, 32^3, FP64
    "helmholtz64": 2,    # anisotropic Helmholtz, 64^3, omega = 4 pi
    "maxwell128": 3,     # anisotropic Maxwell (eps and mu), 128^3, omega = 8 pi
    "batched96": 4,      # Helmholtz, 96^3, omega = 6 pi, 64 right-hand sides
    "serving": 5,        # request stream
    "helmholtz128": 6,   # Helmholtz recipe at 128^3, omega = 8 pi
    "test": 7,           # free-form test inputs
}

KIND_LAPLACE = 0
KIND_HELMHOLTZ = 1
KIND_MAXWELL = 2


def rng_for(config_id: int, item: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(config_id), int(item)]))


# ----------------------------------------------------------------------------
# grid and bump
# ----------------------------------------------------------------------------

def grid_spacing(n: int, width: float = 2.0) -> float:
    return width / n


def grid_axis(n: int, origin: float = -1.0, h: Optional[float] = None) -> np.ndarray:
    """Cell-centred sample positions along one axis."""
    if h is None:
        h = grid_spacing(n)
    return origin + (np.arange(n, dtype=np.float64) + 0.5) * h


def grid_coords(n: int, origin: float = -1.0, h: Optional[float] = None):
    """Return X, Y, Z arrays of shape (n, n, n) indexed [z][y][x]."""
    t = grid_axis(n, origin, h)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    return X, Y, Z


def grid_coords_plane(n: int, origin: float = -1.0, h: Optional[float] = None):
    """X, Y, Z of the z = 0 plane, shape (1, n, n) indexed [z][y][x]."""
    t = grid_axis(n, origin, h)
    Z, Y, X = np.meshgrid(t[:1], t, t, indexing="ij")
    return X, Y, Z


def bump(X, Y, Z, radius: float = 0.8) -> np.ndarray:
    """C-infinity bump exp(1 - 1/(1 - |x|^2/radius^2)) inside the ball, 0 outside; b(0) = 1."""
    q = (X * X + Y * Y + Z * Z) / (radius * radius)
    out = np.zeros_like(q)
    inside = q < 1.0
    out[inside] = np.exp(1.0 - 1.0 / (1.0 - q[inside]))
    return out


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Draws a 3x3 standard normal matrix; Q of its QR with sign(diag R) made positive."""
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def random_unit(rng: np.random.Generator) -> np.ndarray:
    """Draws a standard normal 3-vector and normalises it."""
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def tensor_field(const_part: np.ndarray, b: np.ndarray, mat) -> np.ndarray:
    """I * const_part + b(x) * mat(x) as a [9][n][n][n] complex128 array.

    ``mat`` is either a constant 3x3 matrix or an array [3][3][n][n][n].
    """
    n = b.shape[0]
    out = np.zeros((3, 3) + b.shape, dtype=np.complex128)
    mat = np.asarray(mat)
    for a in range(3):
        for c in range(3):
            m = mat[a, c]
            out[a, c] = b * m
            if a == c:
                out[a, c] += const_part
    return np.ascontiguousarray(out.reshape((9, n, n, n)))


def identity_field(n: int) -> np.ndarray:
    b = np.zeros((n, n, n))
    return tensor_field(1.0, b, np.zeros((3, 3)))


# ----------------------------------------------------------------------------
# media recipes
# ----------------------------------------------------------------------------

def laplace_matrix(rng: np.random.Generator) -> np.ndarray:
    """A = Q diag(lam) Q^T, lam ~ U[0.5, 2]; draw order: lam (3 uniforms), then Q (9 normals)."""
    lam = rng.uniform(0.5, 2.0, 3)
    q = random_rotation(rng)
    return (q @ np.diag(lam) @ q.T).astype(np.complex128)


def laplace_medium(n: int, rng: np.random.Generator) -> np.ndarray:
    """eps(x) = I + b(x) A with A from ``laplace_matrix``."""
    A = laplace_matrix(rng)
    X, Y, Z = grid_coords(n)
    return tensor_field(1.0, bump(X, Y, Z), A)


def helmholtz_matrix(rng: np.random.Generator, norm: float = 0.5, loss: float = 0.05) -> np.ndarray:
    """A + i*loss*I, A = norm * S/||S||_2, S = sym(G), G standard normal; draw order: G (9 normals)."""
    g = rng.standard_normal((3, 3))
    s = 0.5 * (g + g.T)
    A = norm * s / np.max(np.abs(np.linalg.eigvalsh(s)))
    return A + 1j * loss * np.eye(3)


def helmholtz_medium(n: int, rng: np.random.Generator, norm: float = 0.5,
                     loss: float = 0.05) -> np.ndarray:
    """eps^{-1}(x) = I + b(x) M with M from ``helmholtz_matrix``."""
    M = helmholtz_matrix(rng, norm, loss)
    X, Y, Z = grid_coords(n)
    return tensor_field(1.0, bump(X, Y, Z), M)


def sheared_matrix(rng: np.random.Generator, norm: float = 0.5, shear: float = 0.8,
                   loss: float = 0.05) -> np.ndarray:
    """A non-symmetric 3x3 matrix: a rotation composed with a shear, scaled to
    spectral norm ``norm``, plus i*loss*I.  N = Q S with Q from
    ``random_rotation`` and S = I + shear e_x e_y^T.  Draw order: Q (9 normals).
    With norm <= 0.5 the symmetric part of I + b N stays positive definite for
    0 <= b <= 1, so the contrast is a contraction (Lemma 1)."""
    q = random_rotation(rng)
    s = np.eye(3)
    s[0, 1] = shear
    N = q @ s
    N = norm * N / np.linalg.norm(N, 2)
    return N + 1j * loss * np.eye(3)


def sheared_medium(n: int, rng: np.random.Generator, norm: float = 0.5) -> np.ndarray:
    """I + b(x) N with N from ``sheared_matrix``: a tensor field that is not
    (complex-)symmetric at any point of the bump, so that H and H^T differ."""
    N = sheared_matrix(rng, norm)
    X, Y, Z = grid_coords(n)
    return tensor_field(1.0, bump(X, Y, Z), N)


def rot1(theta):
    """Rotation about the first axis (Section 5, dense medium)."""
    c, s = np.cos(theta), np.sin(theta)
    o, z = np.ones_like(theta), np.zeros_like(theta)
    return np.array([[o, z, z], [z, c, -s], [z, s, c]])


def rot2(phi):
    """Rotation about the third axis (Section 5, dense medium)."""
    c, s = np.cos(phi), np.sin(phi)
    o, z = np.ones_like(phi), np.zeros_like(phi)
    return np.array([[c, -s, z], [s, c, z], [z, z, o]])


def _rotated_field(X, Y, diag: np.ndarray) -> np.ndarray:
    """R(x) diag R(x)^T with R(x) = R2(pi x) R1(pi y), as [3][3][1][n][n]:
    it depends on (x, y) only, so it is formed on one z plane and broadcast."""
    X2, Y2 = X[:1], Y[:1]
    R = np.einsum("ab...,bc...->ac...", rot2(np.pi * X2), rot1(np.pi * Y2))
    return np.einsum("ab...,b,cb...->ac...", R, diag, R)


def maxwell_medium(n: int, rng: np.random.Generator, with_mu: bool = True):
    """eps = I + b R (D_eps + 0.05i) R^T, mu = I + b R (D_mu + 0.02i) R^T.

    R(x) = R2(pi x) R1(pi y) (the rotation field of the paper's dense medium).
    Draw order: D_eps (3 uniforms in [0, 1]), D_mu (3 uniforms in [0, 0.5]).
    Returns (eps, mu) (mu None without with_mu; the draws are the same).
    """
    d_eps = rng.uniform(0.0, 1.0, 3)
    d_mu = rng.uniform(0.0, 0.5, 3)
    X, Y, Z = grid_coords(n)
    b = bump(X, Y, Z)
    eps = tensor_field(1.0, b, _rotated_field(X, Y, d_eps + 0.05j))
    mu = tensor_field(1.0, b, _rotated_field(X, Y, d_mu + 0.02j)) if with_mu else None
    return eps, mu


def sphere_medium(n: int, eps_const: np.ndarray, radius: float = 0.5) -> np.ndarray:
    """Constant tensor eps_const inside the ball of the given radius, I outside."""
    X, Y, Z = grid_coords(n)
    inside = ((X * X + Y * Y + Z * Z) < radius * radius).astype(np.float64)
    return tensor_field(1.0, inside, np.asarray(eps_const, dtype=np.complex128) - np.eye(3))


# media of the paper's numerical section, on [0,1]^3 (Section 5)

def paper_bump_W(X, Y, Z) -> np.ndarray:
    return (np.exp(-((X - 0.5) / 0.25) ** 8) * np.exp(-((Y - 0.5) / 0.25) ** 8)
            * np.exp(-((Z - 0.5) / 0.25) ** 8))


def paper_medium(name: str, n: int) -> np.ndarray:
    """eps_222, eps_444, eps_234 or eps_dense sampled on the unit box, cell-centred."""
    X, Y, Z = grid_coords(n, origin=0.0, h=1.0 / n)
    W = paper_bump_W(X, Y, Z)
    if name == "eps222":
        diag = np.array([1.0, 1.0, 1.0])
    elif name == "eps444":
        diag = np.array([3.0, 3.0, 3.0])
    elif name in ("eps234", "epsdense"):
        diag = np.array([1.0, 2.0, 3.0])
    else:
        raise ValueError(name)
    if name == "epsdense":
        R = np.einsum("ab...,bc...->ac...", rot2(np.pi * X), rot1(np.pi * Y))
        mat = np.einsum("ab...,b,cb...->ac...", R, diag, R)
    else:
        mat = np.diag(diag)
    return tensor_field(1.0, W, np.asarray(mat, dtype=np.complex128))


# ----------------------------------------------------------------------------
# incident fields
# ----------------------------------------------------------------------------

def constant_field(n: int, E0) -> np.ndarray:
    """[3][n][n][n] constant vector field (the Laplace applied gradient E0)."""
    out = np.empty((3, n, n, n), dtype=np.complex128)
    for a in range(3):
        out[a] = E0[a]
    return out


def plane_phase(n: int, omega: float, d: np.ndarray, origin: float = -1.0, h: Optional[float] = None):
    """exp(i omega d.x) on the grid, [n][n][n] (z, y, x), as the product of its
    three one-dimensional factors."""
    t = grid_axis(n, origin, h)
    ex, ey, ez = (np.exp(1j * omega * d[a] * t) for a in range(3))
    return ez[:, None, None] * ey[None, :, None] * ex[None, None, :]


def plane_wave_gradient(n: int, omega: float, d: np.ndarray, origin: float = -1.0,
                        h: Optional[float] = None, out: Optional[np.ndarray] = None) -> np.ndarray:
    """grad of phi_inc = exp(i omega d.x): i omega d exp(i omega d.x), as [3][n][n][n]
    (written into `out` when given)."""
    ph = plane_phase(n, omega, d, origin, h)
    if out is None:
        out = np.empty((3, n, n, n), dtype=np.complex128)
    for a in range(3):
        np.multiply(ph, 1j * omega * d[a], out=out[a])
    return out


def plane_wave_em(n: int, omega: float, d: np.ndarray, p: np.ndarray, origin: float = -1.0,
                  h: Optional[float] = None, with_h: bool = True) -> np.ndarray:
    """[E_inc; H_inc] = [p; d x p] exp(i omega d.x) as [6][n][n][n] (free-space,
    eps = mu = 1); [3][n][n][n] (E only) without with_h."""
    ph = plane_phase(n, omega, d, origin, h)
    q = np.cross(d, p)
    coefs = list(p) + (list(q) if with_h else [])
    out = np.empty((len(coefs), n, n, n), dtype=np.complex128)
    for a, c in enumerate(coefs):
        np.multiply(ph, c, out=out[a])
    return out


def random_polarisation(rng: np.random.Generator, d: np.ndarray) -> np.ndarray:
    """Draws a standard normal 3-vector and projects it orthogonal to d, normalised."""
    v = rng.standard_normal(3)
    v = v - np.dot(v, d) * d
    return v / np.linalg.norm(v)


# ----------------------------------------------------------------------------
# random and Gaussian densities
# ----------------------------------------------------------------------------

def random_density(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex standard normal array (real parts drawn first, then imaginary parts)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex128)


def sparse_density(shape, rng: np.random.Generator, count: int):
    """A density that is zero except at ``count`` random points of the grid.

    ``shape`` is (c, n, n, n).  Draw order: for each point, the grid index
    (3 integers), then c complex normals (real, imaginary).  Returns
    (array, list of (z, y, x) indices).
    """
    c, n = shape[0], shape[-1]
    out = np.zeros(shape, dtype=np.complex128)
    pts = []
    for _ in range(count):
        z, y, x = (int(v) for v in rng.integers(0, n, 3))
        vals = rng.standard_normal(c) + 1j * rng.standard_normal(c)
        out[:, z, y, x] += vals
        pts.append((z, y, x))
    return out, pts


def gaussian(n: int, sigma: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """rho(x) = exp(-|x - center|^2 / (2 sigma^2)) on the grid, real, [n][n][n]."""
    X, Y, Z = grid_coords(n)
    r2 = (X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    kind: int
    n: int
    omega: float
    coef: np.ndarray                 # [9][n][n][n] complex128 (eps, eps^{-1} or eps)
    mu: Optional[np.ndarray]         # [9][n][n][n] or None
    inc: np.ndarray                  # [nrhs][c][n][n][n]
    tol: float
    name: str = ""
    h: float = 0.0
    origin: tuple = (-1.0, -1.0, -1.0)
    extra: dict = field(default_factory=dict)

    @property
    def ncomp(self) -> int:
        return 6 if self.mu is not None else 3

    @property
    def nrhs(self) -> int:
        return self.inc.shape[0]


def laplace_problem(n: int = 32, config: str = "laplace32", nrhs: int = 1) -> Problem:
    """Anisotropic Laplace: eps = I + b A, E0 = (0, 0, 1)."""
    cid = CONFIG_IDS[config]
    coef = laplace_medium(n, rng_for(cid, 0))
    inc = np.stack([constant_field(n, (0.0, 0.0, 1.0)) for _ in range(nrhs)])
    return Problem(KIND_LAPLACE, n, 0.0, coef, None, inc, 1e-10, config, 2.0 / n)


def helmholtz_problem(n: int = 64, omega: float = 4 * math.pi, config: str = "helmholtz64",
                      nrhs: int = 1, norm: float = 0.5) -> Problem:
    """Anisotropic Helmholtz: eps^{-1} = I + b (A + 0.05 i I), plane wave along seeded d_j.

    Right-hand side j draws its direction from item 1 + j.
    """
    cid = CONFIG_IDS[config]
    coef = helmholtz_medium(n, rng_for(cid, 0), norm=norm)
    dirs = [random_unit(rng_for(cid, 1 + j)) for j in range(nrhs)]
    inc = np.stack([plane_wave_gradient(n, omega, d) for d in dirs])
    return Problem(KIND_HELMHOLTZ, n, omega, coef, None, inc, 1e-10, config, 2.0 / n,
                   extra={"directions": np.array(dirs)})


def maxwell_problem(n: int = 128, omega: float = 8 * math.pi, config: str = "maxwell128",
                    nrhs: int = 1, with_mu: bool = True) -> Problem:
    """Anisotropic Maxwell: seeded eps, mu; plane wave [p; d x p] e^{i omega d.x}.

    Right-hand side j draws d (3 normals) then the polarisation (3 normals) from item 1 + j.
    """
    cid = CONFIG_IDS[config]
    eps, mu = maxwell_medium(n, rng_for(cid, 0))
    incs = []
    for j in range(nrhs):
        r = rng_for(cid, 1 + j)
        d = random_unit(r)
        p = random_polarisation(r, d)
        f = plane_wave_em(n, omega, d, p)
        incs.append(f if with_mu else f[:3])
    return Problem(KIND_MAXWELL, n, omega, eps, mu if with_mu else None, np.stack(incs), 1e-8,
                   config, 2.0 / n)


def config_problem(name: str, nrhs: Optional[int] = None, n: Optional[int] = None) -> Problem:
    """The named configurations with their default sizes."""
    if name == "laplace32":
        return laplace_problem(n or 32, name, nrhs or 1)
    if name == "helmholtz64":
        return helmholtz_problem(n or 64, 4 * math.pi, name, nrhs or 1)
    if name == "helmholtz128":
        return helmholtz_problem(n or 128, 8 * math.pi, name, nrhs or 1)
    if name == "batched96":
        return helmholtz_problem(n or 96, 6 * math.pi, name, nrhs or 64)
    if name == "maxwell128":
        return maxwell_problem(n or 128, 8 * math.pi, name, nrhs or 1)
    raise ValueError(f"unknown configuration {name!r}")


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------

SERVING_GRIDS = (32, 48, 64, 96, 128, 160)


def serving_requests(count: int = 2000, rate: float = 10.0, grids=SERVING_GRIDS,
                     max_rhs: int = 16, seed_item: int = 0, media: int = 0):
    """Poisson stream of mixed solve requests.

    Draw order (one generator, item ``seed_item`` of the serving config):
    ``count`` exponential inter-arrival times (mean 1/rate), then per request:
    kind (integer in {0,1,2}), grid index, wavelengths w ~ U[2, 10], nrhs in {1..max_rhs}.
    The medium and incident waves of request r use item 1000 + r.

    media > 0: the scatterers come from a pool of ``media`` entries instead,
    so that requests repeat plans.  Entry j draws (kind, grid index, w) from
    item 200000 + j, then its medium; request r draws, after its arrival
    gap, the pool index (integer in [0, media)) and nrhs from the stream
    generator, and its waves from item 1000 + r.
    """
    rng = rng_for(CONFIG_IDS["serving"], seed_item)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    pool = []
    for j in range(media):
        prng = rng_for(CONFIG_IDS["serving"], 200000 + j)
        kind = int(prng.integers(0, 3))
        n = int(grids[int(prng.integers(0, len(grids)))])
        w = float(prng.uniform(2.0, 10.0))
        pool.append((kind, n, 0.0 if kind == KIND_LAPLACE else math.pi * w, 200000 + j))
    reqs = []
    for r in range(count):
        if media > 0:
            kind, n, omega, mitem = pool[int(rng.integers(0, media))]
            nrhs = int(rng.integers(1, max_rhs + 1))
            reqs.append({"id": r, "arrival": float(t[r]), "kind": kind, "n": n, "omega": omega,
                         "nrhs": nrhs, "item": 1000 + r, "medium_item": mitem})
            continue
        kind = int(rng.integers(0, 3))
        n = int(grids[int(rng.integers(0, len(grids)))])
        w = float(rng.uniform(2.0, 10.0))
        nrhs = int(rng.integers(1, max_rhs + 1))
        omega = 0.0 if kind == KIND_LAPLACE else math.pi * w
        reqs.append({"id": r, "arrival": float(t[r]), "kind": kind, "n": n, "omega": omega,
                     "nrhs": nrhs, "item": 1000 + r})
    return reqs


def serving_recipe(req: dict) -> dict:
    """The random draws of one serving request, in the order ``serving_problem``
    makes them, and the small factors its arrays are built from:

    * ``matrix``: [3][3] (Laplace, Helmholtz) or [3][3][1][n][n] (Maxwell,
      R(x, y) diag R^T on one z plane), so that coef = I + bump(x) * matrix;
    * ``waves``: per right-hand side the three components' constant factors,
      multiplied by the separable phase exp(i omega d.x) (``phased``) or not
      (Laplace: constant fields);
    * ``dirs``: the directions d of the phases.
    """
    # the medium from the pool entry's generator when the request has one,
    # else from the request's own (then the waves follow in the same generator)
    rng = rng_for(CONFIG_IDS["serving"], req["item"])
    mrng = rng_for(CONFIG_IDS["serving"], req["medium_item"]) if "medium_item" in req else rng
    n, kind, omega, nrhs = req["n"], req["kind"], req["omega"], req["nrhs"]
    out = {"kind": kind, "n": n, "omega": omega, "nrhs": nrhs, "axis": grid_axis(n)}
    waves, dirs = [], []
    if kind == KIND_LAPLACE:
        out["matrix"] = laplace_matrix(mrng)
        for r in range(nrhs):
            waves.append(random_unit(rng))
        out["phased"] = False
    elif kind == KIND_HELMHOLTZ:
        out["matrix"] = helmholtz_matrix(mrng)
        for r in range(nrhs):
            d = random_unit(rng)
            dirs.append(d)
            waves.append(1j * omega * d)
        out["phased"] = True
    else:
        d_eps = mrng.uniform(0.0, 1.0, 3)
        mrng.uniform(0.0, 0.5, 3)  # D_mu, drawn and unused (mu = I)
        X, Y, _ = grid_coords_plane(n)
        out["matrix"] = _rotated_field(X, Y, d_eps + 0.05j)
        for r in range(nrhs):
            d = random_unit(rng)
            dirs.append(d)
            waves.append(random_polarisation(rng, d))
        out["phased"] = True
    out["waves"], out["dirs"] = waves, dirs
    return out


def serving_problem(req: dict) -> Problem:
    """Materialise the medium and right-hand sides of one serving request.

    Medium: drawn from the request's generator (recipes of the Laplace,
    Helmholtz and Maxwell configurations; Maxwell with mu = I).  Then per
    right-hand side: a direction (and polarisation for Maxwell).
    """
    rc = serving_recipe(req)
    n, kind, omega, nrhs = rc["n"], rc["kind"], rc["omega"], rc["nrhs"]
    X, Y, Z = grid_coords(n)
    coef = tensor_field(1.0, bump(X, Y, Z), rc["matrix"])
    inc = np.empty((nrhs, 3, n, n, n), dtype=np.complex128)
    for r in range(nrhs):
        w = rc["waves"][r]
        if rc["phased"]:
            ph = plane_phase(n, omega, rc["dirs"][r])
            for a in range(3):
                np.multiply(ph, w[a], out=inc[r, a])
        else:
            for a in range(3):
                inc[r, a] = w[a]
    return Problem(kind, n, omega, coef, None, inc, 1e-8, f"req{req['id']}", 2.0 / n)
