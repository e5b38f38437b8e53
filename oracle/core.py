"""Oracle core: grid, DFT, spectral symbols, FD operators, phi-functions.

TEST INFRASTRUCTURE ONLY (see the package header).  All arithmetic is FP64.

Conventions
  * grid: Omega = prod_d [-X_d, X_d), h_d = 2 X_d / N_d, x_i = -X + i h
    (Section 2.1, Section 3.2); arrays are C-order with one axis per
    dimension.
  * DFT: forward unnormalized exp(-2 pi i j k / N); inverse carries 1/N.
  * <f, g>_h = (prod h_d) sum f g  (Section 2.1).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# grid
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Grid:
    n: tuple          # points per axis
    half_len: tuple   # X_d

    @property
    def dim(self):
        return len(self.n)

    @property
    def h(self):
        return tuple(2.0 * X / N for N, X in zip(self.n, self.half_len))

    @property
    def cell(self):
        """h_x h_y (h_z): the weight of <.,.>_h."""
        return float(np.prod(self.h))

    @property
    def volume(self):
        """|Omega| = prod 2 X_d."""
        return float(np.prod([2.0 * X for X in self.half_len]))


def inner(a, b, grid: Grid) -> float:
    """Discrete L2 inner product <a, b>_h (Section 2.1)."""
    return grid.cell * float(np.sum(a * b))


# ---------------------------------------------------------------------------
# DFT: two modes.  "naive" applies the defining sum along each axis with an
# exact-index twiddle matrix (w^(j k mod N)); "library" calls pocketfft
# through scipy.  Both are pinned against a brute-force multidimensional sum.
# ---------------------------------------------------------------------------

_MODE = os.environ.get("ETD_ORACLE_DFT", "library")
_WORKERS = int(os.environ.get("ETD_ORACLE_THREADS", "0")) or (os.cpu_count() or 1)


def set_dft_mode(mode: str):
    global _MODE
    assert mode in ("naive", "library")
    _MODE = mode


def get_dft_mode() -> str:
    return _MODE


def set_threads(n: int):
    global _WORKERS
    _WORKERS = max(1, int(n))


def get_threads() -> int:
    return _WORKERS


_TW = {}


def dft_matrix(n: int, sign: int) -> np.ndarray:
    """W[j, k] = exp(sign * 2 pi i (j k mod n) / n)."""
    key = (n, sign)
    if key not in _TW:
        j = np.arange(n)
        e = np.outer(j, j) % n
        ang = 2.0 * math.pi * e / n
        _TW[key] = np.cos(ang) + 1j * sign * np.sin(ang)
    return _TW[key]


def _naive_axis(a: np.ndarray, axis: int, sign: int) -> np.ndarray:
    W = dft_matrix(a.shape[axis], sign)
    b = np.moveaxis(a, axis, -1)
    return np.moveaxis(b @ W, -1, axis)    # W symmetric: (b W)[..., k] = sum_j b_j W[j, k]


def fft(a: np.ndarray) -> np.ndarray:
    """Forward multidimensional DFT, unnormalized."""
    a = np.asarray(a, dtype=np.complex128)
    if _MODE == "naive":
        for ax in range(a.ndim):
            a = _naive_axis(a, ax, -1)
        return a
    import scipy.fft as sf
    return sf.fftn(a, workers=_WORKERS)


def ifft_complex(A: np.ndarray) -> np.ndarray:
    """Inverse multidimensional DFT with 1/prod(N)."""
    A = np.asarray(A, dtype=np.complex128)
    if _MODE == "naive":
        for ax in range(A.ndim):
            A = _naive_axis(A, ax, +1) / A.shape[ax]
        return A
    import scipy.fft as sf
    return sf.ifftn(A, workers=_WORKERS)


def ifft(A: np.ndarray) -> np.ndarray:
    """Real part of the inverse DFT (the spectra used here are Hermitian)."""
    return ifft_complex(A).real


# ---------------------------------------------------------------------------
# spectral symbols (Section 3.2)
# ---------------------------------------------------------------------------


def lam_axis(N: int, X: float) -> np.ndarray:
    """lambda_x(i) = (pi/X) i for 0 <= i <= N/2, (pi/X)(N - i) above."""
    i = np.arange(N)
    return (math.pi / X) * np.where(i <= N // 2, i, N - i)


def kder_axis(N: int, X: float) -> np.ndarray:
    """First-derivative wavenumber: (pi/X) * (i, 0 at Nyquist, i - N)."""
    i = np.arange(N).astype(np.float64)
    k = np.where(i < N / 2, i, i - N)
    if N % 2 == 0:
        k[N // 2] = 0.0
    return (math.pi / X) * k


def _bcast(v, axis, ndim):
    shape = [1] * ndim
    shape[axis] = v.size
    return v.reshape(shape)


def ksq(grid: Grid) -> np.ndarray:
    """k^2 = lambda_x^2 + lambda_y^2 (+ lambda_z^2) = -lambda_ijk."""
    out = np.zeros(grid.n)
    for d, (N, X) in enumerate(zip(grid.n, grid.half_len)):
        out = out + _bcast(lam_axis(N, X) ** 2, d, grid.dim)
    return out


def kder(grid: Grid, d: int) -> np.ndarray:
    N, X = grid.n[d], grid.half_len[d]
    return np.broadcast_to(_bcast(kder_axis(N, X), d, grid.dim), grid.n)


def spectral_lap(a: np.ndarray, grid: Grid) -> np.ndarray:
    return ifft(-ksq(grid) * fft(a))


def spectral_grad(a: np.ndarray, grid: Grid):
    A = fft(a)
    return [ifft(1j * kder(grid, d) * A) for d in range(grid.dim)]


def fd_symbol(grid: Grid) -> np.ndarray:
    """mu_k = sum_d (4/h_d^2) sin^2(pi k_d / N_d): eigenvalues of -Delta_h."""
    out = np.zeros(grid.n)
    for d, (N, h) in enumerate(zip(grid.n, grid.h)):
        s = np.sin(math.pi * np.arange(N) / N)
        out = out + _bcast(4.0 / (h * h) * s * s, d, grid.dim)
    return out


# ---------------------------------------------------------------------------
# finite differences (Section 2.1, operator:diff), periodic
# ---------------------------------------------------------------------------


# Spatial axes are addressed from the end (axis d of a dim-D grid is array
# axis d - D), so the operators also act on stacks of grid functions.


def d_plus(u, ax, h):
    return (np.roll(u, -1, axis=ax) - u) / h


def d_minus(u, ax, h):
    return (u - np.roll(u, 1, axis=ax)) / h


def g_half(g, ax):
    """g_{i+1/2} = (g_i + g_{i+1}) / 2 along axis ax."""
    return 0.5 * (g + np.roll(g, -1, axis=ax))


def lap_S(u: np.ndarray, g: np.ndarray, grid: Grid, mask=None) -> np.ndarray:
    """Delta_{S,h} u = sum_d D_d^- (g_{i+1/2} D_d^+ u)  (operator:diff).

    With a band mask (bool, grid shape) only the faces whose two nodes are
    both on the band carry flux, so rows off the band are 0 and the band
    nodes see no value off it (the operator set up on the band nodes alone,
    Section 3.2)."""
    out = np.zeros(np.broadcast_shapes(u.shape, g.shape))
    for d, h in enumerate(grid.h):
        ax = d - grid.dim
        gh = g_half(g, ax)
        if mask is not None:
            m = np.asarray(mask, dtype=np.float64)
            gh = gh * (m * np.roll(m, -1, axis=ax))
        out = out + d_minus(gh * d_plus(u, ax, h), ax, h)
    return out


def lap_h(u: np.ndarray, grid: Grid) -> np.ndarray:
    """Constant-coefficient (2d+1)-point Laplacian (Delta_{S,h} with g = 1)."""
    return lap_S(u, np.ones_like(u), grid)


def div_central(F, grid: Grid) -> np.ndarray:
    """sum_d (F_d(i+1) - F_d(i-1)) / (2 h_d)."""
    out = np.zeros_like(F[0])
    for d, h in enumerate(grid.h):
        ax = d - grid.dim
        out = out + (np.roll(F[d], -1, axis=ax) - np.roll(F[d], 1, axis=ax)) / (2.0 * h)
    return out


def lapinv(f: np.ndarray, grid: Grid) -> np.ndarray:
    """(-Delta_h)^{-1} f with the mean removed: zero mode of 1/mu_k set to 0.

    This is the pseudo-inverse of the periodic FD Laplacian; removing the
    zero mode is exactly the mean removal of (-Delta_{S,h})^{-1} in
    Section 2.1 (definition after Lemma lemma:Linfbound's preamble).
    """
    mu = fd_symbol(grid)
    inv = np.zeros_like(mu)
    nz = mu > 0
    inv[nz] = 1.0 / mu[nz]
    return ifft(inv * fft(f))


def band_matrix(g: np.ndarray, mask: np.ndarray, grid: Grid):
    """Band nodes B (flat indices, ascending) and the band matrix A of
    -Delta_{S,h} (operator:diff, Section 2.1) restricted to them: row i is
    sum over band neighbours j of w_ij (psi_i - psi_j), w_ij = (g_i + g_j) /
    (2 h_d^2); faces with a node off the band are left out.  Assembled edge
    by edge (each face once, along +e_d, periodic)."""
    import scipy.sparse as sp
    m = np.asarray(mask).astype(bool)
    B = np.flatnonzero(m.ravel())
    nb = B.size
    pos = -np.ones(m.size, dtype=np.int64)
    pos[B] = np.arange(nb)
    gf = np.asarray(g, dtype=np.float64).ravel()
    shape = m.shape
    rows, cols, vals = [], [], []
    diag = np.zeros(nb)
    for d, h in enumerate(grid.h):
        ax = d - grid.dim + len(shape)
        nbr = np.roll(np.arange(m.size).reshape(shape), -1, axis=ax).ravel()   # node i + e_d (periodic)
        j = nbr[B]
        on = m.ravel()[j]
        a, b = np.arange(nb)[on], pos[j[on]]
        w = 0.5 * (gf[B[on]] + gf[j[on]]) / (h * h)
        rows += [a, b]
        cols += [b, a]
        vals += [-w, -w]
        np.add.at(diag, a, w)
        np.add.at(diag, b, w)
    A = sp.coo_matrix((np.concatenate(vals + [diag]),
                       (np.concatenate(rows + [np.arange(nb)]), np.concatenate(cols + [np.arange(nb)]))),
                      shape=(nb, nb)).tocsr()
    return B, A


def lapinv_S_band(f: np.ndarray, g: np.ndarray, mask: np.ndarray, grid: Grid) -> np.ndarray:
    """(-Delta_{S,h})^{-1} f, set up and inverted on a narrow band.

    Section 2.1 (operator:diff) defines Delta_{S,h} with face coefficients
    g_{i+1/2} = (g_i + g_{i+1})/2 and its inverse on mean-zero functions,
    extended to any f by removing the mean; Section 3.2 assembles and solves
    the nonlocal problem only on the band nodes.  Reading: the unknowns are
    the nodes with mask != 0; a face enters when both of its nodes are on the
    band (faces to nodes off the band carry no flux); the mean removed from f
    and from the solution is the plain mean over the band nodes; the result
    is 0 off the band.  The band must be connected (else the reduced system
    below is singular).

    With A = band_matrix(...): its null space on a connected band is the
    constants and f_B - mean(f_B) lies in its range, so one solution has psi
    at the first band node fixed to 0: the remaining rows and columns are
    nonsingular and go to scipy's sparse direct solver (the library
    primitive); the band mean of that solution is then removed.
    """
    import scipy.sparse.linalg as spla
    m = np.asarray(mask).astype(bool)
    B, A = band_matrix(g, m, grid)
    nb = B.size
    fb = np.asarray(f, dtype=np.float64).ravel()[B]
    rhs = fb - fb.mean()
    sol = np.zeros(nb)
    if nb > 1:
        sol[1:] = spla.spsolve(A[1:, 1:].tocsc(), rhs[1:])
    sol -= sol.mean()
    out = np.zeros(m.size)
    out[B] = sol
    return out.reshape(m.shape)


def lapinv_S_band_inf_norm(g: np.ndarray, mask: np.ndarray, grid: Grid) -> float:
    """C = ||(-Delta_{S,h})^{-1}||_inf on a band (the constant of the MBP
    condition, Section 2.1) by a dense computation: the operator is
    X = A^+ (I - 11^T / nb) (Moore-Penrose inverse of the band matrix after
    the mean removal, numpy's pinv the library primitive), C its largest
    absolute row sum.  Small bands only (dense nb x nb)."""
    B, A = band_matrix(g, mask, grid)
    nb = B.size
    Ad = A.toarray()
    X = np.linalg.pinv(Ad) @ (np.eye(nb) - np.full((nb, nb), 1.0 / nb))
    return float(np.abs(X).sum(axis=1).max())


def lapinv_inf_norm(grid: Grid) -> float:
    """C = ||(-Delta_h)^{-1}||_inf = sum_j |a_j|, a = IDFT(1/mu) (0 at k=0).

    The pseudo-inverse is circulant, so every row has the same absolute sum.
    """
    mu = fd_symbol(grid)
    inv = np.zeros_like(mu)
    nz = mu > 0
    inv[nz] = 1.0 / mu[nz]
    a = ifft(inv)
    return float(np.sum(np.abs(a)))


# ---------------------------------------------------------------------------
# nonlinearities (Section 1)
# ---------------------------------------------------------------------------


def W(s):
    return 18.0 * (s * s - s) ** 2


def Wp(s):
    return 36.0 * (s * s - s) * (2.0 * s - 1.0)


def Wpp(s):
    return 36.0 * (6.0 * s * s - 6.0 * s + 1.0)


def f_ind(s):
    """f(u) = 3u^2 - 2u^3."""
    return 3.0 * s * s - 2.0 * s ** 3


def fp_ind(s):
    return 6.0 * s * (1.0 - s)


def g_loc(phi):
    """g(phi) = 18 (phi^2 - phi)^2 (Section 2.2, Section 3.3)."""
    return 18.0 * (phi * phi - phi) ** 2


# ---------------------------------------------------------------------------
# phi-functions (Section 2.2): phi0 = e^{-z}, phi1 = (1-e^{-z})/z,
# phi2 = (e^{-z} - 1 + z)/z^2.  Small |z| uses the Taylor series
# phi_k(z) = sum_j (-z)^j / (j + k)!, which avoids the cancellation.
# ---------------------------------------------------------------------------

_TAYLOR_Z = 0.1


def _taylor(z, k, terms=20):
    out = np.zeros_like(z)
    for j in reversed(range(terms)):
        out = out * (-z) + 1.0 / math.factorial(j + k)
    return out


def phi0(z):
    return np.exp(-np.asarray(z, dtype=np.float64))


def phi1(z):
    z = np.asarray(z, dtype=np.float64)
    small = np.abs(z) < _TAYLOR_Z
    zs = np.where(small, 1.0, z)
    big = -np.expm1(-zs) / zs
    return np.where(small, _taylor(z, 1), big)


def phi2(z):
    z = np.asarray(z, dtype=np.float64)
    small = np.abs(z) < _TAYLOR_Z
    zs = np.where(small, 1.0, z)
    big = (np.expm1(-zs) + zs) / (zs * zs)
    return np.where(small, _taylor(z, 2), big)
