"""Fixed-membrane OK dynamics: localization-split ETD1 / ETDRK2 (Section 2.2).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64 throughout.

With g > 0 fixed, the FD semi-discrete system (eqn:ODE_eqn) reads
    d(sqrt(g) u)/dt + L (sqrt(g) u) = R(u),
    L = B I - eps_u g^{-1/2} Delta_{S,h} g^{-1/2}  =  B I + eps_u H,
    R(u) = B sqrt(g) u - sqrt(g) W'(u)/eps_u
           - gamma sqrt(g) (-Delta)^{-1}(g f(u)) f'(u)
           - M <g (f(u) - ubar), 1>_h sqrt(g) f'(u).
ETD1 (eqn:ETD1):  sqrt(g) U^{n+1} = phi0(tau L) sqrt(g) U^n + tau phi1(tau L) R(U^n).
ETDRK2 (eqn:ETDRK2): the ETD1 value is the predictor U~, then
    sqrt(g) U^{n+1} = sqrt(g) U~ + tau phi2(tau L) (R(U~) - R(U^n)).

Readings (ambiguity register entries, recorded in the design notes):
  * (-Delta)^{-1} is the constant-coefficient periodic FD pseudo-inverse
    applied by DFT (zero mode removed); the theorems only use its symmetry,
    semidefiniteness and sup-norm bound C.
  * The nonlocal argument is g f(u) as in the discrete R and energy; the
    flag ``nonlocal_with_ubar`` selects g (f(u) - ubar) as in the PDE.
  * phi_k(tau L) v is computed by a dense eigendecomposition of the
    symmetric matrix L on small grids and by Lanczos with full
    reorthogonalization otherwise (the paper does not say how).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import core
from .core import Grid

# constants of Lemma lemma:MBPbdd / Theorem thm:Energy (bounds on [0, 1])
L_W2 = 36.0      # max |W''|
L_F2 = 6.0       # max |f''|
L_F1 = 1.5       # max |f'|
L_G = 9.0 / 8.0  # max g


@dataclass
class FixedParams:
    eps_u: float
    gamma: float
    M: float
    ubar: float
    B: float
    nonlocal_with_ubar: bool = False
    # > 0: the nonlocal term by (-Delta_{S,h})^{-1} solved on the band
    # {g >= band_delta} (Section 3.2; core.lapinv_S_band) instead of (-Delta_h)^{-1}
    band_delta: float = 0.0
    # > 0: the whole step restricted to the band {g >= band_step} (the
    # narrow-band implementation of the fixed-membrane scheme): the unknowns
    # are the band nodes, Delta_{S,h} keeps the faces with both nodes on the
    # band, the nonlinear terms, the nonlocal argument and the mass sum are
    # taken on the band, and U off the band keeps its value
    band_step: float = 0.0


def step_band(g, p: FixedParams):
    """Mask of the band of the restricted step (None: the whole grid)."""
    return (np.asarray(g) >= p.band_step) if p.band_step > 0.0 else None


def B_mbp(eps_u, gamma, M, C, vol):
    """Condition (eqn:cond_MBP): the smallest B with the discrete MBP."""
    return L_W2 / eps_u + gamma * C * L_F2 * L_G + M * vol * L_F2 * L_G


def B_es(eps_u, gamma, M, C, vol):
    """Condition (eqn:cond_ES) of Theorem thm:Energy."""
    return L_W2 / eps_u + (0.5 * gamma * C + 0.5 * M * vol) * (L_F2 + L_F1 ** 2) * L_G


def _on_band(x, g, p: FixedParams):
    m = step_band(g, p)
    return x if m is None else np.where(m, x, 0.0)


def mass_f(U, g, p: FixedParams, grid: Grid) -> float:
    """m_f = <g (f(U) - ubar), 1>_h (on the band of a restricted step)."""
    return grid.cell * float(np.sum(_on_band(g * (core.f_ind(U) - p.ubar), g, p)))


def nonlocal_arg(U, g, p: FixedParams):
    fu = core.f_ind(U)
    return _on_band(g * (fu - p.ubar) if p.nonlocal_with_ubar else g * fu, g, p)


def R_phi(U, g, p: FixedParams, grid: Grid) -> np.ndarray:
    """Nonlinear remainder R(U) of the localization split."""
    sg = np.sqrt(g)
    if p.band_delta > 0.0:
        psi = core.lapinv_S_band(nonlocal_arg(U, g, p), g, g >= p.band_delta, grid)
    else:
        psi = core.lapinv(nonlocal_arg(U, g, p), grid)
    mf = mass_f(U, g, p, grid)
    fp = core.fp_ind(U)
    nonlin = sg * core.Wp(U) / p.eps_u + p.gamma * sg * psi * fp + p.M * mf * sg * fp
    return p.B * sg * U - _on_band(nonlin, g, p)


def H_apply(w, g, grid: Grid, mask=None):
    """H w = -g^{-1/2} Delta_{S,h}(g^{-1/2} w) (faces on the band only, with a mask)."""
    isg = 1.0 / np.sqrt(g)
    return -isg * core.lap_S(isg * w, g, grid, mask)


def L_apply(w, g, p: FixedParams, grid: Grid):
    return p.B * w + p.eps_u * H_apply(w, g, grid, step_band(g, p))


# ---------------------------------------------------------------------------
# actions of phi_k(tau L)
# ---------------------------------------------------------------------------


class DenseExpo:
    """phi(tau L) v through the eigendecomposition L = V diag(lam) V^T."""

    def __init__(self, g, p: FixedParams, grid: Grid):
        n = int(np.prod(grid.n))
        eye = np.eye(n).reshape((n,) + tuple(grid.n))
        cols = L_apply(eye, g, p, grid).reshape(n, n)     # row j = L e_j
        Lm = cols.T
        self.L = 0.5 * (Lm + Lm.T)
        self.asym = float(np.abs(Lm - Lm.T).max())
        self.lam, self.V = np.linalg.eigh(self.L)
        self.shape = tuple(grid.n)

    def apply(self, fun, tau, v):
        c = self.V.T @ v.reshape(-1)
        return (self.V @ (fun(tau * self.lam) * c)).reshape(self.shape)


class UspaceExpo:
    """phi(tau L) w computed in the U variable (small grids, one fixed tau).

    With D = diag(sqrt g), phi(tau L) w = D phi(tau Lt) D^{-1} w where
    Lt = D^{-1} L D = B I - eps_u G^{-1} Delta_{S,h}.  Unlike L, whose entries
    carry factors g^{-1/2} up to ~1e8 where g is tiny, Lt's entries are ratios
    of neighbouring g values, so the block-matrix exponential
        expm([[A, I, 0], [0, 0, I], [0, 0, 0]]),  A = -tau Lt,
    whose first block row is [e^A, phi1, phi2] (phi_k in the convention of
    Section 2.2 evaluated at tau Lt), yields U-space results accurate relative
    to U itself, also where g ~ 1e-17.  scipy's expm is the library primitive.
    """

    def __init__(self, g, p: FixedParams, grid: Grid, tau: float):
        import scipy.linalg as sla
        n = int(np.prod(grid.n))
        eye = np.eye(n).reshape((n,) + tuple(grid.n))
        cols = (p.B * eye - p.eps_u * core.lap_S(eye, g, grid, step_band(g, p)) / g).reshape(n, n)
        Lt = cols.T
        aug = np.zeros((3 * n, 3 * n))
        aug[:n, :n] = -tau * Lt
        aug[:n, n:2 * n] = np.eye(n)
        aug[n:2 * n, 2 * n:] = np.eye(n)
        E = sla.expm(aug)
        self.mats = {core.phi0: E[:n, :n], core.phi1: E[:n, n:2 * n], core.phi2: E[:n, 2 * n:]}
        self.tau, self.sg, self.shape = tau, np.sqrt(g), tuple(grid.n)

    def apply(self, fun, tau, v):
        assert tau == self.tau
        x = (v / self.sg).reshape(-1)
        return self.sg * (self.mats[fun] @ x).reshape(self.shape)


class LanczosExpo:
    """phi(tau L) v by Lanczos with full reorthogonalization.

    Stops once two successive Krylov approximations agree to ``tol``
    relative; the spectrum of tau L lies in [tau B, tau (B + eps_u rho)], where
    the phi-functions are smooth, so convergence is fast.
    """

    def __init__(self, g, p: FixedParams, grid: Grid, tol=1e-15, max_iter=400):
        self.g, self.p, self.grid = g, p, grid
        self.tol, self.max_iter = tol, max_iter
        self.last_iters = 0

    def apply(self, fun, tau, v):
        shape = v.shape
        v = v.reshape(-1)
        beta0 = float(np.linalg.norm(v))
        if beta0 == 0.0:
            return np.zeros(shape)
        Q = [v / beta0]
        alphas, betas = [], []
        prev, prev_diff = None, np.inf
        y = None
        for j in range(self.max_iter):
            w = L_apply(Q[j].reshape(shape), self.g, self.p, self.grid).reshape(-1)
            a = float(w @ Q[j])
            alphas.append(a)
            Qm = np.array(Q)
            for _ in range(2):
                w = w - Qm.T @ (Qm @ w)
            T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
            lam, S = np.linalg.eigh(T)
            coef = S @ (fun(tau * lam) * S[0, :])
            y = beta0 * (Qm.T @ coef)
            b = float(np.linalg.norm(w))
            if prev is not None:
                diff = float(np.linalg.norm(y - prev))
                ny = float(np.linalg.norm(y))
                if diff <= self.tol * ny or (diff <= 1e-13 * ny and diff >= prev_diff):
                    break
                prev_diff = diff
            if b <= 1e-300:
                break
            betas.append(b)
            Q.append(w / b)
            prev = y
        self.last_iters = j + 1
        return y.reshape(shape)


def make_expo(g, p: FixedParams, grid: Grid):
    n = int(np.prod(grid.n))
    return DenseExpo(g, p, grid) if n <= 4096 else LanczosExpo(g, p, grid)


# ---------------------------------------------------------------------------
# schemes
# ---------------------------------------------------------------------------


def etd1_step(U, g, p: FixedParams, grid: Grid, tau: float, expo, R=None):
    """One ETD1 step (eqn:ETD1).  ``R`` overrides the remainder (tests)."""
    R = R or R_phi
    sg = np.sqrt(g)
    w = sg * U
    w1 = expo.apply(core.phi0, tau, w) + tau * expo.apply(core.phi1, tau, R(U, g, p, grid))
    return _keep_off_band(w1 / sg, U, g, p)


def _keep_off_band(U_new, U, g, p: FixedParams):
    """A restricted step leaves U off its band as it was."""
    m = step_band(g, p)
    return U_new if m is None else np.where(m, U_new, U)


def etdrk2_step(U, g, p: FixedParams, grid: Grid, tau: float, expo, R=None):
    """One ETDRK2 step (eqn:ETDRK2)."""
    R = R or R_phi
    sg = np.sqrt(g)
    w = sg * U
    Rn = R(U, g, p, grid)
    wt = expo.apply(core.phi0, tau, w) + tau * expo.apply(core.phi1, tau, Rn)
    Ut = wt / sg
    Ut = _keep_off_band(Ut, U, g, p)
    w2 = wt + tau * expo.apply(core.phi2, tau, R(Ut, g, p, grid) - Rn)
    return _keep_off_band(w2 / sg, U, g, p)


def step(U, g, p, grid, tau, scheme, expo, R=None):
    return (etd1_step if scheme == 1 else etdrk2_step)(U, g, p, grid, tau, expo, R)


# ---------------------------------------------------------------------------
# energy (eqn:Energy_dis) and diagnostics
# ---------------------------------------------------------------------------


def energy(U, g, p: FixedParams, grid: Grid) -> dict:
    """E_{phi,h}[U] and its four terms, each from the literal formula (on the
    band's nodes and faces for a restricted step)."""
    m = step_band(g, p)
    e_grad = 0.5 * p.eps_u * core.inner(-core.lap_S(U, g, grid, m), U, grid)
    e_well = core.inner(_on_band(g * core.W(U), g, p), np.ones_like(U), grid) / p.eps_u
    q = nonlocal_arg(U, g, p)
    e_nl = 0.5 * p.gamma * core.inner(core.lapinv(q, grid), q, grid)
    mf = mass_f(U, g, p, grid)
    e_mass = 0.5 * p.M * mf * mf
    return dict(E=e_grad + e_well + e_nl + e_mass, E_grad=e_grad, E_well=e_well,
                E_nonlocal=e_nl, E_mass=e_mass)


def diagnostics(U, g, p: FixedParams, grid: Grid) -> dict:
    return dict(m=mass_f(U, g, p, grid), Q=grid.cell * float(np.sum(g * U)),
                umin=float(U.min()), umax=float(U.max()),
                bound=float(np.abs(2.0 * U - 1.0).max()))
