"""Seeded synthetic inputs shaped like the paper's 2D and 3D experiments.

This module is shared by the CPU oracle tests and the GPU path.  It holds
only random draws and input geometry (initial phase fields, the fixed
membrane's localization field, parameter draws); none of the scheme's
arithmetic lives here.

Random numbers come from a counter-based SplitMix64 generator keyed by
(seed, instance, field): draw j of a field is the SplitMix64 finalizer of
``key + (j + 1) * 0x9E3779B97F4A7C15`` taken modulo 2**64, in C-order linear
index.  That makes every array reproducible bit for bit on any machine.

Variable convention.  The paper uses phi, u in [0, 1] with the double well
W(s) = 18 (s^2 - s)^2 (Section 1).  The experiment descriptions here are
written in the symmetric +-1 convention (tanh profiles, "|u| <= 1"), so the
builders map phi = (1 + phi_pm)/2 and u = (1 + u_pm)/2.  A +-1 width eps_pm
corresponds to the paper's eps_phi = 3*sqrt(2)*eps_pm, because the paper's
equilibrium profile is 0.5 + 0.5 tanh(3 d / eps_phi) (Section 4.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DEFAULT_SEED = 20260604


def _finalize(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, instance: int, field_id: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = _finalize(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))
        k = _finalize(k ^ np.uint64((instance * 0x10001 + 1) & 0xFFFFFFFFFFFFFFFF))
        k = _finalize(k ^ np.uint64((field_id * 0x1000193 + 7) & 0xFFFFFFFFFFFFFFFF))
    return k[0]


def draws_u64(seed: int, instance: int, field_id: int, n: int) -> np.ndarray:
    """n raw 64-bit draws of the (seed, instance, field) stream."""
    key = _key(seed, instance, field_id)
    j = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _finalize(key + j * _GOLD)


def uniform_pm1(seed, instance, field_id, shape) -> np.ndarray:
    """U(-1, 1) in float64: 2 * ((x >> 11) * 2^-53) - 1."""
    n = int(np.prod(shape))
    x = draws_u64(seed, instance, field_id, n)
    return (2.0 * ((x >> np.uint64(11)).astype(np.float64) * 2.0**-53) - 1.0).reshape(shape)


def uniform_open01(seed, instance, field_id, n) -> np.ndarray:
    """U(0, 1] in float64: ((x >> 11) + 1) * 2^-53."""
    x = draws_u64(seed, instance, field_id, n)
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53


def normal(seed, instance, field_id, n) -> np.ndarray:
    """N(0, 1) by Box-Muller from two U(0,1] streams."""
    a = uniform_open01(seed, instance, field_id, n)
    b = uniform_open01(seed, instance, field_id + 100003, n)
    return np.sqrt(-2.0 * np.log(a)) * np.cos(2.0 * math.pi * b)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def axis_coords(n: int, half_len: float) -> np.ndarray:
    """Grid points x_i = -X + i h, h = 2X/n, i = 0..n-1 (Section 2.1)."""
    h = 2.0 * half_len / n
    return -half_len + h * np.arange(n, dtype=np.float64)


def mesh(shape, half_len):
    axes = [axis_coords(n, X) for n, X in zip(shape, half_len)]
    return np.meshgrid(*axes, indexing="ij")


def _assoc_legendre(l: int, m: int, x: np.ndarray) -> np.ndarray:
    """P_l^m(x) for m >= 0 by the standard upward recurrence (no phase factor)."""
    pmm = np.ones_like(x)
    if m > 0:
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
        fact = 1.0
        for _ in range(m):
            pmm = pmm * fact * s
            fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def real_sph_harm(l: int, m: int, theta: np.ndarray, azim: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonic; theta = polar angle from +z."""
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    p = _assoc_legendre(l, am, np.cos(theta))
    if m == 0:
        return norm * p
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(m * azim)
    return math.sqrt(2.0) * norm * p * np.sin(am * azim)


def sech4(s: np.ndarray) -> np.ndarray:
    """sech(s)^4 without overflow."""
    e = np.exp(-2.0 * np.abs(s))
    return (2.0 * np.sqrt(e) / (1.0 + e)) ** 4


# ----------------------------------------------------------------------------
# fixed membrane inputs (2D 64^2 circle; 3D 128^3 sphere)
# ----------------------------------------------------------------------------

@dataclass
class FixedInputs:
    shape: tuple
    half_len: tuple
    g: np.ndarray           # localization g(phi) > 0, float64
    u0: np.ndarray          # initial protein density in [0, 1]
    eps_u: float
    gamma: float
    M: float
    ubar: float
    tau: float


def fixed_membrane(dim: int = 2, n: int | tuple = 64, radius: float = 0.5, eps_pm: float | None = None,
                   eps_pm_in_h: float | None = None, seed: int = DEFAULT_SEED, instance: int = 0,
                   u_mean_pm: float = -0.2, u_amp_pm: float = 0.05, gamma: float = 1.0,
                   M: float | None = None, tau: float = 0.01, half_len: float = 1.0) -> FixedInputs:
    """Fixed circular/spherical membrane on [-X, X)^d.

    phi_pm = tanh((R - r) / (sqrt(2) eps_pm)); in the [0,1] convention
    g = 18 (phi^2 - phi)^2 equals (9/8) sech^4((R - r)/(sqrt(2) eps_pm)),
    which is used directly so that g stays strictly positive in float64
    (the tanh route saturates to phi = 1 exactly far from the membrane).
    u_pm = u_mean_pm + u_amp_pm * U(-1, 1), mapped u = (1 + u_pm)/2.
    n: the points per axis, or one count per axis; eps_pm_in_h counts the
    coarsest spacing, so the interface is resolved along every axis.
    """
    shape = (n,) * dim if isinstance(n, int) else tuple(n)
    assert len(shape) == dim
    hl = (half_len,) * dim
    h = 2.0 * half_len / min(shape)
    if eps_pm is None:
        eps_pm = (eps_pm_in_h * h) if eps_pm_in_h is not None else 0.0625
    X = mesh(shape, hl)
    r = np.sqrt(sum(x * x for x in X))
    s = (radius - r) / (math.sqrt(2.0) * eps_pm)
    g = 1.125 * sech4(s)
    upm = u_mean_pm + u_amp_pm * uniform_pm1(seed, instance, 1, shape)
    u0 = 0.5 * (1.0 + upm)
    eps_phi = 3.0 * math.sqrt(2.0) * eps_pm
    eps_u = 0.5 * eps_phi
    ubar = float(0.5 * (1.0 + u_mean_pm))
    if M is None:
        M = 600.0 if dim == 2 else 200.0
    return FixedInputs(shape, hl, g, u0, eps_u, gamma, M, ubar, tau)


def fixed_patch_study(n: int = 256, eps_u_in_h: float = 5.0, M: float = 600.0, tau: float = 1e-4,
                      seed: int = DEFAULT_SEED, instance: int = 0, r0: float = 0.4, eps_phi_in_h: float = 10.0,
                      ubar: float = 0.3, gamma: float = 100.0, patch_fraction: float = 0.35,
                      mem_threshold: float = 1e-3) -> FixedInputs:
    """The fixed circle and protein patch of the temporal convergence study
    (Section 4.1, Tables 1-2) on [-1, 1]^2.

    phi = 0.5 + 0.5 tanh(3 (r0 - r) / eps_phi), r0 = 0.4, eps_phi = 10 h, so
    g = 18 (phi^2 - phi)^2 = (9/8) sech^4(3 (r0 - r) / eps_phi), used in that
    form so that g stays strictly positive in float64.  U^0 = 1 on a connected
    patch Gamma_0 of the membrane region {g >= 1e-3} carrying the fraction
    0.35 = ubar + 0.05 of its g-mass, 0 elsewhere.  The paper draws Gamma_0
    at random without fixing how; here it is the annular sector that starts
    at a seeded uniform angle and grows counter-clockwise: the membrane points
    in order of their angle from the start (stable order), kept while the
    running g-sum stays within 0.35 of the total.
    """
    shape = (n, n)
    h = 2.0 / n
    eps_phi = eps_phi_in_h * h
    X = mesh(shape, (1.0, 1.0))
    r = np.sqrt(X[0] * X[0] + X[1] * X[1])
    g = 1.125 * sech4(3.0 * (r0 - r) / eps_phi)
    mem = g >= mem_threshold
    theta0 = math.pi * (1.0 + float(uniform_pm1(seed, instance, 2, (1,))[0]))
    ang = np.mod(np.arctan2(X[1], X[0]) - theta0, 2.0 * math.pi)
    idx = np.flatnonzero(mem.ravel())
    order = idx[np.argsort(ang.ravel()[idx], kind="stable")]
    csum = np.cumsum(g.ravel()[order])
    keep = order[csum <= patch_fraction * csum[-1]]
    u0 = np.zeros(n * n)
    u0[keep] = 1.0
    return FixedInputs(shape, (1.0, 1.0), g, u0.reshape(shape), eps_u_in_h * h, gamma, M, ubar, tau)


COARSENING_RUNS = (   # (geometry, scheme, gamma) of the 2D coarsening experiments (Section 4.2)
    ("circle", 1, 2000.0), ("circle", 2, 3000.0), ("ellipse", 2, 5000.0), ("protrusions", 2, 7000.0))


def fixed_coarsening(geometry: str = "circle", n: int = 256, gamma: float = 2000.0, M: float = 600.0,
                     tau: float = 1e-3, ubar: float = 0.5, eps_u_in_h: float = 5.0, eps_phi_in_h: float = 10.0,
                     r0: float = 0.4, coarse: int = 8, band_delta: float = 1e-3, seed: int = DEFAULT_SEED,
                     instance: int = 0) -> FixedInputs:
    """The fixed cells of the 2D coarsening experiments (Section 4.2) on
    [-1, 1]^2 with N = 256: phi = 0.5 + 0.5 tanh(3 (r0 - r) / eps_phi),
    eps_phi = 10 h, so g = (9/8) sech^4(3 (r0 - r) / eps_phi) (used in that
    form: positive everywhere), with
      circle       r = sqrt(x^2 + y^2), r0 = 0.4;
      ellipse      r = sqrt(x^2 + sqrt(3) y^2), r0 = 0.4;
      protrusions  r = sqrt(x^2 + y^2), r0 = 0.4 (1 + 0.1 sin 7 theta).
    U^0 is drawn on a coarse grid (blocks of coarse x coarse cells, one
    U(0, 1) value each, seeded) on the band {g >= band_delta}, and ubar
    elsewhere; eps_u = 5 h, ubar = 0.5, tau = 1e-3 as the section states."""
    shape = (n, n)
    h = 2.0 / n
    X, Y = mesh(shape, (1.0, 1.0))
    if geometry == "ellipse":
        r = np.sqrt(X * X + math.sqrt(3.0) * Y * Y)
        rr = np.full(shape, r0)
    else:
        r = np.sqrt(X * X + Y * Y)
        rr = r0 * (1.0 + 0.1 * np.sin(7.0 * np.arctan2(Y, X))) if geometry == "protrusions" else np.full(shape, r0)
    if geometry not in ("circle", "ellipse", "protrusions"):
        raise ValueError(geometry)
    g = 1.125 * sech4(3.0 * (rr - r) / (eps_phi_in_h * h))
    nc = n // coarse
    draws = 0.5 * (1.0 + uniform_pm1(seed, instance, 5, (nc, nc)))
    field = np.repeat(np.repeat(draws, coarse, axis=0), coarse, axis=1)
    u0 = np.where(g >= band_delta, field, ubar)
    return FixedInputs(shape, (1.0, 1.0), g, u0, eps_u_in_h * h, gamma, M, ubar, tau)


# ----------------------------------------------------------------------------
# coupled phi/u inputs (3D, [-pi, pi)^3, eps = 3h)
# ----------------------------------------------------------------------------

@dataclass
class CoupledParams:
    """Model parameters in the paper's [0,1] convention (Section 1, Section 3.1)."""
    mu: float = 2.0
    lambda_surf: float = 1.0
    kappa: float = 1.0
    lambda_line: float = 1.0
    M_area: float = 1.0
    alpha: float = 1.0
    u0: float = 0.0
    eps_phi: float = 0.3
    eps_u: float = 0.15
    gamma: float = 4000.0
    ubar: float = 0.5
    M: float = 500.0
    A1: float = 20.0
    A2: float = 50.0
    B1: float = 1.0
    B2: float = 1000.0
    A0: float = 0.0
    A0_from_initial: int = 1

    def as_dict(self):
        return asdict(self)


@dataclass
class CoupledInputs:
    shape: tuple
    half_len: tuple
    phi0: np.ndarray
    u0: np.ndarray
    params: CoupledParams
    tau: float
    seed: int
    instance: int
    a_lm: np.ndarray = field(default=None)


NAMED_COEFFS = ("kappa", "lambda_surf", "M_area", "lambda_line", "alpha")


def coupled_membrane(n=256, seed: int = DEFAULT_SEED, instance: int = 0, R0: float = 1.5,
                     eps_pm_in_h: float = 3.0, tau: float = 1e-4, half_len: float = math.pi,
                     lmax: int = 4, amp: float = 0.05, base: dict | None = None,
                     coeff_range=(0.5, 2.0), u_amp_pm: float = 0.1, u_mask_pm: float = 0.9,
                     overrides: dict | None = None) -> CoupledInputs:
    """Perturbed-sphere vesicle with a random protein field on its membrane.

    phi_pm = tanh((R(theta, azim) - r) / (sqrt(2) eps_pm)),
    R = R0 (1 + amp * sum_{l=1..lmax, m} a_lm Y_lm), a_lm ~ N(0, 1);
    u_pm = u_amp_pm * U(-1, 1) where |phi_pm| < u_mask_pm; mapped to [0, 1]
    inside the mask and set to 0 outside.  The five named coupling
    coefficients are drawn as base * U(coeff_range).
    """
    shape = tuple(n) if isinstance(n, (tuple, list)) else (n, n, n)
    hl = (half_len,) * 3
    h = 2.0 * half_len / min(shape)
    eps_pm = eps_pm_in_h * h
    X, Y, Z = mesh(shape, hl)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    ct = np.clip(np.divide(Z, r, out=np.ones_like(Z), where=r > 0), -1.0, 1.0)   # cos(theta)
    azim = np.arctan2(Y, X)
    del X, Y, Z
    nco = sum(2 * l + 1 for l in range(1, lmax + 1))
    a = normal(seed, instance, 2, nco)
    # sum_{l=1..lmax, m=-l..l} a_lm Y_lm with a_lm in (l, m) order; the Legendre
    # functions of one order m are built once by the upward recurrence in l
    coef = {}
    c = 0
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            coef[(l, m)] = a[c]
            c += 1
    pert = np.zeros(shape)
    for m in range(0, lmax + 1):
        plm = {m: _assoc_legendre(m, m, ct)}
        if m + 1 <= lmax:
            plm[m + 1] = _assoc_legendre(m + 1, m, ct)
        for l in range(m + 2, lmax + 1):
            plm[l] = ((2 * l - 1) * ct * plm[l - 1] - (l + m - 1) * plm[l - 2]) / (l - m)
        if m == 0:
            for l in range(1, lmax + 1):
                nrm = math.sqrt((2 * l + 1) / (4 * math.pi))
                pert += (coef[(l, 0)] * nrm) * plm[l]
        else:
            cm, sm = np.cos(m * azim), np.sin(m * azim)
            for l in range(m, lmax + 1):
                nrm = math.sqrt(2.0) * math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m)
                                                 / math.factorial(l + m))
                pert += (nrm * plm[l]) * (coef[(l, m)] * cm + coef[(l, -m)] * sm)
    del ct, azim
    R = R0 * (1.0 + amp * pert)
    phi_pm = np.tanh((R - r) / (math.sqrt(2.0) * eps_pm))
    phi0 = 0.5 * (1.0 + phi_pm)
    upm = u_amp_pm * uniform_pm1(seed, instance, 3, shape)
    u0 = np.where(np.abs(phi_pm) < u_mask_pm, 0.5 * (1.0 + upm), 0.0)

    eps_phi = 3.0 * math.sqrt(2.0) * eps_pm
    p = CoupledParams(eps_phi=eps_phi, eps_u=0.5 * eps_phi)
    base = dict(base or {})
    draws = uniform_open01(seed, instance, 4, len(NAMED_COEFFS))
    lo, hi = coeff_range
    for i, name in enumerate(NAMED_COEFFS):
        setattr(p, name, float(base.get(name, 1.0) * (lo + (hi - lo) * draws[i])))
    for k, v in (overrides or {}).items():
        setattr(p, k, v)
    return CoupledInputs(shape, hl, phi0, u0, p, tau, seed, instance, a)


def coupled_membrane_2d(n=256, seed: int = DEFAULT_SEED, instance: int = 0, R0: float = 1.5,
                        eps_pm_in_h: float = 3.0, tau: float = 1e-4, half_len: float = math.pi, mmax: int = 4,
                        amp: float = 0.05, base: dict | None = None, coeff_range=(0.5, 2.0), u_amp_pm: float = 0.1,
                        u_mask_pm: float = 0.9, overrides: dict | None = None) -> CoupledInputs:
    """Two-dimensional counterpart of coupled_membrane: a perturbed circle
    phi_pm = tanh((R(theta) - r) / (sqrt(2) eps_pm)) on [-X, X)^2 with
    R = R0 (1 + amp * sum_{m=1..mmax} (a_m cos m theta + b_m sin m theta) / sqrt(pi)),
    a_m, b_m ~ N(0, 1) (orthonormal Fourier modes of the circle); u, the
    width convention and the parameter draws as in coupled_membrane."""
    shape = tuple(n) if isinstance(n, (tuple, list)) else (n, n)
    hl = (half_len,) * 2
    h = 2.0 * half_len / min(shape)
    eps_pm = eps_pm_in_h * h
    X, Y = mesh(shape, hl)
    r = np.sqrt(X * X + Y * Y)
    theta = np.arctan2(Y, X)
    a = normal(seed, instance, 2, 2 * mmax)
    pert = np.zeros(shape)
    for m in range(1, mmax + 1):
        pert += (a[2 * m - 2] * np.cos(m * theta) + a[2 * m - 1] * np.sin(m * theta)) / math.sqrt(math.pi)
    R = R0 * (1.0 + amp * pert)
    phi_pm = np.tanh((R - r) / (math.sqrt(2.0) * eps_pm))
    phi0 = 0.5 * (1.0 + phi_pm)
    upm = u_amp_pm * uniform_pm1(seed, instance, 3, shape)
    u0 = np.where(np.abs(phi_pm) < u_mask_pm, 0.5 * (1.0 + upm), 0.0)
    eps_phi = 3.0 * math.sqrt(2.0) * eps_pm
    p = CoupledParams(eps_phi=eps_phi, eps_u=0.5 * eps_phi)
    base = dict(base or {})
    draws = uniform_open01(seed, instance, 4, len(NAMED_COEFFS))
    lo, hi = coeff_range
    for i, name in enumerate(NAMED_COEFFS):
        setattr(p, name, float(base.get(name, 1.0) * (lo + (hi - lo) * draws[i])))
    for k, v in (overrides or {}).items():
        setattr(p, k, v)
    return CoupledInputs(shape, hl, phi0, u0, p, tau, seed, instance, a)


def frozen_sphere(n: int = 128, radius: float = 0.5, eps_pm_in_h: float = 2.0, tau: float = 0.02,
                  B2: float = 1000.0, seed: int = DEFAULT_SEED, instance: int = 0, u_mean_pm: float = -0.2,
                  u_amp_pm: float = 0.05, gamma: float = 1.0, M: float = 200.0, dim: int = 3,
                  eps_pm: float | None = None) -> CoupledInputs:
    """The sphere (dim 3) or circle (dim 2) of fixed_membrane(dim, ...) as
    coupled-model inputs, for the coupled scheme's u stages on a frozen
    membrane: phi the [0,1] tanh profile of the same radius and width (so
    g(phi) is that membrane's g up to rounding), the same U^0 draws, eps_u,
    gamma, M, ubar, and the stabilizer B2 given (B1 = 1).  The phi-equation
    coefficients are unused."""
    shape = (n,) * dim
    hl = (1.0,) * dim
    eps_pm = eps_pm if eps_pm is not None else eps_pm_in_h * 2.0 / n
    X = mesh(shape, hl)
    r = np.sqrt(sum(x * x for x in X))
    phi0 = 0.5 * (1.0 + np.tanh((radius - r) / (math.sqrt(2.0) * eps_pm)))
    upm = u_mean_pm + u_amp_pm * uniform_pm1(seed, instance, 1, shape)
    u0 = 0.5 * (1.0 + upm)
    eps_phi = 3.0 * math.sqrt(2.0) * eps_pm
    p = CoupledParams(eps_phi=eps_phi, eps_u=0.5 * eps_phi, gamma=gamma, M=M, ubar=float(0.5 * (1.0 + u_mean_pm)),
                      B1=1.0, B2=B2)
    return CoupledInputs(shape, hl, phi0, u0, p, tau, seed, instance, np.zeros(0))


def batch_sweep(seed: int = DEFAULT_SEED + 5000, counts=((64, 32), (96, 12), (128, 4)),
                taus=(5e-5, 1e-4)) -> list:
    """Uneven batch: instance i gets its own seed stream, coefficients and tau."""
    out = []
    i = 0
    for n, cnt in counts:
        for _ in range(cnt):
            coin = draws_u64(seed, i, 9, 1)[0] & np.uint64(1)
            tau = taus[int(coin)]
            out.append(coupled_membrane(n=n, seed=seed, instance=i, tau=tau))
            i += 1
    return out
