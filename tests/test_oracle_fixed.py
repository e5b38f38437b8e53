"""Pins of the fixed-membrane oracle (Section 2) against the paper's lemmas
and theorems, an independent matrix-exponential route and convergence
orders (CPU only)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import core, fixed
from oracle.band import mass_project
from oracle.core import Grid
from paper_2606_04347_amd import inputs


def small_case(n=16, dim=2, gamma=1.0, M=600.0, eps_pm_in_h=2.0, B=None, seed=11, tau=0.01):
    fi = inputs.fixed_membrane(dim=dim, n=n, eps_pm_in_h=eps_pm_in_h, gamma=gamma, M=M,
                               seed=seed, tau=tau)
    grid = Grid(fi.shape, fi.half_len)
    C = core.lapinv_inf_norm(grid)
    if B is None:
        B = fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, C, grid.volume)
    p = fixed.FixedParams(fi.eps_u, fi.gamma, fi.M, fi.ubar, B)
    return fi, grid, p, C


def dense(op, grid):
    n = int(np.prod(grid.n))
    eye = np.eye(n).reshape((n,) + grid.n)
    return op(eye).reshape(n, n).T


def test_H_annihilates_sqrt_g_and_L_is_symmetric_metzler():
    fi, grid, p, _ = small_case(n=8)
    Hm = dense(lambda w: fixed.H_apply(w, fi.g, grid), grid)
    sg = np.sqrt(fi.g).reshape(-1)
    assert np.abs(Hm @ sg).max() <= 1e-9 * np.abs(Hm).max() * sg.max()
    assert np.abs(Hm - Hm.T).max() <= 1e-10 * np.abs(Hm).max()
    off = Hm - np.diag(np.diag(Hm))
    assert off.max() <= 0.0 and np.all(np.diag(Hm) > 0)          # -L is Metzler
    ev = np.linalg.eigvalsh(0.5 * (Hm + Hm.T))
    assert ev.min() >= -1e-9 * ev.max()


@pytest.mark.parametrize("tau", [1e-3, 0.05])
def test_exponential_positive_and_weighted_contraction(tau):
    """Lemma lemma:LuPD and Lemma lemma:phi_bdd on a tiny grid."""
    fi, grid, p, _ = small_case(n=8)
    Lm = dense(lambda w: fixed.L_apply(w, fi.g, p, grid), grid)
    E = sla.expm(-tau * Lm)
    assert E.min() >= -1e-14 * np.abs(E).max()
    w = np.sqrt(fi.g).reshape(-1)
    # induced weighted norm: max_i sum_j |E_ij| w_j / w_i
    nrm = np.max(np.abs(E) @ w / w)
    assert nrm <= math.exp(-p.B * tau) * (1 + 1e-10)


def test_eta_function_nonpositive():
    a = np.logspace(-4, 3, 2000)
    eta1 = a - a / (1 - np.exp(-a))
    eta2 = a - a * a / (np.expm1(-a) + a)
    eta = eta2 - 0.5 * eta1
    closed = a * (np.exp(-a) * (3 + a - np.exp(-a)) - 2) / (2 * (np.expm1(-a) + a) * (-np.expm1(-a)))
    assert np.all(eta <= 1e-9 * a) and np.all(eta1 <= 0) and np.all(eta1[a < 30] < 0)
    assert np.allclose(eta, closed, rtol=1e-6, atol=1e-9)


def test_dense_expo_matches_augmented_expm():
    """phi_k(tau L) v against the block-matrix exponential (Pade, scipy)."""
    fi, grid, p, _ = small_case(n=8)
    ex = fixed.DenseExpo(fi.g, p, grid)
    assert ex.asym <= 1e-9 * p.B
    rng = np.random.default_rng(5)
    v = rng.standard_normal(grid.n)
    n = v.size
    tau = 2e-4
    A = -tau * ex.L
    aug1 = np.zeros((n + 1, n + 1))
    aug1[:n, :n] = A
    aug1[:n, n] = v.reshape(-1)
    ph1 = sla.expm(aug1)[:n, n]
    # exp([[A, b, 0], [0, 0, 1], [0, 0, 0]]) holds phi2(A) b in its top-right column
    aug2 = np.zeros((n + 2, n + 2))
    aug2[:n, :n] = A
    aug2[:n, n] = v.reshape(-1)
    aug2[n, n + 1] = 1.0
    ph2 = sla.expm(aug2)[:n, n + 1]
    e0 = sla.expm(A) @ v.reshape(-1)
    for fn, ref in ((core.phi0, e0), (core.phi1, ph1), (core.phi2, ph2)):
        got = ex.apply(fn, tau, v).reshape(-1)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [16, 32])
def test_lanczos_matches_dense(n):
    fi, grid, p, _ = small_case(n=n)
    d = fixed.DenseExpo(fi.g, p, grid)
    lz = fixed.LanczosExpo(fi.g, p, grid)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(grid.n)
    for tau in (1e-4, 0.01):
        for fn in (core.phi0, core.phi1, core.phi2):
            a, b = d.apply(fn, tau, v), lz.apply(fn, tau, v)
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("scheme", [1, 2])
def test_exact_for_constant_remainder(scheme):
    """Variation of constants: ETD reproduces the exact solution when R is
    constant in time (Section 2.2), for any tau."""
    fi, grid, p, _ = small_case(n=8)
    ex = fixed.DenseExpo(fi.g, p, grid)
    rng = np.random.default_rng(7)
    c = rng.standard_normal(grid.n) * p.B
    Rconst = lambda U, g, pp, gr: c
    sg = np.sqrt(fi.g)
    U = fi.u0.copy()
    tau, nsteps = 3e-4, 5
    for _ in range(nsteps):
        U = fixed.step(U, fi.g, p, grid, tau, scheme, ex, R=Rconst)
    Lm = ex.L
    T = nsteps * tau
    E = sla.expm(-T * Lm)
    w0 = (sg * fi.u0).reshape(-1)
    exact = E @ w0 + (np.eye(Lm.shape[0]) - E) @ np.linalg.solve(Lm, c.reshape(-1))
    got = (sg * U).reshape(-1)
    assert np.abs(got - exact).max() <= 1e-12 * np.abs(exact).max()


def test_lemma_MBPbdd_remainder_bounds():
    """Lemma lemma:MBPbdd: R(u) >= 0 and ||R(u)||_{inf, sqrt g} <= B for 0 <= u <= 1."""
    for gamma in (1.0, 50.0):
        fi, grid, p, _ = small_case(n=16, gamma=gamma)
        rng = np.random.default_rng(8)
        for U in (rng.random(grid.n), (rng.random(grid.n) > 0.5).astype(float),
                  np.zeros(grid.n), np.ones(grid.n)):
            R = fixed.R_phi(U, fi.g, p, grid)
            sg = np.sqrt(fi.g)
            assert R.min() >= -1e-10 * p.B * sg.max()
            assert np.max(np.abs(R) / sg) <= p.B * (1 + 1e-12)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("tau", [0.01, 1.0])
def test_maximum_bound_principle(scheme, tau):
    """Theorem thm:MBP: 0 <= U^n <= 1 for every step when B >= B_MBP."""
    fi, grid, p, _ = small_case(n=16, gamma=20.0)
    ex = fixed.DenseExpo(fi.g, p, grid)
    rng = np.random.default_rng(9)
    for U in (rng.random(grid.n), (rng.random(grid.n) > 0.6).astype(float)):
        for _ in range(20):
            U = fixed.step(U, fi.g, p, grid, tau, scheme, ex)
            assert U.min() >= -1e-12 and U.max() <= 1 + 1e-12


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("which", ["ES", "MBP"])
def test_energy_decay(scheme, which):
    """Theorem thm:Energy: E_{phi,h}[U^{n+1}] <= E_{phi,h}[U^n]."""
    fi, grid, p, C = small_case(n=16, gamma=20.0, M=50.0)
    if which == "ES":
        p.B = fixed.B_es(p.eps_u, p.gamma, p.M, C, grid.volume)
    ex = fixed.DenseExpo(fi.g, p, grid)
    rng = np.random.default_rng(10)
    U = rng.random(grid.n)
    E = fixed.energy(U, fi.g, p, grid)["E"]
    for _ in range(30):
        U = fixed.step(U, fi.g, p, grid, 0.05, scheme, ex)
        E1 = fixed.energy(U, fi.g, p, grid)["E"]
        assert E1 <= E + 1e-13 * abs(E)
        E = E1


def test_energy_terms_two_routes():
    fi, grid, p, _ = small_case(n=16, gamma=20.0)
    U = np.random.default_rng(12).random(grid.n)
    e = fixed.energy(U, fi.g, p, grid)
    # gradient term in edge form: (eps_u/2) h^d sum_d sum g_{i+1/2} (D+ U)^2
    edge = 0.0
    for d, h in enumerate(grid.h):
        gh = 0.5 * (fi.g + np.roll(fi.g, -1, axis=d))
        edge += np.sum(gh * ((np.roll(U, -1, axis=d) - U) / h) ** 2)
    assert abs(e["E_grad"] - 0.5 * p.eps_u * grid.cell * edge) <= 1e-12 * e["E_grad"]
    # nonlocal term by Parseval
    q = fi.g * core.f_ind(U)
    Q = np.fft.fftn(q)
    mu = core.fd_symbol(grid)
    nz = mu > 0
    pars = grid.cell * np.sum(np.abs(Q[nz]) ** 2 / mu[nz]) / q.size
    assert abs(e["E_nonlocal"] - 0.5 * p.gamma * pars) <= 1e-12 * e["E_nonlocal"]


def _rhs_direct(U, g, p, grid):
    """dU/dt of (eqn:model_OK_fix) divided by g, written without the split."""
    fu = core.f_ind(U)
    psi = core.lapinv(g * fu, grid)
    m = grid.cell * np.sum(g * (fu - p.ubar))
    return (p.eps_u * core.lap_S(U, g, grid) - g * core.Wp(U) / p.eps_u
            - p.gamma * g * core.fp_ind(U) * psi - p.M * g * core.fp_ind(U) * m) / g


@pytest.mark.parametrize("scheme", [1, 2])
def test_small_tau_limit_is_the_pde(scheme):
    """(U(tau) - U0)/tau -> RHS, independent of the stabilizer B."""
    fi, grid, p, _ = small_case(n=16, gamma=5.0, M=5.0, eps_pm_in_h=3.0)
    U0 = np.random.default_rng(13).random(grid.n)
    rhs = _rhs_direct(U0, fi.g, p, grid)
    errs = []
    for tau in (1e-8, 5e-9):
        for B in (p.B, 3 * p.B):
            pp = fixed.FixedParams(p.eps_u, p.gamma, p.M, p.ubar, B)
            ex = fixed.DenseExpo(fi.g, pp, grid)
            U1 = fixed.step(U0, fi.g, pp, grid, tau, scheme, ex)
            errs.append(np.abs((U1 - U0) / tau - rhs).max() / np.abs(rhs).max())
    assert max(errs) < 5e-3


def _convergence_errors(scheme):
    fi, grid, p, C = small_case(n=16, gamma=1.0, M=1.0, eps_pm_in_h=4.0)
    ex = fixed.DenseExpo(fi.g, p, grid)
    T = 0.004
    ref = fi.u0.copy()
    nref = 512
    for _ in range(nref):
        ref = fixed.etdrk2_step(ref, fi.g, p, grid, T / nref, ex)
    errs = []
    for k in range(4):
        nst = 4 * 2 ** k
        U = fi.u0.copy()
        for _ in range(nst):
            U = fixed.step(U, fi.g, p, grid, T / nst, scheme, ex)
        errs.append(np.abs(U - ref).max())
    return np.array(errs), p.B * T / 4


@pytest.mark.parametrize("scheme,lo,hi", [(1, 0.85, 1.2), (2, 1.75, 2.3)])
def test_temporal_convergence_order(scheme, lo, hi):
    errs, tauB = _convergence_errors(scheme)
    rates = np.log2(errs[:-1] / errs[1:])
    assert lo <= rates[-1] <= hi, (errs, rates, tauB)


def test_mass_projection_restores_Q():
    fi, grid, p, _ = small_case(n=16)
    U = np.random.default_rng(14).random(grid.n)
    Q0 = 0.123
    U2 = mass_project(U, fi.g, Q0, grid, 1e-3)
    assert abs(grid.cell * np.sum(fi.g * U2) - Q0) <= 1e-14 * max(1, abs(Q0)) + 1e-15


def test_uspace_expo_matches_dense_where_both_are_accurate():
    """The U-space block exponential and the eigendecomposition agree on a
    grid whose g stays well above rounding (g_min ~ 1e-4)."""
    fi, grid, p, _ = small_case(n=16, eps_pm_in_h=4.0)
    assert fi.g.min() > 1e-5
    tau = 1e-4
    d = fixed.DenseExpo(fi.g, p, grid)
    us = fixed.UspaceExpo(fi.g, p, grid, tau)
    v = np.sqrt(fi.g) * np.random.default_rng(15).standard_normal(grid.n)
    for fn in (core.phi0, core.phi1, core.phi2):
        a, b = d.apply(fn, tau, v), us.apply(fn, tau, v)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_uspace_expo_exact_for_constant_remainder_with_tiny_g():
    """Variation of constants in the U variable where g reaches 1e-17: with a
    remainder sqrt(g) c (c constant in time) one ETD1 step of size tau equals
    e^{-tau Lt} U0 + tau phi1(tau Lt) c, evaluated independently in the
    eigenbasis of the symmetric part (valid here: Lt is similar to L)."""
    fi = inputs.fixed_membrane(dim=2, n=16, eps_pm=0.0625)
    grid = Grid(fi.shape, fi.half_len)
    assert fi.g.min() < 1e-12
    C = core.lapinv_inf_norm(grid)
    p = fixed.FixedParams(fi.eps_u, fi.gamma, fi.M, fi.ubar, fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, C, grid.volume))
    tau = 0.01
    us = fixed.UspaceExpo(fi.g, p, grid, tau)
    c = np.cos(np.arange(fi.g.size)).reshape(grid.n)
    sg = np.sqrt(fi.g)
    U1 = fixed.etd1_step(fi.u0, fi.g, p, grid, tau, us, R=lambda U, g, pp, gr: sg * c)
    # U-space operator applied to U1 recovers the ODE balance: for constant forcing the
    # exact solution satisfies (U1 - e^{-tau Lt} U0) = tau phi1(tau Lt) c; check it through
    # the identity (I - e^{-tau Lt}) Lt^{-1} c = tau phi1(tau Lt) c
    n = fi.g.size
    eye = np.eye(n).reshape((n,) + grid.n)
    Lt = (p.B * eye - p.eps_u * core.lap_S(eye, fi.g, grid) / fi.g).reshape(n, n).T
    E0 = us.mats[core.phi0]
    lhs = (U1.reshape(-1) - E0 @ fi.u0.reshape(-1))
    rhs = np.linalg.solve(Lt, (np.eye(n) - E0) @ c.reshape(-1))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_band_nonlocal_enters_only_through_gamma():
    """band_delta > 0 replaces (-Delta_h)^{-1} by the band solve in the gamma
    term of R_phi only: with gamma = 0 the remainders agree bit for bit."""
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
    grid = Grid(fi.shape, fi.half_len)
    U = fi.u0
    out = {}
    for gamma in (0.0, 5.0):
        r = [fixed.R_phi(U, fi.g, fixed.FixedParams(fi.eps_u, gamma, fi.M, fi.ubar, 100.0, False, d), grid)
             for d in (0.0, 1e-3)]
        out[gamma] = r
    assert np.array_equal(out[0.0][0], out[0.0][1])
    assert np.abs(out[5.0][0] - out[5.0][1]).max() > 1e-6


def test_band_inverse_norm_of_the_config1_circle():
    """C of the band inverse for the 64^2 circle of config 1 on {g >= 1e-3},
    by the dense oracle, beside the circulant C of (-Delta_h)^{-1}: the band
    operator has much weaker coefficients (g <= 9/8, small at the band edge),
    so its inverse is larger; both are finite and positive."""
    fi = inputs.fixed_membrane(dim=2, n=64)
    grid = Grid(fi.shape, fi.half_len)
    Cb = core.lapinv_S_band_inf_norm(fi.g, fi.g >= 1e-3, grid)
    C = core.lapinv_inf_norm(grid)
    print(f"C band {Cb:.6g}, C periodic {C:.6g}")
    assert np.isfinite(Cb) and Cb > C > 0


def test_stabilizer_constants_of_the_64sq_circle():
    """eqn:cond_MBP and eqn:cond_ES evaluated by hand for the 64^2 circle
    (eps_pm = 0.0625 so eps_u = 3 sqrt(2) 0.0625 / 2 = 0.1325825, gamma = 1,
    M = 600, |Omega| = 4, C = ||(-Delta_h)^{-1}||_inf = 0.1678365 on
    [-1, 1)^2, L_W'' = 36, L_f'' = 6, L_f' = 3/2, L_g = 9/8):
      B_MBP = 36/eps_u + (gamma C + M |Omega|) L_f'' L_g
            = 271.5290 + 2400.1678 * 6.75 = 16,472.66
      B_ES  = 36/eps_u + (gamma C / 2 + M |Omega| / 2) (L_f'' + L_f'^2) L_g
            = 271.5290 + 1200.0839 * 9.28125 = 11,409.81"""
    fi = inputs.fixed_membrane(dim=2, n=64, eps_pm=0.0625)
    grid = Grid(fi.shape, fi.half_len)
    C = core.lapinv_inf_norm(grid)
    assert abs(C - 0.1678365) < 1e-6
    assert abs(fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, C, grid.volume) - 16472.66) < 0.01
    assert abs(fixed.B_es(fi.eps_u, fi.gamma, fi.M, C, grid.volume) - 11409.81) < 0.01


def test_band_step_on_a_band_holding_every_node_is_the_full_step():
    """The restricted step with a band that holds every node (threshold below
    min g) is the full-grid step, bit for bit."""
    fi, grid, p, _ = small_case(n=16)
    pb = fixed.FixedParams(p.eps_u, p.gamma, p.M, p.ubar, p.B, band_step=0.5 * float(fi.g.min()))
    for scheme in (1, 2):
        a = fixed.step(fi.u0, fi.g, p, grid, fi.tau, scheme, fixed.DenseExpo(fi.g, p, grid))
        b = fixed.step(fi.u0, fi.g, pb, grid, fi.tau, scheme, fixed.DenseExpo(fi.g, pb, grid))
        assert np.array_equal(a, b)


@pytest.mark.parametrize("scheme", [1, 2])
def test_band_step_keeps_the_theorems_and_the_off_band_values(scheme):
    """The step restricted to {g >= 1e-3} (faces with both nodes on the band):
    H on the band is symmetric positive semidefinite with H sqrt(g) = 0 on
    its rows (the properties the proofs of Lemma lemma:LuPD and Theorems
    thm:MBP, thm:Energy use), so with B = B_MBP the band system keeps
    0 <= U <= 1 and a non-increasing energy; U off the band never changes."""
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm_in_h=2.0, tau=0.01, seed=13)
    grid = Grid(fi.shape, fi.half_len)
    C = core.lapinv_inf_norm(grid)
    B = fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, C, grid.volume)
    p = fixed.FixedParams(fi.eps_u, fi.gamma, fi.M, fi.ubar, B, band_step=1e-3)
    band = fixed.step_band(fi.g, p)
    assert 0 < band.sum() < band.size
    n = band.size
    eye = np.eye(n).reshape((n,) + fi.shape)
    H = fixed.H_apply(eye, fi.g, grid, band).reshape(n, n).T
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    Hb = H[np.ix_(band.ravel(), band.ravel())]
    assert np.linalg.eigvalsh(0.5 * (Hb + Hb.T)).min() >= -1e-9 * np.abs(Hb).max()
    assert np.abs(fixed.H_apply(np.sqrt(fi.g), fi.g, grid, band)).max() <= 1e-9 * np.abs(H).max()
    ex = fixed.UspaceExpo(fi.g, p, grid, fi.tau)
    U = fi.u0.copy()
    E0 = fixed.energy(U, fi.g, p, grid)["E"]
    for _ in range(12):
        U1 = fixed.step(U, fi.g, p, grid, fi.tau, scheme, ex)
        assert np.array_equal(U1[~band], fi.u0[~band])
        assert U1.min() >= -1e-14 and U1.max() <= 1.0 + 1e-14
        E1 = fixed.energy(U1, fi.g, p, grid)["E"]
        assert E1 <= E0 + 1e-13 * abs(E0)
        U, E0 = U1, E1
    assert np.abs(U - fi.u0)[band].max() > 1e-6     # the band moved
