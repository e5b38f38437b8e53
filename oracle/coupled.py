"""Coupled phi/u system: stabilized spectral ETD1 / ETDRK2 (Section 3).

TEST INFRASTRUCTURE ONLY (see the package header).  FP64, full complex
spectra (indices 0..N-1 per axis, as in Section 3.2), real parts taken after
each inverse transform.

Splitting (Section 3.1):
  phi_t + L_phi phi = R1(phi, u),   (g u)_t + L_u (g u) = R2(phi, u),
  symbol l_phi = (kappa/mu) k^4 + [kappa (A1 + A2) + lambda_surf eps^2]/(mu eps^2) k^2
                 + [kappa A1 A2 + lambda_surf A1 eps^2]/(mu eps^4)      (eqn:linear_force)
  symbol l_u   = B2 + eps_u B1 k^2                                       (eqn:linear_OK)
with k^2 = -lambda_ijk.  R1 collects every other term of (eqn:model_force)/mu:
  R1 = (kappa/(mu eps^2)) Delta(W'(phi) - A1 phi) + P1, where
  P1 = (kappa/(mu eps^2)) (W''(phi) - A2)(Delta phi - A1 phi/eps^2)
       - (kappa W''(phi)/(mu eps^4) + lambda_surf/(mu eps^2)) (W'(phi) - A1 phi)
       + (lambda_line/mu)(eps_u Delta_S u - g W'(u)/eps_u)|grad phi|
       - (M_area/mu)(int phi - A0)|grad phi|
       + (alpha/mu)(u + u0)|grad phi| (eps_phi Delta phi - W'(phi)/eps_phi);
and R2 = -eps_u B1 Delta(g u) + P2 with
  P2 = eps_u Delta_S u + B2 g u - g W'(u)/eps_u - gamma g (-Delta)^{-1}(g (u - ubar))
       - M g int g (u - ubar) - div(g u v).

Readings (ambiguity register; listed in the design notes):
  * every derivative of phi is spectral (Delta: -k^2; first derivatives:
    i k_d with the Nyquist bin zeroed); every derivative involving u is the
    second-order FD of Section 2.1 (Delta_S u with g(phi) of the stage, and a
    central-difference divergence for the advection flux);
  * the stabilizer -eps_u B1 Delta(g u) is folded in Fourier space with the
    same k^2 as l_u, so it cancels L_u exactly;
  * (-Delta)^{-1} is the constant-coefficient periodic FD pseudo-inverse;
  * v = -((phi^{n+1} - phi^n)/tau) grad phi^{n+1} / |grad phi^{n+1}|^2 where
    g(phi^{n+1}) > recover threshold and |grad phi^{n+1}|^2 > 0, else 0;
  * the phi stages freeze u at u^n; the u stages use g(phi^{n+1}) and restart
    from FFT(g(phi^{n+1}) u^n) (Section 3.3);
  * A0 = int phi^0 when ``A0_from_initial``;
  * ``surface_nonlocal``: the nonlocal term uses (-Delta_{S,h})^{-1}
    set up and inverted on the band (core.lapinv_S_band, with g = g+ of
    the stage) instead of the constant-coefficient (-Delta_h)^{-1}; the
    energy diagnostic keeps (-Delta_h)^{-1};
  * ``frozen_membrane``: phi keeps its initial value and only the g u
    stages run, with g = g(phi^0) and v = 0 (the stabilized scheme of
    Section 3.1 on a fixed membrane);
  * with a narrow band (mask from |2 phi - 1| < threshold, rebuilt every
    ``band_rebuild_every`` steps from the current phi), P2, the nonlocal input
    g (u - ubar) and the three |grad phi|-weighted terms of P1 are zero off the
    band.

Pins (tests/test_oracle_coupled.py): the splitting identities of R1 and R2
against the model equations written directly, the exact per-mode solution
for constant remainders, the small-tau limits of both stages, symmetry, the
decoupled-limit orders, the velocity of a translating wave, and the energy
terms through their first variations.  The paper prints no coupled
trajectory values, so long runs are held against this oracle, not against
printed numbers.
"""
from __future__ import annotations

import numpy as np

from . import core
from .band import band_mask, mass_project, recover
from .core import Grid


class CoupledOracle:
    def __init__(self, grid: Grid, p, tau: float, scheme: int = 2,
                 recover_threshold: float = 1e-3, band_threshold: float = 0.0,
                 band_rebuild_every: int = 10, mass_projection: bool = False,
                 frozen_membrane: bool = False, surface_nonlocal: bool = False):
        self.grid, self.p, self.tau, self.scheme = grid, p, float(tau), int(scheme)
        self.thr = float(recover_threshold)
        self.band_thr = float(band_threshold)
        self.band_every = max(1, int(band_rebuild_every))
        self.mass_projection = bool(mass_projection)
        self.frozen = bool(frozen_membrane)
        self.surface = bool(surface_nonlocal)
        if self.surface and self.band_thr <= 0.0:
            raise ValueError("the band solve of the nonlocal term needs a band")
        k2 = core.ksq(grid)
        self.k2 = k2
        self.kd = [core.kder(grid, d) for d in range(grid.dim)]
        e2 = p.eps_phi ** 2
        self.lphi = (p.kappa / p.mu) * k2 * k2 \
            + (p.kappa * (p.A1 + p.A2) + p.lambda_surf * e2) / (p.mu * e2) * k2 \
            + (p.kappa * p.A1 * p.A2 + p.lambda_surf * p.A1 * e2) / (p.mu * e2 * e2)
        self.lu = p.B2 + p.eps_u * p.B1 * k2
        self.set_tau(tau)
        self.mask = None
        self.n = 0

    def set_tau(self, tau):
        """Step size tau_{n+1} of the next steps (Section 3.3 writes both schemes
        with a per-step tau: the phi-functions, the step and phi_t take it)."""
        self.tau = float(tau)
        zt, zu = self.tau * self.lphi, self.tau * self.lu
        self.E0p, self.E1p, self.E2p = core.phi0(zt), core.phi1(zt), core.phi2(zt)
        self.E0u, self.E1u, self.E2u = core.phi0(zu), core.phi1(zu), core.phi2(zu)

    # ------------------------------------------------------------------ state
    def set_state(self, phi, u):
        self.phi_hat = core.fft(phi)
        self.u = np.array(u, dtype=np.float64)
        self.A0 = self.grid.cell * float(np.sum(phi)) if self.p.A0_from_initial else float(self.p.A0)
        self.Q0 = self.grid.cell * float(np.sum(core.g_loc(np.asarray(phi)) * self.u))
        self.n = 0
        self.mask = None

    def phi(self):
        return core.ifft(self.phi_hat)

    # ------------------------------------------------------------- remainders
    def _derivs(self, phi_hat):
        phi = core.ifft(phi_hat)
        lap = core.ifft(-self.k2 * phi_hat)
        grad = [core.ifft(1j * k * phi_hat) for k in self.kd]
        return phi, lap, grad

    def R1_hat(self, phi_hat, u):
        p, grid = self.p, self.grid
        phi, lap, grad = self._derivs(phi_hat)
        gnorm = np.sqrt(sum(gd * gd for gd in grad))
        g = core.g_loc(phi)
        S = core.lap_S(u, g, grid)
        I_phi = grid.cell * float(np.sum(phi))
        e2 = p.eps_phi ** 2
        c1 = p.kappa / (p.mu * e2)
        Wp, Wpp = core.Wp(phi), core.Wpp(phi)
        Q1 = Wp - p.A1 * phi
        P1 = c1 * (Wpp - p.A2) * (lap - p.A1 * phi / e2) \
            - (p.kappa * Wpp / (p.mu * e2 * e2) + p.lambda_surf / (p.mu * e2)) * Q1
        surf = (p.lambda_line / p.mu) * (p.eps_u * S - g * core.Wp(u) / p.eps_u) * gnorm \
            - (p.M_area / p.mu) * (I_phi - self.A0) * gnorm \
            + (p.alpha / p.mu) * (u + p.u0) * gnorm * (p.eps_phi * lap - Wp / p.eps_phi)
        if self.mask is not None:
            surf = surf * self.mask
        return core.fft(P1 + surf) - c1 * self.k2 * core.fft(Q1)

    def velocity(self, phi_old, phi_new_hat, g_new):
        phi_new, _, grad = self._derivs(phi_new_hat)
        gn2 = sum(gd * gd for gd in grad)
        sel = (g_new > self.thr) & (gn2 > 0.0)
        dphidt = (phi_new - phi_old) / self.tau
        safe = np.where(sel, gn2, 1.0)
        return [np.where(sel, -dphidt * gd / safe, 0.0) for gd in grad]

    def R2_hat(self, u, g, v):
        p, grid = self.p, self.grid
        S = core.lap_S(u, g, grid)
        q = g * (u - p.ubar)
        if self.mask is not None:
            q = q * self.mask
        m = grid.cell * float(np.sum(q))
        psi = core.lapinv_S_band(q, g, self.mask, grid) if self.surface else core.lapinv(q, grid)
        flux = [g * u * vd for vd in v]
        P2 = p.eps_u * S + p.B2 * g * u - g * core.Wp(u) / p.eps_u \
            - p.gamma * g * psi - p.M * g * m - core.div_central(flux, grid)
        if self.mask is not None:
            P2 = P2 * self.mask
        return core.fft(P2) + p.eps_u * p.B1 * self.k2 * core.fft(g * u)

    # ------------------------------------------------------------------- step
    def step(self):
        """One step of Algorithm 1 (ETD1 or ETDRK2)."""
        tau = self.tau
        phi_n = self.phi()
        if self.band_thr > 0.0 and self.n % self.band_every == 0:
            self.mask = band_mask(phi_n, self.band_thr)
        u = self.u
        if self.frozen:
            # fixed membrane: phi^{n+1} = phi^n, so g+ = g(phi^n) and v = 0
            phi_new_hat = self.phi_hat
            g_new = core.g_loc(phi_n)
            v = [np.zeros_like(u) for _ in range(self.grid.dim)]
        else:
            # phi update, u frozen at u^n
            R1a = self.R1_hat(self.phi_hat, u)
            phit_hat = self.E0p * self.phi_hat + tau * self.E1p * R1a
            if self.scheme == 1:
                phi_new_hat = phit_hat
            else:
                R1b = self.R1_hat(phit_hat, u)
                phi_new_hat = phit_hat + tau * self.E2p * (R1b - R1a)
            phi_new = core.ifft(phi_new_hat)
            g_new = core.g_loc(phi_new)
            v = self.velocity(phi_n, phi_new_hat, g_new)
        # g u update with g = g(phi^{n+1})
        GU0 = core.fft(g_new * u)
        R2a = self.R2_hat(u, g_new, v)
        GUt_hat = self.E0u * GU0 + tau * self.E1u * R2a
        Ut = recover(core.ifft(GUt_hat), g_new, self.thr)
        if self.scheme == 1:
            u_new = Ut
        else:
            R2b = self.R2_hat(Ut, g_new, v)
            GU_hat = GUt_hat + tau * self.E2u * (R2b - R2a)
            u_new = recover(core.ifft(GU_hat), g_new, self.thr)
        if self.mass_projection:
            u_new = mass_project(u_new, g_new, self.Q0, self.grid, self.thr)
        self.phi_hat, self.u = phi_new_hat, u_new
        self.n += 1

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    # ----------------------------------------------------------- diagnostics
    def energy(self) -> dict:
        p, grid = self.p, self.grid
        phi, lap, grad = self._derivs(self.phi_hat)
        e2 = p.eps_phi ** 2
        one = np.ones_like(phi)
        gn2 = sum(gd * gd for gd in grad)
        e_surf = p.lambda_surf * core.inner(0.5 * gn2 + core.W(phi) / e2, one, grid)
        e_bend = 0.5 * p.kappa * core.inner((lap - core.Wp(phi) / e2) ** 2, one, grid)
        I_phi = grid.cell * float(np.sum(phi))
        e_area = 0.5 * p.M_area * (I_phi - self.A0) ** 2
        u = self.u
        g = core.g_loc(phi)
        e_ok = 0.5 * p.eps_u * core.inner(-core.lap_S(u, g, grid), u, grid) \
            + core.inner(g * core.W(u), one, grid) / p.eps_u
        q = g * (u - p.ubar)
        e_nl = 0.5 * p.gamma * core.inner(core.lapinv(q, grid), q, grid)
        mq = grid.cell * float(np.sum(q))
        e_mass = 0.5 * p.M * mq * mq
        return dict(E_surf=e_surf, E_bend=e_bend, E_area=e_area, E_ok=e_ok,
                    E_nonlocal=e_nl, E_mass=e_mass)

    def diagnostics(self) -> dict:
        phi = self.phi()
        g = core.g_loc(phi)
        u = self.u
        return dict(I_phi=self.grid.cell * float(np.sum(phi)),
                    m=self.grid.cell * float(np.sum(g * (u - self.p.ubar))),
                    Q=self.grid.cell * float(np.sum(g * u)),
                    umin=float(u.min()), umax=float(u.max()),
                    bound=float(np.abs(2.0 * u - 1.0).max()))
