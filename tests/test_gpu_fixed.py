"""GPU: the fixed-membrane localization-split ETD1/ETDRK2 step (Section 2.2)
through the C ABI against the FP64 oracle, plus the discrete maximum bound
principle and energy decay on the GPU."""
import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, rel_linf, report, torch
from oracle import core, fixed
from oracle.core import Grid
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


def oracle_params(fi, B=None):
    grid = Grid(fi.shape, fi.half_len)
    C = core.lapinv_inf_norm(grid)
    Bm = fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, C, grid.volume)
    return grid, fixed.FixedParams(fi.eps_u, fi.gamma, fi.M, fi.ubar, Bm if B is None else B), C


def gpu_run(fi, scheme, nsteps, precision=etd.FP64, B=0.0, flags=0, **kw):
    plan = etd.Plan(etd.fixed_instance(fi, B=B, scheme=scheme, precision=precision, flags=flags, **kw))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    plan.step(nsteps)
    _, u = plan.get_state(0)
    return plan, host(u)


def test_constants_match_oracle():
    fi = inputs.fixed_membrane(dim=2, n=64)
    grid, p, C = oracle_params(fi)
    plan = etd.Plan(etd.fixed_instance(fi))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    assert abs(plan.query(0, etd.Q_C) - C) <= 1e-12 * C
    assert abs(plan.query(0, etd.Q_B_MBP) - p.B) <= 1e-12 * p.B
    assert abs(plan.query(0, etd.Q_B) - p.B) <= 1e-12 * p.B
    Bes = fixed.B_es(fi.eps_u, fi.gamma, fi.M, C, grid.volume)
    assert abs(plan.query(0, etd.Q_B_ES) - Bes) <= 1e-12 * Bes
    report("fixed_constants", C=plan.query(0, etd.Q_C), B=plan.query(0, etd.Q_B),
           rho=plan.query(0, etd.Q_RHO), deg=plan.query(0, etd.Q_CHEB_DEG))
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_fp64_2d_matches_uspace_oracle(scheme):
    """Config-1 geometry (eps = 0.0625) on 32^2: g reaches 1e-17, and the U-space
    block-exponential oracle resolves U there to rounding."""
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
    assert fi.g.min() < 1e-15
    grid, p, _ = oracle_params(fi)
    ex = fixed.UspaceExpo(fi.g, p, grid, fi.tau)
    U = fi.u0.copy()
    for _ in range(10):
        U = fixed.step(U, fi.g, p, grid, fi.tau, scheme, ex)
    plan, Ug = gpu_run(fi, scheme, 10)
    err = rel_linf(Ug, U)
    report("fixed2d_fp64", scheme=scheme, err=err)
    assert err <= 1e-12
    e, oe = plan.energy(0), fixed.energy(U, fi.g, p, grid)
    for k in ("E", "E_grad", "E_well", "E_nonlocal", "E_mass"):
        assert abs(e[k] - oe[k]) <= 1e-11 * max(abs(oe[k]), 1e-12), (k, e[k], oe[k])
    d, od = plan.diagnostics(0), fixed.diagnostics(U, fi.g, p, grid)
    for k in ("mass", "Q", "umin", "umax", "bound"):
        ok = {"mass": "m"}.get(k, k)
        assert abs(d[k] - od[ok]) <= 1e-11 * max(1.0, abs(od[ok])), (k, d[k], od[ok])
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_variable_step_matches_uspace_oracle(scheme):
    """etd_set_tau between steps re-forms the Chebyshev coefficients; the
    U-space oracle steps the same tau sequence (one exponential per tau)."""
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
    grid, p, _ = oracle_params(fi)
    seq = (fi.tau, 2 * fi.tau, 0.5 * fi.tau, fi.tau)
    ex = {t: fixed.UspaceExpo(fi.g, p, grid, t) for t in set(seq)}
    U = fi.u0.copy()
    plan = etd.Plan(etd.fixed_instance(fi, scheme=scheme))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    degs = []
    for t in seq:
        U = fixed.step(U, fi.g, p, grid, t, scheme, ex[t])
        plan.set_tau(0, t)
        degs.append(plan.query(0, etd.Q_CHEB_DEG))
        plan.step(1)
    _, u = plan.get_state(0)
    err = rel_linf(host(u), U)
    report("fixed_variable_tau", scheme=scheme, err=err, degrees=str(degs))
    assert err <= 1e-12
    plan.close()


def test_fp64_config1_64x64_etd1_matches_oracle():
    """64^2 config 1 against the eigendecomposition oracle, compared in the
    scheme's own variable w = sqrt(g) U (eqn:ODE_eqn): the dense route is
    accurate to rounding relative to max |w|, not where sqrt(g) ~ 4e-9."""
    fi = inputs.fixed_membrane(dim=2, n=64)
    grid, p, _ = oracle_params(fi)
    ex = fixed.DenseExpo(fi.g, p, grid)
    U = fi.u0.copy()
    for _ in range(5):
        U = fixed.etd1_step(U, fi.g, p, grid, fi.tau, ex)
    plan, Ug = gpu_run(fi, etd.ETD1, 5)
    sg = np.sqrt(fi.g)
    err_w = rel_linf(sg * Ug, sg * U)
    sel = fi.g >= 1e-4          # where the dense route's w-space rounding stays below 1e-12 in U
    err_u = rel_linf(Ug[sel], U[sel])
    report("fixed_config1", err_w=err_w, err_u_g_ge_1e4=err_u, err_u_all=rel_linf(Ug, U))
    assert err_w <= 1e-12 and err_u <= 1e-12
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_fp64_3d_matches_lanczos_oracle(scheme):
    fi = inputs.fixed_membrane(dim=3, n=24, eps_pm_in_h=2.0, tau=0.02)
    grid, p, _ = oracle_params(fi)
    ex = fixed.LanczosExpo(fi.g, p, grid)
    U = fi.u0.copy()
    for _ in range(3):
        U = fixed.step(U, fi.g, p, grid, fi.tau, scheme, ex)
    plan, Ug = gpu_run(fi, scheme, 3)
    err = rel_linf(Ug, U)
    report("fixed3d_fp64", scheme=scheme, err=err)
    assert err <= 1e-12
    plan.close()


@pytest.mark.parametrize("n", [12, (16, 24, 48)])
def test_fp64_3d_two_term_passes_on_ragged_tiles(n):
    """On 3D grids the recurrence runs two terms per pass over tiles of 8 x
    planes, 16 y rows and 32 z nodes: 12^3 has a ragged x segment and y and z
    tiles wider than the grid (their halos wrap more than once), 16 x 24 x 48
    ragged y and z tiles.  ETDRK2 against the Lanczos oracle."""
    fi = inputs.fixed_membrane(dim=3, n=n, eps_pm_in_h=2.0, tau=0.02)
    grid, p, _ = oracle_params(fi)
    ex = fixed.LanczosExpo(fi.g, p, grid)
    U = fi.u0.copy()
    for _ in range(2):
        U = fixed.step(U, fi.g, p, grid, fi.tau, etd.ETDRK2, ex)
    plan, Ug = gpu_run(fi, etd.ETDRK2, 2)
    err = rel_linf(Ug, U)
    report("fixed3d_pair", n=str(n), err=err, degree=plan.query(0, etd.Q_CHEB_DEG))
    assert err <= 1e-12
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_mbp_and_energy_decay_on_gpu(scheme):
    """Theorems thm:MBP and thm:Energy on the 64^2 configuration, 200 steps."""
    fi = inputs.fixed_membrane(dim=2, n=64)
    plan = etd.Plan(etd.fixed_instance(fi, scheme=scheme))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    E0 = plan.energy(0)["E"]
    for k in range(20):
        plan.step(10)
        d = plan.diagnostics(0)
        E1 = plan.energy(0)["E"]
        assert d["umin"] >= 0.0 and d["umax"] <= 1.0 and d["bound"] <= 1.0
        assert E1 <= E0 + 1e-13 * abs(E0)
        E0 = E1
    report("fixed_mbp_energy", scheme=scheme, E=E0, bound=d["bound"])
    plan.close()


def test_fp32_fft_variant_close_and_bounded():
    fi = inputs.fixed_membrane(dim=2, n=64)
    grid, p, _ = oracle_params(fi)
    _, U64 = gpu_run(fi, etd.ETDRK2, 20)
    plan, U32 = gpu_run(fi, etd.ETDRK2, 20, precision=etd.FP32)
    err = rel_linf(U32, U64)
    report("fixed_fp32fft", err=err)
    assert err <= 1e-5
    d = plan.diagnostics(0)
    assert d["umin"] >= 0.0 and d["umax"] <= 1.0
    plan.close()


def test_fixed_128cubed_tau_sweep_bound_and_energy():
    """The 3D fixed-membrane configuration (128^3 sphere, eps = 2h, B = B_MBP)
    with tau halved over 0.08 ... 0.005 to T = 0.96, on the FP64 path and the
    FP32-FFT path: every run keeps the discrete maximum bound (thm:MBP) and
    a non-increasing energy (thm:Energy) at each checkpoint, the two paths
    agree to 1e-5, and the error against tau = 0.00125 falls with tau.  (At
    these steps tau B_MBP is large and U relaxes within a fraction of T, so
    the errors fall faster than the asymptotic order; the order itself is
    checked by the 2D convergence study and the oracle pins.)"""
    import dataclasses
    fi0 = inputs.fixed_membrane(dim=3, n=128, eps_pm_in_h=2.0, tau=0.08)
    T = 0.96

    def run(tau, precision):
        fi = dataclasses.replace(fi0, tau=tau)
        plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETDRK2, precision=precision))
        plan.set_state(0, dev(fi.g), dev(fi.u0))
        nsteps = int(round(T / tau))
        E = [plan.energy(0)["E"]]
        for chunk in (nsteps // 4,) * 3 + (nsteps - 3 * (nsteps // 4),):
            plan.step(chunk)
            d = plan.diagnostics(0)
            assert d["umin"] >= 0.0 and d["umax"] <= 1.0 and d["bound"] <= 1.0, (tau, d)
            E.append(plan.energy(0)["E"])
        _, u = plan.get_state(0)
        plan.close()
        assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:])), (tau, E)
        return host(u)

    ref = run(0.00125, etd.FP64)
    errs, gaps = [], []
    for t in (0.08, 0.04, 0.02, 0.01, 0.005):
        u64, u32 = run(t, etd.FP64), run(t, etd.FP32)
        errs.append(float(np.abs(u64 - ref).max()))
        gaps.append(rel_linf(u32, u64))
    report("fixed3d_tau_sweep", errs=" ".join(f"{e:.3e}" for e in errs), fp32_gap=max(gaps))
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))
    assert max(gaps) <= 1e-5


def test_config1_200_steps_with_mass_projection():
    """Config 1 (64^2 circle, ETD1, tau = 0.01, B = B_MBP, 200 steps) with the
    per-step FP64 mean correction (ETD_F_MASS_PROJECT): <g U, 1>_h keeps its
    initial value and U stays in [0, 1]."""
    fi = inputs.fixed_membrane(dim=2, n=64)
    plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETD1, flags=etd.F_MASS_PROJECT))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    Q0 = plan.diagnostics(0)["Q"]
    for _ in range(4):
        plan.step(50)
        d = plan.diagnostics(0)
        assert abs(d["Q"] - Q0) <= 1e-12 * abs(Q0), (d["Q"], Q0)
        assert d["umin"] >= 0.0 and d["umax"] <= 1.0
    report("fixed_config1_mass", Q=Q0, drift=abs(d["Q"] - Q0) / abs(Q0), umin=d["umin"], umax=d["umax"])
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_split_and_stabilized_schemes_on_one_circle(scheme):
    """The two discretizations of the OK dynamics on a fixed membrane, on the
    same 64^2 circle (eps_pm = 0.0625, the fixed configuration) with the same
    U^0, tau = 0.01 and stabilizer B = B_MBP: the localization split of
    Section 2 (its MBP and energy theorems: asserted) and the stabilized
    spectral u-step of Section 3.1 with phi frozen and v = 0 (no such
    theorems: its bound and energy are reported).  The two discretize the
    nonlocal and mass terms differently (g f(u) in the split, g (u - ubar)
    here), so their trajectories differ."""
    fi = inputs.fixed_membrane(dim=2, n=64, eps_pm=0.0625)
    split = etd.Plan(etd.fixed_instance(fi, scheme=scheme))
    split.set_state(0, dev(fi.g), dev(fi.u0))
    B = split.query(0, etd.Q_B)
    ci = inputs.frozen_sphere(n=64, radius=0.5, dim=2, eps_pm=0.0625, tau=fi.tau, B2=B, gamma=fi.gamma, M=fi.M)
    assert np.abs(18.0 * (ci.phi0 * ci.phi0 - ci.phi0) ** 2 - fi.g).max() <= 1e-12
    assert np.array_equal(ci.u0, fi.u0)
    stab = etd.Plan(etd.coupled_instance(ci, scheme=scheme, flags=etd.F_FROZEN_MEMBRANE))
    stab.set_state(0, dev(ci.phi0), dev(ci.u0))
    E_split = [split.energy(0)["E"]]
    e = stab.energy(0)
    E_stab = [e["E_ok"] + e["E_nonlocal"] + e["E_mass"]]
    lo, hi = 1.0, 0.0
    for _ in range(10):
        split.step(5)
        stab.step(5)
        d = split.diagnostics(0)
        assert d["umin"] >= 0.0 and d["umax"] <= 1.0
        E_split.append(split.energy(0)["E"])
        assert E_split[-1] <= E_split[-2] + 1e-13 * abs(E_split[-2])
        ds = stab.diagnostics(0)
        lo, hi = min(lo, ds["umin"]), max(hi, ds["umax"])
        e = stab.energy(0)
        E_stab.append(e["E_ok"] + e["E_nonlocal"] + e["E_mass"])
        assert np.isfinite(E_stab[-1])
    report("split_vs_stabilized_2d", scheme=scheme, split_U=f"[{d['umin']:.4g},{d['umax']:.4g}]",
           split_E=f"{E_split[0]:.5g}->{E_split[-1]:.5g}", stab_U=f"[{lo:.4g},{hi:.4g}]",
           stab_E=f"{E_stab[0]:.5g}->{E_stab[-1]:.5g}",
           stab_E_monotone=bool(all(b <= a + 1e-12 * abs(a) for a, b in zip(E_stab, E_stab[1:]))))
    split.close()
    stab.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("precision", [etd.FP64, etd.FP32])
def test_band_step_matches_oracle(scheme, precision):
    """ETD_F_BAND_STEP: the step restricted to {g >= 1e-3} against the oracle's
    restricted step (U-space block exponential), 2D config-1 geometry on
    32^2; U off the band keeps its initial value exactly; the band energy."""
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
    grid, p, _ = oracle_params(fi)
    p.band_step = 1e-3
    band = fixed.step_band(fi.g, p)
    ex = fixed.UspaceExpo(fi.g, p, grid, fi.tau)
    U = fi.u0.copy()
    for _ in range(8):
        U = fixed.step(U, fi.g, p, grid, fi.tau, scheme, ex)
    plan, Ug = gpu_run(fi, scheme, 8, precision=precision, flags=etd.F_BAND_STEP, band_threshold=1e-3)
    err = rel_linf(Ug, U)
    report("fixed_band_step", scheme=scheme, precision=precision, err=err, band=int(band.sum()),
           deg=plan.query(0, etd.Q_CHEB_DEG))
    assert err <= (1e-12 if precision == etd.FP64 else 1e-5)
    assert np.array_equal(Ug[~band], fi.u0[~band])
    e, oe = plan.energy(0), fixed.energy(U, fi.g, p, grid)
    for k in ("E", "E_grad", "E_well", "E_nonlocal", "E_mass"):
        assert abs(e[k] - oe[k]) <= 1e-9 * max(abs(oe[k]), 1e-12), (k, e[k], oe[k])
    plan.close()


def test_band_step_3d_matches_lanczos_oracle():
    fi = inputs.fixed_membrane(dim=3, n=24, eps_pm_in_h=2.0, tau=0.02)
    grid, p, _ = oracle_params(fi)
    p.band_step = 1e-4
    ex = fixed.LanczosExpo(fi.g, p, grid)
    U = fi.u0.copy()
    for _ in range(3):
        U = fixed.step(U, fi.g, p, grid, fi.tau, etd.ETDRK2, ex)
    plan, Ug = gpu_run(fi, etd.ETDRK2, 3, flags=etd.F_BAND_STEP, band_threshold=1e-4)
    err = rel_linf(Ug, U)
    report("fixed3d_band_step", err=err)
    assert err <= 1e-12
    plan.close()


def test_band_step_tames_the_protrusion_cell_and_full_grid_refuses_it():
    """The seven-protrusion cell of Section 4.2: r0 = 0.4 (1 + 0.1 sin 7 theta)
    makes g jump by ~1e5 between neighbouring nodes near the centre, where
    g ~ 1e-67, and the full-grid operator's spectrum (Gershgorin bound
    ~5e9) needs a Chebyshev series beyond 4096 terms: plan set-up refuses
    it.  On the band {g >= 1e-3} the spectrum is that of the circle."""
    fi = inputs.fixed_coarsening("protrusions", gamma=7000.0, M=200.0)
    full = etd.Plan(etd.fixed_instance(fi, B=2000.0, scheme=etd.ETDRK2))
    with pytest.raises(etd.EtdError) as ei:
        full.set_state(0, dev(fi.g), dev(fi.u0))
    assert ei.value.status == etd.ETD_E_ARG
    full.close()
    plan = etd.Plan(etd.fixed_instance(fi, B=2000.0, scheme=etd.ETDRK2, flags=etd.F_BAND_STEP,
                                       band_threshold=1e-3))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    deg, rho = plan.query(0, etd.Q_CHEB_DEG), plan.query(0, etd.Q_RHO)
    report("protrusions_band", deg=deg, rho=rho)
    assert deg <= 40
    plan.step(10)
    d = plan.diagnostics(0)
    assert d["umin"] >= -1e-14 and d["umax"] <= 1.0 + 1e-14
    plan.close()
