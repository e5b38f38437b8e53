"""GPU: (-Delta_S,h)^{-1} on a narrow band (etd_surface_lapinv, and the
coupled step with ETD_F_SURFACE_NONLOCAL) against the oracle's bordered
sparse direct solve (oracle.core.lapinv_S_band)."""
import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, rel_linf, report, torch
from oracle import core
from oracle.core import Grid
from oracle.coupled import CoupledOracle
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


def shell_case(n, thr=0.995, seed=31):
    # interface width 1.5 h: a band of a few cells, small enough for the
    # oracle's sparse direct solve
    ci = inputs.coupled_membrane(n=n, seed=seed, tau=1e-4, eps_pm_in_h=1.5)
    g = 18.0 * (ci.phi0 * ci.phi0 - ci.phi0) ** 2
    mask = np.abs(2.0 * ci.phi0 - 1.0) < thr
    return ci, g, mask


def gpu_solve(plan, g, f, mask, dtype=torch.float64, tol=1e-12):
    psi, it, rr = plan.surface_lapinv(0, dev(g, dtype), dev(f, dtype), dev(mask.astype(np.uint8), torch.uint8),
                                      tol=tol)
    return host(psi), it, rr


@pytest.mark.parametrize("n", [16, 32, 64])
def test_band_solve_matches_oracle_3d(n):
    ci, g, mask = shell_case(n)
    grid = Grid(ci.shape, ci.half_len)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(ci.shape) * mask
    ref = core.lapinv_S_band(f, g, mask, grid)
    plan = etd.Plan(etd.coupled_instance(ci))
    psi, it, rr = gpu_solve(plan, g, f, mask)
    err = rel_linf(psi, ref)
    report("surface_band_3d", n=n, band=int(mask.sum()), iters=it, relres=rr, err=err)
    assert rr <= 1e-12 and err <= 1e-8
    # the Chebyshev polynomial preconditioner: 30 and 31 iterations on the 16^3
    # and 32^3 shells, where Jacobi alone took 179 on the 32^3 shell
    assert it <= 120
    assert (psi[~mask] == 0).all() and abs(psi[mask].mean()) <= 1e-12 * np.abs(psi).max()
    # FP32 data through the same FP64 iteration
    p32, _, rr32 = gpu_solve(plan, g, f, mask, torch.float32, tol=1e-7)
    assert rel_linf(p32, ref) <= 1e-5
    plan.close()


def test_band_solve_at_the_benchmark_size():
    """The band of the 256^3 benchmark (eps = 3h, |2 phi - 1| < 0.995: about
    1.2e6 band nodes), where the oracle's direct solve is out of reach: the
    GPU solution is checked through the oracle's band matrix (a property that
    holds at any size): A psi_B equals the band-mean-free right-hand side to
    the solver's tolerance times the operator's scale, psi has zero band mean
    and is 0 off the band."""
    ci = inputs.coupled_membrane(n=256, tau=1e-4)
    g = 18.0 * (ci.phi0 * ci.phi0 - ci.phi0) ** 2
    mask = np.abs(2.0 * ci.phi0 - 1.0) < 0.995
    rng = np.random.default_rng(7)
    f = rng.standard_normal(ci.shape) * mask
    plan = etd.Plan(etd.coupled_instance(ci))
    psi, it, rr = gpu_solve(plan, g, f, mask, tol=1e-10)
    plan.close()
    B, A = core.band_matrix(g, mask, Grid(ci.shape, ci.half_len))
    fb = f.ravel()[B]
    rhs = fb - fb.mean()
    pb = psi.ravel()[B]
    res = A @ pb - rhs
    rel = float(np.linalg.norm(res) / np.linalg.norm(rhs))
    report("surface_band_256", band=int(B.size), iters=it, relres=rr, oracle_relres=rel)
    assert rr <= 1e-10 and rel <= 1e-9
    assert (psi[~mask] == 0).all() and abs(pb.mean()) <= 1e-12 * np.abs(pb).max()


def test_band_solve_2d_shell_and_full_band():
    """2D grid (fixed-model instance): a shell band with g of the fixed circle,
    and the whole grid with g = 1, where the band solve is the FFT
    pseudo-inverse (-Delta_h)^{-1} of etd_spectral_apply."""
    fi = inputs.fixed_membrane(dim=2, n=64)
    grid = Grid(fi.shape, fi.half_len)
    plan = etd.Plan(etd.fixed_instance(fi))
    rng = np.random.default_rng(6)
    f = rng.standard_normal(fi.shape)
    mask = fi.g >= 1e-3
    ref = core.lapinv_S_band(f, fi.g, mask, grid)
    psi, it, rr = gpu_solve(plan, fi.g, f, mask)
    err = rel_linf(psi, ref)
    report("surface_band_2d", band=int(mask.sum()), iters=it, relres=rr, err=err)
    assert err <= 1e-8
    full = np.ones(fi.shape, dtype=bool)
    psi1, _, _ = gpu_solve(plan, np.ones(fi.shape), f, full)
    out = torch.empty(fi.shape, dtype=torch.float64, device="cuda")
    plan.spectral_apply(0, etd.OP_LAPINV, dev(f), out)
    assert rel_linf(psi1, host(out)) <= 1e-9
    # an empty band gives psi = 0 without iterating
    psi0, it0, _ = gpu_solve(plan, fi.g, f, np.zeros(fi.shape, dtype=bool))
    assert it0 == 0 and (psi0 == 0).all()
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_coupled_step_with_band_solve_matches_oracle(scheme):
    ci = inputs.coupled_membrane(n=(24, 24, 24), seed=31, tau=1e-4, eps_pm_in_h=1.5)
    grid = Grid(ci.shape, ci.half_len)
    o = CoupledOracle(grid, ci.params, ci.tau, scheme, band_threshold=0.995, band_rebuild_every=2,
                      surface_nonlocal=True)
    o.set_state(ci.phi0, ci.u0)
    o.run(3)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=scheme, band_threshold=0.995, band_rebuild_every=2,
                                         flags=etd.F_SURFACE_NONLOCAL))
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    plan.set_schedule(etd.EXEC_GRAPH, 2)      # plans with the band solve step eagerly
    plan.step(3)
    phi, u = (host(t) for t in plan.get_state(0))
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_surface_nonlocal", scheme=scheme, err_phi=ephi, err_u=eu,
           iters=plan.query(0, etd.Q_SURF_ITERS), relres=plan.query(0, etd.Q_SURF_RELRES))
    assert ephi <= 1e-12 and eu <= 1e-10
    assert plan.query(0, etd.Q_SURF_RELRES) <= 1e-12
    plan.close()


@pytest.mark.parametrize("scheme,precision", [(etd.ETD1, etd.FP64), (etd.ETDRK2, etd.FP64), (etd.ETDRK2, etd.FP32)])
def test_fixed_step_with_band_solve_matches_oracle(scheme, precision):
    """The fixed-membrane step with R_phi's nonlocal term by the band solve on
    {g >= 1e-3} (both of its paths take the FP64 solve) against the U-space
    oracle with the same band."""
    from oracle import fixed
    fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
    grid = Grid(fi.shape, fi.half_len)
    B = fixed.B_mbp(fi.eps_u, fi.gamma, fi.M, core.lapinv_inf_norm(grid), grid.volume)
    p = fixed.FixedParams(fi.eps_u, fi.gamma, fi.M, fi.ubar, B, False, 1e-3)
    ex = fixed.UspaceExpo(fi.g, p, grid, fi.tau)
    U = fi.u0.copy()
    for _ in range(5):
        U = fixed.step(U, fi.g, p, grid, fi.tau, scheme, ex)
    plan = etd.Plan(etd.fixed_instance(fi, scheme=scheme, precision=precision, band_threshold=1e-3,
                                       flags=etd.F_SURFACE_NONLOCAL))
    plan.set_state(0, dev(fi.g), dev(fi.u0))
    plan.step(5)
    _, u = plan.get_state(0)
    err = rel_linf(host(u), U)
    report("fixed_surface_nonlocal", scheme=scheme, precision=precision, err=err,
           iters=plan.query(0, etd.Q_SURF_ITERS))
    assert err <= 1e-11
    plan.close()


def test_band_solve_warm_start_depends_on_the_state_alone():
    """Each band solve of a step starts from the previous solve's result; a new
    state (etd_set_state) starts cold again, so stepping the same state twice
    gives the same trajectory bit for bit, and the warm-started solves stop at
    the same relative residual as a cold one."""
    ci = inputs.coupled_membrane(n=(24, 24, 24), seed=31, tau=1e-4, eps_pm_in_h=1.5)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, band_threshold=0.995, band_rebuild_every=2,
                                         flags=etd.F_SURFACE_NONLOCAL))
    runs = []
    for _ in range(2):
        plan.set_state(0, dev(ci.phi0), dev(ci.u0))
        plan.step(3)
        runs.append([host(t) for t in plan.get_state(0)] + [plan.query(0, etd.Q_SURF_ITERS)])
        assert plan.query(0, etd.Q_SURF_RELRES) <= 1e-12
    report("surface_warm_start", iters_last=runs[0][2])
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][2] == runs[1][2]
    plan.close()
