"""GPU: the coupled stabilized ETD1/ETDRK2 step (Algorithm 1) through the C
ABI against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, recovery_flips, rel_linf, report, torch, u_gap_outside_flips
from oracle import band as oband
from oracle.core import Grid
from oracle.coupled import CoupledOracle
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


def make_case(shape, tau=1e-4, seed=31, **kw):
    return inputs.coupled_membrane(n=shape, seed=seed, tau=tau, **kw)


def run_pair(ci, scheme, precision, nsteps, **inst_kw):
    grid = Grid(ci.shape, ci.half_len)
    o = CoupledOracle(grid, ci.params, ci.tau, scheme,
                      band_threshold=inst_kw.get("band_threshold", 0.0),
                      band_rebuild_every=inst_kw.get("band_rebuild_every", 10),
                      mass_projection=bool(inst_kw.get("flags", 0) & etd.F_MASS_PROJECT),
                      frozen_membrane=bool(inst_kw.get("flags", 0) & etd.F_FROZEN_MEMBRANE))
    o.set_state(ci.phi0, ci.u0)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=scheme, precision=precision, **inst_kw))
    dt = torch.float64 if precision == etd.FP64 else torch.float32
    plan.set_state(0, dev(ci.phi0, dt), dev(ci.u0, dt))
    o.run(nsteps)
    plan.step(nsteps)
    phi_g, u_g = plan.get_state(0)
    return o, plan, host(phi_g), host(u_g)


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("shape,nsteps", [((16, 16, 16), 1), ((16, 16, 16), 5), ((24, 16, 32), 3),
                                          ((48, 48, 48), 2), ((64, 96, 128), 1), ((96, 64, 192), 1),
                                          ((16, 24, 512), 1), ((384, 8, 16), 1), ((8, 512, 8), 1),
                                          ((8, 8, 8), 2), ((512, 8, 12), 1)])
def test_fp64_step_matches_oracle(shape, nsteps, scheme):
    ci = make_case(shape)
    o, plan, phi, u = run_pair(ci, scheme, etd.FP64, nsteps)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_fp64", shape=str(shape), scheme=scheme, steps=nsteps, err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12
    # diagnostics and energy components, FP64
    d = plan.diagnostics(0)
    od = o.diagnostics()
    for k_gpu, k_or in (("int_phi", "I_phi"), ("mass", "m"), ("Q", "Q"), ("umin", "umin"), ("umax", "umax"),
                        ("bound", "bound")):
        assert abs(d[k_gpu] - od[k_or]) <= 1e-11 * max(1.0, abs(od[k_or])), (k_gpu, d[k_gpu], od[k_or])
    e = plan.energy(0)
    oe = o.energy()
    for k in ("E_surf", "E_bend", "E_area", "E_ok", "E_nonlocal", "E_mass"):
        assert abs(e[k] - oe[k]) <= 1e-10 * max(1e-8, abs(oe[k])) + 1e-14, (k, e[k], oe[k])
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("shape,nsteps", [((32, 32, 32), 20), ((96, 64, 192), 3), ((8, 512, 8), 3),
                                          ((512, 8, 12), 1)])
def test_fp32_step_close_to_oracle(scheme, shape, nsteps):
    """FP32 path against the FP64 oracle, step by step.  phi within 1e-4
    (relative L-inf) everywhere; u within 1e-4 everywhere except at the
    points where the two paths' G fell on opposite sides of the recovery
    threshold in some step (counted, at most 1e-4 of the grid) and their
    two-cell neighbourhood; g u within 1e-4 everywhere -- or, where rounding
    the state to FP32 alone moves the oracle's u further (rounding_floor:
    the 8 x 512 x 8 grid), within twice that.  The 512 x 8 x 12
    grid (dx = 2 pi / 512 beside dy = 2 pi / 8) is unstable at tau = 1e-4
    even in exact arithmetic (the oracle's u grows thirtyfold a step and
    overflows by step 3), so it runs one step only."""
    ci = make_case(shape)
    grid = Grid(ci.shape, ci.half_len)
    o = CoupledOracle(grid, ci.params, ci.tau, scheme)
    o.set_state(ci.phi0, ci.u0)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=scheme, precision=etd.FP32))
    plan.set_state(0, dev(ci.phi0, torch.float32), dev(ci.u0, torch.float32))
    flips = np.zeros(ci.shape, dtype=bool)
    for _ in range(nsteps):
        o.step()
        plan.step(1)
        phi = host(plan.get_state(0, torch.float32)[0])
        flips |= recovery_flips(phi, o.phi())
    phi, u = (host(t) for t in plan.get_state(0))
    po = o.phi()
    ephi = rel_linf(phi, po)
    eu, near, egu, eall = u_gap_outside_flips(u, o.u, po, flips)
    tol = 1e-4
    if eu > tol or egu > tol:
        tol = max(tol, 2.0 * rounding_floor(ci, scheme, nsteps))
    report("coupled_fp32", shape=str(shape), scheme=scheme, steps=nsteps, err_phi=ephi, err_u=eu,
           flips=int(flips.sum()), near=near, err_gu=egu, err_u_all=eall, tol_u=tol)
    assert np.isfinite(phi).all() and np.isfinite(u).all()
    assert ephi <= 1e-4 and eu <= tol and egu <= tol
    assert flips.sum() <= max(1, 1e-4 * flips.size)
    plan.close()


def rounding_floor(ci, scheme, nsteps):
    """What rounding the state alone does to the oracle's u: the relative
    L-inf change of u (and of g u) when the velocity v = -phi_t grad phi /
    |grad phi|^2 (defined with eqn:model_OK) is formed from phi^n and
    phi^{n+1} rounded to FP32.  phi_t is a difference quotient of two states
    tau apart, so a rounding of 6e-8 becomes 6e-4 in phi_t, and where |grad
    phi| is small v carries it further.  On grids whose cells are far from
    cubic (8 x 512 x 8: the membrane spans a fraction of an x or z cell) this
    alone moves u by more than 1e-4 within three steps; no FP32 state can do
    better there."""
    from oracle import core
    grid = Grid(ci.shape, ci.half_len)
    ref = CoupledOracle(grid, ci.params, ci.tau, scheme)
    per = CoupledOracle(grid, ci.params, ci.tau, scheme)
    ref.set_state(ci.phi0, ci.u0)
    per.set_state(ci.phi0, ci.u0)
    vel = per.velocity

    def vel32(phi_old, phi_new_hat, g_new):
        r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        return vel(r32(phi_old), core.fft(r32(core.ifft(phi_new_hat))), g_new)

    per.velocity = vel32
    ref.run(nsteps)
    per.run(nsteps)
    d = np.abs(per.u - ref.u)
    g = core.g_loc(ref.phi())
    return max(float(d.max() / np.abs(ref.u).max()), float((g * d).max() / np.abs(g * ref.u).max()))


def test_fp64_step_matches_naive_dft_oracle():
    """The oracle with its own exact-index DFT (no library transform anywhere
    in the reference): ETDRK2 on a 24 x 16 x 32 grid (radix-3 length) and
    ETD1 at 16^3, FP64 within 1e-12."""
    from oracle import core
    mode = core.get_dft_mode()
    core.set_dft_mode("naive")
    try:
        for shape, scheme, nsteps in (((24, 16, 32), etd.ETDRK2, 2), ((16, 16, 16), etd.ETD1, 3)):
            ci = make_case(shape)
            o, plan, phi, u = run_pair(ci, scheme, etd.FP64, nsteps)
            ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
            report("coupled_fp64_naive_dft", shape=str(shape), scheme=scheme, err_phi=ephi, err_u=eu)
            assert ephi <= 1e-12 and eu <= 1e-12
            plan.close()
    finally:
        core.set_dft_mode(mode)


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("precision,tol", [(etd.FP64, 1e-12), (etd.FP32, 1e-4)])
def test_frozen_membrane_matches_oracle(scheme, precision, tol):
    """ETD_F_FROZEN_MEMBRANE: only the g u stages, with g = g(phi^0), v = 0;
    phi stays at its set_state value (its spectral round trip)."""
    ci = make_case((32, 32, 32))
    o, plan, phi, u = run_pair(ci, scheme, precision, 6, flags=etd.F_FROZEN_MEMBRANE)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_frozen", scheme=scheme, precision=precision, err_phi=ephi, err_u=eu)
    assert ephi <= (1e-14 if precision == etd.FP64 else 1e-6) and eu <= tol
    d, od = plan.diagnostics(0), o.diagnostics()
    assert abs(d["mass"] - od["m"]) <= 10 * tol * max(1.0, abs(od["m"]))
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
def test_variable_step_matches_oracle(scheme):
    """etd_set_tau between steps (per-step tau_{n+1}, Section 3.3) against the
    oracle stepping the same tau sequence."""
    ci = make_case((16, 16, 16))
    grid = Grid(ci.shape, ci.half_len)
    o = CoupledOracle(grid, ci.params, ci.tau, scheme)
    o.set_state(ci.phi0, ci.u0)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=scheme, precision=etd.FP64))
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    for tau in (1e-4, 2e-4, 5e-5, 3e-4):
        o.set_tau(tau)
        o.step()
        plan.set_tau(0, tau)
        plan.step(1)
    phi, u = (host(t) for t in plan.get_state(0))
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_variable_tau", scheme=scheme, err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12
    plan.close()


def test_band_restricted_step_matches_oracle():
    ci = make_case((32, 32, 32))
    o, plan, phi, u = run_pair(ci, etd.ETDRK2, etd.FP64, 12, band_threshold=0.995, band_rebuild_every=10)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_band", err_phi=ephi, err_u=eu, band=plan.diagnostics(0)["band_count"])
    assert ephi <= 1e-12 and eu <= 1e-12
    # the band in use was rebuilt from phi^10
    assert plan.diagnostics(0)["band_count"] > 0
    plan.close()


def test_mass_projection_matches_oracle_and_conserves():
    ci = make_case((16, 16, 16))
    o, plan, phi, u = run_pair(ci, etd.ETDRK2, etd.FP64, 4, flags=etd.F_MASS_PROJECT)
    assert rel_linf(u, o.u) <= 1e-12
    # <g(phi^n) U^n, 1>_h is the set_state value Q0
    assert abs(plan.diagnostics(0)["Q"] - o.Q0) <= 1e-12 * abs(o.Q0)
    plan.close()


@pytest.mark.parametrize("precision", [etd.FP64, etd.FP32])
def test_narrowband_list_bit_exact(precision):
    for shape in ((32, 32, 32), (128, 128, 128)):
        ci = make_case(shape)
        dt = torch.float64 if precision == etd.FP64 else torch.float32
        phi_d = dev(ci.phi0, dt)
        ref = oband.band_list(host(phi_d), 0.995)      # decided in FP64 on the same values
        plan = etd.Plan(etd.coupled_instance(ci, precision=precision))
        idx = plan.narrowband(0, phi_d, 0.995).cpu().numpy()
        report("band", shape=str(shape), n=len(ref))
        assert idx.dtype == np.int32 and np.array_equal(idx, ref)
        with pytest.raises(etd.EtdError) as ei:
            plan.narrowband(0, phi_d, 0.995, capacity=len(ref) - 1)
        assert ei.value.status == etd.ETD_E_CAPACITY
        plan.close()


def test_steps_are_deterministic():
    ci = make_case((24, 24, 24))
    outs = []
    for _ in range(2):
        plan = etd.Plan(etd.coupled_instance(ci))
        plan.set_state(0, dev(ci.phi0), dev(ci.u0))
        plan.step(3)
        outs.append([host(t) for t in plan.get_state(0)])
        plan.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


# ----------------------------------------------------------------------------- two-dimensional grids
def make_case_2d(shape, tau=1e-4, seed=31, **kw):
    return inputs.coupled_membrane_2d(n=shape, seed=seed, tau=tau, **kw)


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("shape,nsteps", [((64, 64), 5), ((96, 128), 3), ((256, 256), 2), ((8, 512), 2),
                                          ((384, 24), 1)])
def test_fp64_2d_step_matches_oracle(shape, nsteps, scheme):
    """The coupled scheme on two-dimensional grids (Section 3 is written for
    d = 2, 3): the perturbed circle of inputs.coupled_membrane_2d."""
    ci = make_case_2d(shape)
    o, plan, phi, u = run_pair(ci, scheme, etd.FP64, nsteps)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_2d_fp64", shape=str(shape), scheme=scheme, steps=nsteps, err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12
    d, od = plan.diagnostics(0), o.diagnostics()
    for k_gpu, k_or in (("int_phi", "I_phi"), ("mass", "m"), ("Q", "Q"), ("umin", "umin"), ("umax", "umax"),
                        ("bound", "bound")):
        assert abs(d[k_gpu] - od[k_or]) <= 1e-11 * max(1.0, abs(od[k_or])), (k_gpu, d[k_gpu], od[k_or])
    e, oe = plan.energy(0), o.energy()
    for k in ("E_surf", "E_bend", "E_area", "E_ok", "E_nonlocal", "E_mass"):
        assert abs(e[k] - oe[k]) <= 1e-10 * max(1e-8, abs(oe[k])) + 1e-14, (k, e[k], oe[k])
    plan.close()


@pytest.mark.parametrize("scheme", [etd.ETD1, etd.ETDRK2])
@pytest.mark.parametrize("shape,nsteps", [((128, 128), 20), ((96, 128), 5)])
def test_fp32_2d_step_close_to_oracle(scheme, shape, nsteps):
    """FP32 on two-dimensional grids, step by step, under the comparison of
    test_fp32_step_close_to_oracle."""
    ci = make_case_2d(shape)
    grid = Grid(ci.shape, ci.half_len)
    o = CoupledOracle(grid, ci.params, ci.tau, scheme)
    o.set_state(ci.phi0, ci.u0)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=scheme, precision=etd.FP32))
    plan.set_state(0, dev(ci.phi0, torch.float32), dev(ci.u0, torch.float32))
    flips = np.zeros(ci.shape, dtype=bool)
    for _ in range(nsteps):
        o.step()
        plan.step(1)
        flips |= recovery_flips(host(plan.get_state(0, torch.float32)[0]), o.phi())
    phi, u = (host(t) for t in plan.get_state(0))
    po = o.phi()
    ephi = rel_linf(phi, po)
    eu, near, egu, eall = u_gap_outside_flips(u, o.u, po, flips)
    report("coupled_2d_fp32", shape=str(shape), scheme=scheme, steps=nsteps, err_phi=ephi, err_u=eu,
           flips=int(flips.sum()), near=near, err_gu=egu, err_u_all=eall)
    assert ephi <= 1e-4 and eu <= 1e-4 and egu <= 1e-4
    assert flips.sum() <= max(1, 1e-4 * flips.size)
    plan.close()


@pytest.mark.parametrize("kw", [dict(flags=etd.F_FROZEN_MEMBRANE), dict(flags=etd.F_MASS_PROJECT),
                                dict(band_threshold=0.995, band_rebuild_every=3)])
def test_2d_options_match_oracle(kw):
    """Frozen membrane, mass projection and the narrow band on a 2D grid."""
    ci = make_case_2d((64, 96))
    o, plan, phi, u = run_pair(ci, etd.ETDRK2, etd.FP64, 6, **kw)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("coupled_2d_options", opts=str(kw), err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12
    plan.close()
