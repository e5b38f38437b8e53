"""GPU: degenerate inputs of the coupled step through the C ABI: zero steps,
an empty narrow band (the list and a band-restricted step), and a grid with
no membrane (phi = 0, so g = 0 and every surface term vanishes), each
against the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, rel_linf, report, torch
from oracle import band as oband
from oracle.core import Grid
from oracle.coupled import CoupledOracle
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


def case(shape=(16, 16, 16)):
    return inputs.coupled_membrane(n=shape, seed=31, tau=1e-4)


def test_zero_steps_keep_the_state_and_negative_counts_are_rejected():
    ci = case()
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2))
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    before = [host(t) for t in plan.get_state(0)]
    plan.step(0)
    after = [host(t) for t in plan.get_state(0)]
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    assert plan.diagnostics(0)["step"] == 0
    with pytest.raises(etd.EtdError) as ei:
        plan.step(-1)
    assert ei.value.status == etd.ETD_E_ARG
    plan.close()


@pytest.mark.parametrize("precision", [etd.FP64, etd.FP32])
def test_empty_narrow_band_list(precision):
    ci = case()
    dt = torch.float64 if precision == etd.FP64 else torch.float32
    phi = torch.zeros(ci.shape, dtype=dt, device="cuda")     # |2 phi - 1| = 1 everywhere
    plan = etd.Plan(etd.coupled_instance(ci, precision=precision))
    assert len(plan.narrowband(0, phi, 0.995)) == 0
    assert len(plan.narrowband(0, phi, 0.995, capacity=0)) == 0
    plan.close()


def run_pair(ci, phi0, nsteps, **kw):
    o = CoupledOracle(Grid(ci.shape, ci.half_len), ci.params, ci.tau, etd.ETDRK2,
                      band_threshold=kw.get("band_threshold", 0.0), band_rebuild_every=kw.get("band_rebuild_every", 10))
    o.set_state(phi0, ci.u0)
    o.run(nsteps)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, **kw))
    plan.set_state(0, dev(phi0), dev(ci.u0))
    plan.step(nsteps)
    phi, u = (host(t) for t in plan.get_state(0))
    d = plan.diagnostics(0)
    plan.close()
    return o, phi, u, d


def test_step_with_an_empty_band_matches_oracle():
    """A threshold no point meets: the band is empty at set_state and at the
    rebuild after step 2, and the band-restricted surface terms vanish."""
    ci = case()
    assert len(oband.band_list(ci.phi0, 1e-9)) == 0
    o, phi, u, d = run_pair(ci, ci.phi0, 3, band_threshold=1e-9, band_rebuild_every=2)
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    report("edge_empty_band", err_phi=ephi, err_u=eu, band=d["band_count"])
    assert d["band_count"] == 0
    assert ephi <= 1e-12 and eu <= 1e-12


@pytest.mark.parametrize("level", [0.0, 1.0])
def test_no_membrane_matches_oracle(level):
    """phi constant at a pure phase: g = 0 and grad phi = 0 everywhere, so the
    recovery takes its G <= threshold branch at every point."""
    ci = case()
    phi0 = np.full(ci.shape, level)
    o, phi, u, d = run_pair(ci, phi0, 2)
    ephi = float(np.abs(phi - o.phi()).max())
    eu = rel_linf(u, o.u)
    report("edge_no_membrane", level=level, abs_err_phi=ephi, err_u=eu)
    assert np.isfinite(u).all() and np.isfinite(phi).all()
    assert ephi <= 1e-13 and eu <= 1e-12


@pytest.mark.parametrize("bad", ["zero", "negative", "nan"])
def test_fixed_set_state_rejects_g_not_positive_and_finite(bad):
    fi = inputs.fixed_membrane(dim=2, n=16, eps_pm=0.0625)
    g = fi.g.copy()
    g.flat[7] = {"zero": 0.0, "negative": -1e-3, "nan": np.nan}[bad]
    plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETD1))
    with pytest.raises(etd.EtdError) as ei:
        plan.set_state(0, dev(g), dev(fi.u0))
    assert ei.value.status == etd.ETD_E_ARG
    plan.set_state(0, dev(fi.g), dev(fi.u0))   # the plan stays usable
    plan.step(1)
    plan.close()


def test_nonfinite_state_is_reported():
    ci = case()
    u0 = ci.u0.copy()
    u0.flat[123] = np.nan
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2))
    plan.set_state(0, dev(ci.phi0), dev(u0))
    assert plan.diagnostics(0)["nonfinite"] == 1
    plan.close()


def raw_get_state(plan, i=0):
    """etd_get_state through the C ABI: (status, a, u) as FP64 host arrays,
    without raising on a non-OK status."""
    import ctypes as C
    shape = tuple(plan.instances[i].shape)
    a = torch.empty(shape, dtype=torch.float64, device="cuda")
    u = torch.empty_like(a)
    st = etd.lib().etd_get_state(plan._ptr, i, C.c_void_p(a.data_ptr()), C.c_void_p(u.data_ptr()), etd.F64)
    return st, host(a), host(u)


def same(x, y):
    return np.array_equal(x, y, equal_nan=True)


@pytest.mark.parametrize("schedule", [etd.EXEC_EAGER, etd.EXEC_GRAPH])
@pytest.mark.parametrize("model", ["coupled_fp64", "coupled_fp32", "fixed"])
def test_steps_after_a_nonfinite_state_are_no_ops(model, schedule):
    """A NaN loaded by etd_set_state is the detected non-finite state: every
    later step leaves (phi, u) / U as they are, eagerly and under a captured
    graph, etd_get_state returns ETD_E_NONFINITE with the state copied out,
    and a finite etd_set_state clears it."""
    if model == "fixed":
        fi = inputs.fixed_membrane(dim=2, n=32, eps_pm=0.0625)
        plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETDRK2))
        a0, u_ok = fi.g, fi.u0
    else:
        ci = case()
        prec = etd.FP64 if model == "coupled_fp64" else etd.FP32
        plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=prec))
        a0, u_ok = ci.phi0, ci.u0
    dt = torch.float32 if model == "coupled_fp32" else torch.float64
    u_bad = u_ok.copy()
    u_bad.flat[123] = np.nan
    plan.set_schedule(schedule, 1)
    plan.set_state(0, dev(a0, dt), dev(u_bad, dt))
    st0, a_set, u_set = raw_get_state(plan)
    assert st0 == etd.ETD_E_NONFINITE
    assert np.isnan(u_set.flat[123]) and np.isfinite(np.delete(u_set.ravel(), 123)).all()
    plan.step(3)
    plan.step(1)
    st, a, u = raw_get_state(plan)
    report("nonfinite_noop", model=model, schedule=schedule, status=st)
    assert st == etd.ETD_E_NONFINITE
    assert same(a, a_set) and same(u, u_set)
    assert plan.diagnostics(0)["nonfinite"] == 1
    # a finite state clears the flag and the steps run again
    plan.set_state(0, dev(a0, dt), dev(u_ok, dt))
    st1, _, u1 = raw_get_state(plan)
    plan.step(2)
    st2, _, u2 = raw_get_state(plan)
    assert st1 == etd.ETD_OK and st2 == etd.ETD_OK and not np.array_equal(u1, u2)
    plan.close()


def test_nonfinite_values_arising_in_a_step_freeze_the_state():
    """The 512 x 8 x 12 grid (dx = 2 pi / 512 beside dy = 2 pi / 8) is
    unstable at tau = 1e-4: u grows by orders of magnitude a step until it
    overflows.  The step's own FP64 sums detect the first non-finite value;
    from the next step on the state no longer changes."""
    ci = inputs.coupled_membrane(n=(512, 8, 12), seed=31, tau=1e-4)
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=etd.FP64))
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    detected = None
    for k in range(1, 60):
        plan.step(1)
        st, a, u = raw_get_state(plan)
        if st == etd.ETD_E_NONFINITE:
            detected = k
            break
        assert st == etd.ETD_OK
    report("nonfinite_in_step", detected_at_step=detected)
    assert detected is not None
    assert not (np.isfinite(a).all() and np.isfinite(u).all())
    plan.step(3)
    st2, a2, u2 = raw_get_state(plan)
    assert st2 == etd.ETD_E_NONFINITE and same(a2, a) and same(u2, u)
    plan.close()
