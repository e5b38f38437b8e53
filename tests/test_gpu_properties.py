"""GPU property tests of the step that hold at any size: translation
commutes with a step on the periodic grid, a state with the grid's
octahedral symmetry keeps it, an instance steps bit for bit the same alone
and inside a batch, and a run resumed from a checkpoint continues bit for
bit (every operator of both schemes is translation invariant and isotropic
on cubic grids: spectral symbols in |k|^2, the 7-point Delta_S,h, central
differences)."""
import dataclasses
import itertools

import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, rel_linf, report, torch
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]

SHIFT = (3, 5, 7)


def coupled_run(ci, nsteps, **kw):
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, **kw))
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    plan.step(nsteps)
    out = [host(t) for t in plan.get_state(0)]
    plan.close()
    return out


@pytest.mark.parametrize("kw", [{}, dict(band_threshold=0.995, band_rebuild_every=2)])
def test_coupled_step_commutes_with_translation(kw):
    ci = inputs.coupled_membrane(n=(24, 32, 48), seed=31, tau=1e-4)
    shifted = dataclasses.replace(ci, phi0=np.roll(ci.phi0, SHIFT, axis=(0, 1, 2)),
                                  u0=np.roll(ci.u0, SHIFT, axis=(0, 1, 2)))
    phi, u = coupled_run(ci, 3, **kw)
    phis, us = coupled_run(shifted, 3, **kw)
    ephi = rel_linf(phis, np.roll(phi, SHIFT, axis=(0, 1, 2)))
    eu = rel_linf(us, np.roll(u, SHIFT, axis=(0, 1, 2)))
    report("translation_coupled", band=bool(kw), err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12


def test_fixed_step_commutes_with_translation():
    fi = inputs.fixed_membrane(dim=3, n=24, eps_pm_in_h=2.0, tau=0.02)
    runs = []
    for g, u0 in ((fi.g, fi.u0), (np.roll(fi.g, SHIFT, axis=(0, 1, 2)), np.roll(fi.u0, SHIFT, axis=(0, 1, 2)))):
        plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETDRK2))
        plan.set_state(0, dev(g), dev(u0))
        plan.step(3)
        runs.append(host(plan.get_state(0)[1]))
        plan.close()
    err = rel_linf(runs[1], np.roll(runs[0], SHIFT, axis=(0, 1, 2)))
    report("translation_fixed", err=err)
    assert err <= 1e-12


def _reflect(f, ax):
    return np.roll(np.flip(f, axis=ax), 1, axis=ax)      # index i -> N - i (mod N)


def _octahedral_average(f):
    """Mean of f over the 48 symmetries of the cubic grid about the point
    x = 0 (index N/2): axis permutations and reflections i -> N - i."""
    acc = np.zeros_like(f)
    for perm in itertools.permutations(range(3)):
        g = np.transpose(f, perm)
        for mask in range(8):
            h = g
            for ax in range(3):
                if mask >> ax & 1:
                    h = _reflect(h, ax)
            acc += h
    return acc / 48.0


def test_octahedral_symmetry_is_kept():
    """A sphere centred on the grid point x = 0 (index N/2) and u the
    octahedral average of the seeded draw: the state after three steps is
    invariant, to rounding, under the axis permutations and the reflections
    i -> N - i (48^3: at 32^3 the symmetric state is unstable in the oracle
    too, the interface being a third of the radius wide)."""
    ci = inputs.coupled_membrane(n=48, seed=31, tau=1e-4, amp=0.0)
    sym = dataclasses.replace(ci, u0=_octahedral_average(ci.u0))
    phi, u = coupled_run(sym, 3)
    worst = 0.0
    for f in (phi, u):
        assert np.isfinite(f).all()
        for perm in ((0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
            worst = max(worst, rel_linf(np.transpose(f, perm), f))
        for ax in range(3):
            worst = max(worst, rel_linf(_reflect(f, ax), f))
    report("octahedral", err=worst)
    assert worst <= 1e-12


@pytest.mark.parametrize("mode", [etd.EXEC_EAGER, etd.EXEC_GRAPH])
def test_instance_alone_and_in_a_batch_step_alike(mode):
    """The same coupled instance alone and as the second of three instances
    (another size and a fixed-membrane instance beside it): bit for bit."""
    ci = inputs.coupled_membrane(n=(24, 24, 32), seed=31, tau=1e-4)
    other = inputs.coupled_membrane(n=16, seed=5, tau=5e-5)
    fi = inputs.fixed_membrane(dim=2, n=32, tau=0.01)
    alone = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2))
    alone.set_state(0, dev(ci.phi0), dev(ci.u0))
    alone.set_schedule(mode, 1)
    alone.step(4)
    want = [host(t) for t in alone.get_state(0)]
    alone.close()
    batch = etd.Plan([etd.coupled_instance(other, scheme=etd.ETD1), etd.coupled_instance(ci, scheme=etd.ETDRK2),
                      etd.fixed_instance(fi, scheme=etd.ETDRK2)])
    batch.set_state(0, dev(other.phi0), dev(other.u0))
    batch.set_state(1, dev(ci.phi0), dev(ci.u0))
    batch.set_state(2, dev(fi.g), dev(fi.u0))
    batch.set_schedule(mode, 3)
    batch.step(4)
    got = [host(t) for t in batch.get_state(1)]
    batch.close()
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def _resume_case(make_plan, set_state, nsave, nmore):
    """Run nsave + nmore steps in one plan; save a checkpoint after nsave and
    resume it in a fresh plan for nmore steps: the states agree bit for bit."""
    a = make_plan()
    set_state(a)
    a.step(nsave)
    image = a.checkpoint(0)
    a.step(nmore)
    want = [host(t) for t in a.get_state(0)]
    a.close()
    b = make_plan()
    b.load_checkpoint(0, image)
    b.step(nmore)
    got = [host(t) for t in b.get_state(0)]
    assert b.diagnostics(0)["step"] == nsave + nmore
    b.close()
    return image.nbytes, want, got


@pytest.mark.parametrize("precision,kw", [(etd.FP64, {}),
                                          (etd.FP32, dict(band_threshold=0.995, band_rebuild_every=3)),
                                          (etd.FP64, dict(band_threshold=0.995, band_rebuild_every=3,
                                                          flags=etd.F_SURFACE_NONLOCAL))])
def test_coupled_checkpoint_resumes_bit_for_bit(precision, kw):
    """Saved after 4 steps (band rebuilt at steps 0 and 3, so the list in use
    came from phi^3), resumed for 5: the band list, the spectrum of phi, A0
    and the band solve's starting iterate all come back."""
    ci = inputs.coupled_membrane(n=(24, 24, 32), seed=31, tau=1e-4, eps_pm_in_h=1.5,
                                 overrides=dict(B2=16000.0))
    dt = torch.float64 if precision == etd.FP64 else torch.float32

    def make():
        return etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=precision, **kw))

    nbytes, want, got = _resume_case(make, lambda p: p.set_state(0, dev(ci.phi0, dt), dev(ci.u0, dt)), 4, 5)
    report("checkpoint_coupled", precision=precision, opts=str(kw), nbytes=nbytes)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_fixed_checkpoint_resumes_bit_for_bit():
    fi = inputs.fixed_membrane(dim=3, n=24, eps_pm_in_h=2.0, tau=0.02)

    def make():
        return etd.Plan(etd.fixed_instance(fi, scheme=etd.ETDRK2, flags=etd.F_MASS_PROJECT))

    nbytes, want, got = _resume_case(make, lambda p: p.set_state(0, dev(fi.g), dev(fi.u0)), 3, 4)
    report("checkpoint_fixed", nbytes=nbytes)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_checkpoint_rejects_a_different_instance():
    ci = inputs.coupled_membrane(n=16, seed=31, tau=1e-4)
    a = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2))
    with pytest.raises(etd.EtdError) as ei:
        a.checkpoint(0)
    assert ei.value.status == etd.ETD_E_STATE
    a.set_state(0, dev(ci.phi0), dev(ci.u0))
    image = a.checkpoint(0)
    b = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETD1))
    with pytest.raises(etd.EtdError) as ei:
        b.load_checkpoint(0, image)
    assert ei.value.status == etd.ETD_E_ARG
    with pytest.raises(etd.EtdError):
        a.load_checkpoint(0, image[:100])
    bad = image.copy()
    bad[:8] = 0
    with pytest.raises(etd.EtdError):
        a.load_checkpoint(0, bad)
    a.close()
    b.close()


@pytest.mark.parametrize("mode", [etd.EXEC_EAGER, etd.EXEC_GRAPH])
def test_diagnostics_ring_records_every_step(mode):
    """A ring of 6 entries over 9 steps (4 eager, then 5 under the schedule
    tested): the last 6 entries hold steps 4..9, each equal to etd_diagnostics
    of a second plan stepped one step at a time; set_state starts the record
    again."""
    ci = inputs.coupled_membrane(n=32, seed=31, tau=5e-5)
    kw = dict(scheme=etd.ETDRK2, band_threshold=0.995, band_rebuild_every=3)
    ref = etd.Plan(etd.coupled_instance(ci, **kw))
    ref.set_state(0, dev(ci.phi0), dev(ci.u0))
    want = []
    for _ in range(9):
        ref.step(1)
        want.append(ref.diagnostics(0))
    ref.close()
    plan = etd.Plan(etd.coupled_instance(ci, **kw))
    plan.diag_ring(0, 6)
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    plan.step(4)
    plan.set_schedule(mode, 1)
    plan.step(5)
    got, rec = plan.read_diag_ring(0)
    assert rec == 9 and [d["step"] for d in got] == [4, 5, 6, 7, 8, 9]
    for d, w in zip(got, want[3:]):
        assert d["nonfinite"] == 0
        for k in ("step", "int_phi", "mass", "Q", "umin", "umax", "bound", "band_count", "nonfinite"):
            assert d[k] == w[k], (d["step"], k, d[k], w[k])
    plan.set_state(0, dev(ci.phi0), dev(ci.u0))
    plan.set_schedule(etd.EXEC_EAGER, 1)
    plan.step(2)
    got, rec = plan.read_diag_ring(0, max_entries=1)
    assert rec == 2 and [d["step"] for d in got] == [2]
    plan.diag_ring(0, 0)
    with pytest.raises(etd.EtdError) as ei:
        plan.read_diag_ring(0)
    assert ei.value.status == etd.ETD_E_STATE
    plan.close()
