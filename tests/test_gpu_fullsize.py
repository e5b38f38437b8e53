"""GPU: parity at the benchmark's full sizes, in the configuration bench.py
times -- the coupled ETDRK2 step on the perturbed-sphere vesicle
(inputs.coupled_membrane defaults, eps = 3h, tau = 1e-4) at 128^3 and
256^3 -- against the FP64 oracle: one step against the live oracle, and
200 steps against the oracle's stored trajectory (sampled values written by
tests/golden/make_coupled_trajectories.py); and the FP32 path against the
FP64 path after 100 steps."""
import json
import os

import numpy as np
import pytest

from gpu_util import dev, host, needs_gpu, recovery_flips_dev, rel_linf, report, torch, u_gap_outside_flips_dev
from oracle.core import Grid
from oracle.coupled import CoupledOracle
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def workload():
    return inputs.coupled_membrane(n=256, tau=1e-4)


def make_plan(ci, precision):
    dt = torch.float64 if precision == etd.FP64 else torch.float32
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=precision))
    plan.set_state(0, dev(ci.phi0, dt), dev(ci.u0, dt))
    return plan


def test_fp64_256cubed_step_matches_oracle(workload):
    ci = workload
    plan = make_plan(ci, etd.FP64)
    plan.step(1)
    phi, u = (host(t) for t in plan.get_state(0))
    d = plan.diagnostics(0)
    plan.close()
    o = CoupledOracle(Grid(ci.shape, ci.half_len), ci.params, ci.tau, etd.ETDRK2)
    o.set_state(ci.phi0, ci.u0)
    o.step()
    ephi, eu = rel_linf(phi, o.phi()), rel_linf(u, o.u)
    od = o.diagnostics()
    report("fullsize_fp64", grid="256^3", err_phi=ephi, err_u=eu)
    assert ephi <= 1e-12 and eu <= 1e-12
    assert abs(d["int_phi"] - od["I_phi"]) <= 1e-11 * abs(od["I_phi"])
    assert abs(d["mass"] - od["m"]) <= 1e-11 * max(1.0, abs(od["m"]))


@pytest.mark.parametrize("n", [128, 256])
def test_fp64_trajectory_matches_stored_oracle(n):
    """200 FP64 ETDRK2 steps against the oracle's trajectory, sampled after
    steps 1, 100 and 200 (relative to the oracle's full-grid maxima), with the
    diagnostics."""
    path = os.path.join(GOLDEN, f"coupled_trajectory_{n}.json")
    ref = json.load(open(path))
    ci = inputs.coupled_membrane(n=n, tau=ref["tau"])
    assert list(ci.shape) == ref["grid"] and ci.seed == ref["seed"]
    idx = torch.as_tensor(np.array(ref["sample"], dtype=np.int64), device="cuda")
    plan = make_plan(ci, etd.FP64)
    done = 0
    for k in sorted(int(s) for s in ref["steps"]):
        plan.step(k - done)
        done = k
        r = ref["steps"][str(k)]
        phi, u = plan.get_state(0)
        ephi = float((phi.reshape(-1)[idx].cpu().numpy() - np.array(r["phi"])).__abs__().max() / r["phi_absmax"])
        eu = float((u.reshape(-1)[idx].cpu().numpy() - np.array(r["u"])).__abs__().max() / r["u_absmax"])
        gmax = (float(phi.abs().max()), float(u.abs().max()))
        d = plan.diagnostics(0)
        od = r["diagnostics"]
        report("trajectory_fp64", grid=f"{n}^3", step=k, err_phi=ephi, err_u=eu)
        assert ephi <= 1e-12 and eu <= 1e-12, (k, ephi, eu)
        assert abs(gmax[0] - r["phi_absmax"]) <= 1e-12 * r["phi_absmax"]
        assert abs(gmax[1] - r["u_absmax"]) <= 1e-12 * r["u_absmax"]
        for kg, ko in (("int_phi", "I_phi"), ("mass", "m"), ("Q", "Q"), ("umin", "umin"), ("umax", "umax"),
                       ("bound", "bound")):
            assert abs(d[kg] - od[ko]) <= 1e-11 * max(1.0, abs(od[ko])), (k, kg, d[kg], od[ko])
    plan.close()


@pytest.mark.parametrize("n", [128, 256])
def test_fp32_within_1e_4_of_fp64_after_100_steps(n):
    """The FP32 path against the FP64 path (itself within 1e-12 of the
    oracle's trajectory above) after 100 steps, step by step: phi within
    1e-4 everywhere; u within 1e-4 everywhere except at the points where the
    two paths' G fell on opposite sides of the recovery threshold in some
    step and their two-cell neighbourhood (at most 1e-4 of the grid flips);
    g u within 1e-4 everywhere."""
    ci = inputs.coupled_membrane(n=n, tau=1e-4)
    p32, p64 = make_plan(ci, etd.FP32), make_plan(ci, etd.FP64)
    flips = torch.zeros(ci.shape, dtype=torch.bool, device="cuda")
    for _ in range(100):
        p32.step(1)
        p64.step(1)
        f32 = p32.get_state(0, torch.float32)[0]
        f64 = p64.get_state(0)[0]
        flips |= recovery_flips_dev(f32, f64)
    phi32, u32 = p32.get_state(0)
    phi64, u64 = p64.get_state(0)
    ephi = float((phi32 - phi64).abs().max() / phi64.abs().max())
    eu, near, egu, eall = u_gap_outside_flips_dev(u32, u64, phi64, flips)
    nflip = int(flips.sum())
    report("fullsize_fp32_vs_fp64", grid=f"{n}^3", steps=100, err_phi=ephi, err_u=eu, flips=nflip, near=near,
           err_gu=egu, err_u_all=eall)
    assert bool(torch.isfinite(phi32).all()) and bool(torch.isfinite(u32).all())
    assert ephi <= 1e-4 and eu <= 1e-4 and egu <= 1e-4
    assert nflip <= 1e-4 * flips.numel()
    p32.close()
    p64.close()
