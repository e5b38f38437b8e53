"""Benchmark: grid-point steps/s of the coupled ETDRK2 step on a 256^3 grid,
FP32 path (headline) with the FP64 path timed beside it, on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]

Prints ONE JSON line.  Inputs are the seeded synthetic perturbed-sphere
vesicle (inputs.coupled_membrane), resident in HBM before timing starts.
Besides the headline it reports
  fp64           the FP64 path on the same workload
  fp32_vs_fp64   relative L-inf gap of the two GPU paths after --err-steps steps
  roofline       the dominant kernel (the FFT pass kind with the largest
                 event-timed total) against the 8 TB/s HBM peak
  cpu_baseline   the FP64 oracle timed on this host on one step of the same
                 workload
  batched        the uneven 48-instance sweep (32 x 64^3, 12 x 96^3, 4 x
                 128^3) under the grouped schedule against sequential
                 per-instance launches, measured in a child process first
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--err-steps", type=int, default=100,
                    help="FP32 vs FP64 GPU gap after this many steps (0 = skip)")
    ap.add_argument("--no-band", action="store_true",
                    help="skip the 512^3 narrow-band measurement")
    ap.add_argument("--band-n", type=int, default=512)
    ap.add_argument("--band-steps", type=int, default=50)
    ap.add_argument("--no-fixed", action="store_true",
                    help="skip the 128^3 fixed-membrane measurement")
    ap.add_argument("--fixed-n", type=int, default=128)
    ap.add_argument("--no-surface", action="store_true",
                    help="skip the band-solve leg ((-Delta_S,h)^{-1} on the band, 256^3)")
    ap.add_argument("--surface-n", type=int, default=256)
    ap.add_argument("--surface-steps", type=int, default=4)
    ap.add_argument("--no-batch", action="store_true",
                    help="leave out the uneven-batch measurement (32x64^3 + 12x96^3 + 4x128^3 instances, run in a "
                         "child process)")
    ap.add_argument("--batch-only", action="store_true", help="only the uneven-batch measurement (one JSON line)")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--coarsening", type=float, default=0.0,
                    help="run the four 2D coarsening experiments to this final time (the paper's: 1000); 0 = off")
    ap.add_argument("--coarsening-every", type=float, default=1.0, help="checkpoint interval (time units)")
    ap.add_argument("--coarsening-runs", default="0,1,2,3",
                    help="which of the four coarsening runs (circle ETD1, circle, ellipse, protrusions ETDRK2)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 256 MiB device copies (a reference kernel of known size "
                         "for hardware byte counters)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn the counter CSVs of a FETCH_SIZE and a WRITE_SIZE pass "
                         "(rocprofv3 --pmc, both with --copy-calibration) into "
                         "profiles/traffic_fp32_256cubed.json and exit")
    return ap.parse_args()


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def timed_steps(plan, steps, warmup):
    import torch
    plan.step(warmup)
    torch.cuda.synchronize()
    s = plan.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    plan.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)      # ms


def run_precision(ci, prec, dt, steps, warmup, pass_steps):
    import torch

    from paper_2606_04347_amd import etd
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=prec))
    plan.set_state(0, torch.as_tensor(ci.phi0, dtype=dt, device="cuda"),
                   torch.as_tensor(ci.u0, dtype=dt, device="cuda"))
    ms = timed_steps(plan, steps, warmup)
    # per-pass event timing on the same stream, right after the timed region
    plan.pass_timing(True)
    plan.step(pass_steps)
    passes = plan.pass_timing(False)
    plan.close()
    return ms, passes


# Sources that are not compiled into the passes of the 3D coupled step
# (fixed-membrane stencils, the band solve, the band list, the 2D coupled
# kernels): a change there leaves the counters of those passes valid.
TRAFFIC_HASH_EXCLUDES = ("fixed.hip", "surface.hip", "band.hip", "coupled.hip")


def kernel_source_hash():
    """sha256 over the sources of the 3D coupled step's kernels and launches
    (file names and contents)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_04347_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        if os.path.basename(p) in TRAFFIC_HASH_EXCLUDES:
            continue
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic(kind, n, precision):
    """HBM bytes per launch of a kernel kind from the committed counter summary
    (profiles/traffic_fp32_256cubed.json: calibrated FETCH_SIZE + WRITE_SIZE),
    only while the kernel sources are the ones the counters were taken on."""
    path = os.path.join(ROOT, "profiles", "traffic_fp32_256cubed.json")
    try:
        rec = json.load(open(path))
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("grid") != n or \
            rec.get("precision") != precision:
        return None
    p = rec.get("passes", {}).get(kind)
    return p["bytes_per_launch"] if p else None


# kernel name -> pass kind of the ledger (the FP32 instantiations are read)
KERNEL_KINDS = (("k_x_etd<", "pair_x_etd"), ("k_y_pair<", "pair_y_lines"), ("k_fft_ylines<", "fft_y_lines"),
                ("k_fft_xlines<", "fft_x_lines"), ("k_deriv_y<", "deriv_y"), ("k_deriv_x<", "deriv_x"),
                ("k_deriv_z<", "deriv_z_c2r"), ("k_lapinv_lines<", "lapinv_lines"),
                ("k_z_c2r_recover<", "z_c2r_recover"), ("k_z_r2c_r1<", "z_r2c_r1"), ("k_z_r2c_p2<", "z_r2c_p2"),
                ("k_z_r2c_q<", "z_r2c_q"), ("k_z_r2c_pair<", "pair_z_r2c"), ("k_fft_z_r2c<", "fft_z_r2c"),
                ("k_fft_z_c2r<", "fft_z_c2r"))
COPY_BYTES = 64 * 2 ** 20 * 4      # one --copy-calibration copy: 256 MiB read, 256 MiB written


def summarize_traffic(fetch_csv, write_csv):
    """Per-kind HBM bytes per launch from a FETCH_SIZE and a WRITE_SIZE counter
    pass (KiB per dispatch), each scaled by what the counter reads for the
    calibration copy of COPY_BYTES."""
    import csv

    def per_kernel(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")

    def calib(d):
        vals = [v for k, vs in d.items() if "copyBuffer" in k for v in vs]
        vals = [v for v in vals if v > 0.25 * COPY_BYTES / 1024]   # the 256 MiB copies only
        return (COPY_BYTES / 1024) / (sum(vals) / len(vals)) if vals else None

    ff, wf = calib(fetch), calib(write)
    if ff is None or wf is None:
        raise SystemExit("no calibration copy in the counter CSVs (run them with --copy-calibration); copy-like "
                         f"kernels seen: {sorted(k for k in fetch if 'copy' in k.lower())}")
    rec = {"kernel_source_sha256": kernel_source_hash(), "grid": 256, "precision": "fp32",
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_factor": ff, "write_factor": wf}, "passes": {}}
    for name in fetch:
        if "float" not in name or name not in write:
            continue
        kind = next((k for pat, k in KERNEL_KINDS if pat in name), None)
        if kind is None:
            continue
        fk = sum(fetch[name]) / len(fetch[name])
        wk = sum(write[name]) / len(write[name])
        p = rec["passes"].setdefault(kind, {"fetch_kib": 0.0, "write_kib": 0.0, "n": 0})
        m = len(fetch[name])
        p["fetch_kib"] = (p["fetch_kib"] * p["n"] + fk * m) / (p["n"] + m)
        p["write_kib"] = (p["write_kib"] * p["n"] + wk * m) / (p["n"] + m)
        p["n"] += m
    for p in rec["passes"].values():
        p["bytes_per_launch"] = 1024.0 * (p["fetch_kib"] * ff + p["write_kib"] * wf)
    path = os.path.join(ROOT, "profiles", "traffic_fp32_256cubed.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(path)


def roofline(passes, pass_steps, n, precision):
    kind = max(passes, key=lambda k: passes[k]["ms"])
    p = passes[kind]
    avg_ms = p["ms"] / max(p["launches"], 1)
    per_launch = p["bytes"] / max(p["launches"], 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kind, n, precision),
            "kernel": kind, "launches_per_step": p["launches"] / pass_steps,
            "avg_launch_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": per_launch}


FFT_KINDS = ("fft_z_r2c", "fft_z_c2r", "fft_y_lines", "fft_x_lines", "deriv_x", "deriv_y", "deriv_z_c2r",
             "pair_z_r2c", "pair_y_lines", "pair_x_etd", "lapinv_lines", "z_c2r_recover")
# z passes with the R1 / P2 stencils formed in their load
FUSED_STENCIL_KINDS = ("z_r2c_r1", "z_r2c_p2", "z_r2c_q")


def ledger(passes, pass_steps, npts, ms_per_step):
    """Per-kind and whole-step algorithmic bytes from the pass-timed steps."""
    kinds = {k: {"launches_per_step": v["launches"] / pass_steps, "ms_per_step": v["ms"] / pass_steps,
                 "bytes_per_step": v["bytes"] / pass_steps,
                 "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None}
             for k, v in passes.items() if v["launches"]}
    tot_b = sum(v["bytes"] for v in passes.values()) / pass_steps
    tot_ms = sum(v["ms"] for v in passes.values()) / pass_steps
    return {"bytes_per_step": tot_b, "bytes_per_point_step": tot_b / npts,
            "kernel_ms_per_step": tot_ms,
            "achieved_GBps_kernel_time": tot_b / (tot_ms * 1e-3) / 1e9,
            "achieved_GBps_wall": tot_b / (ms_per_step * 1e-3) / 1e9,
            "frac_wall": tot_b / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kinds": kinds}


def band_measure(n, steps, warmup):
    """Coupled FP32 ETDRK2 at n^3 with the narrow band |2 phi - 1| < 0.995
    rebuilt every 10 steps: throughput, and the band kernels, the stencil
    kernels and the FFT passes timed separately over 10 steps."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    t0 = time.time()
    ci = inputs.coupled_membrane(n=n, tau=1e-4)
    log(f"band inputs {n}^3 {time.time() - t0:.1f}s")
    plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=etd.FP32, band_threshold=0.995,
                                         band_rebuild_every=10))
    plan.set_state(0, torch.as_tensor(ci.phi0, dtype=torch.float32, device="cuda"),
                   torch.as_tensor(ci.u0, dtype=torch.float32, device="cuda"))
    del ci
    ms = timed_steps(plan, steps, warmup) / steps
    plan.pass_timing(True)
    plan.step(10)
    passes = plan.pass_timing(False)
    d = plan.diagnostics(0)
    plan.close()
    npts = n ** 3
    group = lambda ks: sum(passes[k]["ms"] for k in ks) / 10
    return {"workload": f"coupled ETDRK2 FP32, {n}^3 grid, eps=3h, tau=1e-4, narrow band |2 phi - 1| < 0.995 "
                        "rebuilt every 10 steps", "grid": [n, n, n], "steps": steps,
            "value": npts / (ms * 1e-3), "unit": "grid-pt steps/s", "ms_per_step": ms,
            "band_points": d["band_count"], "band_fraction": d["band_count"] / npts,
            "ms_per_step_by_group": {"fft_passes": group(FFT_KINDS), "band_flags_and_compaction": group(("band",)),
                                     "stencils_R1_P2": group(("r1_stencil", "p2_stencil")),
                                     "z_r2c_with_R1_P2": group(FUSED_STENCIL_KINDS),
                                     "pointwise_and_reductions": group(("pointwise", "reduce"))},
            "band_kernels_per_rebuild_ms": passes["band"]["ms"] / max(1, passes["band"]["launches"]),
            "ledger": ledger(passes, 10, npts, ms)}


def surface_measure(n, steps):
    """Coupled FP32 ETDRK2 at n^3 with the narrow band |2 phi - 1| < 0.995 and
    the nonlocal term by the band solve of (-Delta_S,h)^{-1}
    (ETD_F_SURFACE_NONLOCAL): step time, iterations and final relative
    residual of the last solve, beside the same step with (-Delta_h)^{-1}."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    ci = inputs.coupled_membrane(n=n, tau=1e-4)
    out = {"workload": f"coupled ETDRK2 FP32, {n}^3 grid, eps=3h, tau=1e-4, band |2 phi - 1| < 0.995, nonlocal "
                       f"term by the band solve (FP64 CG, 16-term Chebyshev polynomial preconditioner, relative residual 1e-9)", "grid": [n, n, n],
           "steps": steps}
    for name, flags in (("band_solve", etd.F_SURFACE_NONLOCAL), ("fft_inverse", 0)):
        plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=etd.FP32, band_threshold=0.995,
                                             band_rebuild_every=10, flags=flags))
        plan.set_state(0, torch.as_tensor(ci.phi0, dtype=torch.float32, device="cuda"),
                       torch.as_tensor(ci.u0, dtype=torch.float32, device="cuda"))
        ms = timed_steps(plan, steps, 1) / steps
        r = {"ms_per_step": ms, "value": n ** 3 / (ms * 1e-3), "unit": "grid-pt steps/s"}
        d = plan.diagnostics(0)
        r["umin"], r["umax"], r["mass"] = d["umin"], d["umax"], d["mass"]   # the state stays finite and bounded
        if flags:
            r["iterations_last_solve"] = plan.query(0, etd.Q_SURF_ITERS)
            r["relres_last_solve"] = plan.query(0, etd.Q_SURF_RELRES)
            r["band_points"] = d["band_count"]
        out[name] = r
        plan.close()
    return out


def fixed_measure(n, warmup):
    """Fixed-membrane ETDRK2 at n^3 on [-1, 1)^3 (sphere R = 0.5, eps = 2h,
    M = 200, tau = 0.02; 2 untimed steps, which capture the two-step graph of
    the graph schedule, then 48 timed steps, to T = 1.0), FP64 and FP32-FFT
    paths: throughput, the maximum bound, energy and mass."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    fi = inputs.fixed_membrane(dim=3, n=n, eps_pm_in_h=2.0, tau=0.02)
    nsteps = 48
    out = {"workload": f"fixed-membrane ETDRK2, {n}^3 grid on [-1,1)^3, sphere R=0.5, eps=2h, M=200, tau=0.02, "
                       f"2 + {nsteps} steps (T=1.0), graph schedule", "grid": [n, n, n]}
    for prec, name in ((etd.FP64, "fp64"), (etd.FP32, "fp32_fft")):
        plan = etd.Plan(etd.fixed_instance(fi, scheme=etd.ETDRK2, precision=prec))
        plan.set_state(0, torch.as_tensor(fi.g, device="cuda"), torch.as_tensor(fi.u0, device="cuda"))
        e0 = plan.energy(0)["E"]
        mass0 = plan.diagnostics(0)["mass"]
        plan.set_schedule(etd.EXEC_GRAPH, 1)
        ms = timed_steps(plan, nsteps, 2) / nsteps
        d = plan.diagnostics(0)
        e1 = plan.energy(0)["E"]
        plan.pass_timing(True)
        plan.step(2)
        passes = plan.pass_timing(False)
        out[name] = {"value": n ** 3 / (ms * 1e-3), "unit": "grid-pt steps/s", "ms_per_step": ms,
                     "steps": nsteps, "B": plan.query(0, etd.Q_B), "cheb_degree": plan.query(0, etd.Q_CHEB_DEG),
                     "umin": d["umin"], "umax": d["umax"], "max_abs_2u_minus_1": d["bound"],
                     "energy_start": e0, "energy_end": e1, "mass_start": mass0, "mass_end": d["mass"],
                     "ledger": ledger(passes, 2, n ** 3, ms)}
        plan.close()
    out["frozen_coupled"] = frozen_measure(n, out["fp64"]["B"], nsteps)
    return out


def frozen_measure(n, B2, nsteps):
    """The coupled scheme's u stages on the same frozen sphere (ETD_F_FROZEN_MEMBRANE,
    ETDRK2, B2 = the fixed scheme's B, B1 = 1, tau = 0.02; 2 untimed steps,
    which take the first launches of every kernel, then nsteps timed ones):
    throughput, bounds and the u part of the coupled energy, beside the
    localization split above."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    ci = inputs.frozen_sphere(n=n, B2=B2, tau=0.02)
    out = {"workload": f"coupled u stages on a frozen sphere, {n}^3 on [-1,1)^3, ETDRK2, B2={B2:.6g}, B1=1, "
                       f"tau=0.02, 2 + {nsteps} steps"}
    for prec, name, dt in ((etd.FP64, "fp64", torch.float64), (etd.FP32, "fp32", torch.float32)):
        plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=prec, flags=etd.F_FROZEN_MEMBRANE))
        plan.set_state(0, torch.as_tensor(ci.phi0, dtype=dt, device="cuda"),
                       torch.as_tensor(ci.u0, dtype=dt, device="cuda"))
        e = plan.energy(0)
        e0 = e["E_ok"] + e["E_nonlocal"] + e["E_mass"]
        ms = timed_steps(plan, nsteps, 2) / nsteps
        d = plan.diagnostics(0)
        e = plan.energy(0)
        out[name] = {"value": n ** 3 / (ms * 1e-3), "unit": "grid-pt steps/s", "ms_per_step": ms, "steps": nsteps,
                     "umin": d["umin"], "umax": d["umax"], "energy_u_start": e0,
                     "energy_u_end": e["E_ok"] + e["E_nonlocal"] + e["E_mass"]}
        plan.close()
    return out


def precision_gap(ci, nsteps):
    """Relative L-inf gap between the FP32 and FP64 GPU paths after nsteps from
    the same initial state, stepped side by side (the FP64 path is itself
    checked against the oracle's trajectory).  The recovery U = GU/G on
    {G > 1e-3} (after Algorithm 1) is discontinuous in G: where the two
    paths' G fall on opposite sides of the threshold they take different
    branches and U differs by O(U) there, which the stencils of later steps
    carry to the neighbours.  Reported: the all-points gap, the gap outside
    those points (counted over all steps) and their two-cell neighbourhood,
    and the gap of g u, the quantity the scheme carries."""
    import torch
    import torch.nn.functional as F

    from paper_2606_04347_amd import etd
    plans = {}
    for prec, dt in ((etd.FP32, torch.float32), (etd.FP64, torch.float64)):
        plan = etd.Plan(etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=prec))
        plan.set_state(0, torch.as_tensor(ci.phi0, dtype=dt, device="cuda"),
                       torch.as_tensor(ci.u0, dtype=dt, device="cuda"))
        plans[prec] = plan
    flips = torch.zeros(ci.shape, dtype=torch.bool, device="cuda")
    for _ in range(nsteps):
        for p in plans.values():
            p.step(1)
        f32 = plans[etd.FP32].get_state(0, torch.float32)[0]
        f64 = plans[etd.FP64].get_state(0)[0]
        a = f32 * f32 - f32
        g32 = (18.0 * a * a).double()
        g64 = 18.0 * (f64 * f64 - f64) ** 2
        flips |= ((g32 > 1e-3) != (g64 > 1e-3)) | ((g32 / 1e-3 - 1.0).abs() < 1e-5)
    p32, u32 = plans[etd.FP32].get_state(0)
    p64, u64 = plans[etd.FP64].get_state(0)
    for p in plans.values():
        p.close()
    r = 2
    near = F.max_pool3d(F.pad(flips.to(torch.float32)[None, None], (r,) * 6, mode="circular"), 2 * r + 1,
                        stride=1)[0, 0] > 0
    d = (u32 - u64).abs()
    scale = u64.abs().max()
    g = 18.0 * (p64 * p64 - p64) ** 2
    rel = lambda a, b: float((a - b).abs().max() / b.abs().max())
    return {"steps": nsteps, "phi": rel(p32, p64), "u": rel(u32, u64),
            "u_outside_flips": float(d[~near].max() / scale), "flips": int(flips.sum()),
            "flip_neighbourhood_points": int(near.sum()), "flip_radius": r,
            "gu": float((g * d).max() / (g * u64).abs().max()),
            "g_at_max_u_gap": float(g.reshape(-1)[int(torch.argmax(d))])}


def batch_measure(steps, warmup):
    """Uneven batch of 48 coupled FP32 ETDRK2 instances (32 x 64^3, 12 x 96^3,
    4 x 128^3 = 27,394,048 points) in one plan, each with its own seed,
    coefficients and tau: sequential per-instance launches (eager, one
    instance after another) against the grouped schedule (one launch per pass
    per shape class, captured two steps at a time) over its branch and tile
    candidates, with the graph schedule on four branches beside them."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    t0 = time.time()
    cis = inputs.batch_sweep()
    log(f"batch inputs {time.time() - t0:.1f}s")
    npts = sum(int(ci.phi0.size) for ci in cis)
    plan = etd.Plan([etd.coupled_instance(ci, scheme=etd.ETDRK2, precision=etd.FP32) for ci in cis])
    for i, ci in enumerate(cis):
        plan.set_state(i, torch.as_tensor(ci.phi0, dtype=torch.float32, device="cuda"),
                       torch.as_tensor(ci.u0, dtype=torch.float32, device="cuda"))
    base_steps = max(2, (steps // 5) & ~1)
    ms_eager = timed_steps(plan, base_steps, warmup) / base_steps
    log(f"batch eager: {ms_eager:.3f} ms/step")
    cands = {}
    for name, mode, branches, xlines in (("grouped1", etd.EXEC_GROUPED, 1, 0), ("grouped3", etd.EXEC_GROUPED, 3, 0),
                                         ("grouped1_x8", etd.EXEC_GROUPED, 1, 8),
                                         ("grouped3_x8", etd.EXEC_GROUPED, 3, 8), ("graph4", etd.EXEC_GRAPH, 4, 0)):
        plan.set_schedule(mode, branches, xlines)
        n = steps if mode == etd.EXEC_GROUPED else base_steps
        cands[name] = timed_steps(plan, n, warmup) / n
        log(f"batch {name}: {cands[name]:.3f} ms/step")
    plan.close()
    best = min((k for k in cands if k.startswith("grouped")), key=lambda k: cands[k])
    rate = lambda ms: npts / (ms * 1e-3)
    return {"workload": "32 x 64^3 + 12 x 96^3 + 4 x 128^3 coupled ETDRK2 FP32 instances in one plan "
                        f"({npts} points), per-instance seeds, coefficients and tau in {{5e-5, 1e-4}}",
            "value": rate(cands[best]), "unit": "grid-pt steps/s", "ms_per_step": cands[best], "steps": steps,
            "schedule": best, "candidates_ms_per_step": cands,
            "eager_sequential": {"value": rate(ms_eager), "ms_per_step": ms_eager, "steps": base_steps},
            "speedup_vs_eager": ms_eager / cands[best],
            "speedup_graph4_vs_eager": ms_eager / cands["graph4"]}


def batch_in_child(steps, warmup, timeout=300):
    """The batch leg in a child process (started before this process touches
    the GPU): its result, or its exit status and last lines of output."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--batch-only", "--batch-steps", str(steps),
           "--warmup", str(warmup)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout)
    except subprocess.TimeoutExpired:
        return {"error": f"timed out after {timeout} s"}
    sys.stderr.write(r.stderr)
    sys.stderr.flush()
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"exit status {r.returncode}", "stderr_tail": r.stderr.splitlines()[-5:]}
    return json.loads(lines[-1])


def coarsening_measure(T, every, which=(0, 1, 2, 3)):
    """The 2D coarsening experiments of the fixed-membrane OK model (Section
    4.2): ETD1 on the circle (gamma = 2000), ETDRK2 on the circle (3000), the
    ellipse (5000) and the seven-protrusion cell (7000); N = 256 on [-1, 1]^2,
    ubar = 0.5, eps_u = 5h, tau = 1e-3, B = 2000, M = 600 (ETD1) / 200
    (ETDRK2), each step on the narrow band {g >= 1e-3} (the region the initial
    field is drawn on), one plan of four instances under the graph schedule.  Records
    E_phi,h and max|2U - 1| at every checkpoint."""
    import torch

    from paper_2606_04347_amd import etd, inputs
    runs = [inputs.COARSENING_RUNS[k] for k in which]
    fis = [inputs.fixed_coarsening(geo, gamma=gam, M=600.0 if sch == 1 else 200.0, instance=k)
           for k, (geo, sch, gam) in zip(which, runs)]
    plan = etd.Plan([etd.fixed_instance(fi, B=2000.0, scheme=sch, flags=etd.F_BAND_STEP, band_threshold=1e-3)
                     for fi, (_, sch, _) in zip(fis, runs)])
    for k, fi in enumerate(fis):
        plan.set_state(k, torch.as_tensor(fi.g, device="cuda"), torch.as_tensor(fi.u0, device="cuda"))
    plan.set_schedule(etd.EXEC_GRAPH, len(runs))
    tau = fis[0].tau
    chunk = max(2, int(round(every / tau)) & ~1)
    nchk = int(round(T / (chunk * tau)))
    curves = [dict(t=[0.0], E=[plan.energy(k)["E"]], bound=[plan.diagnostics(k)["bound"]]) for k in range(len(runs))]
    umin = [1.0] * len(runs)
    t0 = time.time()
    ms_steps = 0.0
    for c in range(nchk):
        torch.cuda.synchronize()
        s = time.perf_counter()
        plan.step(chunk)
        torch.cuda.synchronize()
        ms_steps += (time.perf_counter() - s) * 1e3
        for k in range(len(runs)):
            d = plan.diagnostics(k)
            curves[k]["t"].append((c + 1) * chunk * tau)
            curves[k]["E"].append(plan.energy(k)["E"])
            curves[k]["bound"].append(d["bound"])
            umin[k] = min(umin[k], d["umin"])
        if (c + 1) % max(1, nchk // 20) == 0:
            log(f"coarsening t={(c + 1) * chunk * tau:.0f} ({time.time() - t0:.0f} s)")
    out = []
    for k, (geo, sch, gam) in enumerate(runs):
        E, bd = curves[k]["E"], curves[k]["bound"]
        out.append({"geometry": geo, "scheme": "ETD1" if sch == 1 else "ETDRK2", "gamma": gam,
                    "M": 600.0 if sch == 1 else 200.0, "B": 2000.0, "B_MBP": plan.query(k, etd.Q_B_MBP),
                    "B_ES": plan.query(k, etd.Q_B_ES), "E_start": E[0], "E_end": E[-1],
                    "E_non_increasing": bool(all(b <= a + 1e-13 * abs(a) for a, b in zip(E, E[1:]))),
                    "max_bound": max(bd), "min_U": umin[k], "curve": curves[k]})
    plan.close()
    npts = sum(fi.g.size for fi in fis)
    return {"workload": "2D coarsening on fixed membranes (Section 4.2), four 256^2 instances in one plan",
            "T": nchk * chunk * tau, "steps": nchk * chunk, "ms_per_step": ms_steps / (nchk * chunk),
            "value": npts * nchk * chunk / (ms_steps * 1e-3), "unit": "grid-pt steps/s", "runs": out}


def cpu_baseline(ci, nsteps=3):
    """The FP64 oracle, as it stands, timed on the first nsteps ETDRK2 steps
    of the workload (about 15 s of CPU work at 256^3)."""
    from oracle import core
    from oracle.core import Grid
    from oracle.coupled import CoupledOracle
    o = CoupledOracle(Grid(ci.shape, ci.half_len), ci.params, ci.tau, 2)
    o.set_state(ci.phi0, ci.u0)
    t0 = time.perf_counter()
    o.run(nsteps)
    dt = time.perf_counter() - t0
    npts = int(ci.phi0.size)
    out = {"value": nsteps * npts / dt, "unit": "grid-pt steps/s", "cores": core.get_threads(), "kind": "oracle",
           "sample": f"the first {nsteps} ETDRK2 steps of the {ci.shape[0]}^3 workload (FP64 numpy/scipy.fft, "
                     f"{core.get_threads()} threads), {dt:.1f} s"}
    # context beside it: one thread, and the oracle's own exact-index DFT, on
    # smaller grids of the same workload family (one step each, a few seconds)
    from paper_2606_04347_amd import inputs
    threads, mode = core.get_threads(), core.get_dft_mode()
    for key, n, nthr, dft in (("single_thread", 128, 1, "library"), ("naive_dft", 64, threads, "naive")):
        core.set_threads(nthr)
        core.set_dft_mode(dft)
        cs = inputs.coupled_membrane(n=n, tau=ci.tau)
        o = CoupledOracle(Grid(cs.shape, cs.half_len), cs.params, cs.tau, 2)
        o.set_state(cs.phi0, cs.u0)
        t0 = time.perf_counter()
        o.run(1)
        dt = time.perf_counter() - t0
        # the naive DFT is a matrix product per axis: BLAS threads, not the FFT workers
        cores = nthr if dft == "library" else int(os.environ.get("OMP_NUM_THREADS", "0") or os.cpu_count() or 1)
        out[key] = {"value": n ** 3 / dt, "unit": "grid-pt steps/s", "cores": cores,
                    "sample": f"one ETDRK2 step at {n}^3 ({dft} DFT, {cores} thread{'s' if cores > 1 else ''}), "
                              f"{dt:.1f} s"}
    core.set_threads(threads)
    core.set_dft_mode(mode)
    return out


def main():
    a = parse()
    if a.summarize_traffic:
        summarize_traffic(*a.summarize_traffic)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU slab "
              "decomposition is designed but not implemented.", file=sys.stderr)
        sys.exit(2)
    if a.batch_only:
        print(json.dumps(batch_measure(a.batch_steps, a.warmup)))
        return
    batched = None if a.no_batch else batch_in_child(a.batch_steps, a.warmup)
    import torch

    from paper_2606_04347_amd import etd, inputs

    if a.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = a.n
    t0 = time.time()
    ci = inputs.coupled_membrane(n=n, tau=1e-4)
    log(f"inputs {time.time() - t0:.1f}s")
    npts = n ** 3
    pass_steps = 3
    res = {}
    for prec, name, dt in ((etd.FP32, "fp32", torch.float32), (etd.FP64, "fp64", torch.float64)):
        if prec == etd.FP64 and a.no_fp64:
            continue
        ms, passes = run_precision(ci, prec, dt, a.steps, a.warmup, pass_steps)
        res[name] = dict(ms_per_step=ms / a.steps, value=npts * a.steps / (ms * 1e-3),
                         roofline=roofline(passes, pass_steps, n, name),
                         ledger=ledger(passes, pass_steps, npts, ms / a.steps))
        log(f"{name}: {ms / a.steps:.3f} ms/step, {res[name]['value']:.3e} pt-steps/s, "
            f"dominant {res[name]['roofline']['kernel']} {res[name]['roofline']['achieved']:.0f} GB/s")
    out = {
        "metric": "grid-pt steps/s, 256^3 coupled ETDRK2: FP32 vs FP64 at <=1e-4 err; % HBM peak",
        "value": res["fp32"]["value"],
        "unit": "grid-pt steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["fp32"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"coupled phi/u ETDRK2 step, {n}^3 grid on [-pi,pi)^3, eps=3h, tau=1e-4, "
                               "perturbed-sphere vesicle (real harmonics l<=4), FP32 path",
                   "grid": [n, n, n], "scheme": "ETDRK2", "precision": "fp32"},
        "roofline": res["fp32"]["roofline"],
        "ledger": res["fp32"]["ledger"],
    }
    if "fp64" in res:
        out["fp64"] = {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                       "roofline": res["fp64"]["roofline"], "ledger": res["fp64"]["ledger"]}
        out["fp32_over_fp64"] = res["fp32"]["value"] / res["fp64"]["value"]
    if not a.no_band:
        out["band"] = band_measure(a.band_n, a.band_steps, a.warmup)
        log(f"band {a.band_n}^3: {out['band']['ms_per_step']:.3f} ms/step, {out['band']['band_points']} band points, "
            f"{out['band']['ms_per_step_by_group']}")
    if not a.no_fixed:
        out["fixed"] = fixed_measure(a.fixed_n, a.warmup)
        log(f"fixed {a.fixed_n}^3: fp64 {out['fixed']['fp64']['ms_per_step']:.3f} ms/step, "
            f"fp32-fft {out['fixed']['fp32_fft']['ms_per_step']:.3f} ms/step, U in "
            f"[{out['fixed']['fp64']['umin']:.4g}, {out['fixed']['fp64']['umax']:.4g}]")
        fz = out["fixed"]["frozen_coupled"]
        log(f"frozen-membrane coupled u stages {a.fixed_n}^3: fp64 {fz['fp64']['ms_per_step']:.3f} ms/step, "
            f"fp32 {fz['fp32']['ms_per_step']:.3f} ms/step, U in [{fz['fp64']['umin']:.4g}, {fz['fp64']['umax']:.4g}], "
            f"E_u {fz['fp64']['energy_u_start']:.6g} -> {fz['fp64']['energy_u_end']:.6g}")
    if not a.no_surface:
        out["surface"] = surface_measure(a.surface_n, a.surface_steps)
        sf = out["surface"]
        log(f"band solve {a.surface_n}^3: {sf['band_solve']['ms_per_step']:.2f} ms/step "
            f"({sf['band_solve']['iterations_last_solve']:.0f} PCG iterations, relres "
            f"{sf['band_solve']['relres_last_solve']:.1e}, {sf['band_solve']['band_points']} band points) vs "
            f"{sf['fft_inverse']['ms_per_step']:.3f} ms/step with (-Delta_h)^-1; U in [{sf['band_solve']['umin']:.4g}, "
            f"{sf['band_solve']['umax']:.4g}] vs [{sf['fft_inverse']['umin']:.4g}, {sf['fft_inverse']['umax']:.4g}]")
    if batched is not None:
        out["batched"] = batched
        if "error" in batched:
            log(f"batched: failed, {batched}")
        else:
            log(f"batched: {batched['ms_per_step']:.3f} ms/step ({batched['schedule']}), "
                f"x{batched['speedup_vs_eager']:.2f} vs sequential per-instance launches")
    if a.coarsening > 0:
        out["coarsening"] = coarsening_measure(a.coarsening, a.coarsening_every,
                                               tuple(int(k) for k in a.coarsening_runs.split(",")))
        for r in out["coarsening"]["runs"]:
            log(f"coarsening {r['geometry']} {r['scheme']} gamma={r['gamma']:.0f}: E {r['E_start']:.6g} -> "
                f"{r['E_end']:.6g} non-increasing={r['E_non_increasing']} max|2U-1|={r['max_bound']:.6f}")
    if a.err_steps > 0:
        out["fp32_vs_fp64"] = precision_gap(ci, a.err_steps)
        log(f"fp32 vs fp64 after {a.err_steps} steps: {out['fp32_vs_fp64']}")
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ci)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
