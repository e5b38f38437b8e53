"""The C-ABI library loads, exports every declared entry point, and rejects
invalid descriptors before any HIP call (CPU only: no compute is run)."""
import ctypes as C
import os
import re

import pytest

from paper_2606_04347_amd import etd

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "etd.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:etd_status|const char\*)\s+(etd_[a-z_]+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = etd.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(etd.EXPORTS) == set(names)


def _desc(model=etd.COUPLED, shape=(16, 16, 16), tau=1e-4, scheme=2, prec=0):
    d = (etd.InstanceDesc * 1)()
    d[0].model, d[0].scheme, d[0].precision = model, scheme, prec
    d[0].grid = etd.make_grid(shape, (1.0,) * len(shape))
    d[0].tau = tau
    d[0].recover_threshold = 1e-3
    cp = etd.CoupledParams()
    cp.mu, cp.eps_phi, cp.eps_u = 2.0, 0.3, 0.15
    fp = etd.FixedParams(0.1, 1.0, 0.4, 600.0, 0.0, 0)
    d[0].coupled = C.pointer(cp)
    d[0].fixed = C.pointer(fp)
    return d, (cp, fp)


@pytest.mark.parametrize("mutate,status", [
    (lambda d: setattr(d[0], "tau", 0.0), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "tau", float("nan")), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "grid", etd.make_grid((15, 16, 16), (1, 1, 1))), etd.ETD_E_SIZE),
    (lambda d: setattr(d[0], "grid", etd.make_grid((20, 16, 16), (1, 1, 1))), etd.ETD_E_SIZE),
    (lambda d: setattr(d[0], "grid", etd.make_grid((1024, 16, 16), (1, 1, 1))), etd.ETD_E_SIZE),
    (lambda d: setattr(d[0], "grid", etd.make_grid((16, 15), (1, 1))), etd.ETD_E_SIZE),   # odd 2D length
    (lambda d: setattr(d[0].grid, "dim", 4), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "model", 7), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "scheme", 3), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "coupled", C.POINTER(etd.CoupledParams)()), etd.ETD_E_ARG),
    (lambda d: setattr(d[0].coupled.contents, "eps_phi", -1.0), etd.ETD_E_ARG),
    (lambda d: setattr(d[0].coupled.contents, "gamma", float("inf")), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "recover_threshold", -1.0), etd.ETD_E_ARG),
    (lambda d: (setattr(d[0], "band_threshold", 0.995), setattr(d[0], "band_rebuild_every", 0)), etd.ETD_E_ARG),
    (lambda d: setattr(d[0], "flags", 0x10), etd.ETD_E_ARG),                              # unknown flag bit
    (lambda d: setattr(d[0], "flags", etd.F_BAND_STEP), etd.ETD_E_ARG),                   # fixed model only
    (lambda d: setattr(d[0], "flags", etd.F_SURFACE_NONLOCAL), etd.ETD_E_ARG),            # band solve without a band
])
def test_plan_create_rejects_invalid_descriptors(mutate, status):
    L = etd.lib()
    d, keep = _desc()
    mutate(d)
    p = C.c_void_p()
    assert L.etd_plan_create(d, 1, None, C.byref(p)) == status
    assert not p.value
    assert L.etd_last_error(None)


def test_fixed_membrane_validation():
    L = etd.lib()
    d, keep = _desc(model=etd.FIXED_MEMBRANE, shape=(64, 64), scheme=1)
    d[0].fixed.contents.eps_u = 0.0
    p = C.c_void_p()
    assert L.etd_plan_create(d, 1, None, C.byref(p)) == etd.ETD_E_ARG
    d[0].fixed.contents.eps_u = 0.1
    d[0].flags = etd.F_FROZEN_MEMBRANE          # a coupled-model flag
    assert L.etd_plan_create(d, 1, None, C.byref(p)) == etd.ETD_E_ARG
    d[0].flags = 0
    d[0].fixed = C.POINTER(etd.FixedParams)()
    assert L.etd_plan_create(d, 1, None, C.byref(p)) == etd.ETD_E_ARG


def test_null_arguments_and_status_strings():
    L = etd.lib()
    p = C.c_void_p()
    assert L.etd_plan_create(None, 1, None, C.byref(p)) == etd.ETD_E_ARG
    d, keep = _desc()
    assert L.etd_plan_create(d, 0, None, C.byref(p)) == etd.ETD_E_ARG
    assert L.etd_step(None, 1) == etd.ETD_E_ARG
    assert L.etd_set_tau(None, 0, 1e-4) == etd.ETD_E_ARG
    assert L.etd_surface_lapinv(None, 0, None, None, None, None, 0, 1e-12, 10, None, None) == etd.ETD_E_ARG
    n = C.c_size_t(0)
    assert L.etd_checkpoint_size(None, 0, C.byref(n)) == etd.ETD_E_ARG
    assert L.etd_checkpoint_save(None, 0, None, 0) == etd.ETD_E_ARG
    assert L.etd_checkpoint_load(None, 0, None, 0) == etd.ETD_E_ARG
    assert L.etd_diag_ring_enable(None, 0, 8) == etd.ETD_E_ARG
    assert L.etd_diag_ring_read(None, 0, None, 0, None) == etd.ETD_E_ARG
    assert L.etd_plan_destroy(None) == etd.ETD_OK
    for s in range(-7, 1):
        assert L.etd_status_string(s)


def test_ctypes_layouts_match_the_header(tmp_path):
    """Every structure and array length the binding marshals has the size and
    field offsets the header gives it, as a C compiler lays them out (so no
    call can write past a buffer the binding allocated)."""
    import json
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"etd_grid": etd.Grid, "etd_coupled_params": etd.CoupledParams, "etd_fixed_params": etd.FixedParams,
               "etd_instance_desc": etd.InstanceDesc, "etd_pass_times": etd.PassTimes,
               "etd_schedule": etd.Schedule, "etd_diag": etd.Diag}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "etd.h"', 'int main(void) {', 'printf("{");']
    for cname, cls in structs.items():
        lines.append(f'printf("\\"{cname}\\": [%zu", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf(", %zu", offsetof({cname}, {fname}));')
        lines.append('printf("], ");')
    lines.append('printf("\\"pass_kinds\\": %d, \\"autotune\\": %d}", ETD_PASS_KINDS, ETD_AUTOTUNE_CANDIDATES);')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)
    for cname, cls in structs.items():
        want = [C.sizeof(cls)] + [getattr(cls, f).offset for f, _ in cls._fields_]
        assert got[cname] == want, cname
    assert got["pass_kinds"] == etd.N_PASS_SLOTS
    assert got["autotune"] == len(etd.AUTOTUNE_CANDIDATES)


def test_etd_log_reports_errors_on_stderr():
    """ETD_LOG=1 sends every error status with its message to stderr; the
    default is quiet (each run in a fresh process: the level is read once)."""
    import subprocess
    import sys
    code = ("import ctypes as C\n"
            "from paper_2606_04347_amd import etd\n"
            "p = C.c_void_p()\n"
            "assert etd.lib().etd_plan_create(None, 1, None, C.byref(p)) == etd.ETD_E_ARG\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = {}
    for level in ("0", "1"):
        env = dict(os.environ, ETD_LOG=level)
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        outs[level] = r.stderr
    assert "[etd]" not in outs["0"]
    assert f"[etd] error {etd.ETD_E_ARG}: need at least one instance descriptor" in outs["1"]
