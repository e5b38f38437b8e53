"""ctypes binding of libetd.so (the C ABI declared in include/etd.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (tensor data pointers) and the
HIP stream.  If the library is missing this module raises; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libetd.so")

# enums (etd.h)
ETD_OK, ETD_E_ARG, ETD_E_SIZE, ETD_E_STATE, ETD_E_HIP, ETD_E_NOMEM, ETD_E_NONFINITE, ETD_E_CAPACITY = \
    0, -1, -2, -3, -4, -5, -6, -7
FIXED_MEMBRANE, COUPLED = 0, 1
ETD1, ETDRK2 = 1, 2
FP64, FP32 = 0, 1
F64, F32 = 0, 1
F_MASS_PROJECT = 0x1
F_FROZEN_MEMBRANE = 0x2
F_SURFACE_NONLOCAL = 0x4
F_BAND_STEP = 0x8
OP_IDENTITY, OP_LAPLACE, OP_DX, OP_DY, OP_DZ, OP_LAPINV = range(6)
Q_B, Q_B_MBP, Q_B_ES, Q_C, Q_RHO, Q_CHEB_DEG, Q_A0, Q_WORKSPACE, Q_SURF_ITERS, Q_SURF_RELRES = range(10)

EXPORTS = ("etd_plan_create", "etd_plan_destroy", "etd_set_state", "etd_set_tau", "etd_get_state", "etd_step",
           "etd_energy", "etd_diagnostics", "etd_narrowband_build", "etd_spectral_apply",
           "etd_pass_timing", "etd_plan_query", "etd_set_schedule", "etd_get_schedule", "etd_autotune",
           "etd_surface_lapinv", "etd_narrowband_build_noalloc",
           "etd_checkpoint_size", "etd_checkpoint_save", "etd_checkpoint_load",
           "etd_diag_ring_enable", "etd_diag_ring_read",
           "etd_status_string", "etd_last_error")
EXEC_EAGER, EXEC_GRAPH, EXEC_GROUPED = 0, 1, 2
AUTOTUNE_CANDIDATES = (("eager", 1), ("graph", 1), ("graph", 2), ("graph", 4), ("graph", 8), ("graph", 16),
                       ("graph", 32), ("grouped", 1), ("grouped", 8), ("best_xlines", 8))
PASS_KINDS = ("fft_z_r2c", "fft_z_c2r", "fft_y_lines", "fft_x_lines", "deriv_x", "deriv_y", "deriv_z_c2r",
              "pair_z_r2c", "pair_y_lines", "pair_x_etd", "lapinv_lines", "z_c2r_recover",
              "band", "r1_stencil", "p2_stencil", "pointwise", "reduce", "fixed_stencil", "fixed_pointwise",
              "z_r2c_r1", "z_r2c_p2", "z_r2c_q")
N_PASS_SLOTS = 24


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("half_len", C.c_double * 3)]


class CoupledParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "mu", "lambda_surf", "kappa", "lambda_line", "M_area", "alpha", "u0",
        "eps_phi", "eps_u", "gamma", "ubar", "M", "A1", "A2", "B1", "B2", "A0")] + \
        [("A0_from_initial", C.c_int)]


class FixedParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("eps_u", "gamma", "ubar", "M", "B")] + \
        [("nonlocal_with_ubar", C.c_int)]


class InstanceDesc(C.Structure):
    _fields_ = [("model", C.c_int), ("scheme", C.c_int), ("precision", C.c_int), ("grid", Grid),
                ("tau", C.c_double), ("coupled", C.POINTER(CoupledParams)),
                ("fixed", C.POINTER(FixedParams)), ("band_threshold", C.c_double),
                ("band_rebuild_every", C.c_int), ("recover_threshold", C.c_double),
                ("flags", C.c_uint)]


class PassTimes(C.Structure):
    _fields_ = [("launches", C.c_int64 * N_PASS_SLOTS), ("total_ms", C.c_double * N_PASS_SLOTS),
                ("bytes", C.c_double * N_PASS_SLOTS)]


class Schedule(C.Structure):
    _fields_ = [("mode", C.c_int), ("branches", C.c_int), ("xlines", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("int_phi", C.c_double), ("mass", C.c_double), ("Q", C.c_double),
                ("umin", C.c_double), ("umax", C.c_double), ("bound", C.c_double),
                ("band_count", C.c_int64), ("nonfinite", C.c_int), ("b_warning", C.c_int)]


_lib = None


def lib():
    """Load libetd.so (built in-tree by paper_2606_04347_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2606_04347_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.etd_plan_create.argtypes = [C.POINTER(InstanceDesc), i, vp, C.POINTER(vp)]
        L.etd_plan_destroy.argtypes = [vp]
        L.etd_set_state.argtypes = [vp, i, vp, vp, i]
        L.etd_set_tau.argtypes = [vp, i, d]
        L.etd_get_state.argtypes = [vp, i, vp, vp, i]
        L.etd_step.argtypes = [vp, i]
        L.etd_energy.argtypes = [vp, i, C.POINTER(d), i]
        L.etd_diagnostics.argtypes = [vp, i, C.POINTER(Diag)]
        L.etd_narrowband_build.argtypes = [vp, i, vp, i, d, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.etd_spectral_apply.argtypes = [vp, i, i, vp, vp, i]
        L.etd_plan_query.argtypes = [vp, i, i, C.POINTER(d)]
        L.etd_pass_timing.argtypes = [vp, i, C.POINTER(PassTimes)]
        L.etd_set_schedule.argtypes = [vp, C.POINTER(Schedule)]
        L.etd_get_schedule.argtypes = [vp, C.POINTER(Schedule)]
        L.etd_autotune.argtypes = [vp, i, C.c_char_p, C.POINTER(Schedule), C.POINTER(d)]
        L.etd_surface_lapinv.argtypes = [vp, i, vp, vp, vp, vp, i, d, i, C.POINTER(i), C.POINTER(d)]
        L.etd_narrowband_build_noalloc.argtypes = [vp, vp, i, C.c_int64, d, vp, C.c_int64, C.POINTER(C.c_int64)]
        L.etd_checkpoint_size.argtypes = [vp, i, C.POINTER(C.c_size_t)]
        L.etd_checkpoint_save.argtypes = [vp, i, vp, C.c_size_t]
        L.etd_checkpoint_load.argtypes = [vp, i, vp, C.c_size_t]
        L.etd_diag_ring_enable.argtypes = [vp, i, i]
        L.etd_diag_ring_read.argtypes = [vp, i, C.POINTER(Diag), i, C.POINTER(C.c_int64)]
        L.etd_status_string.argtypes = [i]
        L.etd_status_string.restype = C.c_char_p
        L.etd_last_error.argtypes = [vp]
        L.etd_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("etd_status_string", "etd_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class EtdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().etd_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status, plan_ptr=None):
    if status != ETD_OK:
        raise EtdError(status, lib().etd_last_error(plan_ptr).decode())


# ----------------------------------------------------------------------------- descriptors

def make_grid(shape, half_len):
    g = Grid()
    g.dim = len(shape)
    for k, (n, X) in enumerate(zip(shape, half_len)):
        g.n[k] = int(n)
        g.half_len[k] = float(X)
    return g


def coupled_params(p) -> CoupledParams:
    """From any object with the CoupledParams attribute names (e.g. inputs.CoupledParams)."""
    out = CoupledParams()
    for name, _ in CoupledParams._fields_:
        setattr(out, name, type(getattr(out, name))(getattr(p, name)))
    return out


@dataclass
class Instance:
    """Python-side description of one instance (converted to InstanceDesc)."""
    model: int
    shape: tuple
    half_len: tuple
    tau: float
    scheme: int = ETDRK2
    precision: int = FP64
    coupled: object = None      # object with CoupledParams attributes
    fixed: object = None        # dict/obj with eps_u, gamma, ubar, M, B, nonlocal_with_ubar
    band_threshold: float = 0.0
    band_rebuild_every: int = 10
    recover_threshold: float = 1e-3
    flags: int = 0


class Plan:
    """One etd_plan over one or more instances, bound to a torch stream."""

    def __init__(self, instances, stream=None):
        import torch
        L = lib()
        if isinstance(instances, Instance):
            instances = [instances]
        n = len(instances)
        self._descs = (InstanceDesc * n)()
        self._keep = []
        self.instances = list(instances)
        for k, ins in enumerate(instances):
            d = self._descs[k]
            d.model, d.scheme, d.precision = ins.model, ins.scheme, ins.precision
            d.grid = make_grid(ins.shape, ins.half_len)
            d.tau = ins.tau
            d.band_threshold = ins.band_threshold
            d.band_rebuild_every = ins.band_rebuild_every
            d.recover_threshold = ins.recover_threshold
            d.flags = ins.flags
            if ins.coupled is not None:
                cp = coupled_params(ins.coupled)
                self._keep.append(cp)
                d.coupled = C.pointer(cp)
            if ins.fixed is not None:
                f = ins.fixed
                get = (lambda k_: f[k_]) if isinstance(f, dict) else (lambda k_: getattr(f, k_))
                fp = FixedParams(get("eps_u"), get("gamma"), get("ubar"), get("M"), get("B"),
                                 int(get("nonlocal_with_ubar")))
                self._keep.append(fp)
                d.fixed = C.pointer(fp)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._ptr = C.c_void_p()
        _check(L.etd_plan_create(self._descs, n, C.c_void_p(stream.cuda_stream), C.byref(self._ptr)))

    # -------------------------------------------------------------------- helpers
    def _dt(self, t):
        import torch
        if t.dtype == torch.float64:
            return F64
        if t.dtype == torch.float32:
            return F32
        raise TypeError("float32 or float64 tensors only")

    @staticmethod
    def _dev(t):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("contiguous device tensors required")
        return C.c_void_p(t.data_ptr())

    def _c(self, st):
        _check(st, self._ptr)

    # -------------------------------------------------------------------- API
    def set_state(self, i, a, u):
        assert a.dtype == u.dtype
        self._c(lib().etd_set_state(self._ptr, i, self._dev(a), self._dev(u), self._dt(a)))

    def set_tau(self, i, tau):
        """Time step of the next steps of instance i (variable-step scheme)."""
        self._c(lib().etd_set_tau(self._ptr, i, float(tau)))
        self.instances[i].tau = float(tau)

    def surface_lapinv(self, i, g, f, mask, tol=1e-12, max_iter=20000, psi=None):
        """psi = (-Delta_S,h)^{-1} f on the band {mask != 0} of instance i's grid;
        returns (psi, iterations, final relative residual)."""
        import torch
        assert g.dtype == f.dtype and mask.dtype == torch.uint8
        psi = torch.empty_like(f) if psi is None else psi
        it, rr = C.c_int(0), C.c_double(0.0)
        self._c(lib().etd_surface_lapinv(self._ptr, i, self._dev(g), self._dev(f), self._dev(mask), self._dev(psi),
                                         self._dt(f), float(tol), int(max_iter), C.byref(it), C.byref(rr)))
        return psi, it.value, rr.value

    def get_state(self, i, dtype=None):
        import torch
        ins = self.instances[i]
        dtype = dtype or torch.float64
        a = torch.empty(tuple(ins.shape), dtype=dtype, device="cuda")
        u = torch.empty_like(a)
        self._c(lib().etd_get_state(self._ptr, i, self._dev(a), self._dev(u), self._dt(a)))
        return a, u

    def checkpoint(self, i):
        """The instance's checkpoint image (etd_checkpoint_save) as a numpy uint8 array."""
        import numpy as np
        n = C.c_size_t(0)
        self._c(lib().etd_checkpoint_size(self._ptr, i, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._c(lib().etd_checkpoint_save(self._ptr, i, C.c_void_p(buf.ctypes.data), n.value))
        return buf

    def load_checkpoint(self, i, image):
        """Resume instance i from an image of checkpoint() (etd_checkpoint_load)."""
        import numpy as np
        buf = np.ascontiguousarray(image, dtype=np.uint8)
        self._c(lib().etd_checkpoint_load(self._ptr, i, C.c_void_p(buf.ctypes.data), buf.nbytes))

    def step(self, nsteps=1):
        self._c(lib().etd_step(self._ptr, int(nsteps)))

    def energy(self, i=0):
        out = (C.c_double * 6)()
        n = 6 if self.instances[i].model == COUPLED else 5
        self._c(lib().etd_energy(self._ptr, i, out, n))
        names = (["E_surf", "E_bend", "E_area", "E_ok", "E_nonlocal", "E_mass"]
                 if n == 6 else ["E", "E_grad", "E_well", "E_nonlocal", "E_mass"])
        return dict(zip(names, list(out)[:n]))

    def diagnostics(self, i=0):
        d = Diag()
        st = lib().etd_diagnostics(self._ptr, i, C.byref(d))
        out = {k: getattr(d, k) for k, _ in Diag._fields_}
        if st not in (ETD_OK, ETD_E_NONFINITE):
            self._c(st)
        return out

    def diag_ring(self, i, capacity):
        """Record the diagnostics of the last `capacity` steps on the device (0: off)."""
        self._c(lib().etd_diag_ring_enable(self._ptr, i, int(capacity)))
        if not hasattr(self, "_ring_cap"):
            self._ring_cap = {}
        self._ring_cap[i] = int(capacity)

    def read_diag_ring(self, i, max_entries=1 << 20):
        """(entries oldest first as dicts, steps recorded since the record started)."""
        n = int(max_entries)
        buf = (Diag * max(n, 1))()
        rec = C.c_int64(0)
        self._c(lib().etd_diag_ring_read(self._ptr, i, buf, n, C.byref(rec)))
        k = min(rec.value, n, getattr(self, "_ring_cap", {}).get(i, 0))
        return [{f: getattr(buf[j], f) for f, _ in Diag._fields_} for j in range(k)], rec.value

    def narrowband(self, i, phi, threshold, capacity=None):
        import torch
        cap = phi.numel() if capacity is None else int(capacity)
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        cnt = C.c_int64(0)
        st = lib().etd_narrowband_build(self._ptr, i, self._dev(phi), self._dt(phi), float(threshold),
                                        C.c_void_p(idx.data_ptr()), cap, C.byref(cnt))
        if st == ETD_E_CAPACITY:
            raise EtdError(st, f"band has {cnt.value} points")
        self._c(st)
        return idx[: cnt.value]

    def narrowband_noalloc(self, phi, threshold, capacity=None):
        """The band list of narrowband() for the values of phi (any shape), built
        with no device allocation (etd_narrowband_build_noalloc)."""
        import torch
        cap = phi.numel() if capacity is None else int(capacity)
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        cnt = C.c_int64(0)
        st = lib().etd_narrowband_build_noalloc(self._ptr, self._dev(phi), self._dt(phi), phi.numel(),
                                                float(threshold), C.c_void_p(idx.data_ptr()), cap, C.byref(cnt))
        if st == ETD_E_CAPACITY:
            raise EtdError(st, f"band has {cnt.value} points")
        self._c(st)
        return idx[: cnt.value]

    def spectral_apply(self, i, op, x, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        self._c(lib().etd_spectral_apply(self._ptr, i, int(op), self._dev(x), self._dev(out), self._dt(x)))
        return out

    def pass_timing(self, enable):
        """Start (True) or stop (False) FFT pass timing; stop returns per-kind totals."""
        t = PassTimes()
        self._c(lib().etd_pass_timing(self._ptr, 1 if enable else 0, C.byref(t)))
        if enable:
            return None
        return {k: dict(launches=t.launches[n], ms=t.total_ms[n], bytes=t.bytes[n])
                for n, k in enumerate(PASS_KINDS)}

    def query(self, i, what):
        v = C.c_double(0.0)
        self._c(lib().etd_plan_query(self._ptr, i, int(what), C.byref(v)))
        return v.value

    def set_schedule(self, mode, branches=1, xlines=0):
        """Step schedule: EXEC_EAGER; EXEC_GRAPH with `branches` concurrent capture branches;
        EXEC_GROUPED (one launch per pass per group of like instances, groups on `branches`
        branches); xlines: the FP32 ETD x-pass tile (0 or 16: default, 8)."""
        self._c(lib().etd_set_schedule(self._ptr, C.byref(Schedule(int(mode), int(branches), int(xlines)))))

    def get_schedule(self):
        """(mode, branches); the tile is get_xlines()."""
        s = Schedule()
        self._c(lib().etd_get_schedule(self._ptr, C.byref(s)))
        return s.mode, s.branches

    def get_xlines(self):
        s = Schedule()
        self._c(lib().etd_get_schedule(self._ptr, C.byref(s)))
        return s.xlines

    def autotune(self, trial_steps=10, cache_path=None):
        """Time the candidate schedules, keep the fastest; returns (mode, branches, {candidate: ms/step}).
        cache_path None: the ETD_AUTOTUNE_CACHE file of the environment, if set."""
        s = Schedule()
        ms = (C.c_double * len(AUTOTUNE_CANDIDATES))()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._c(lib().etd_autotune(self._ptr, int(trial_steps), path, C.byref(s), ms))
        times = {f"{m}{b if m in ('graph', 'grouped') else ''}": ms[k] for k, (m, b) in enumerate(AUTOTUNE_CANDIDATES)
                 if ms[k] >= 0}
        return s.mode, s.branches, times

    def close(self):
        if getattr(self, "_ptr", None) and self._ptr.value:
            lib().etd_plan_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def coupled_instance(ci, scheme=ETDRK2, precision=FP64, **kw) -> Instance:
    """Instance from inputs.CoupledInputs."""
    return Instance(COUPLED, tuple(ci.shape), tuple(ci.half_len), ci.tau, scheme, precision,
                    coupled=ci.params, **kw)


def fixed_instance(fi, B=0.0, scheme=ETD1, precision=FP64, nonlocal_with_ubar=0, **kw) -> Instance:
    """Instance from inputs.FixedInputs (B <= 0: B = B_MBP)."""
    return Instance(FIXED_MEMBRANE, tuple(fi.shape), tuple(fi.half_len), fi.tau, scheme, precision,
                    fixed=dict(eps_u=fi.eps_u, gamma=fi.gamma, ubar=fi.ubar, M=fi.M, B=B,
                               nonlocal_with_ubar=nonlocal_with_ubar), **kw)
