"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="needs an MI355X")


def dev(a, dtype=None):
    dtype = dtype or torch.float64
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def rel_linf(x, ref):
    """max |x - ref| / max |ref| (the relative L-infinity error)."""
    return float(np.abs(np.asarray(x) - np.asarray(ref)).max() / max(np.abs(ref).max(), 1e-300))


def report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


# ----------------------------------------------------------------------------
# FP32 against an FP64 reference through the recovery U = GU / G on G > 1e-3
# (Section 3.3, after Algorithm 1).  The rule is discontinuous in G: where the
# FP32 path's G and the reference G fall on opposite sides of the threshold
# the two take different branches and U differs by O(U) there; the scheme's
# stencils (Delta_S u, the divergence of g u v) then carry that difference to
# the neighbours in later steps.  The relative L-infinity gap of u is taken
# outside those points and their RADIUS-cell neighbourhood; the points are
# counted; the g-weighted gap (of g u, the quantity the scheme carries) and
# the all-points gap are reported beside it.
FLIP_RADIUS = 2


def recovery_flips(phi32, phi_ref, thr=1e-3, ambiguity=1e-5):
    """Points where G from the FP32 phi (in FP32, as the kernels form it) and
    G from the reference phi (FP64) fall on opposite sides of thr; points
    whose FP32 G lies within the relative `ambiguity` of thr are counted
    too (the kernels' rounding of G may differ from numpy's by an ulp)."""
    p = np.asarray(phi32, dtype=np.float32)
    a = p * p - p
    g32 = (np.float32(18.0) * a * a).astype(np.float64)
    pr = np.asarray(phi_ref, dtype=np.float64)
    gref = 18.0 * (pr * pr - pr) ** 2
    return ((g32 > thr) != (gref > thr)) | (np.abs(g32 / thr - 1.0) < ambiguity)


def u_gap_outside_flips(u32, u_ref, phi_ref, flips, radius=FLIP_RADIUS):
    """(gap outside the flip neighbourhood, neighbourhood size, g-weighted gap, all-points gap)."""
    from scipy.ndimage import maximum_filter
    near = maximum_filter(flips, size=2 * radius + 1, mode="wrap") if flips.any() else flips
    d = np.abs(np.asarray(u32) - np.asarray(u_ref))
    scale = np.abs(u_ref).max()
    out = float(d[~near].max() / scale)
    pr = np.asarray(phi_ref)
    g = 18.0 * (pr * pr - pr) ** 2
    gw = float((g * d).max() / np.abs(g * u_ref).max())
    return out, int(near.sum()), gw, float(d.max() / scale)


def recovery_flips_dev(phi32, phi_ref, thr=1e-3, ambiguity=1e-5):
    """recovery_flips on device tensors (phi32 float32, phi_ref float64)."""
    a = phi32 * phi32 - phi32
    g32 = (18.0 * a * a).double()
    gref = 18.0 * (phi_ref * phi_ref - phi_ref) ** 2
    return ((g32 > thr) != (gref > thr)) | ((g32 / thr - 1.0).abs() < ambiguity)


def u_gap_outside_flips_dev(u32, u_ref, phi_ref, flips, radius=FLIP_RADIUS):
    """u_gap_outside_flips on device tensors (3D grids)."""
    import torch.nn.functional as F
    x = flips.to(torch.float32)[None, None]
    x = F.pad(x, (radius,) * 6, mode="circular")
    near = F.max_pool3d(x, 2 * radius + 1, stride=1)[0, 0] > 0
    d = (u32.double() - u_ref).abs()
    scale = u_ref.abs().max()
    g = 18.0 * (phi_ref * phi_ref - phi_ref) ** 2
    return (float(d[~near].max() / scale), int(near.sum()), float((g * d).max() / (g * u_ref).abs().max()),
            float(d.max() / scale))
