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
