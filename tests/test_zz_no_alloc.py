"""GPU: the allocation-free band build (etd_narrowband_build_noalloc) through
the C ABI against etd_narrowband_build on the same inputs: bit-exact lists
and counts on two calls in a row, the second with a smaller input, in FP32
and FP64; its argument and size errors."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import dev, needs_gpu, report, torch
from oracle import band as oband
from paper_2606_04347_amd import etd, inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


def noalloc(plan, phi, n, thr, capacity):
    L = etd.lib()
    idx = torch.full((max(capacity, 1),), -7, dtype=torch.int32, device="cuda")
    cnt = C.c_int64(-1)
    dt = etd.F64 if phi.dtype == torch.float64 else etd.F32
    st = L.etd_narrowband_build_noalloc(plan._ptr, C.c_void_p(phi.data_ptr()), dt, n, thr,
                                        C.c_void_p(idx.data_ptr()), capacity, C.byref(cnt))
    return st, cnt.value, idx


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_band_matches_narrowband_build(dtype):
    big = inputs.coupled_membrane(n=96, seed=41)
    small = inputs.coupled_membrane(n=(24, 16, 32), seed=42)
    plan = etd.Plan([etd.coupled_instance(big), etd.coupled_instance(small)])
    for k, ci in enumerate((big, small)):   # the second call is the smaller input
        phi = dev(ci.phi0, dtype)
        n = phi.numel()
        ref = plan.narrowband(k, phi, 0.995).cpu().numpy()
        st, cnt, idx = noalloc(plan, phi, n, 0.995, n)
        got = idx[:cnt].cpu().numpy()
        report("noalloc_band", n=n, count=cnt, ref=len(ref))
        assert st == etd.ETD_OK and cnt == len(ref) and np.array_equal(got, ref)
        assert np.array_equal(got, oband.band_list(phi.cpu().double().numpy(), 0.995))
        assert (idx[cnt:] == -7).all()   # nothing written past the list
    plan.close()


def test_noalloc_band_errors():
    ci = inputs.coupled_membrane(n=16, seed=43)
    plan = etd.Plan(etd.coupled_instance(ci))
    phi = dev(ci.phi0)
    n = phi.numel()
    full = len(oband.band_list(ci.phi0, 0.995))
    st, cnt, idx = noalloc(plan, phi, n, 0.995, full - 1)
    assert st == etd.ETD_E_CAPACITY and cnt == full and (idx == -7).all()
    st, cnt, _ = noalloc(plan, phi, 0, 0.995, 4)
    assert st == etd.ETD_OK and cnt == 0
    assert noalloc(plan, phi, -1, 0.995, 4)[0] == etd.ETD_E_ARG
    assert noalloc(plan, phi, n, 0.0, 4)[0] == etd.ETD_E_ARG
    assert noalloc(plan, phi, 268435456 + 1, 0.995, 4)[0] == etd.ETD_E_SIZE
    plan.close()
