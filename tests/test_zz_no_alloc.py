"""dmwf_alm2map_static, the synthesis that allocates nothing (its scratch is
the library's fixed device array), against dmwf_alm2map with a workspace:
the same kernels, so the maps must agree bit for bit; two calls in a row, the
second on a smaller plan, and a plan too large for the fixed scratch is
refused with a clear error."""
import ctypes

import numpy as np
import pytest

import dmwf_inputs as inp
from gpu_util import device

pytestmark = pytest.mark.gpu


def _call_static(plan, alm, out):
    import torch
    from paper_1702_08852_amd import dmwf as b
    lib = b.load()
    return lib.dmwf_alm2map_static(plan._h, ctypes.c_void_p(alm.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_static_synthesis_equals_workspace_synthesis_twice():
    import torch
    from paper_1702_08852_amd import Plan
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    for nside, lmax, nm, seed in ((64, 128, 3, 11), (16, 32, 1, 12)):
        plan = Plan(nside, lmax, nmaps=nm, device=dev)
        a = np.stack([inp.random_alm(lmax, seed + k) for k in range(nm)])
        a_t = torch.tensor(a if nm > 1 else a[0], device=dev)
        ref = plan.alm2map(a_t).cpu().numpy()
        out = torch.full(ref.shape, np.nan, dtype=torch.float64, device=dev)
        assert _call_static(plan, a_t, out) == b.OK
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        assert np.isfinite(got).all()


def test_static_synthesis_refuses_plans_beyond_its_scratch():
    import torch
    from paper_1702_08852_amd import Plan
    from paper_1702_08852_amd import dmwf as b
    dev = device()
    plan = Plan(512, 1024, nmaps=2, device=dev)  # about 80 MiB of scratch
    a = torch.zeros((2, (1025 * 1026) // 2, 2), dtype=torch.float64, device=dev)
    out = torch.zeros((2, 12 * 512 * 512), dtype=torch.float64, device=dev)
    assert _call_static(plan, a, out) == b.ERR_WORKSPACE
    assert b"static scratch" in b.load().dmwf_last_error()
