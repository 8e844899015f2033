"""The pipelined iteration on the GPU: the synthesis runs group by group of
ring pairs and each group's ring stage overlaps the synthesis of the next
groups.  Every value is computed by the same launches' arithmetic as without
the pipeline, so solves, single iterations and batches must come out bit for
bit the same with the pipeline on (several group counts) and off.
"""
import numpy as np
import pytest

import dmwf_inputs as inp
from gpu_util import device

pytestmark = pytest.mark.gpu

# The pipelined path is switched off and its internals are removed from the
# library: its first solve (nside 128, one map, two groups) ended the test
# process with a host segmentation fault inside dmwf_solve, and no cause was
# found in the host code.  Its ring stage forked side streams from a stream
# that had joined the graph capture through an event; a later variant of the
# multi-plan solve with that same shape faulted the same way.  The tests that
# ran it stay here, skipped.
OFF = ("pipelined iteration switched off (removed): host segmentation fault in its first solve, "
       "cause not found")


def _problem(nside, nmaps, first=0):
    # spectrum, mask and noise of members of the batched workload; any data
    # serve a comparison of two launch orders, so d is white noise at the
    # members' noise level
    import torch
    ps = [inp.make_problem("cfg4", nside=nside, index=first + k) for k in range(nmaps)]
    ds = [inp.random_map(nside, 900 + first + k) * np.sqrt(1.0 / p.ninv.max())
          for k, p in enumerate(ps)]
    dev = device()
    stack = lambda xs: torch.tensor(np.stack(xs) if nmaps > 1 else xs[0], device=dev)
    return ps[0].lmax, (stack([p.cl for p in ps]), stack(ds), stack([p.ninv for p in ps]))


def _plan(nside, lmax, nmaps):
    from paper_1702_08852_amd import Plan
    return Plan(nside, lmax, nmaps=nmaps, device=device())


def _same(x, y):
    np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.skip(reason=OFF)
@pytest.mark.parametrize("nside,nmaps,groups", [(128, 1, 2), (256, 1, 4), (128, 3, 2)])
def test_pipelined_solve_is_bit_identical(nside, nmaps, groups):
    lmax, args = _problem(nside, nmaps)
    plan = _plan(nside, lmax, nmaps)
    plan.set_pipeline(groups)
    assert plan.pipeline_groups == groups
    a_p, s_p, st_p = plan.solve(*args, eps_final=1e-7)
    plan.profile(2)  # the analysis between events, the rest from the graph
    a_t, s_t, _ = plan.solve(*args, eps_final=1e-7)
    plan.profile_read()
    plan.profile(False)
    plan.set_pipeline(0)
    assert plan.pipeline_groups == 0
    a_o, s_o, st_o = plan.solve(*args, eps_final=1e-7)
    for x, y in ((a_p, a_o), (s_p, s_o), (a_t, a_o), (s_t, s_o)):
        _same(x, y)
    st_p = st_p if isinstance(st_p, list) else [st_p]
    st_o = st_o if isinstance(st_o, list) else [st_o]
    assert [s.iters_per_level for s in st_p] == [s.iters_per_level for s in st_o]
    assert all(s.n_iter > 10 for s in st_p)


@pytest.mark.skip(reason=OFF)
def test_group_counts_and_single_iterations():
    """dm_iterate gives the same bits at every group count; counts that ask
    for groups below 128 ring pairs get fewer, larger groups."""
    import torch
    nside = 256
    lmax, (cl, d, w) = _problem(nside, 1, first=5)
    plan = _plan(nside, lmax, 1)
    alpha = float(1.0 / w.max())
    outs = {}
    for groups, expect in ((0, 0), (1, 0), (2, 2), (3, 2), (4, 4), (8, 4)):
        plan.set_pipeline(groups)
        assert plan.pipeline_groups == expect
        a = torch.zeros((lmax + 1) * (lmax + 2) // 2, 2, dtype=torch.float64, device=device())
        s = torch.zeros_like(d)
        c2 = torch.zeros(2, dtype=torch.float64, device=device())
        for it in range(4):
            plan.dm_iterate(alpha * 30.0 if it < 2 else alpha, alpha, cl, d, w, a, s, c2,
                            first=(it == 0))
        outs[groups] = (a.cpu().numpy(), s.cpu().numpy(), c2.cpu().numpy())
    ref = outs[0]
    for g, out in outs.items():
        for x, y in zip(out, ref):
            np.testing.assert_array_equal(x, y)


def test_set_pipeline_is_off_and_rejects_bad_counts():
    """No plan pipelines; asking for groups is an error, naming the reason,
    and leaves the plan unpipelined."""
    from paper_1702_08852_amd import DmwfError
    from paper_1702_08852_amd.dmwf import ERR_UNSUPPORTED
    plan = _plan(128, 256, 1)
    assert plan.pipeline_groups == 0
    for bad in (-1, 9):
        with pytest.raises(DmwfError):
            plan.set_pipeline(bad)
    with pytest.raises(DmwfError) as e:
        plan.set_pipeline(4)
    assert e.value.status == ERR_UNSUPPORTED and "switched off" in str(e.value)
    plan.set_pipeline(0)
    plan.set_pipeline(1)
    assert plan.pipeline_groups == 0
