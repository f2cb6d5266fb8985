"""The entry point that allocates nothing (spx_run_noalloc) against spx_run_ex, through the
C-ABI: two calls in a row, the second on a smaller plan, each bit-identical to the plan's
ordinary run (tallies, counters, records, profiles, arrival tallies)."""
import numpy as np
import pytest

import sputter_inputs as si
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2411_14413_amd as spx  # noqa: E402

PARAMS = si.Params()


def _compare(plan, seed, arrivals):
    ref = plan.allocate(profiles=True, records=True, arrivals=arrivals)
    plan.run_into(seed, ref)
    got = plan.allocate(profiles=True, records=True, arrivals=arrivals)
    for v in got.values():
        if v is not None:
            v.fill_(255 if v.dtype == torch.uint8 else -1)     # stale values must be overwritten
    torch.cuda.synchronize()
    plan.run_noalloc_into(seed, got)
    torch.cuda.synchronize()
    for k, v in ref.items():
        if v is not None:
            assert torch.equal(v, got[k]), k
    C = got["counters"].view(plan.n_segments, -1).cpu().numpy()
    assert np.array_equal(C[:, 0], C[:, 1] + C[:, 2] + C[:, 3])
    assert int(C[:, 0].sum()) == plan.n_particles


def test_noalloc_matches_run_twice_second_smaller():
    # first call: 3.4e6 particles, more than one round of the 64 MiB scratch (~1.07e6 tickets
    # per round at the default launch shape), with the arrival tallies
    big = [si.single_ni(0.5, 2_000_000), si.single_ni(2.0, 200_000),
           si.quaternary(0.5, 25.0, 150.0, [600_000, 100_000, 300_000, 200_000])]
    say("no-alloc run: 3.4e6 particles in several scratch rounds, with arrival tallies")
    _compare(spx.Plan(big, PARAMS), seed=13, arrivals=True)
    # second call: a smaller plan, without arrival tallies; the scratch keeps the first call's
    # queue and counters, which the run must not depend on
    small = [si.single_ni(2.0, 3000), si.quaternary(0.9, 30.0, 120.0, [2000, 500, 1500, 800])]
    say("no-alloc run: a smaller plan after it")
    _compare(spx.Plan(small, PARAMS), seed=14, arrivals=False)


def test_noalloc_rejects_fp64_plans():
    plan = spx.Plan([si.single_ni(0.5, 100)], PARAMS, precision=64)
    bufs = plan.allocate()
    with pytest.raises(spx.SpxError, match="precision 32"):
        plan.run_noalloc_into(1, bufs)
