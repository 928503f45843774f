"""tc_stats_noalloc (the statistics with their reduction scratch in the
library's static device array, for callers that cannot allocate) against
tc_stats, through the C ABI: two calls in a row, the second on a smaller grid,
so that anything the first call left in the shared array would show, then the
larger grid again.  Collected last, so a failure here hides no other test."""

import numpy as np
import pytest

from tests.helpers import pair, workload

pytestmark = pytest.mark.gpu

KEYS = ("time", "torque_in", "torque_out", "tau_in", "tau_out", "retau_in", "retau_out", "energy",
        "energy_pert", "steps", "nonfinite")


def _noalloc(solver, inst=0):
    return solver.stats_noalloc(inst)


def _check(got, want, label):
    for k in KEYS:
        a, b = got[k], want[k]
        if isinstance(b, float) and b != 0:
            assert abs(a / b - 1) <= 1e-12, (label, k, a, b)
        else:
            assert a == b, (label, k, a, b)


def test_stats_noalloc_matches_tc_stats_twice_second_smaller():
    big_w = workload("tc-medium-fp64")
    small_w = workload("tc-small-fp64", nr=9, ntheta=8, nz=8)
    _, big = pair(big_w)
    _, small = pair(small_w)
    big.step(2)
    small.step(3)
    for label, g in (("medium", big), ("tiny", small)):
        want = g.stats()
        got = _noalloc(g)
        print(label, {k: got[k] for k in ("torque_in", "energy", "energy_pert")}, flush=True)
        _check(got, want, label)
        # the reduction order is the same, so the values agree bit for bit
        assert got["energy"] == want["energy"] and got["torque_in"] == want["torque_in"], label
    # and once more on the larger grid after the smaller one
    _check(_noalloc(big), big.stats(), "medium again")
