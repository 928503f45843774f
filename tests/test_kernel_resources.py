"""The compiler's resource report of the kernels the benchmark and batched
workloads launch by default: no scratch memory, no vector-register spills, and the
waves per SIMD their launch shapes were tuned for.  (A conditional between
two complex values as whole objects once compiled into a choice of address
between two stack copies: 40 bytes of scratch per lane in the FP64 theta
kernel, 8 % more HBM writes than its model, with no spill reported.)  The
report is written by the package's build (paper_0711_1429_amd/build.py)."""
import os
import re

import pytest

from paper_0711_1429_amd.build import RESOURCES


def _report():
    if not os.path.exists(RESOURCES):
        pytest.skip("no resource report: build the library with paper_0711_1429_amd.build")
    rows, cur = {}, None
    for line in open(RESOURCES):
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            rows[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs Spill|SGPRs Spill|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur:
            rows[cur][m.group(1).split(" [")[0]] = int(m.group(2))
    return rows


# mangled-name fragments of the default kernels, with the waves per SIMD each
# needs (None: not checked)
DEFAULT_KERNELS = {
    # 129 x 768 x 384, FP64 and mixed
    "k_theta_waveIdLi768ELi1ELi2E": 2,
    "k_theta_waveIfLi768ELi4ELi3E": 4,
    "k_zinv_laneIdLi384ELi8E": 2,
    "k_zinv_laneIfLi384ELi16E": 4,
    "k_zfwd_laneIdLi384ELi8E": 2,
    "k_zfwd_laneIfLi384ELi16E": 4,
    "k_rhsIdLi0ELb1E": None,
    "k_rhsIdLi1ELb1E": None,
    "k_rhsIdLi2ELb1E": None,
    "k_rhsIfLi0ELb0E": None,
    "k_rhsIfLi1ELb0E": None,
    "k_rhsIfLi2ELb0E": None,
    "k_solve_segILi8ELi16ELb0ELb1E": 4,
    "k_solve_segILi8ELi16ELb0ELb0E": 4,
    "k_dv_segILi16ELi8E": 4,
    # the batched workload's lengths and segment shapes (untuned defaults)
    "k_theta_waveIfLi64ELi2ELi0E": None,
    "k_theta_waveIfLi96ELi2ELi0E": None,
    "k_theta_waveIfLi128ELi2ELi0E": None,
    "k_zinv_laneIfLi64ELi32E": None,
    "k_zinv_laneIfLi128ELi16E": None,
    "k_zfwd_laneIfLi64ELi32E": None,
    "k_zfwd_laneIfLi128ELi16E": None,
    "k_solve_segILi8ELi8ELb0ELb0E": None,
    "k_solve_segILi4ELi8ELb0ELb0E": None,
    "k_dv_segILi8ELi8E": None,
    "k_dv_segILi4ELi8E": None,
}


def test_default_kernels_use_no_scratch_and_keep_their_occupancy():
    rows = _report()
    assert rows, "empty resource report"
    for frag, waves in DEFAULT_KERNELS.items():
        hits = [n for n in rows if frag in n]
        assert hits, f"{frag}: not in the resource report"
        for n in hits:
            r = rows[n]
            assert r.get("ScratchSize", 0) == 0, f"{n}: {r.get('ScratchSize')} bytes of scratch per lane"
            # (scalar spills go to vector-register lanes, not memory)
            assert r.get("VGPRs Spill", 0) == 0, f"{n}: vector register spills {r}"
            if waves is not None:
                assert r.get("Occupancy", 0) >= waves, f"{n}: {r.get('Occupancy')} waves per SIMD, expected {waves}"
