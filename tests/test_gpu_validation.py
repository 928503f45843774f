"""Validation runs of the paper's Sec. 3 on the GPU path (long runs that the
oracle cannot afford; the GPU path equals the oracle step by step to 1e-12 in
test_gpu_parity.py, so these runs pin the discrete method itself).

* Onset of Taylor vortices (Sec. 3): the paper brackets the critical Re
  at radius ratio 0.5 as 68.2 < Re_c < 68.4 by watching the perturbation
  energy of a small random disturbance.  At Re = 68.0 it must decay and at
  Re = 68.4 grow, at the rate of the least stable eigenvalue of the discrete
  linear operator about Couette flow (built from the oracle's operators).
* Saturated straight Taylor vortices (Table 2): the torque at Re = 70, 75
  and 80 in the straight-vortex box of Table 1.  This is the only check of
  the nonlinear terms far from the linear regime against numbers the paper
  prints.

Box and resolution follow Table 1: L_z = 4h = 2d, L_theta = pi h at mid-gap
(Theta = pi / 3 at radius ratio 0.5), N_r = 64 uniform, 64 axial and 32
azimuthal Fourier modes (N_z = 96, N_theta = 48 physical points under the
3/2 rule).  The steady state of the scheme does not depend on dt.
"""

import os

import numpy as np
import pytest

from paper_0711_1429_amd import tc as tcb
from tests.helpers import abi_geometry, fields_for

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BOX = dict(zeta=0.5, nr=64, ntheta=48, nz=96, dt=0.02, lz=2.0, theta_period=np.pi / 3, stretch=0.0,
           amplitude=1e-2, seed=7)


def _solver(re, precision=tcb.TC_PREC_FP64):
    w = dict(BOX, re=re)
    g = tcb.Solver(abi_geometry(w, precision))
    g.load_fields(*fields_for(w, g.grid()))
    return g


@pytest.mark.gpu
@pytest.mark.parametrize("re", [68.0, 68.4])
def test_onset_growth_rate_brackets_the_critical_reynolds_number(re):
    from tests.test_oracle_dynamics import _oracle_growth
    lam = _oracle_growth(0.5, re, nr=BOX["nr"])[0].real
    g = _solver(re)
    g.step(5000)  # t = 100: the other modes have decayed
    e1 = g.stats()["energy_pert"]
    g.step(2500)  # t = 150
    e2 = g.stats()["energy_pert"]
    sigma = np.log(e2 / e1) / (2 * 50.0)
    print(f"Re {re}: DNS growth rate {sigma:.6e}, eigenvalue {lam:.6e}", flush=True)
    assert (sigma > 0) == (re > 68.2) and (lam > 0) == (re > 68.2)
    assert abs(sigma / lam - 1) < 2e-3


@pytest.mark.gpu
@pytest.mark.parametrize("re,precision", [(70.0, tcb.TC_PREC_FP64), (75.0, tcb.TC_PREC_FP64),
                                          (80.0, tcb.TC_PREC_FP64), (80.0, tcb.TC_PREC_MIXED)])
def test_taylor_vortex_torque_matches_table2(re, precision):
    table = {r: t for r, t in np.loadtxt(os.path.join(GOLDEN, "table2_taylor_vortex_torque.txt"))}
    g = _solver(re, precision)
    prev = None
    for _ in range(40):  # at most 2000 time units
        g.step(2500)
        s = g.stats()
        if prev is not None and abs(s["torque_in"] / prev - 1) < 1e-8:
            break
        prev = s["torque_in"]
    print(f"Re {re}: torque {s['torque_in']:.6f} (outer {s['torque_out']:.6f}) at t = {s['time']:.0f}, "
          f"Table 2 {table[re]}", flush=True)
    assert prev is not None and abs(s["torque_in"] / prev - 1) < 1e-8, "not steady"
    assert s["torque_in"] > 16.7552  # vortices, not the laminar torque
    assert abs(s["torque_in"] / table[re] - 1) < 2e-4
    assert abs(s["torque_out"] / s["torque_in"] - 1) < 2e-5  # radial resolution: 7e-6 measured
