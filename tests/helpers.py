"""Shared test helpers: workloads for both sides and parity metrics."""

import numpy as np

from oracle import Geometry, Oracle
from paper_0711_1429_amd import tc as tcb
from paper_0711_1429_amd.synth import WORKLOADS, initial_fields

GEO_KEYS = ("zeta", "re", "nr", "ntheta", "nz", "dt", "stretch")


def workload(name, **override):
    w = dict(WORKLOADS[name])
    w.update(override)
    return w


def oracle_geometry(w):
    return Geometry(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"], dt=w["dt"],
                    stretch=w.get("stretch", 0.0), re_outer=w.get("re_outer", 0.0),
                    lz=w.get("lz", 0.0), theta_period=w.get("theta_period", 0.0))


def abi_geometry(w, precision=tcb.TC_PREC_FP64, flags=0):
    return tcb.make_geometry(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"],
                             dt=w["dt"], stretch=w.get("stretch", 0.0), re_outer=w.get("re_outer", 0.0),
                             lz=w.get("lz", 0.0), theta_period=w.get("theta_period", 0.0),
                             precision=precision, flags=flags)


def fields_for(w, r):
    return initial_fields(r, w["zeta"], w["ntheta"], w["nz"], w["amplitude"], w["seed"],
                          w_outer=w.get("re_outer", 0.0) / w["re"])


def pair(w, precision=tcb.TC_PREC_FP64, flags=0):
    """(oracle, gpu solver) loaded with the same seeded fields."""
    orc = Oracle(oracle_geometry(w))
    gpu = tcb.Solver(abi_geometry(w, precision, flags))
    flds = fields_for(w, orc.disc.r)
    orc.load(*flds)
    gpu.load_fields(*flds)
    return orc, gpu


def cweights(nj):
    return np.where(np.arange(nj) == 0, 1.0, 2.0)[None, :, None]


def rel_l2(a, b):
    """Relative L2 difference over all stored (r, j, l) with the Hermitian
    weights c_0 = 1, c_{j>0} = 2 (b is the reference)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 1:
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    c = cweights(b.shape[1])
    num = np.sum(c * np.abs(a - b) ** 2)
    den = np.sum(c * np.abs(b) ** 2)
    return float(np.sqrt(num / den))
