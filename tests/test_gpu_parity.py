"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar (FP64 path): relative L2 <= 1e-12 per field per step, with the Hermitian
weights of the stored half spectrum; statistics to the same relative bar.
Fields compared: v, eta, u (mean included), w (mean included), w' (mean
excluded) and the mean profiles.
"""

import numpy as np
import pytest

from paper_0711_1429_amd import tc as tcb
from tests.helpers import pair, rel_l2, workload

pytestmark = pytest.mark.gpu

TOL = 1e-12
# both transform paths: the fixed-length lane kernels (default for the
# compiled lengths) and the run-time-length kernels
PATHS = pytest.mark.parametrize("flags", [0, tcb.TC_FLAG_GENERIC_FFT], ids=["lane-fft", "generic-fft"])


def _compare_state(orc, gpu, tol=TOL, label=""):
    v, e, um, wm = gpu.get_fields()
    rv, re_, rum, rwm = orc.fields()
    errs = {"v": rel_l2(v, rv), "eta": rel_l2(e, re_)}
    errs["w_mean"] = rel_l2(wm, rwm)
    gu, gw = gpu.velocity()
    dv, u, w, c = orc.velocity()
    shape = v.shape
    u = u.reshape(shape)
    w = w.reshape(shape)
    errs["u"] = rel_l2(gu, u)
    errs["w"] = rel_l2(gw, w)
    kz = (shape[2] - 1) // 2
    wp, gwp = w.copy(), gw.copy()
    wp[:, 0, kz] = 0
    gwp[:, 0, kz] = 0
    errs["w_pert"] = rel_l2(gwp, wp)
    # the mean axial flow is the (0,0) mode of u, measured also against the
    # whole u field as the metric defines
    errs["u_mean_in_u"] = float(np.linalg.norm(um - rum) / np.sqrt(np.sum(np.abs(u) ** 2)))
    info = {}
    bad = {}
    if np.linalg.norm(rum) > 0:
        # the mean axial flow against itself.  It is the response to the plane
        # average of uv, a sum of products of random-phase modes that cancel to
        # a small fraction of their magnitudes, so its relative rounding is
        # about ten times that of the fields (measured up to 2e-12): held to
        # ten times the FP64 bar.  In mixed precision it carries the FP32
        # rounding of those products and is only reported (it is part of u,
        # which is held to the bar).
        info["u_mean_self"] = rel_l2(um, rum)
        if tol <= TOL and not info["u_mean_self"] <= 10 * tol:
            bad["u_mean_self"] = info["u_mean_self"]
    bad.update({k: x for k, x in errs.items() if not x <= tol})
    print(label, {k: f"{x:.2e}" for k, x in errs.items()}, {k: f"{x:.2e}" for k, x in info.items()}, flush=True)
    assert not bad, (label, bad)
    return errs


@PATHS
def test_velocity_and_products_small(flags):
    orc, gpu = pair(workload("tc-small-fp64"), flags=flags)
    _compare_state(orc, gpu, label="loaded")
    dv, u, w, c = orc.velocity()
    P = orc.products(u, orc.v, w)
    G = gpu.products()
    for k in P:
        ref = P[k].reshape(G[k].shape)
        err = rel_l2(G[k], ref)
        print(k, f"{err:.2e}", flush=True)
        assert err < 1e-13, (k, err)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_single_substep_small(k):
    orc, gpu = pair(workload("tc-small-fp64"))
    # advance both by the earlier substeps so that substep k sees non-zero
    # explicit-term registers
    for kk in range(1, k):
        orc.substep(kk - 1)
        gpu.substep(kk)
    orc.substep(k - 1)
    gpu.substep(k)
    _compare_state(orc, gpu, label=f"substep {k}")


@PATHS
def test_ten_steps_small_every_step(flags):
    w = workload("tc-small-fp64")
    orc, gpu = pair(w, flags=flags)
    for s in range(w["steps"]):
        orc.step(1)
        gpu.step(1)
        _compare_state(orc, gpu, label=f"step {s + 1}")
    so, sg = orc.stats(), gpu.stats()
    for key in ("torque_in", "torque_out", "retau_in", "retau_out", "energy", "energy_pert"):
        assert abs(sg[key] / so[key] - 1) < TOL, (key, sg[key], so[key])
    assert sg["steps"] == w["steps"] and sg["nonfinite"] == 0
    assert abs(sg["time"] - so["time"]) < 1e-15


@PATHS
def test_medium_grid_three_steps(flags):
    w = workload("tc-medium-fp64")
    orc, gpu = pair(w, flags=flags)
    for s in range(3):
        orc.step(1)
        gpu.step(1)
    _compare_state(orc, gpu, label="medium step 3")


@pytest.mark.parametrize("name,steps,prec", [("tc-small-fp64", 5, tcb.TC_PREC_FP64),
                                              ("tc-medium-fp64", 2, tcb.TC_PREC_FP64),
                                              ("tc-medium-fp64", 2, tcb.TC_PREC_MIXED)])
def test_radial_profiles(name, steps, prec):
    """Mean profiles and fluctuation (co)variances per radial node (Sec. 5
    statistics) against the oracle's Parseval sums: on the seeded initial
    state, then after both sides stepped on their own (to FP64 rounding; the
    mixed path to its FP32 transform error)."""
    w = workload(name)
    orc, gpu = pair(w, precision=prec)
    tol = TOL if prec == tcb.TC_PREC_FP64 else 1e-5
    for stage in ("initial", "stepped"):
        if stage == "stepped":
            orc.step(steps)
            gpu.step(steps)
        ref = orc.profiles()
        got = gpu.profiles()
        for k in ref:
            scale = np.abs(ref[k]).max()
            if scale == 0:  # e.g. no axial mean flow in the initial state
                assert np.all(got[k] == 0), k
                continue
            err = np.abs(got[k] - ref[k]).max() / scale
            print("profile", name, prec, stage, k, f"{err:.2e}", flush=True)
            assert err < (TOL if stage == "initial" else tol)
        assert np.all(got["vv"] >= 0) and got["vv"][0] == 0 and got["vv"][-1] == 0


@PATHS
@pytest.mark.parametrize("sizes", [dict(nr=7, ntheta=4, nz=4), dict(nr=9, ntheta=48, nz=36, stretch=1.0),
                                   dict(nr=20, ntheta=12, nz=96), dict(nr=11, ntheta=96, nz=6),
                                   dict(nr=13, ntheta=768, nz=8), dict(nr=10, ntheta=24, nz=768),
                                   dict(nr=12, ntheta=384, nz=64)])
def test_ragged_and_degenerate_sizes(sizes, flags):
    w = workload("tc-small-fp64", amplitude=1e-2, **sizes)
    orc, gpu = pair(w, flags=flags)
    for s in range(2):
        orc.step(1)
        gpu.step(1)
    _compare_state(orc, gpu, tol=TOL, label=str(sizes))


@PATHS
@pytest.mark.parametrize("nr", [131, 140])
def test_radial_sweeps_beyond_the_segmented_shapes(nr, flags):
    """N_r above the largest segmented shape of the solve (N_r - 2 > 128 rows)
    and of the D v sweep (N_r > 132) takes the one-lane-per-column kernels
    (k_solve_lu, k_dv): both against the oracle for three steps."""
    w = workload("tc-small-fp64", nr=nr, ntheta=12, nz=24, amplitude=1e-2, stretch=1.2)
    orc, gpu = pair(w, flags=flags)
    assert gpu.tuning()["solve_shape"] == 0
    for s in range(3):
        orc.step(1)
        gpu.step(1)
        _compare_state(orc, gpu, label=f"nr={nr} step {s + 1}")


@pytest.mark.parametrize("sizes", [dict(nr=9, ntheta=729, nz=192), dict(nr=9, ntheta=96, nz=384)])
def test_mixed_precision_paired_column_groups(sizes):
    """Mixed precision where the FP32 z kernels pair their column groups
    across XCDs (16 or more groups per plane): N_theta = 729 gives 243
    columns, so the last group of 16 is partial (3 columns); N_z = 384 with
    N_theta = 96 gives 4 groups (no pairing).  The products of the FP32
    transforms match the FP64 ones to single-precision rounding (a column
    handled by the wrong block would be off by O(1)), and two steps track the
    oracle to the FP32 transform error (eta, the smallest field, carries the
    largest relative error)."""
    from tests.helpers import abi_geometry, fields_for
    w = workload("tc-small-fp64", amplitude=1e-2, **sizes)
    ref = tcb.Solver(abi_geometry(w))
    mix = tcb.Solver(abi_geometry(w, tcb.TC_PREC_MIXED))
    f = fields_for(w, ref.grid())
    ref.load_fields(*f)
    mix.load_fields(*f)
    pr, pm = ref.products(), mix.products()
    for k in pr:
        err = rel_l2(pm[k], pr[k])
        print("mixed products", sizes, k, f"{err:.2e}", flush=True)
        assert 1e-10 < err < 2e-6
    del ref, mix
    orc, gpu = pair(w, precision=tcb.TC_PREC_MIXED)
    for s in range(2):
        orc.step(1)
        gpu.step(1)
    errs = _compare_state(orc, gpu, tol=1e-4, label="mixed " + str(sizes))
    assert max(errs.values()) > 1e-12  # the FP32 stages really ran


def test_rotating_outer_wall_and_custom_domain():
    w = workload("tc-small-fp64", zeta=0.5, re=120.0, re_outer=-30.0, lz=2.0, theta_period=np.pi,
                 amplitude=1e-2)
    orc, gpu = pair(w)
    orc.step(3)
    gpu.step(3)
    _compare_state(orc, gpu, label="outer rotation")
    so, sg = orc.stats(), gpu.stats()
    assert abs(sg["torque_out"] / so["torque_out"] - 1) < TOL


@PATHS
def test_turbulent_size_one_substep_sampled(flags):
    """Full turbulent-case grid (129 x 768 x 384, tanh clustering), in the
    launch configuration the benchmark times: one substep on the GPU, checked
    on a sample of modes the oracle solves one by one (its products still
    cover the whole grid)."""
    w = workload("tc-turbulent-fp64")
    orc, gpu = pair(w, flags=flags)
    gpu.substep(1)
    rng = np.random.default_rng(7)
    nmodes = orc.nmodes
    sample = rng.choice(np.flatnonzero(~orc.mc.is_mean), size=48, replace=False)
    # the lowest wavenumbers, whose mass operator carries the largest 1/k^2
    # (j <= 2, |l| <= 2, both signs of l), and the highest
    nl = orc.disc.nl
    kz = (nl - 1) // 2
    low = [j * nl + kz + l for j in range(3) for l in range(-2, 3) if (j, l) != (0, 0)]
    hi = [nmodes - 1, nmodes - 2, 2 * kz, 0]  # (K_theta, K_z), (K_theta, K_z - 1), (0, +-K_z)
    sample = np.unique(np.concatenate([sample, low, hi]))
    assert not np.any(orc.mc.is_mean[sample])
    assert np.min(np.hypot(orc.m_flat[sample], orc.alpha_flat[sample])) == np.min(
        np.hypot(orc.m_flat, orc.alpha_flat)[~orc.mc.is_mean])
    vs, es = orc.substep_sample(0, sample)
    v, e, um, wm = gpu.get_fields()
    v = v.reshape(v.shape[0], -1)[:, sample]
    e = e.reshape(e.shape[0], -1)[:, sample]
    ev = np.linalg.norm(v - vs) / np.linalg.norm(vs)
    ee = np.linalg.norm(e - es) / np.linalg.norm(es)
    print("turbulent sampled", ev, ee, flush=True)
    assert ev < TOL and ee < TOL


@pytest.mark.parametrize("nz", [96, 128, 256, 384])
def test_paired_solve_layout_matches_oracle(nz):
    """The radial solve with the two signs of l of each wavenumber pair in the
    two halves of a wavefront (an autotuner candidate, set here through
    tc_set_solve_shape): three steps against the oracle with one full group
    of 32 pairs per j (N_z = 96, K_z = 31), two groups the second partial
    (N_z = 128, K_z = 42), three groups the last partial (N_z = 256, K_z = 85)
    and four full groups (N_z = 384, K_z = 127)."""
    w = workload("tc-small-fp64", nr=33, ntheta=12, nz=nz, amplitude=1e-2)
    orc, gpu = pair(w)
    gpu.set_solve_shape(10000 + gpu.tuning()["solve_shape"])
    assert gpu.tuning()["solve_shape"] >= 10000
    for s in range(3):
        orc.step(1)
        gpu.step(1)
        _compare_state(orc, gpu, label=f"paired nz={nz} step {s + 1}")


@pytest.mark.parametrize("name", ["tc-medium-fp64", "tc-turbulent-fp64"])
def test_tile_shapes_are_bit_identical(name):
    """Every compiled tile shape of the transform kernels (z kernels at half,
    the default and twice the columns per block; theta at 1, 2 and 4
    wavefronts per block) gives the default's products bit for bit, in both
    precisions; a shape that is not compiled is refused."""
    from tests.helpers import abi_geometry, fields_for
    w = workload(name)
    for prec in (tcb.TC_PREC_FP64, tcb.TC_PREC_MIXED):
        g = tcb.Solver(abi_geometry(w, prec))
        g.load_fields(*fields_for(w, g.grid()))
        want = g.products()
        tried = 0
        for zi, th, zf in ((1, 0, 1), (2, 0, 2), (0, 1, 0), (0, 2, 0), (0, 3, 0)):
            try:
                g.set_tiles(zi, th, zf)
            except tcb.TcError as e:
                assert e.code == tcb.TC_EINVAL
                continue
            assert g.tiles() == {"zinv": zi, "theta": th, "zfwd": zf}
            got = g.products()
            tried += 1
            for k in want:
                assert np.array_equal(got[k], want[k]), (name, prec, zi, th, zf, k)
        assert tried >= 3
        with pytest.raises(tcb.TcError):
            g.set_tiles(0, 7, 0)
        g.close()


def test_loaded_field_validation():
    w = workload("tc-small-fp64")
    orc, gpu = pair(w)
    v, e, um, wm = gpu.get_fields()
    bad = v.copy()
    bad[3, 2, 4] = np.nan
    with pytest.raises(tcb.TcError) as ex:
        gpu.load_fields(bad, e, um, wm)
    assert ex.value.code == tcb.TC_ENONFINITE
    bad = v.copy()
    bad[0, 1, 1] = 1e-3
    with pytest.raises(tcb.TcError) as ex:
        gpu.load_fields(bad, e, um, wm)
    assert ex.value.code == tcb.TC_ESHAPE
    bad = v.copy()
    kz = (v.shape[2] - 1) // 2
    bad[5, 0, kz + 1] += 1e-3j
    with pytest.raises(tcb.TcError) as ex:
        gpu.load_fields(bad, e, um, wm)
    assert ex.value.code == tcb.TC_ESHAPE
    wm2 = wm.copy()
    wm2[0] = 0.9
    with pytest.raises(tcb.TcError) as ex:
        gpu.load_fields(v, e, um, wm2)
    assert ex.value.code == tcb.TC_ESHAPE
    # the state was left untouched by the failed loads
    v2 = gpu.get_fields()[0]
    assert np.array_equal(v, v2)


def test_blow_up_is_reported():
    """A time step far beyond the explicit stability limit makes the state
    non-finite; the step reports it instead of returning garbage."""
    w = workload("tc-small-fp64", dt=50.0, amplitude=0.5, re=5000.0)
    orc, gpu = pair(w)
    with pytest.raises(tcb.TcError) as ex:
        gpu.step(40)
    assert ex.value.code == tcb.TC_ENONFINITE
    assert gpu.stats()["nonfinite"] == 1


def test_deterministic_and_checkpoint_restart():
    w = workload("tc-medium-fp64")
    _, a = pair(w)
    _, b = pair(w)
    a.step(4)
    b.step(2)
    ckpt = b.get_fields()
    b.load_fields(*ckpt)  # restart from the saved fields at a step boundary
    # the explicit-term registers are not needed at step boundaries (the
    # first substep has no N^{k-2} term), so the restarted run is identical
    b.step(2)
    fa, fb = a.get_fields(), b.get_fields()
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)


def test_mixed_precision_small_ten_steps():
    """Mixed precision (FP32 transforms and products, FP64 radial solves,
    mean flow and statistics) against the FP64 oracle."""
    w = workload("tc-small-fp64")
    orc, gpu = pair(w, precision=tcb.TC_PREC_MIXED)
    orc.step(w["steps"])
    gpu.step(w["steps"])
    errs = _compare_state(orc, gpu, tol=1e-5, label="mixed 10 steps")
    so, sg = orc.stats(), gpu.stats()
    assert abs(sg["torque_in"] / so["torque_in"] - 1) < 1e-6
    assert max(errs.values()) > 1e-12  # the FP32 stages really ran


def test_lane_and_generic_paths_agree_at_turbulent_size():
    """The two transform implementations give the same products on the full
    turbulent-case grid (to FP64 rounding)."""
    w = workload("tc-turbulent-fp64")
    from tests.helpers import abi_geometry, fields_for
    a = tcb.Solver(abi_geometry(w))
    b = tcb.Solver(abi_geometry(w, flags=tcb.TC_FLAG_GENERIC_FFT))
    f = fields_for(w, a.grid())
    a.load_fields(*f)
    b.load_fields(*f)
    pa, pb_ = a.products(), b.products()
    for k in pa:
        err = rel_l2(pa[k], pb_[k])
        print("lane vs generic", k, f"{err:.2e}", flush=True)
        assert err < 1e-13


def test_theta_transform_variants_agree_at_turbulent_size():
    """The three 768-point theta transforms (lane-digit swaps with the low
    digits through LDS, the default; Stockham passes through LDS, tile code 4;
    every lane exchange in registers, tile code 5) give the same products to
    the rounding of each precision (codes 0 and 5 differ only in how data move
    between lanes, so they may agree bit for bit); the other form of w's fetch
    (code 6: into LDS by DMA in FP64, into registers in FP32) runs the same
    arithmetic in another instruction order and agrees to rounding too; and
    each code is refused at a length where only the Stockham transform is
    compiled."""
    w = workload("tc-turbulent-fp64")
    from tests.helpers import abi_geometry, fields_for
    for prec, tol in ((tcb.TC_PREC_FP64, 1e-13), (tcb.TC_PREC_MIXED, 2e-6)):
        g = tcb.Solver(abi_geometry(w, prec))
        g.load_fields(*fields_for(w, g.grid()))
        ref = g.products()
        for code in (4, 5, 6):
            g.set_tiles(0, code, 0)
            got = g.products()
            for k in ref:
                err = rel_l2(got[k], ref[k])
                print("theta code", code, prec, k, f"{err:.2e}", flush=True)
                assert err < tol
        g.close()
    small = tcb.Solver(abi_geometry(workload("tc-medium-fp64")))
    for code in (4, 5, 6):
        with pytest.raises(tcb.TcError):
            small.set_tiles(0, code, 0)
    small.close()


def test_mixed_products_at_turbulent_size():
    """FP32 transforms on the full turbulent-case grid, the size at which the
    FP32 z kernels pair their column groups across XCDs, give the products of
    the FP64 transforms to single-precision rounding (both lane and generic
    kernels)."""
    w = workload("tc-turbulent-fp64")
    from tests.helpers import abi_geometry, fields_for
    ref = tcb.Solver(abi_geometry(w))
    f = fields_for(w, ref.grid())
    ref.load_fields(*f)
    pr = ref.products()
    for flags in (0, tcb.TC_FLAG_GENERIC_FFT):
        m = tcb.Solver(abi_geometry(w, tcb.TC_PREC_MIXED, flags=flags))
        m.load_fields(*f)
        pm = m.products()
        for k in pr:
            err = rel_l2(pm[k], pr[k])
            print("mixed vs fp64", flags, k, f"{err:.2e}", flush=True)
            assert 1e-10 < err < 2e-6
        del m


@pytest.mark.parametrize("prec", [tcb.TC_PREC_FP64, tcb.TC_PREC_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name", ["tc-small-fp64", "tc-medium-fp64"])
def test_forward_elimination_in_rhs_matches_oracle(name, prec):
    """With whole-column chunks the explicit-term kernel runs the solves'
    forward elimination along each column (boundary-row folds and the mean
    profiles' wall terms included) and the solve substitutes back: three
    steps against the oracle, in both precisions (mixed: the FP32 transform
    error).  The solve's byte model drops the two factor fields it no longer
    reads, which shows the form is in use; switched off, the solve does both
    sweeps again."""
    w = workload(name)
    orc, gpu = pair(w, precision=prec)
    nr = gpu.mode_shape()[0]
    plain = gpu.kernel_bytes()["radial_solve"]
    gpu.set_rhs_rows(nr - 4)
    fused = gpu.kernel_bytes()["radial_solve"]
    assert fused < plain
    tol = TOL if prec == tcb.TC_PREC_FP64 else 1e-5
    for s in range(3):
        orc.step(1)
        gpu.step(1)
        _compare_state(orc, gpu, tol=tol, label=f"{name} fused elimination step {s + 1}")
    gpu.set_rhs_elimination(False)
    assert gpu.kernel_bytes()["radial_solve"] == plain
    orc.step(1)
    gpu.step(1)
    _compare_state(orc, gpu, tol=tol, label=f"{name} after switching it off")


@pytest.mark.parametrize("name", ["tc-small-fp64", "tc-medium-fp64"])
def test_rhs_chunking_is_bit_identical(name):
    """The explicit-term kernel walks each radial column in chunks; every row's
    terms are summed in the same order whatever the chunk length, including
    lengths whose rr + 4 points are not whole periods of the rolled loop (the
    walk then starts up to 4 points early).  One step for each chunk length
    gives the default's state bit for bit, in both precisions (with the
    solve's forward elimination in the solve: whole-column chunks would
    otherwise move it into the explicit-term kernel, which changes rounding;
    that form has its own tests)."""
    from tests.helpers import abi_geometry, fields_for
    w = workload(name)
    for prec in (tcb.TC_PREC_FP64, tcb.TC_PREC_MIXED):
        ref = tcb.Solver(abi_geometry(w, prec))
        ref.set_rhs_elimination(False)
        f = fields_for(w, ref.grid())
        ref.load_fields(*f)
        ref.step(1)
        want = ref.get_fields()
        nr = ref.mode_shape()[0]
        rows = sorted({1, 2, 3, 4, 7, 13, 22, 25, (nr - 4 + 1) // 2, nr - 4} & set(range(1, nr - 3)))
        g = tcb.Solver(abi_geometry(w, prec))
        g.set_rhs_elimination(False)
        for rr in rows:
            g.set_rhs_rows(rr)
            assert g.tuning()["rhs_rows"] == rr
            g.load_fields(*f)
            g.step(1)
            got = g.get_fields()
            for a, b, k in zip(got, want, ("v", "eta", "u_mean", "w_mean")):
                assert np.array_equal(a, b), (name, prec, rr, k)
        with pytest.raises(tcb.TcError):
            g.set_rhs_rows(nr - 3)
        with pytest.raises(tcb.TcError):
            g.set_rhs_rows(0)


def test_graph_replays_match_eager_steps():
    """Whole-step graph replays, with eager work (field reads) and
    synchronisation between them, give bit-identical states to eager launches."""
    w = workload("tc-medium-fp64")
    _, a = pair(w)
    _, b = pair(w)
    b.use_graphs(False)
    for s in range(4):
        a.step(1)
        b.step(1)
        fa, fb = a.get_fields(), b.get_fields()
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y), s
    a.step(3)
    b.step(3)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.array_equal(x, y)


def test_batched_instances_equal_single_runs():
    """A context holding several instances of different shapes (several per
    launch) gives each instance exactly the state it has when run alone; one
    of them is also checked against the oracle."""
    from paper_0711_1429_amd.synth import batched_instances
    from tests.helpers import abi_geometry, fields_for
    ws = batched_instances(64)[:6] + [dict(workload("tc-small-fp64"), amplitude=1e-2)]
    for prec in (tcb.TC_PREC_FP64, tcb.TC_PREC_MIXED):
        multi = tcb.Solver([abi_geometry(w, prec) for w in ws])
        singles = [tcb.Solver(abi_geometry(w, prec)) for w in ws]
        for i, w in enumerate(ws):
            f = fields_for(w, multi.grid(i))
            multi.load_fields(*f, inst=i)
            singles[i].load_fields(*f)
        multi.step(3)
        for i, one in enumerate(singles):
            one.step(3)
            for x, y in zip(multi.get_fields(i), one.get_fields()):
                assert np.array_equal(x, y), (prec, i)
            pm, ps_ = multi.profiles(i), one.profiles()
            for k in pm:
                assert np.array_equal(pm[k], ps_[k]), (prec, i, k)
    orc, _ = pair(ws[0])
    orc.step(3)
    multi = tcb.Solver([abi_geometry(w) for w in ws])
    for i, w in enumerate(ws):
        multi.load_fields(*fields_for(w, multi.grid(i)), inst=i)
    multi.step(3)
    v, e, um, wm = multi.get_fields(0)
    rv, re_, rum, rwm = orc.fields()
    assert rel_l2(v, rv) < TOL and rel_l2(e, re_) < TOL


def test_batched_workload_all_64_instances_equal_single_runs():
    """The whole batched workload (64 instances of nine grid shapes, mixed
    precision, as the benchmark runs it: launch parameters autotuned, steps
    replayed from the captured graph) gives every instance bit for bit the
    state it reaches alone in a context of its own with the same launch
    parameters, after 5 steps."""
    from paper_0711_1429_amd.synth import batched_instances
    from tests.helpers import abi_geometry, fields_for
    ws = batched_instances(64)
    prec = tcb.TC_PREC_MIXED
    multi = tcb.Solver([abi_geometry(w, prec) for w in ws])
    fields = [fields_for(w, multi.grid(i)) for i, w in enumerate(ws)]
    for i, f in enumerate(fields):
        multi.load_fields(*f, inst=i)
    multi.autotune(2)
    multi.step(5)
    for i, w in enumerate(ws):
        one = tcb.Solver(abi_geometry(w, prec))
        one.set_rhs_rows(multi.tuning(i)["rhs_rows"])
        one.load_fields(*fields[i])
        one.step(5)
        got, want = multi.get_fields(i), one.get_fields()
        same_shape = multi.tuning(i)["solve_shape"] == one.tuning()["solve_shape"]
        for x, y, k in zip(got, want, ("v", "eta", "u_mean", "w_mean")):
            if same_shape:
                assert np.array_equal(x, y), (i, k)
            else:  # the autotuner chose another segmentation of the same solve
                assert rel_l2(np.atleast_1d(x), np.atleast_1d(y)) < 1e-12, (i, k)
        one.close()
    multi.close()


def test_linear_flag_matches_oracle_without_products():
    """TC_FLAG_LINEAR: the step with the six products set to zero equals the
    oracle's step with its products replaced by zeros (a mixed instance set:
    one linear and one full instance of different shapes in one context)."""
    from tests.helpers import abi_geometry, fields_for, oracle_geometry
    from oracle import Oracle
    w = workload("tc-small-fp64", amplitude=1e-2)
    orc = Oracle(oracle_geometry(w))
    orc.products = lambda u, v, ww: {k: np.zeros((orc.geo.nr, orc.disc.nj * orc.disc.nl), complex)
                                     for k in ("uu", "uv", "uw", "vv", "vw", "ww")}
    w2 = workload("tc-medium-fp64")
    gpu = tcb.Solver([abi_geometry(w, flags=tcb.TC_FLAG_LINEAR), abi_geometry(w2)])
    f = fields_for(w, orc.disc.r)
    orc.load(*f)
    gpu.load_fields(*f, inst=0)
    orc2, one = pair(w2)
    gpu.load_fields(*fields_for(w2, gpu.grid(1)), inst=1)
    for s in range(3):
        orc.step(1)
        gpu.step(1)
        v, e, um, wm = gpu.get_fields(0)
        rv, re_, rum, rwm = orc.fields()
        assert rel_l2(v, rv) < TOL and rel_l2(e, re_) < TOL and rel_l2(wm, rwm) < TOL, s
    assert all(np.all(p == 0) for p in gpu.products(0).values())
    one.step(3)
    for x, y in zip(gpu.get_fields(1), one.get_fields()):
        assert np.array_equal(x, y)


def test_linear_flag_decays_at_the_stokes_eigenvalue():
    """Without products the perturbation obeys the Stokes problem about the
    (unadvected) mean flow: seeded with the least stable Stokes eigenvector of
    the discrete operator (radius ratio 0.5, Re = 100, axial wavenumber pi,
    m = 0), its energy decays at twice the eigenvalue, -0.20088 (a value the
    eigenproblem fixes independently of the time integrator)."""
    from scipy.linalg import eig
    from oracle import Geometry, Oracle
    from tests.test_oracle_dynamics import linear_operator
    geo = Geometry(zeta=0.5, re=100.0, nr=33, ntheta=4, nz=4, dt=1e-2, lz=2.0)
    orc = Oracle(geo)
    A, B = linear_operator(orc, 0, 1, np.zeros(geo.nr))
    lam, vec = eig(A, B)
    ok = np.isfinite(lam) & (np.abs(lam) < 1e6)
    k = np.argmax(np.where(ok, lam.real, -np.inf))
    assert abs(lam[k].real + 0.20088) < 1e-4 and abs(lam[k].imag) < 1e-8
    # at m = 0 without base flow v and eta decouple, and the least stable mode
    # may be a pure eta mode: scale by the whole eigenvector
    x = vec[:, k] * (1e-6 / np.max(np.abs(vec[:, k])))
    nr, kz = geo.nr, orc.disc.kz
    v = np.zeros((nr, orc.disc.nj, orc.disc.nl), dtype=complex)
    e = np.zeros_like(v)
    v[:, 0, kz + 1], e[:, 0, kz + 1] = x[:nr], x[nr:]
    v[:, 0, kz - 1], e[:, 0, kz - 1] = np.conj(x[:nr]), np.conj(x[nr:])
    v[[0, -1]] = 0
    e[[0, -1]] = 0
    from paper_0711_1429_amd.synth import couette_profile
    wlam = couette_profile(orc.disc.r, 0.5, 1.0, 0.0)
    gpu = tcb.Solver(tcb.make_geometry(zeta=0.5, re=100.0, nr=33, ntheta=4, nz=4, dt=1e-2, lz=2.0,
                                       flags=tcb.TC_FLAG_LINEAR))
    gpu.load_fields(v, e, np.zeros(geo.nr), wlam)
    e0 = gpu.stats()["energy_pert"]
    gpu.step(100)  # t = 1
    e1 = gpu.stats()["energy_pert"]
    sigma = np.log(e1 / e0) / 2.0
    print(f"decay rate {sigma:.6f}, eigenvalue {lam[k].real:.6f}", flush=True)
    assert abs(sigma / lam[k].real - 1) < 1e-4


def test_autotune_keeps_the_state_and_the_results():
    """tc_autotune times launch variants that do not change the method: the
    state is bit-identical afterwards, the chosen parameters are valid, and the
    following steps still match the oracle."""
    from paper_0711_1429_amd.synth import batched_instances
    from tests.helpers import abi_geometry, fields_for
    w = workload("tc-medium-fp64")
    orc, gpu = pair(w)
    before = gpu.get_fields()
    gpu.autotune(2)
    for x, y in zip(gpu.get_fields(), before):
        assert np.array_equal(x, y)
    t = gpu.tuning()
    assert t["rhs_rows"] in (6, 11, 16, 21) and t["solve_shape"] % 10000 in (804, 808, 1608)
    tl = gpu.tiles()
    assert tl["zinv"] in (0, 1, 2) and tl["zfwd"] in (0, 1, 2) and tl["theta"] in (0, 1, 2, 3)
    orc.step(2)
    gpu.step(2)
    _compare_state(orc, gpu, label="after autotune")
    # a batched context keeps its per-instance results as well
    ws = batched_instances(64)[:5]
    multi = tcb.Solver([abi_geometry(x, tcb.TC_PREC_MIXED) for x in ws])
    for i, x in enumerate(ws):
        multi.load_fields(*fields_for(x, multi.grid(i)), inst=i)
    ref = tcb.Solver([abi_geometry(x, tcb.TC_PREC_MIXED) for x in ws])
    for i, x in enumerate(ws):
        ref.load_fields(*fields_for(x, ref.grid(i)), inst=i)
    multi.autotune(2)
    print("tiles chosen:", [multi.tiles(i) for i in range(len(ws))], flush=True)
    multi.step(2)
    ref.step(2)
    for i in range(len(ws)):
        for x, y in zip(multi.get_fields(i), ref.get_fields(i)):
            if multi.tuning(i)["solve_shape"] == ref.tuning(i)["solve_shape"]:
                assert np.array_equal(x, y), i
            else:  # another segmentation of the same solve: equal to rounding
                assert rel_l2(np.atleast_1d(x), np.atleast_1d(y)) < 1e-12, i
