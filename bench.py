"""Throughput of the Taylor--Couette RK3 substep on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                [--precision fp64|mixed] [--no-cpu-baseline]

Workloads: tc-turbulent-fp64 (default; 129 x 768 x 384), tc-medium-fp64,
tc-small-fp64, tc-batched-64 (64 independent instances, mixed precision).

A step is one full RK3 step (3 substeps: velocity recovery, inverse
transforms, products, forward transforms, explicit terms, banded solves and
the mean flow) of the whole grid, on synthetic seeded fields already resident
in HBM.  value = grid points x substeps per second / 1e6.  Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="tc-turbulent-fp64")
    p.add_argument("--precision", choices=("fp64", "mixed"), default=None,
                   help="default: fp64, or mixed for the batched workload")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the mixed-precision and batched sub-records of the default line")
    p.add_argument("--autotune", choices=("on", "off", "auto"), default="auto",
                   help="time the launch variants before the run (auto: on for the batched workload)")
    p.add_argument("--eager", action="store_true",
                   help="launch every kernel from the host instead of replaying the step graph "
                        "(for profilers that see only host-launched kernels)")
    p.add_argument("--cpu-modes", type=int, default=16384,
                   help="modes the CPU baseline solves radially (the transforms cover the whole grid)")
    p.add_argument("--copy-calib", action="store_true",
                   help="only run a device copy of known size (counter calibration)")
    p.add_argument("--accuracy", type=str, default="",
                   help="comma-separated step counts: run the FP64 and mixed paths side by side "
                        "and report the mixed path's relative L2 error after those steps")
    return p.parse_args()


def copy_calibration():
    """A plain 512 MiB device copy: the reference reading for the HBM traffic
    counters, and the copy bandwidth the device reaches in practice."""
    import torch
    n = 512 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 20
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 25,
                      "copy_GBs": 2 * n * 8 / dt / 1e9}))


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter table in
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a device-copy calibration),
    or None when the table has no row for it or was taken on other kernel
    sources than the ones built here."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_step_kernels.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_lane.h", "fft_xlane.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_0711_1429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha, rows = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if not parts or parts[0].startswith("#"):
                continue
            if parts[0] == "kernels_sha256":
                sha = parts[1]
            elif len(parts) == 5:
                rows[tuple(parts[:3])] = float(parts[3]) + float(parts[4])
    if sha != h.hexdigest():
        return None
    return rows.get((workload, precision, kernel))


def _cpu_workers():
    n = os.cpu_count() or 1
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        pass
    return max(1, min(n, 16))


def cpu_baseline(w, nmodes_sample, workers=None):
    """The FP64 oracle on the host's cores: one substep of the same workload.
    The oracle's own functions run unchanged; the harness splits their
    independent work over `workers` forked processes that share the arrays:
    the velocity recovery by modes (each mode's D v solve is independent), the
    dealiased products by radial planes (each plane's transforms are
    independent), and the explicit terms and banded solves by modes, on a
    sample of modes scaled to all of them."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    from oracle import Geometry, Oracle
    from oracle import equations as oeq
    from oracle.spectral import products as oracle_products
    from paper_0711_1429_amd.synth import initial_fields

    workers = workers or _cpu_workers()
    geo = Geometry(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"],
                   dt=w["dt"], stretch=w["stretch"])
    orc = Oracle(geo)
    orc.load(*initial_fields(orc.disc.r, w["zeta"], w["ntheta"], w["nz"], w["amplitude"], w["seed"]))
    idx = np.flatnonzero(~orc.mc.is_mean)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(idx, size=min(nmodes_sample, idx.size), replace=False))
    nr, nj, nl = geo.nr, orc.disc.nj, orc.disc.nl
    M = nj * nl
    keys = ("uu", "uv", "uw", "vv", "vw", "ww")
    shm = shared_memory.SharedMemory(create=True, size=9 * nr * M * 16)
    ctx = mp.get_context("fork")

    def one_thread(target):
        def wrapped(*a):
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):  # one core per process (BLAS threads off)
                target(*a)
        return wrapped

    def run(target, args_list):
        procs = [ctx.Process(target=one_thread(target), args=a) for a in args_list]
        for p in procs:
            p.start()
        for p in procs:
            p.join()
        assert all(p.exitcode == 0 for p in procs)

    try:
        A = np.ndarray((9, nr, M), dtype=np.complex128, buffer=shm.buf)
        U, W, Cc, P = A[0], A[1], A[2], A[3:]
        t0 = time.perf_counter()

        def recover(sub):
            dv = orc.ops.radial_derivative(orc.v[:, sub])
            u, ww, c = oeq.recover_velocity(orc.ops, orc._sub_mc(sub), orc.v[:, sub], orc.eta[:, sub], dv)
            U[:, sub], W[:, sub], Cc[:, sub] = u, ww, c

        run(recover, [(part,) for part in np.array_split(np.arange(M), workers)])
        U[:, orc.mean_index] = orc.u_mean
        W[:, orc.mean_index] = orc.w_mean

        def planes(r0, r1):
            sh = (r1 - r0, nj, nl)
            out = oracle_products(U[r0:r1].reshape(sh), orc.v[r0:r1].reshape(sh), W[r0:r1].reshape(sh),
                                  geo.ntheta, geo.nz)
            for q, k in enumerate(keys):
                P[q, r0:r1] = out[k].reshape(r1 - r0, -1)

        bounds = np.linspace(0, nr, workers + 1).astype(int)
        run(planes, [(int(bounds[i]), int(bounds[i + 1])) for i in range(workers)])
        t1 = time.perf_counter()
        prods = {k: P[q] for q, k in enumerate(keys)}

        def radial(sub):
            nv, ne = orc.explicit_terms(sub, U, orc.v, W, Cc, prods)
            orc.radial_update(0, sub, orc.v, orc.eta, nv, ne, orc.nv_prev[:, sub], orc.neta_prev[:, sub])

        run(radial, [(part,) for part in np.array_split(sample, workers)])
        t2 = time.perf_counter()
    finally:
        shm.close()
        shm.unlink()
    t_sub = (t1 - t0) + (t2 - t1) * idx.size / sample.size
    pts = w["nr"] * w["ntheta"] * w["nz"] / 1e6
    return {
        "value": pts / t_sub,
        "unit": "Mpts*substeps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"one substep of {w['nr']}x{w['ntheta']}x{w['nz']} on {workers} forked processes "
                   f"(host reports {os.cpu_count()} CPUs): velocity recovery split by modes and dealiased "
                   f"products on the whole grid split by radial planes ({t1 - t0:.1f} s), explicit terms "
                   f"and banded solves on {sample.size} of {idx.size} modes split by modes "
                   f"({t2 - t1:.1f} s) scaled to all modes; numpy FFT and LAPACK single-threaded in each "
                   f"process"),
        "seconds_per_substep": t_sub,
    }


def method_bytes(w, precision):
    """Minimum HBM bytes of one substep of the staged method: every stage
    reads its inputs and writes its outputs once; FP64 448 S + 288 Q, mixed
    (complex64 transform-side arrays) 304 S + 144 Q."""
    kt, kz = (w["ntheta"] - 1) // 3, (w["nz"] - 1) // 3
    S = w["nr"] * (kt + 1) * (2 * kz + 1)
    Q = w["nr"] * w["nz"] * (kt + 1)
    return (448.0 * S + 288.0 * Q) if precision == "fp64" else (304.0 * S + 144.0 * Q)


def _rel(a, b, cj):
    return float(np.sqrt(np.sum(cj * np.abs(a - b) ** 2) / np.sum(cj * np.abs(b) ** 2)))


def accuracy(w, checkpoints):
    """Mixed-precision error growth: the FP64 GPU path (which matches the FP64
    oracle to <= 1e-12 per step in the parity tests) is the reference."""
    from paper_0711_1429_amd import tc
    from paper_0711_1429_amd.synth import initial_fields
    geo = dict(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"],
               dt=w["dt"], stretch=w["stretch"])
    ref = tc.Solver(tc.make_geometry(**geo))
    mix = tc.Solver(tc.make_geometry(precision=tc.TC_PREC_MIXED, **geo))
    fields = initial_fields(ref.grid(), w["zeta"], w["ntheta"], w["nz"], w["amplitude"], w["seed"])
    ref.load_fields(*fields)
    mix.load_fields(*fields)
    nj = ref.mode_shape()[1]
    cj = np.where(np.arange(nj) == 0, 1.0, 2.0)[None, :, None]
    done = 0
    out = []
    for target in checkpoints:
        ref.step(target - done)
        mix.step(target - done)
        done = target
        v0, e0, u0m, w0m = ref.get_fields()
        v1, e1, u1m, w1m = mix.get_fields()
        uu0, ww0 = ref.velocity()
        uu1, ww1 = mix.velocity()
        kz = (v0.shape[2] - 1) // 2
        wp0, wp1 = ww0.copy(), ww1.copy()
        wp0[:, 0, kz] = 0
        wp1[:, 0, kz] = 0
        s0, s1 = ref.stats(), mix.stats()
        rec = {"steps": target, "v": _rel(v1, v0, cj), "eta": _rel(e1, e0, cj), "u": _rel(uu1, uu0, cj),
               "w": _rel(ww1, ww0, cj), "w_pert": _rel(wp1, wp0, cj),
               "torque_in": abs(s1["torque_in"] / s0["torque_in"] - 1),
               "torque_out": abs(s1["torque_out"] / s0["torque_out"] - 1),
               "energy_pert": abs(s1["energy_pert"] / s0["energy_pert"] - 1)}
        print(json.dumps(rec), file=sys.stderr, flush=True)
        out.append(rec)
    return out


def _sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:  # pragma: no cover
        pass


STEP_KERNELS = ("radial_derivative", "zfft_inverse", "theta_rows_products", "zfft_forward",
                "radial_rhs", "radial_solve")


def measure(workload, precision, steps, warmup, eager=False, autotune="auto"):
    """Time `steps` whole RK3 steps of a workload (inputs resident in HBM):
    first replayed from the captured step graph (the value), then launched
    eagerly with HIP events around every kernel on the solver's stream (the
    per-kernel figures)."""
    from paper_0711_1429_amd import tc
    from paper_0711_1429_amd.synth import WORKLOADS, batched_instances, initial_fields

    batched = workload == "tc-batched-64"
    ws = batched_instances() if batched else [dict(WORKLOADS[workload])]
    prec = tc.TC_PREC_MIXED if precision == "mixed" else tc.TC_PREC_FP64
    geos = [tc.make_geometry(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"],
                             dt=w["dt"], stretch=w["stretch"], precision=prec) for w in ws]
    solver = tc.Solver(geos)
    if eager:
        solver.use_graphs(False)
    for i, w in enumerate(ws):
        solver.load_fields(*initial_fields(solver.grid(i), w["zeta"], w["ntheta"], w["nz"], w["amplitude"],
                                           w["seed"]), inst=i)
    tuned = autotune == "on" or (autotune == "auto" and batched)
    if tuned:
        print(f"bench: {workload} autotune", file=sys.stderr, flush=True)
        solver.autotune(5)
    tuning = sorted({tuple(solver.tuning(i).items()) + tuple(solver.tiles(i).items()) for i in range(len(ws))})
    print(f"bench: {workload} {precision} warmup {warmup}", file=sys.stderr, flush=True)
    solver.step(warmup)

    # timed region 1 (the value): whole steps replayed from the captured graph
    _sync()
    t0 = time.perf_counter()
    solver.step(steps)
    _sync()
    elapsed = time.perf_counter() - t0
    # timed region 2 (per-kernel figures): the same steps launched eagerly,
    # each launch bracketed by HIP events on the solver's stream
    solver.timing(True)
    _sync()
    t1 = time.perf_counter()
    solver.step(steps)
    _sync()
    elapsed_events = time.perf_counter() - t1
    ktimes = solver.kernel_times()
    solver.timing(False)
    print(f"bench: {workload} {precision}: timed {steps} steps in {elapsed:.3f} s (graph), "
          f"{elapsed_events:.3f} s (events)", file=sys.stderr, flush=True)

    substeps = 3 * steps
    pts = sum(w["nr"] * w["ntheta"] * w["nz"] for w in ws)
    kbytes = {}
    for i in range(len(ws)):
        for name, bts in solver.kernel_bytes(i).items():
            kbytes[name] = kbytes.get(name, 0.0) + bts
    ncls = len({(w["nr"], w["ntheta"], w["nz"]) for w in ws})
    per_kernel = {}
    for name, (ms, calls) in ktimes.items():
        if calls:
            rec = {"avg_ms": ms / calls, "calls": calls}
            if name in STEP_KERNELS:
                # each step kernel is launched once per substep and launch
                # group, covering every instance of the group: the algorithmic
                # bytes of all instances over the summed launch time
                rec["model_GBs"] = kbytes[name] * substeps / (ms * 1e-3) / 1e9
            per_kernel[name] = rec
    dom = max(STEP_KERNELS, key=lambda k: ktimes[k][0])
    # whole-substep byte models.  method: each stage of the staged substep
    # reads its inputs and writes its outputs in HBM once (448 S + 288 Q bytes
    # in FP64, 304 S + 144 Q with complex64 transform-side arrays; S spectral
    # and Q mixed-space points); implementation: the sum of the step kernels'
    # own models, which also count this build's design traffic (the LU-factor
    # table of the solve, the right-hand sides between the explicit-term and
    # solve kernels, the separate D v array)
    model = sum(method_bytes(w, precision) for w in ws)
    impl = sum(kbytes[k] for k in STEP_KERNELS)
    t_sub = elapsed / substeps
    solver.close()
    return {
        "ws": ws, "batched": batched, "ncls": ncls, "pts": pts,
        "value": pts * substeps / elapsed / 1e6,
        "ms_per_step": elapsed / steps * 1e3,
        "ms_per_step_events": elapsed_events / steps * 1e3,
        "dominant": dom, "kbytes": kbytes, "kernels": per_kernel,
        "substep_model": {"bytes": model, "ms_per_substep": t_sub * 1e3,
                          "GBs": model / t_sub / 1e9, "frac": model / t_sub / 1e9 / HBM_PEAK_GBS,
                          "implementation_bytes": impl,
                          "implementation_frac": impl / t_sub / 1e9 / HBM_PEAK_GBS},
        "launch_tuning": {"autotuned": tuned, "choices": [dict(t) for t in tuning]},
    }


def batched_accuracy(steps):
    """The batched workload in mixed precision against the same instances in
    FP64 after `steps` steps: the largest per-instance relative L2 error of
    v, eta and w (mean included) and of the inner torque."""
    from paper_0711_1429_amd import tc
    from paper_0711_1429_amd.synth import batched_instances, initial_fields
    ws = batched_instances()
    out = {}
    solvers = {}
    for name, prec in (("fp64", tc.TC_PREC_FP64), ("mixed", tc.TC_PREC_MIXED)):
        g = tc.Solver([tc.make_geometry(zeta=w["zeta"], re=w["re"], nr=w["nr"], ntheta=w["ntheta"], nz=w["nz"],
                                        dt=w["dt"], stretch=w["stretch"], precision=prec) for w in ws])
        for i, w in enumerate(ws):
            g.load_fields(*initial_fields(g.grid(i), w["zeta"], w["ntheta"], w["nz"], w["amplitude"], w["seed"]),
                          inst=i)
        g.step(steps)
        solvers[name] = g
    worst = {"v": 0.0, "eta": 0.0, "w": 0.0, "torque_in": 0.0}
    for i in range(len(ws)):
        a, b = solvers["fp64"], solvers["mixed"]
        v0, e0, _, _ = a.get_fields(i)
        v1, e1, _, _ = b.get_fields(i)
        cj = np.where(np.arange(v0.shape[1]) == 0, 1.0, 2.0)[None, :, None]
        _, w0 = a.velocity(i)
        _, w1 = b.velocity(i)
        worst["v"] = max(worst["v"], _rel(v1, v0, cj))
        worst["eta"] = max(worst["eta"], _rel(e1, e0, cj))
        worst["w"] = max(worst["w"], _rel(w1, w0, cj))
        worst["torque_in"] = max(worst["torque_in"], abs(b.stats(i)["torque_in"] / a.stats(i)["torque_in"] - 1))
    for g in solvers.values():
        g.close()
    out["steps"] = steps
    out["max_over_instances_mixed_vs_fp64"] = worst
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the solver holds the whole grid in one GPU's HBM", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration()
        return
    if args.accuracy:
        from paper_0711_1429_amd.synth import WORKLOADS
        w = dict(WORKLOADS[args.workload])
        cps = sorted(int(x) for x in args.accuracy.split(","))
        print(json.dumps({"workload": args.workload, "reference": "FP64 GPU path",
                          "mixed_vs_fp64": accuracy(w, cps)}), flush=True)
        return
    batched = args.workload == "tc-batched-64"
    precision = args.precision or ("mixed" if batched else "fp64")
    m = measure(args.workload, precision, args.steps, args.warmup, args.eager, args.autotune)
    ws, w0 = m["ws"], m["ws"][0]
    config = ({"workload": args.workload, "instances": len(ws), "shape_classes": m["ncls"],
               "precision": precision, "total_points": m["pts"]}
              if batched else
              {"workload": args.workload, "nr": w0["nr"], "ntheta": w0["ntheta"], "nz": w0["nz"],
               "zeta": w0["zeta"], "re": w0["re"], "dt": w0["dt"], "stretch": w0["stretch"],
               "precision": precision})
    dom = m["dominant"]
    achieved = m["kernels"][dom]["model_GBs"]
    out = {
        "metric": "Mpts*RK3 substeps/s on 1 GPU (FP64 vs mixed at stated L2 error); HBM GB/s",
        "value": m["value"],
        "unit": "Mpts*substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-transforms/f64-radial",
        "data": "synthetic: laminar Couette profile plus seeded random-phase divergence-free perturbation",
        "config": config,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes": m["kbytes"][dom] / m["ncls"],
                     "traffic": None if batched else measured_traffic(args.workload, precision, dom)},
        "substep_model": m["substep_model"],
        "ms_per_step_events": m["ms_per_step_events"],
        "launch_tuning": m["launch_tuning"],
        "kernels": m["kernels"],
    }
    default_line = args.workload == "tc-turbulent-fp64" and precision == "fp64" and not args.eager
    if default_line and not args.no_variants:
        # the mixed-precision form on the same grid and the batched form, each
        # timed the same way, with their errors against the FP64 path
        mx = measure(args.workload, "mixed", args.steps, args.warmup)
        out["mixed"] = {"value": mx["value"], "ms_per_step": mx["ms_per_step"],
                        "speedup_vs_fp64": mx["value"] / m["value"],
                        "substep_model": mx["substep_model"],
                        "kernels": {k: v["avg_ms"] for k, v in mx["kernels"].items()},
                        "accuracy_vs_fp64": accuracy(dict(w0), [1, 100, 1000])}
        bt = measure("tc-batched-64", "mixed", args.steps, args.warmup)
        out["batched"] = {"value": bt["value"], "ms_per_step": bt["ms_per_step"], "instances": len(bt["ws"]),
                          "total_points": bt["pts"], "speedup_vs_fp64": bt["value"] / m["value"],
                          "substep_model": bt["substep_model"], "launch_tuning": bt["launch_tuning"],
                          "accuracy": batched_accuracy(100)}
    if not args.no_cpu_baseline and not batched:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w0, args.cpu_modes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
