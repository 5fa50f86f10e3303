"""Benchmark of the forcing-loop hot path on one MI355X.

One step = the pair pass (cell/pair/wall lists, collision forces, marker
mask) + one ibmx_forcing call (marker geometry, then n_iter passes of
interpolate -> force -> spread -> update) on the resident synthetic workload.
The tile shape is autotuned first (ibmx_tune, untimed).  The steps are timed
three times: as eager calls with per-kernel HIP events (the roofline's kernel
durations), with the forcing call replayed as one HIP graph, and as eager
calls without the events (the headline value).
The reported value is whole-step throughput in marker-updates/s
(active markers x passes / step time).  Also reported: the FP64 instance of
the same kernels, per-kernel durations from HIP events recorded by the
library on its own stream, the roofline of the dominant kernel, and the CPU
oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, public figure


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(s: int, n_act: int, shell: int) -> float:
    """Algorithmic bytes of one forcing pass (interpolation + spreading), the
    roofline's numerator (s = bytes of the grid type).

    Per marker-update a record of 20 B (FP32: base cell, three fractions,
    particle id) or 32 B (FP64); per shell node (a node in the delta support
    of an active marker) the three velocity components read twice in the
    interpolation (u^0 and the accumulated correction) and the accumulator
    read and written in the spreading: 4 x 3s bytes.
    """
    b_rec = 20 if s == 4 else 32
    return float(n_act * b_rec + 12 * s * shell)


def design_bytes(kind: str, s: int, n_act: int, shell: int, halo: int) -> float:
    """Bytes the tile kernels must move per launch at least (reported beside
    the roofline): marker records of T4 = 4s bytes, halo = (marker,
    neighbouring tile) entries.

    interp: per own marker the fractions and base node (4s) and the
            rigid-body velocity and volume (4s) read, the amplitude G (4s)
            written; the three velocity components of every shell node read
            (3s).  Each tile stages its whole region, shell or not, with a
            margin of W - 1 nodes shared with its neighbours: its reads
            exceed this bound.
    spread: per own and halo entry the fractions and base node (4s) and G
            (4s) read, plus the halo list (4 B); per shell node the three
            components read and written (6s).
    """
    if kind == "interp":
        return float(n_act * 12 * s + shell * 3 * s)
    if kind == "spread":
        return float((n_act + halo) * 8 * s + halo * 4 + shell * 6 * s)
    raise KeyError(kind)


# what the roofline of the smaller workloads means
ROOFLINE_NOTES = {
    "single_sphere_64": "805 markers: launch and latency bound, no roofline claim",
    "suspension_128": "90,600 markers, about 20 MB per pass: launch and latency bound, "
                      "no roofline claim",
    "gradient_suspension_128": "90,600 markers: launch and latency bound, no roofline claim",
    "bidisperse_bed_256x256x512": "the shell's working set (about 70 MB per component "
                                  "array) fits the 256 MB Infinity Cache: the rate is a "
                                  "fabric bandwidth, not an HBM one",
}

COUNTER_FILES = {
    "polydisperse_bed_512": "profiles/k_interp_k_spread_polydisperse_bed_512_f32_hbm_counters.md",
}
# what the forcing kernels' machine code is built from: their sources and
# the compiler flags
KERNEL_SOURCES = ("paper_2109_03972_amd/csrc/ibmx_forcing.hip",
                  "paper_2109_03972_amd/csrc/ibmx_device.hpp",
                  "paper_2109_03972_amd/csrc/ibmx_delta.hpp")


def _strip_comments(src: str) -> str:
    """C/C++ source without its comments, indentation and blank lines (such
    edits do not change the kernels)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.strip() for line in src.splitlines() if line.strip())


def kernel_sources_hash() -> str:
    import hashlib
    from paper_2109_03972_amd import build_lib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            h.update(_strip_comments(fh.read()).encode())
    # the flags, without include paths (they name where the tree sits)
    h.update(" ".join(f for f in build_lib.HIPCC_FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()


def fluid_bytes(kind: str, s: int, nodes: int, walls_z: bool = True) -> float:
    """Bytes one fluid call must move (s = bytes of the field type; the
    solves work in FP64 on the half spectrum of nx/2 + 1 complex modes per
    row, about 8 B per node, and on an FP64 real grid, 8 B per node).

    spectrum (one solve between the x passes): the y pass forward and back
           (read and write 8 each: 16 + 16), and across walls the elimination
           (read and write the spectrum twice: 32; the eliminated coefficient
           is stored only until it becomes constant along z, not counted) or
           along a periodic z two more passes and the division (48).
    predictor: reads u, N (3s each) and P (s); writes u~, N and nu L u (3s each).
    project: face values and divergence (reads 3s, writes 3s + 8), the
           forward x pass from the real grid (read 8, write 8), the spectrum,
           the inverse x pass into the real grid (16), the correction (reads
           the solution, u, u_f, P; writes u, u_f, P: 8 + 14s; phi is not
           asked for).
    helmholtz (theta = 0, no pressure term): per component the forward x
           pass computing the right-hand side from u and nu L u as it reads
           (2s + 8), the spectrum, the inverse x pass writing the result
           (8 + s).
    """
    spectrum = 16 + 16 + (32 if walls_z else 48)
    if kind == "predictor":
        per = 16 * s
    elif kind == "project":
        per = (6 * s + 8) + 16 + spectrum + 16 + (8 + 14 * s)
    elif kind == "helmholtz":
        per = 3 * ((2 * s + 8) + spectrum + (8 + s))
    else:
        raise KeyError(kind)
    return float(per) * nodes


def measured_traffic(workload: str, kind: str, tile) -> "float | None":
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes, copy-calibrated), or None when
    there is none for this workload and tile, or the kernel sources changed
    since the counters were taken."""
    rel = COUNTER_FILES.get(workload)
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    fields = {}
    with open(os.path.join(ROOT, rel)) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0] in (
                    "traffic_per_launch_bytes", "tile", "kernel_sources_sha256"):
                k, v = line.split(":", 1)
                fields[k] = v.strip()
    if fields.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    if fields.get("tile") != ",".join(str(int(t)) for t in tile):
        return None
    for item in fields.get("traffic_per_launch_bytes", "").split():
        k, _, v = item.partition("=")
        if k == kind:
            return float(v)
    return None


def run_gpu(case, precision, steps, warmup, profile=True, tune=True, tile=None, launch=None):
    import torch
    from paper_2109_03972_amd import ibmx

    dev = torch.device("cuda:0")
    T = torch.float64 if precision == "f64" else torch.float32
    f64 = torch.float64
    D = {k: torch.as_tensor(getattr(case, k), dtype=f64).to(dev).contiguous()
         for k in ("xp", "up", "wp", "radius", "mass", "body", "dV")}
    u = case.field(device=dev).to(T).contiguous()
    f = torch.zeros_like(u)
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])
    n_iter = int(case.params["n_iter"])
    mask = torch.empty(case.nm, dtype=torch.uint8, device=dev)
    resid = torch.zeros(n_iter + 1, dtype=f64, device=dev)
    res = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], mask=mask)
    plan.check("pairs")
    t = ibmx.trim_pairs(res)
    prev = dict(pairs=t["pairs"].contiguous(), hist=t["hist"].contiguous(),
                walls=t["walls"].contiguous(), whist=t["whist"].contiguous())
    caps = dict(pair_cap=res["pair_cap"], wall_cap=res["wall_cap"])
    tuned = None
    if tile is not None:
        plan.set_tiles(*tile)
        if launch is not None:
            plan.set_launch(*launch)
    elif tune:
        ts = plan.tune(u, f, D["xp"], D["up"], D["wp"], mask=mask)
        plan.check("tune")
        tuned = ts["tile"]
        log(f"bench: {precision} tuned tile {tuned}, {ts['block']} threads, "
            f"{'persistent' if ts['persistent'] else 'one workgroup per tile'}")

    def step(graph):
        r = plan.pairs(D["xp"], D["radius"], D["mass"], D["up"], D["wp"], prev=prev, mask=mask,
                       **caps)
        plan.forcing(u, f, D["xp"], D["up"], D["wp"], mask=mask, resid=resid, graph=graph)
        return r

    def timed(graph, prof):
        # a graph call captures on its first use: keep that out of the timing
        for _ in range(max(warmup, 1) if graph else warmup):
            step(graph)
        torch.cuda.synchronize()
        plan.check("warmup")
        if prof:
            plan.profile(True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        for _ in range(steps):
            step(graph)
        stop.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        plan.check("timed steps")
        st = plan.stats() if prof else None
        if prof:
            plan.profile(False)
        return start.elapsed_time(stop) / steps, wall, st

    # eager calls with per-kernel events (roofline), then the same steps
    # with the forcing call replayed as one HIP graph
    ms_prof, wall, st = timed(False, profile)
    ms_graph, _, _ = timed(True, False)
    # the same eager steps without the per-kernel events (the step's time)
    ms, wall, _ = timed(False, False)

    # the particle solver's fluid integrals and the mean IBM force, timed on
    # their own (not part of the step)
    def time_call(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    extras = dict(
        particle_integrals_ms=time_call(lambda: plan.particle_integrals(u, D["xp"], D["radius"])),
        grid_mean_ms=time_call(lambda: plan.grid_mean(f)))
    plan.check("integrals")
    # reverse-mode derivative of one forcing call (replay + adjoint passes)
    g_S = torch.ones((3, case.np_), dtype=f64, device=dev)
    extras["backward_ms"] = time_call(
        lambda: plan.forcing_backward(u, D["xp"], D["up"], D["wp"], mask, f, None, g_S, None),
        reps=2)
    plan.check("backward")
    # particle sub-stepping over the step's contact lists: Hertz law with
    # ACTM coefficients, the paper's 15 sub-steps of dt/15 (90 stage launches)
    prm = dict(case.params)
    prm["normal_model"] = 1
    plan.set_params(prm)
    xs, us, ws = D["xp"].clone(), D["up"].clone(), D["wp"].clone()
    hist, whist = res["hist"].clone(), res["whist"].clone()
    n_sub = 15
    extras["substeps_ms"] = time_call(
        lambda: plan.particle_substeps(float(prm["dt"]), n_sub, xs, us, ws, D["radius"],
                                       D["mass"], res, hist, whist, want_forces=False), reps=5)
    extras["substeps_n_sub"] = n_sub
    plan.check("substeps")
    plan.set_params(case.params)
    # the other steps of a fluid Runge-Kutta stage on the same grid: the
    # predictor (stencils), the implicit viscous step and the projection
    # (FP64 FFT / tridiagonal solves)
    if precision == "f32":
        uc = u.clone()
        P = torch.zeros(u.shape[1:], dtype=u.dtype, device=dev)
        Nb = torch.zeros_like(u)
        ut = torch.empty_like(u)
        lapnu = torch.empty_like(u)
        dt = 1.0
        extras["predictor_ms"] = time_call(
            lambda: plan.fluid_predictor(uc, Nb, P, dt, 8.0 / 15.0, 0.0, u_out=ut, lapnu=lapnu),
            reps=3)
        extras["helmholtz_ms"] = time_call(lambda: plan.fluid_helmholtz(ut, lapnu, P, dt, 0.0),
                                           reps=3)
        extras["project_ms"] = time_call(lambda: plan.project(uc, P, 0.0, want_phi=False), reps=3)
        plan.check("fluid stage")
        del uc, P, Nb, ut, lapnu
    if not profile:
        st = plan.stats()
    out = dict(ms_per_step=ms, ms_per_step_profiled=ms_prof, ms_per_step_graph=ms_graph,
               wall_s=wall, stats=st, n_iter=n_iter,
               extras=extras,
               resid=resid.cpu().numpy().tolist(), tile=tuned or list(plan.stats()["tile"]),
               block=plan.stats()["block"], persistent=plan.stats()["persistent"])
    del u, f, D
    plan.close()
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(torch, gib: float = 2.0, reps: int = 5) -> float:
    """Achievable HBM bandwidth for reference: a device-to-device copy of a
    2 GiB buffer, (read + written bytes) / time, best of a few."""
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 4 / best / 1e9


def cpu_substeps(case, pl):
    """The oracle's sub-stepping of one call (bed particles, Hertz law, 15
    sub-steps) on the host, for scale; pl = the oracle's lists."""
    import oracle
    prm = dict(case.params)
    prm["normal_model"] = 1
    ref = oracle.pair_forces(case, pl, params=prm)
    t0 = time.perf_counter()
    oracle.particle_substeps(case, pl, float(prm["dt"]), 15, hist=ref["hist"], whist=ref["whist"],
                             params=prm)
    return (time.perf_counter() - t0) * 1e3


def cpu_baseline(case, mask_np):
    """Oracle (plain FP64, single thread) timed on one forcing pass over all
    markers of the workload on its full grid."""
    import numpy as np
    import oracle
    u0 = case.field().numpy()
    case.u0 = u0
    t0 = time.perf_counter()
    oracle.forcing(case, mask=mask_np, n_iter=1, final_resid=False)
    t = time.perf_counter() - t0
    n_act = int(mask_np.sum()) if mask_np is not None else case.nm
    case.u0 = None
    del u0
    return dict(value=n_act / t, unit="marker-updates/s", cores=1, kind="oracle",
                sample=f"1 forcing pass over all {n_act} active markers of the workload on its "
                       f"full {case.n[0]}x{case.n[1]}x{case.n[2]} grid ({t:.1f} s)",
                host=host_cpu())


def host_cpu():
    """The host the CPU baseline ran on: threads this process may use and the
    processor model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        threads = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        threads = os.cpu_count()
    return dict(threads_available=threads, cpu_model=model)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="polydisperse_bed_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shape")
    ap.add_argument("--tile", default=None,
                    help="FP32 tile shape tx,ty,tz instead of tuning (for counter runs)")
    ap.add_argument("--launch", default=None,
                    help="with --tile: threads per workgroup and persistence, e.g. 256,0")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference kernel for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (--gpus 1); the forcing loop is not "
              "sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2109_03972_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied 1 GiB device-to-device (counter calibration)")
        del src, dst
    copy_gbs = copy_bandwidth(torch)
    log(f"bench: device copy {copy_gbs:.0f} GB/s (read + write)")
    log(f"bench: generating {args.workload}")
    case = synth.make_case(args.workload, lazy_field=True)
    log(f"bench: {case.np_} particles, {case.nm} markers, grid {case.n}")

    log("bench: FP32 run")
    tile = None if args.tile is None else [int(v) for v in args.tile.split(",")]
    launch = None if args.launch is None else [int(v) for v in args.launch.split(",")]
    r32 = run_gpu(case, "f32", args.steps, args.warmup, tune=not args.no_tune, tile=tile,
                  launch=launch)
    st = r32["stats"]
    n_act, shell, n_iter = int(st["n_active"]), int(st["shell_nodes"]), r32["n_iter"]
    value = n_act * n_iter / (r32["ms_per_step"] * 1e-3)
    nodes = int(case.n[0]) * int(case.n[1]) * int(case.n[2])
    value_graph = n_act * n_iter / (r32["ms_per_step_graph"] * 1e-3)
    km, kn = st["kernel_ms"], st["kernel_launches"]
    steps_done = args.steps
    per_launch = {k: (km[k] / kn[k] if kn[k] else None) for k in km}
    # roofline of the forcing pass: one interpolation and one spreading launch
    # (n_iter of each per step), algorithmic bytes over their average durations
    halo = int(st["halo_entries"])
    t_pass = per_launch["interp"] + per_launch["spread"]
    b_pass = pass_bytes(4, n_act, shell)
    achieved = b_pass / (t_pass * 1e-3) / 1e9
    tr = [measured_traffic(args.workload, k, r32["tile"]) for k in ("interp", "spread")]
    traffic = None if None in tr else tr[0] + tr[1]
    roof = dict(bound="hbm", kernel="k_interp + k_spread (one forcing pass)",
                achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                bytes_per_pass=b_pass, ms_per_pass=t_pass,
                ms_per_launch=dict(interp=per_launch["interp"], spread=per_launch["spread"]),
                design_bytes=dict(interp=design_bytes("interp", 4, n_act, shell, halo),
                                  spread=design_bytes("spread", 4, n_act, shell, halo)),
                copy_GBs=round(copy_gbs, 1))
    if traffic is not None:
        roof["traffic_GBs"] = round(traffic / (t_pass * 1e-3) / 1e9, 1)
    if args.workload != "polydisperse_bed_512":
        roof["note"] = ROOFLINE_NOTES.get(args.workload, "")
    log(f"bench: FP32 {r32['ms_per_step']:.3f} ms/step, {value:.3e} marker-updates/s")

    fp64 = None
    if not args.no_fp64:
        log("bench: FP64 run")
        r64 = run_gpu(case, "f64", args.steps, args.warmup, tune=not args.no_tune)
        v64 = n_act * n_iter / (r64["ms_per_step"] * 1e-3)
        fp64 = dict(value=v64, ms_per_step=r64["ms_per_step"], speedup_f32_over_f64=value / v64,
                    ms_per_step_graph=r64["ms_per_step_graph"], tile=r64["tile"],
                    kernel_ms_per_launch={k: (r64["stats"]["kernel_ms"][k] / n if n else None)
                                          for k, n in r64["stats"]["kernel_launches"].items()})

    cpu = None
    cpu_sub_ms = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        import oracle
        pl = oracle.pairs(case)
        mask_np = oracle.marker_mask(case, pl)
        cpu = cpu_baseline(case, mask_np)
        cpu_sub_ms = cpu_substeps(case, pl)

    line = dict(
        metric="marker-updates/s per forcing iter (FP32 batched vs FP64) at stated tol; HBM GB/s",
        value=value, unit="marker-updates/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=r32["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32", data="synthetic",
        config=dict(workload=args.workload, grid=list(case.n), particles=case.np_,
                    markers=case.nm, active_markers=n_act, shell_nodes=shell, n_iter=n_iter,
                    precision="FP32 grid/delta, FP64 geometry, particle sums and pair pass",
                    step="pair pass + marker geometry + n_iter forcing passes",
                    tile=r32["tile"], block=r32["block"], persistent=r32["persistent"]),
        roofline=roof, cpu_baseline=cpu, fp64=fp64,
        kernel_ms_per_launch=per_launch,
        graph=dict(ms_per_step=r32["ms_per_step_graph"], value=value_graph),
        ms_per_step_with_kernel_events=r32["ms_per_step_profiled"],
        particle_integrals=dict(
            ms=r32["extras"]["particle_integrals_ms"],
            note="level-set fluid integrals over all particles (one call, FP32 grid, "
                 "FP64 geometry and sums); not part of the step"),
        grid_mean_ms=r32["extras"]["grid_mean_ms"],
        fluid_stage=dict(predictor_ms=r32["extras"]["predictor_ms"],
                         helmholtz_ms=r32["extras"]["helmholtz_ms"],
                         project_ms=r32["extras"]["project_ms"],
                         roofline={k: dict(
                             bytes=fluid_bytes(k, 4, nodes, not case.periodic[2]),
                             achieved_GBs=round(fluid_bytes(k, 4, nodes, not case.periodic[2])
                                                / (r32["extras"][k + "_ms"] * 1e-3) / 1e9, 1),
                             frac=round(fluid_bytes(k, 4, nodes, not case.periodic[2])
                                        / (r32["extras"][k + "_ms"] * 1e-3) / 1e9
                                        / HBM_PEAK_GBS, 4))
                             for k in ("predictor", "helmholtz", "project")},
                         note="the collocated solver's other steps of one Runge-Kutta stage on "
                              "the workload's grid (FP32 fields): ibmx_fluid_predictor, "
                              "ibmx_fluid_helmholtz and ibmx_project (FP64 FFT/tridiagonal "
                              "solves); not part of the step"),
        substeps=dict(ms=r32["extras"]["substeps_ms"], n_sub=r32["extras"]["substeps_n_sub"],
                      particles=case.np_, cpu_oracle_ms=cpu_sub_ms,
                      note="ibmx_particle_substeps of one time step (Hertz/ACTM contacts, "
                           "15 three-stage sub-steps, FP64) on the step's contact lists; "
                           "not part of the step"),
        backward=dict(ms=r32["extras"]["backward_ms"],
                      note="ibmx_forcing_backward of one call (FP32): binning, replay of the "
                           "passes with the Jacobians, adjoint passes; not part of the step"),
        pass_rate=n_act * n_iter / (sum(km[k] for k in ("interp", "spread")) / steps_done
                                    * 1e-3),
        # the call's rate per pass with its once-per-call work other than the
        # binning (f_tot, final residual, particle sums) spread over the
        # passes: N / ((graph step - pair pass - binning) / n_iter)
        pass_rate_call=n_act * n_iter / ((r32["ms_per_step_graph"] - per_launch["pairs"]
                                          - per_launch["geometry"]) * 1e-3),
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
