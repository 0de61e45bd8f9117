#!/usr/bin/env python3
"""Throughput of the fused D2Q37 step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole hot path (pull streaming, wall rows,
force-shifted BGK collide) over the lattice, in the fused kernel, with the
populations already resident in HBM.  The default workload is the FP64
three-layer Rayleigh-Taylor lattice of one GPU's production share,
4096 x 12288 sites.  Prints one JSON line with MLUPS, the HBM roofline of the
step kernel (algorithmic bytes / kernel time, timed with HIP events on the
stream the kernel runs on, plus the HBM bytes of the committed counter
summary while it matches the kernel code) and the CPU oracle timed on the
host cores (one process per core, each on its own strip of the lattice).
Also: the fused step against streaming alone on the same buffers, in
interleaved windows; the same lattice in FP32 deviation storage (also with
the collision in double, LBM_COLLIDE_F64), with the diffuse
(mass-conserving) walls and on a single buffer, both precisions;
streaming alone in pull and in push form; the adjoint rollouts' cost
relative to a plain forward and the adjoint step's bandwidth (gather form,
the push form's time beside it).  Before the timed steps each lattice keeps
the fastest of a few allocations of its buffers (Lattice.tune_placement,
every trial reported; --no-placement times the first).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q37 MLUPS (fwd FP64 vs FP32) + % HBM roofline; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
Q = 37
STEP_SRC = os.path.join(ROOT, "paper_1405_1253_amd", "csrc", "step.hip")
PROFILES = os.path.join(ROOT, "profiles")


def bytes_per_site(precision):
    return 2 * Q * (8 if precision == "f64" else 4)      # 37 reads + 37 writes


def code_hash(names):
    """sha256 (16 hex digits) of the named kernel sources with comments and
    blank lines removed: a counter summary stays valid across comment edits
    and is invalidated by any change to the code."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1405_1253_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for line in text.splitlines():
            line = line.strip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def step_source_hash():
    return code_hash(("step.hip", "common.h", "lattice_constants.h"))


def adjoint_source_hash():
    return code_hash(("adjoint.hip", "common.h", "lattice_constants.h"))


def measured_adjoint_traffic(workload):
    """HBM bytes per all-float adjoint launch from the committed counter
    summary, if it was taken on the current adjoint source (else None)."""
    path = os.path.join(PROFILES, f"adjoint_f32_{workload.replace('_adj', '')}_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"adjoint_source_sha:\s*(\w+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != adjoint_source_hash():
        return None
    return float(m_b.group(1))


def measured_traffic(workload, precision):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(PROFILES, f"step_{precision}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"kernel_source_sha:\s*(\w+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != step_source_hash():
        return None
    return float(m_b.group(1))


def time_steps(lat, steps, warmup):
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def interleaved_windows(lat, windows=5, k=20):
    """The fused step and streaming alone (LBM_NO_COLLIDE) on the same two
    buffers of ``lat``, alternating windows of ``k`` launches (HIP events on
    the current stream): median, min and max ms per launch of each, and the
    ratio of the medians (the cost of the collision over the pattern's own)."""
    import statistics

    import torch
    from paper_1405_1253_amd import abi
    p = lat.params
    p_nc = abi.make_params(p.lx, p.lz, p.tau, p.g, p.precision, p.flags | abi.NO_COLLIDE)
    stream = torch.cuda.current_stream()

    def window(params):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            abi.lbm_step(params, lat.ghost, lat.buf[lat.cur], lat.buf[1 - lat.cur])
            lat.cur = 1 - lat.cur
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / k

    window(p_nc)
    t = {"fused": [], "streaming": []}
    for _ in range(windows):
        t["fused"].append(window(p))
        t["streaming"].append(window(p_nc))
    out = {}
    for key, ts in t.items():
        out[f"{key}_ms"] = {"median": round(statistics.median(ts), 4), "min": round(min(ts), 4),
                            "max": round(max(ts), 4)}
    out["fused_over_streaming"] = round(statistics.median(t["fused"]) / statistics.median(t["streaming"]), 4)
    out["windows"], out["launches_per_window"] = windows, k
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_strip_worker(name, x0, columns, min_seconds, max_steps, barrier, out):
    """One host core: the oracle on its own strip of `columns` full-height
    columns of the workload (periodic across the strip), one BLAS/OpenMP
    thread, stepped for at least `min_seconds` once every worker is ready."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import lbm as O
    from paper_1405_1253_amd.workload import WORKLOADS, draw_modes
    wl = WORKLOADS[name]
    m = draw_modes(wl.seed)
    with threadpool_limits(limits=1):
        p_full = O.Params(wl.lx, wl.lz, wl.tau, wl.g)
        desc = O.RT3(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase)
        f, ghost = O.init_rt3(p_full, desc, m.amp, columns=np.arange(x0, x0 + columns))
        p = O.Params(columns, wl.lz, wl.tau, wl.g)
        barrier.wait()
        steps, t0 = 0, time.perf_counter()
        while steps < max_steps and (steps < 2 or time.perf_counter() - t0 < min_seconds):
            f = O.step(f, ghost, p)
            steps += 1
        dt = time.perf_counter() - t0
    out.put((x0, steps, dt, columns * wl.lz))


def cpu_baseline(wl, columns=32, min_seconds=12.0, max_steps=64, max_workers=16):
    """The oracle on the host cores: one process per core (at most
    ``max_workers``, the host share of one GPU), each stepping its own strip
    of `columns` full-height columns of the same workload, all at once.  The
    rate is the sum of the workers' site updates per second.  Runs before
    anything touches the GPU (the workers are started by spawning fresh
    interpreters)."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), max_workers, max(1, wl.lx // columns))
    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(cores), ctx.Queue()
    procs = [ctx.Process(target=_oracle_strip_worker,
                         args=(wl.name, i * columns, columns, min_seconds, max_steps, barrier, out))
             for i in range(cores)]
    for pr in procs:
        pr.start()
    res = [out.get() for _ in procs]
    for pr in procs:
        pr.join()
        if pr.exitcode != 0:
            raise RuntimeError(f"oracle worker exited with {pr.exitcode}")
    rate = sum(steps * sites / dt for _, steps, dt, sites in res)
    steps = sorted(r[1] for r in res)
    secs = max(r[2] for r in res)
    return {"value": rate / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"{cores} processes, one per core, each stepping its own {columns} x {wl.lz} column "
                      f"strip of the {wl.name} lattice ({steps[0]}-{steps[-1]} steps, {secs:.1f} s; numpy "
                      f"FP64 oracle, one thread per process); rate = sum of the processes' rates"}


def adjoint_ratio(name, budget_bytes=None, warm=True):
    """Wall time of the rollout's forward pass (with checkpoints and stored
    moments) and of its backward pass (recomputation + adjoint sweep + init
    VJP), against a plain forward of the same steps on the rollout's own
    state buffers (so that both run on the same memory): the plain forward
    is timed twice after a warm-up (the mean is the reference), the rollout
    once (after one warm-up run of every phase if ``warm``).  Also the
    adjoint step alone (20 launches on the rollout's buffers, HIP events)
    with its HBM bandwidth at 37 x 2 adjoint elements + 4 moments per site."""
    import torch
    from paper_1405_1253_amd import abi
    from paper_1405_1253_amd.rollout import Rollout, RolloutConfig
    from paper_1405_1253_amd.workload import WORKLOADS, draw_modes
    wl = WORKLOADS[name]
    m = draw_modes(wl.seed)
    kw = {} if budget_bytes is None else {"moment_budget_bytes": budget_bytes}
    amp = torch.as_tensor(m.amp, device="cuda")

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    r = Rollout(RolloutConfig.from_workload(wl, m, **kw))
    if warm:
        r.forward(amp)
        r.backward()
    r.recomputed_steps = 0
    t_fwd, _ = timed(lambda: r.forward(amp))
    t_bwd, grad = timed(r.backward)

    def plain_forward(n):
        for i in range(n):
            abi.lbm_step(r.params, r.ghost, r.buf[i % 2], r.buf[1 - i % 2])

    abi.lbm_init_rt3(r.params, r.desc, r.amp, r.buf[0], r.ghost)
    plain_forward(wl.steps if warm else 200)             # warm-up
    t_plain = []
    for _ in range(2):
        abi.lbm_init_rt3(r.params, r.desc, r.amp, r.buf[0], r.ghost)
        t_plain.append(timed(lambda: plain_forward(wl.steps))[0])
    plain = sum(t_plain) / len(t_plain)

    # the adjoint step alone, on the rollout's buffers: the gather form the
    # rollout uses, and the push form for comparison
    mom = r.kept[0] if r.keep else r.segbuf[0]
    stream = torch.cuda.current_stream()

    def adj_time(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn(0)
        e0.record(stream)
        for i in range(20):
            fn(i)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 20 / 1e3

    t_push = adj_time(lambda i: abi.lbm_adjoint_step(r.params, r.ghost, mom, r.lam[i % 2], r.lam[1 - i % 2]))
    t_adj = (t_push if r.form == "push" else
             adj_time(lambda i: abi.lbm_adjoint_gather(r.params, r.ghost, mom, r.lam[i % 2], r.lam[1 - i % 2])))
    site_bytes = 2 * abi.Q * r.lam[0].element_size() + 4 * mom.element_size()
    adj_gbs = site_bytes * wl.lx * wl.lz / t_adj / 1e9
    out = {"workload": name, "steps": wl.steps, "plain_forward_s": [round(t, 4) for t in t_plain],
           "rollout_forward_s": round(t_fwd, 4), "backward_s": round(t_bwd, 4),
           "backward_over_plain_forward": round(t_bwd / plain, 3),
           "gradient_over_plain_forward": round((t_fwd + t_bwd) / plain, 3),
           "recomputed_steps": r.recomputed_steps, "moments_kept": r.keep,
           "ckpt_every": r.ckpt_every, "state_checkpoints": len(r.ckpt),
           "moments_dtype": str(mom.dtype).replace("torch.", ""),
           "adjoint_form": r.form, "adjoint_step_ms": round(t_adj * 1e3, 4),
           "adjoint_push_step_ms": round(t_push * 1e3, 4),
           "adjoint_step_over_forward_step": round(t_adj / (plain / wl.steps), 3),
           "adjoint_hbm_gbs": round(adj_gbs, 1), "adjoint_frac": round(adj_gbs / HBM_PEAK_GBS, 4),
           "adjoint_traffic": (measured_adjoint_traffic(name)
                               if r.lam[0].dtype == torch.float32 and mom.dtype == torch.float32 else None),
           "grad_finite": bool(torch.isfinite(grad).all().item())}
    del r, mom
    torch.cuda.empty_cache()
    return out


def propagate_pull_vs_push(wl, launches=20, rounds=2):
    """Streaming alone, in the two forms Sec. III.B compares for the
    propagate kernel: pull = lbm_step with LBM_NO_COLLIDE (reads shifted by
    -e_l, aligned writes); push = lbm_adjoint_step with LBM_NO_COLLIDE, which
    moves each input element along -e_l (aligned reads, shifted writes).
    Both move 37 + 37 elements per site; HIP events on the current stream,
    the two forms interleaved ``rounds`` times (means reported)."""
    import torch
    from paper_1405_1253_amd import abi
    stream = torch.cuda.current_stream()
    out = {}
    for prec in ("f64", "f32dev"):
        f32 = prec != "f64"
        pr = abi.F32_DEV if f32 else abi.F64
        p_pull = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, pr, abi.NO_COLLIDE)
        p_push = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, pr, abi.NO_COLLIDE | (abi.ADJ_F32 if f32 else 0))
        dt = torch.float32 if f32 else torch.float64
        buf = [torch.rand(abi.population_elems(p_pull), dtype=dt, device="cuda") for _ in range(2)]
        gh = torch.rand((2, 3, abi.Q), dtype=dt, device="cuda")

        def timed(fn):
            for i in range(4):
                fn(i)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(launches):
                fn(i)
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / launches / 1e3

        t = {"pull": [], "push": []}
        for _ in range(rounds):
            t["pull"].append(timed(lambda i: abi.lbm_step(p_pull, gh, buf[i % 2], buf[1 - i % 2])))
            t["push"].append(timed(lambda i: abi.lbm_adjoint_step(p_push, gh, None, buf[i % 2], buf[1 - i % 2])))
        del buf, gh
        torch.cuda.empty_cache()
        nbytes = bytes_per_site(prec) * wl.lx * wl.lz
        for form, ts in t.items():
            sec = sum(ts) / len(ts)
            out[f"{prec}_{form}_ms"] = round(sec * 1e3, 4)
            out[f"{prec}_{form}_hbm_gbs"] = round(nbytes / sec / 1e9, 1)
        out[f"{prec}_pull_over_push"] = round(out[f"{prec}_pull_hbm_gbs"] / out[f"{prec}_push_hbm_gbs"], 3)
    return out


def copy_calibration(nbytes=4 << 30, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "copy_calibration_bytes_written": nbytes,
                      "launches": reps}), flush=True)


def adjoint_counter_run(launches=6):
    """A short sequence for the HBM counters of the adjoint step: at the
    2048 x 6144 float rollout's shape, ``launches`` all-float adjoint steps in
    gather form (lbm_adjoint_gather: float buffers and moments), then
    ``launches`` streaming-only ones (S^T alone)."""
    import torch
    from paper_1405_1253_amd import abi
    from paper_1405_1253_amd.workload import WORKLOADS, draw_modes
    wl = WORKLOADS["rt3_2048x6144_adj"]
    m = draw_modes(wl.seed)
    base = abi.F32_DEV
    p_fwd = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, base, abi.MOM_F32)
    p_adj = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, base, abi.MOM_F32 | abi.ADJ_F32)
    p_str = abi.make_params(wl.lx, wl.lz, wl.tau, wl.g, base, abi.NO_COLLIDE | abi.ADJ_F32)
    shape = (abi.population_elems(p_fwd),)
    f = torch.empty(shape, dtype=torch.float32, device="cuda")
    gh = torch.empty((2, 3, abi.Q), dtype=torch.float32, device="cuda")
    abi.lbm_init_rt3(p_fwd, abi.RT3Desc(wl.t_d, wl.t_m, wl.t_u, wl.width, m.k, m.phase),
                     torch.as_tensor(m.amp, device="cuda"), f, gh)
    mom = torch.empty((4, wl.lx, wl.lz), dtype=torch.float32, device="cuda")
    abi.lbm_step(p_fwd, gh, f, torch.empty_like(f), mom)
    gen = torch.Generator(device="cuda").manual_seed(wl.seed)
    lam = [torch.randn(shape, dtype=torch.float32, device="cuda", generator=gen), torch.empty_like(f)]
    for i in range(launches):
        abi.lbm_adjoint_gather(p_adj, gh, mom, lam[i % 2], lam[1 - i % 2])
    for i in range(launches):
        abi.lbm_adjoint_gather(p_str, gh, None, lam[i % 2], lam[1 - i % 2])
    torch.cuda.synchronize()
    print(json.dumps({"adjoint_counter_run": wl.name, "sites": wl.lx * wl.lz,
                      "launches_all_float": launches, "launches_streaming_only": launches}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="rt3_4096x12288")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-placement", action="store_true",
                    help="time the lattice's first allocation instead of the fastest of several")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for the HBM counters)")
    ap.add_argument("--adjoint-counter-run", action="store_true",
                    help="only run a short adjoint sequence (for the HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.adjoint_counter_run:
        adjoint_counter_run()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU x-slab "
              "decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    from paper_1405_1253_amd.workload import WORKLOADS
    wl = WORKLOADS[args.workload]
    # the host-core oracle first: its worker processes start before this
    # process initialises the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)

    import torch
    from paper_1405_1253_amd import abi
    from paper_1405_1253_amd.runtime import Lattice

    abi.load()
    lat = Lattice.from_workload(wl)
    placement = None if args.no_placement else lat.tune_placement()
    secs, wall = time_steps(lat, args.steps, args.warmup)
    lat.sums()                                       # raises on a diverged state
    sites = wl.lx * wl.lz
    ms = secs / args.steps * 1e3
    mlups = sites * args.steps / secs / 1e6
    bpl = bytes_per_site(wl.precision) * sites
    achieved = bpl / (secs / args.steps) / 1e9
    traffic = measured_traffic(wl.name, wl.precision)
    windows = None if args.no_secondary else interleaved_windows(lat)
    lat.sums()
    del lat
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if wl.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "lx": wl.lx, "lz": wl.lz, "sites": sites,
                   "precision": wl.precision, "tau": wl.tau, "g": wl.g},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_launch": bpl,
                     "kernel": "lbm::step_kernel", "wall_s": round(wall, 3)},
    }
    if placement is not None:
        # ms per step of each allocation tried before the timed steps (the
        # first is the lattice's own); the timed steps run on the fastest
        out["placement_trials_ms"] = placement
    if windows is not None:
        out["fused_vs_streaming"] = windows
    if not args.no_secondary and wl.precision == "f64":
        # the same lattice in FP32 deviation storage (float collision, and
        # double collision with LBM_COLLIDE_F64), both precisions with the
        # diffuse (mass-conserving) wall rule, and both on a single buffer
        # (in-place steps come in pairs: step counts rounded up to even)
        sec = {}
        for suffix, key, flags in (("_f32", "f32dev", 0), ("_f32", "f32dev_collide_f64", abi.COLLIDE_F64),
                                   ("_diffuse", "diffuse_f64", 0), ("_f32_diffuse", "diffuse_f32dev", 0),
                                   ("_inplace", "inplace_f64", 0), ("_f32_inplace", "inplace_f32dev", 0)):
            w2 = WORKLOADS.get(wl.name + suffix)
            if w2 is None:
                continue
            n2 = args.steps + (args.steps % 2 if w2.inplace else 0)
            lat = Lattice.from_workload(w2, flags=flags)
            pl2 = None if args.no_placement else lat.tune_placement()
            s2, _ = time_steps(lat, n2, args.warmup + (args.warmup % 2 if w2.inplace else 0))
            if pl2 is not None:
                sec[f"{key}_placement_trials_ms"] = pl2
            if key == "f32dev":
                out["fused_vs_streaming_f32dev"] = interleaved_windows(lat)
            lat.sums()
            del lat
            torch.cuda.empty_cache()
            a2 = bytes_per_site(w2.precision) * sites / (s2 / n2) / 1e9
            sec.update({f"{key}_mlups": round(sites * n2 / s2 / 1e6, 1),
                        f"{key}_ms_per_step": round(s2 / n2 * 1e3, 4),
                        f"{key}_hbm_gbs": round(a2, 1),
                        f"{key}_frac": round(a2 / HBM_PEAK_GBS, 4)})
        out["secondary"] = sec
        out["propagate_pull_vs_push"] = propagate_pull_vs_push(wl)
    if not args.no_adjoint:
        c4 = WORKLOADS["rt3_512x1536_adj"]
        out["adjoint"] = [adjoint_ratio("rt3_512x1536_adj"),
                          # the same rollout with moments for one 100-step segment only: the
                          # backward sweep recomputes each segment from its state checkpoint
                          adjoint_ratio("rt3_512x1536_adj", c4.ckpt_every * 4 * c4.lx * c4.lz * 8),
                          adjoint_ratio("rt3_512x1536_adj_diffuse"),
                          adjoint_ratio("rt3_2048x6144_adj", 232 << 30, warm=False)]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
