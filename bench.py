#!/usr/bin/env python3
"""Benchmark of the lattice-Boltzmann + momentum-exchange step on one MI355X.

Headline workload: the D3Q19 duct 256x128x128 with a static sphere of
radius 16 (interpolated bounce-back, force and torque on the sphere by
momentum exchange every step), FP32 storage with FP64 force accumulation --
the configuration whose two population buffers (2 x 411 MB) exceed the
256 MB last-level cache, so that the stream-collide kernel is measured
against HBM. A step is the whole hot path: the boundary rule and momentum
exchange at the body, and the fused stream-collide with the domain faces.

Prints ONE JSON line (rank 0). `value` = million lattice-node updates per
second over the timed steps (every node of the box counts). `roofline` is
the stream-collide kernel: algorithmic bytes (2 Q s per active node) over its
average duration from HIP events around its launches in the timed region
(every launch while the window is short), against 8 TB/s, with the HBM
traffic of its counter runs when they were taken on the current kernel
source. `cpu_baseline` is the FP64 CPU oracle on a bounded sample of the same
workload. Secondary lines: the same duct in FP16-shifted storage and with Zou-He
faces (quasi-incompressible), the oscillating-cylinder channel 2000x800
(MALL-resident), a 32-body suspension in a 2048x1024 channel, a 4.8 GB channel
(8192x8192), the force-noise comparison of the ME forms and refill rules, the
paper's sedimenting disc moved by each force form, the 64-domain batch and
the served request stream, each with its configuration stated.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS incl. ME force/torque; batched solves/s + p99 latency vs plain"
HEADLINE = "duct_sphere_f32"
MIN_TIMED = 20  # the roofline needs at least this many timed launches (or every launch of a shorter run)


def workload(name):
    import lbm_workloads as W
    if name == "channel_oscillating_f32":
        return W.channel_oscillating_f32(scale=1)
    if name == "duct_sphere_f32":
        return W.duct_sphere(scale=1, storage="f32")
    if name == "duct_sphere_f16":
        return W.duct_sphere(scale=1, storage="f16")
    if name == "channel_cylinder_f64":
        return W.channel_cylinder_f64()
    if name == "channel_large_f32":
        return W.channel_large(storage="f32")
    if name == "suspension_f32":
        return W.suspension("f32")
    if name == "duct_sphere_zouhe_f32":
        w = W.with_changes(W.duct_sphere(scale=1, storage="f32"), eq="heluo",
                           faces=(W.ZOUHE_VELOCITY, W.ZOUHE_PRESSURE, W.WALL, W.WALL, W.WALL, W.WALL))
        w["name"] = "duct_sphere_zouhe_heluo_f32_256x128x128"
        return w
    if name == "sedimenting_disc_f32":
        return W.sedimenting_disc(ratio=1.03, storage="f32")
    raise SystemExit(f"unknown workload {name}")


def active_nodes(w):
    """nodes the stream-collide kernel updates (all but the wall layers)"""
    n = [w["nx"], w["ny"], w["nz"] if w["lattice"] == "D3Q19" else 1]
    faces = w["faces"]
    dims = 2 if w["lattice"] == "D2Q9" else 3
    tot = 1
    for a in range(3):
        k = n[a]
        if a < dims:
            k -= (faces[2 * a] == 1) + (faces[2 * a + 1] == 1)
        tot *= k
    return tot


def bytes_per_node(w):
    q = 9 if w["lattice"] == "D2Q9" else 19
    s = {"f64": 8, "f32": 4, "f16": 2}[w["storage"]]
    return 2 * q * s


def measured_traffic(name, symbol):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{symbol}_{name}_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    from paper_1407_4524_amd.hbm_traffic import kernel_source_hash
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


KERNEL_SYMBOLS = {"stream_collide": "k_stream_collide", "body": "k_links/k_body_step",
                  "near_box": "k_stream_collide (near box)"}


def timing_period(steps):
    """time every launch while the window is short (up to 255 steps); beyond
    it every n-th, at least 128 launches of each kind: a launch timed with
    start/stop events costs the step about 4.5 us on the GPU (the duct: 119.4
    us per step with every launch timed against 110.5 us untimed), which the
    whole-step rate should not carry"""
    return max(1, steps // 128)


# lbm_domain_desc.split_schedule of each --schedule choice
SCHEDULES = {"auto": 0, "split": 1, "plain": -1}


def run_gpu(name, steps, warmup, split_schedule=0):
    import torch
    from paper_1407_4524_amd import Domain
    w = workload(name)
    stream = torch.cuda.Stream()  # the domain's own stream, as a serving process would give it
    with torch.cuda.stream(stream):
        dom = Domain.from_spec(w, split_schedule=split_schedule)
    dom.step(warmup)
    dom.synchronize()
    every = timing_period(steps)
    dom.timing_enable(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps)
    dom.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    kernels = {}
    for k in ("stream_collide", "near_box", "body"):
        kms, timed, nodes, issued = dom.timing_read(k, issued=True)
        if not timed:
            continue
        avg_s = kms / timed / 1e3
        per_step = issued / steps
        entry = dict(symbol=KERNEL_SYMBOLS[k], launches_per_step=round(per_step, 3), avg_us=round(avg_s * 1e6, 3),
                     share_of_step=round(avg_s * per_step / (sec / steps), 4), timed_launches=timed,
                     timing_period=every)
        if nodes:
            algo = nodes * bytes_per_node(w) / timed  # algorithmic bytes per launch
            entry.update(algorithmic_bytes_per_launch=round(algo), achieved_gbs=round(algo / avg_s / 1e9, 1),
                         node_fraction=round(nodes / timed / active_nodes(w), 4))
        kernels[k] = entry
    # the timed launch of a domain stepped as its own one-member batch updates
    # the nodes away from its bodies; a roofline stands for the sweep only
    # while that is nearly every node (not for the suspension, whose bodies'
    # box holds most of the domain)
    kd = kernels.get("stream_collide")
    need = min(MIN_TIMED, steps)
    if kd and kd["timed_launches"] >= need and kd.get("node_fraction", 0.0) >= 0.9:
        roofline = dict(bound="hbm", achieved=kd["achieved_gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(kd["achieved_gbs"] / HBM_PEAK_GBS, 4),
                        traffic=measured_traffic(w["name"], kd["symbol"]), kernel=kd["symbol"],
                        avg_us=kd["avg_us"], timed_launches=kd["timed_launches"],
                        algorithmic_bytes_per_launch=kd["algorithmic_bytes_per_launch"])
    else:
        roofline = None  # too few timed launches to stand for the kernel
    ft = dom.force_torque(0, dom.t - 1, 1)[0] if w["bodies"] else [0.0] * 6
    cells = w["nx"] * w["ny"] * (w["nz"] if w["lattice"] == "D3Q19" else 1)
    footprint = dom.footprint()
    dom.close()
    return dict(w=w, cells=cells, seconds=sec, ms_per_step=sec / steps * 1e3, mlups=cells * steps / sec / 1e6,
                kernels=kernels, roofline=roofline, footprint_bytes=footprint,
                last_force_torque=[float(x) for x in ft])


def copy_ceiling(nbytes, reps=20, variant=0):
    """The library's hand-written copy kernel (lbm_copy) moving nbytes per
    launch (half read, half written), timed with HIP events on the current
    stream: the copy ceiling at a kernel's footprint. Torch's own copy of the
    same bytes is reported beside it."""
    import torch
    from paper_1407_4524_amd import lbm
    half = max(16, nbytes // 2 // 16 * 16)
    a = torch.empty(half, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)

    def timed(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    sec = timed(lambda: lbm.copy(a.data_ptr(), b.data_ptr(), half, variant))
    sec_t = timed(lambda: b.copy_(a))
    moved = 2 * half
    out = dict(bytes_per_copy=moved, kernel="lbm::k_copy", variant=variant, avg_us=round(sec * 1e6, 3),
               gbs=round(moved / sec / 1e9, 1), frac_of_peak=round(moved / sec / 1e9 / HBM_PEAK_GBS, 4),
               torch_copy_gbs=round(moved / sec_t / 1e9, 1))
    del a, b
    torch.cuda.empty_cache()
    return out


def run_batch(steps, count=64, seed=0, tune_steps=5):
    """The 64-domain batch (sides 64..512, one circle or ellipse each, half of
    them rotating, tau in [0.52, 1]): every domain advanced `steps` steps by
    the batched launches -- the launch shape chosen by the autotuner on a
    separate copy of the batch, timed both with every launch enqueued from
    the host and replayed from a captured HIP graph -- against the same
    domains advanced one after another by lbm_step, one domain per launch.
    Every run is timed whole."""
    import torch
    import lbm_workloads as W
    from paper_1407_4524_amd import Batch, Domain
    ws = W.batched_domains(count=count, seed=seed)
    nodes = sum(w["nx"] * w["ny"] for w in ws)

    stream = torch.cuda.Stream()

    def fresh():
        with torch.cuda.stream(stream):
            return [Domain.from_spec(w) for w in ws]

    tb = Batch(stream=stream.cuda_stream)
    tdoms = fresh()
    for d in tdoms:
        tb.add(d)
    chosen, trials = tb.tune(trial_steps=tune_steps)
    tb.close()
    for d in tdoms:
        d.close()

    def batched(cfg):
        doms = fresh()
        batch = Batch(stream=stream.cuda_stream)
        for d in doms:
            batch.add(d)
        batch.config = cfg
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(steps)
        for d in doms:
            d.synchronize()
        sec = time.perf_counter() - t0
        finite = sum(bool(np.isfinite(d.records(0, steps - 1, 1)).all()) for d in doms)
        batch.close()
        for d in doms:
            d.close()
        return dict(seconds=round(sec, 4), solves_per_s=round(count / sec, 3), mlups=round(nodes * steps / sec / 1e6, 1),
                    us_per_step=round(sec / steps * 1e6, 2), finite_members=finite,
                    config={k: v for k, v in cfg.items() if k != "us_per_step"})

    ordinary = batched(dict(chosen, graph=0))
    graphed = batched(dict(chosen, graph=1))

    doms = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in doms:
        d.step(steps)
    for d in doms:
        d.synchronize()
    t_plain = time.perf_counter() - t0
    for d in doms:
        d.close()
    best = graphed if graphed["seconds"] < ordinary["seconds"] else ordinary
    return dict(workload=f"batch{count}_channels_f32", domains=count, steps_per_domain=steps, nodes=nodes,
                batched=best, batched_ordinary=ordinary, batched_graph=graphed,
                plain=dict(seconds=round(t_plain, 4), solves_per_s=round(count / t_plain, 3),
                           mlups=round(nodes * steps / t_plain / 1e6, 1)),
                speedup=round(t_plain / best["seconds"], 2), tuner_choice=chosen, tuner_trials=len(trials))


def run_serving(count, max_steps, seed=0, rate=200.0, budget_gb=64.0, progress=False,
                parts=("batched", "plain", "loaded")):
    """Served solves: a Poisson stream of requests (80 % D2Q9 sides
    128..1024, 20 % D3Q19 sides 48..160, FP32/FP16-shifted, static or
    rotating bodies) with continuous batching and admission by device
    footprint, against the same stream served one request at a time; then a
    second batched run offered 70 % of the measured batched capacity, for
    latency under load. Requests stop at a relative drag change below 1e-6
    over 500 steps, or at max_steps."""
    import torch
    import lbm_workloads as W
    from paper_1407_4524_amd.serve import GpuEngine, Server, serve_plain, summary

    def report(label):
        if not progress:
            return None
        done = [0]

        def cb(r):
            done[0] += 1
            state = "failed: " + r.error if r.failed else ("steady" if r.converged else "capped")
            print(f"served ({label}) {done[0]}/{count}: request {r.id}, {r.steps} steps, {state}",
                  file=sys.stderr, flush=True)
        return cb

    def batched(reqs, label="batched"):
        eng = GpuEngine()
        srv = Server(eng, budget_gb * 2 ** 30, epoch=500, window=500, tol=1e-6, on_result=report(label))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        eng.close()
        out = summary(res, wall)
        out.update(peak_active=srv.peak_active, peak_memory_gb=round(srv.peak_memory / 2 ** 30, 2))
        return out, res

    reqs = W.serving_requests(count=count, seed=seed, rate=rate, max_steps=max_steps)
    note = ("the configured stream (256 requests, 50000-step cap)" if (count, max_steps) == (256, 50000) else
            f"reduced from the configured 256 requests / 50000-step cap to {count} requests / {max_steps} steps")
    out = dict(workload=f"served_{count}_requests_cap{max_steps}", requests=count, max_steps=max_steps,
               offered_rate_per_s=rate, note=note)
    sat = res_b = None
    if "batched" in parts:
        sat, res_b = batched(reqs)
        out["batched"] = sat
    if "plain" in parts:
        t0 = time.perf_counter()
        res_p = serve_plain(reqs, epoch=500, window=500, tol=1e-6, on_result=report("one at a time"))
        out["plain"] = summary(res_p, time.perf_counter() - t0)
        if res_b is not None:
            by_id = {r.id: r for r in res_p}
            ok = [r for r in res_b if not r.failed]
            out["speedup"] = round(out["plain"]["seconds"] / sat["seconds"], 2)
            out["results_equal_alone"] = all(r.force_torque == by_id[r.id].force_torque and
                                             r.steps == by_id[r.id].steps for r in ok)
            out["same_requests_failed"] = sorted(r.id for r in res_b if r.failed) == sorted(
                r.id for r in res_p if r.failed)
    if "loaded" in parts and sat is not None:
        load_rate = 0.7 * sat["solves_per_s"]
        loaded, _ = batched(W.serving_requests(count=count, seed=seed + 1, rate=load_rate, max_steps=max_steps),
                            "at 70 % of capacity")
        out["at_70pct_capacity"] = dict(offered_rate_per_s=round(load_rate, 3), **loaded)
    return out


def cpu_baseline(name, budget_s, single_thread_s):
    """The FP64 oracle (untuned, OpenMP on its bulk loops) on the first steps
    of the same workload, until about budget_s seconds of CPU time, then the
    same at one thread for about single_thread_s seconds."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    from oracle_helpers import make_oracle
    w = workload(name)
    cells = w["nx"] * w["ny"] * (w["nz"] if w["lattice"] == "D3Q19" else 1)
    o = make_oracle(w)
    o.step(1)

    def sample(budget):
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget or n == 0:
            o.step(1)
            n += 1
        return n, time.perf_counter() - t0

    threads = oracle.nthreads()
    n, sec = sample(budget_s)
    out = dict(value=round(cells * n / sec / 1e6, 3), unit="MLUPS", cores=threads, kind="oracle",
               sample=f"{w['name']}: steps 2..{n + 1} ({n} steps, {sec:.1f} s), FP64 oracle, {threads} threads")
    if single_thread_s > 0:
        oracle.set_threads(1)
        n1, sec1 = sample(single_thread_s)
        oracle.set_threads(threads)
        out["single_thread"] = dict(value=round(cells * n1 / sec1 / 1e6, 3), unit="MLUPS", cores=1,
                                    sample=f"the next {n1} steps ({sec1:.1f} s) at one thread")
    o.close()
    return out


def force_noise(x, win=41):
    """RMS of x minus its centred win-step moving average (short-time noise)"""
    k = np.ones(win) / win
    r = x[win // 2: len(x) - win // 2] - np.convolve(x, k, mode="valid")
    return float(np.sqrt((r * r).mean()))


def run_noise(steps=4000, warmup=200):
    """The force-noise comparison of Sec. III.B.3 on the full oscillating
    cylinder (2000x800, R=40, one period of 4000 steps): for each refill
    rule, the short-time noise (force minus its 41-step moving average, RMS)
    of the lattice-frame force (forward and backward sets) and of the
    comoving-frame force, drag and lift."""
    import lbm_workloads as W
    from paper_1407_4524_amd import Domain
    out = {}
    for refill in ("mean", "aidun", "extrapolate"):
        w = W.channel_oscillating_f32(scale=1)
        w["bodies"][0]["refill"] = refill
        dom = Domain.from_spec(w)
        t0 = time.perf_counter()
        dom.step(warmup + steps)
        dom.synchronize()
        sec = time.perf_counter() - t0
        rec = dom.records(0, warmup, steps)
        dom.close()
        prev = np.vstack([np.zeros((1, 3)), rec[:-1, 6:9]])
        forms = {"lattice": rec[:, 0:3] + rec[:, 6:9], "lattice_backward": rec[:, 0:3] + prev,
                 "comoving": rec[:, 12:15]}
        out[refill] = {k: {"drag": round(force_noise(v[:, 0]), 6), "lift": round(force_noise(v[:, 1]), 6)}
                       for k, v in forms.items()}
        out[refill]["us_per_step"] = round(sec / (warmup + steps) * 1e6, 2)
    return dict(workload="channel_oscillating_f32_2000x800", steps=steps, window=41,
                note="RMS of force minus its centred 41-step moving average, lattice units", noise=out)


def run_sedimentation(steps=20000, shape="disc"):
    """The paper's sedimenting disc (135x1073, density ratio 1.03, FP32) or
    ellipse (135x1676, aspect ratio 2, density ratio 1.1, released at 45
    degrees), from rest, for `steps` steps (0.59 s of the physical time) with
    each force form moving it: the classical static sum, the lattice-frame
    force with the previous step's covered/uncovered terms, and the comoving
    form. Reports the speed and the lateral/vertical positions and angle
    reached and the largest difference of the lateral position (and angle)
    between the classical and the corrected forms (the transient difference
    the paper points at)."""
    import lbm_workloads as W
    from paper_1407_4524_amd import Domain
    make = (lambda **kw: W.sedimenting_disc(ratio=1.03, **kw)) if shape == "disc" else \
        (lambda **kw: W.sedimenting_ellipse(ratio=1.1, **kw))
    out, traj = {}, {}
    for me in ("static", "lattice", "comoving"):
        w = make(storage="f32", me=me)
        dom = Domain.from_spec(w)
        t0 = time.perf_counter()
        dom.step(steps)
        dom.synchronize()
        sec = time.perf_counter() - t0
        tr = dom.trajectory(0, 0, steps + 1)
        dom.close()
        traj[me] = tr
        out[me] = dict(us_per_step=round(sec / steps * 1e6, 2), mlups=round(w["nx"] * w["ny"] * steps / sec / 1e6, 1),
                       x_end=round(float(tr[-1, 0]), 4), y_end=round(float(tr[-1, 1]), 4),
                       v_end=[round(float(v), 7) for v in tr[-1, 4:6]], theta_end=round(float(tr[-1, 3]), 6))
    dx = {me: round(float(np.abs(traj[me][:, 0] - traj["static"][:, 0]).max()), 5) for me in ("lattice", "comoving")}
    w = make()
    res = dict(workload=w["name"], steps=steps, seconds_physical=round(steps * w["dt_s"], 4), forms=out,
               max_lateral_difference_vs_classical_nodes=dx)
    if shape != "disc":
        res["max_angle_difference_vs_classical_rad"] = {
            me: round(float(np.abs(traj[me][:, 3] - traj["static"][:, 3]).max()), 6) for me in ("lattice", "comoving")}
    return res


def run_small_graph(name, steps):
    """A small, launch-bound domain stepped as a one-member batch whose
    steps are replayed from captured HIP graphs, timed whole (compare with
    its plain lbm_step line)."""
    import torch
    from paper_1407_4524_amd import Batch, Domain
    w = workload(name)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        dom = Domain.from_spec(w)
    batch = Batch(stream=stream.cuda_stream)
    batch.add(dom)
    batch.config = dict(batch.config, graph=1)
    batch.step(64)
    dom.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    dom.synchronize()
    sec = time.perf_counter() - t0
    batch.close()
    dom.close()
    cells = w["nx"] * w["ny"] * w.get("nz", 1)
    return dict(us_per_step=round(sec / steps * 1e6, 2), mlups=round(cells * steps / sec / 1e6, 1), steps=steps)


def secondary_line(r):
    w = r["w"]
    return dict(workload=w["name"], value=round(r["mlups"], 1), unit="MLUPS", storage=w["storage"],
                ms_per_step=round(r["ms_per_step"], 5), footprint_bytes=r["footprint_bytes"],
                roofline=r["roofline"], kernels=r["kernels"])


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=6.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 4.8 GB channel line")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-domain batched line")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-requests line")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-max-steps", type=int, default=2000)
    ap.add_argument("--serve-progress", action="store_true", help="a line on stderr per finished request")
    ap.add_argument("--serve-parts", default="batched,plain,loaded",
                    help="which served runs: batched, plain (one at a time), loaded (batched at 70%% of capacity)")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--no-physics", action="store_true",
                    help="skip the force-noise comparison and the sedimenting-disc line")
    ap.add_argument("--sediment-steps", type=int, default=20000)
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the copy-kernel reference at the stream-collide footprint")
    ap.add_argument("--schedule", choices=sorted(SCHEDULES), default="auto",
                    help="a single body's step: auto (the library's default: a moving body's domain steps as "
                         "a one-member batch, a fixed body's in the plain schedule), split (the nodes away from "
                         "the body updated on a second stream beside the body work) or plain (one launch after "
                         "another)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(a domain larger than one GPU would be split into x-slabs with a one-layer halo "
              "exchange; that is described, not implemented).", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    main_run = run_gpu(args.workload, args.steps, args.warmup, SCHEDULES[args.schedule])
    w = main_run["w"]
    line = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f16"}[w["storage"]],
        "data": "synthetic",
        "config": {"workload": w["name"], "lattice": w["lattice"], "nx": w["nx"], "ny": w["ny"],
                   "nz": w["nz"], "tau": w["tau"], "storage": w["storage"],
                   "force_accumulation": "f64", "bodies": len(w["bodies"]),
                   "me": w["bodies"][0]["me"] if w["bodies"] else None, "parallelism": "single-gpu",
                   "footprint_bytes": main_run["footprint_bytes"],
                   "schedule": args.schedule, "near_box_launches": "near_box" in main_run["kernels"]},
        "roofline": main_run["roofline"],
        "kernels": main_run["kernels"],
    }
    if not args.no_copy_ceiling and main_run["roofline"]:
        line["copy_ceiling"] = copy_ceiling(main_run["roofline"]["algorithmic_bytes_per_launch"])
    if not args.no_secondary and args.workload == HEADLINE:
        sec = {}
        for name in ("duct_sphere_f16", "duct_sphere_zouhe_f32", "channel_oscillating_f32", "suspension_f32",
                     "channel_cylinder_f64"):
            r = run_gpu(name, args.steps, args.warmup, SCHEDULES[args.schedule])
            sec[r["w"]["name"]] = secondary_line(r)
            if name == "channel_cylinder_f64":
                sec[r["w"]["name"]]["note"] = ("5000 nodes: bound by launches and their latency, not by HBM (the "
                                               "roofline fields only restate the kernel's byte rate); "
                                               "graph_batch: the same domain as a one-member batch replayed from "
                                               "captured HIP graphs")
                sec[r["w"]["name"]]["graph_batch"] = run_small_graph(name, args.steps)
            if name == "suspension_f32":
                sec[r["w"]["name"]]["note"] = ("lbm_step steps the 32 bodies through batched launches (one for the "
                                               "link rule of the 16 static bodies, one for the advance of the 16 "
                                               "moving ones); the timed launch updates the nodes outside the "
                                               "bodies' box only, so no roofline; kernel times from the rocprofv3 "
                                               "summary")
            if name == "channel_oscillating_f32":
                sec[r["w"]["name"]]["note"] = ("lbm_step steps the domain as a one-member batch; the timed "
                                               "launch updates every node but the moving body's near box")
        if not args.no_large:
            r = run_gpu("channel_large_f32", min(args.steps, 200), min(args.warmup, 10))
            ent = secondary_line(r)
            if r["roofline"] and not args.no_copy_ceiling:
                ent["copy_ceiling"] = copy_ceiling(r["roofline"]["algorithmic_bytes_per_launch"], reps=10)
            sec[r["w"]["name"]] = ent
        line["secondary"] = sec
    if not args.no_physics and args.workload == HEADLINE:
        line["force_noise"] = run_noise()
        line["sedimentation"] = run_sedimentation(args.sediment_steps)
        line["sedimentation_ellipse"] = run_sedimentation(args.sediment_steps, shape="ellipse")
    if not args.no_batch and args.workload == HEADLINE:
        line["batched"] = run_batch(args.batch_steps)
    if not args.no_serve and args.workload == HEADLINE:
        line["served"] = run_serving(args.serve_requests, args.serve_max_steps, progress=args.serve_progress,
                                     parts=tuple(args.serve_parts.split(",")))
    if not args.no_cpu_baseline and rank == 0:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds, args.cpu_single_seconds)
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
