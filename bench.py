#!/usr/bin/env python3
"""Benchmark of the FP64 semi-implicit step of the 4D generalized SUBSURF model.

Workload (one GPU's share of the pectoral-fin problem at real shape):
512 x 512 x 96 voxels x 16 frames, uint8, ~2000 ellipsoidal nuclei with
Brownian tracks, background 20 + Poisson noise; K=1000, delta=vartheta=0.5,
lambda=0.5, r=8, one implicit presmoothing step tau=0.1; multi-seed initial
function (v=1, R=8); eps=1e-3, tau=0.5, omega=1.8, tol=1e-8, FP64 throughout.

A timed "step" is one semi-implicit time step of the job: assembly of the
finite-volume system, red-black SOR to tolerance with the fused residual,
unsplit and local rescaling.  Inputs (image, G, owner map, u) are resident in
HBM before the timed region; the per-job preparation runs before it.

value = SOR voxel-updates/s over the timed steps (iterations x interior cells
per step, divided by the wall time of the steps).  roofline: the red-black
sweep kernel, 96 algorithmic bytes per voxel-update, timed with HIP events on
the library's stream; traffic from the committed rocprofv3 counter summary
when it was taken on the current kernel sources.

The same JSON line also carries:
* mixed: the same job with the mixed-precision solve (FP32 sweeps on BF16
  coefficients in FP64 refinement; 20 sweeps per pass at the FP64 omega) at
  the FP64 stopping rule and at 1e-10;
* cpu_baseline: the oracle's red-black SOR on the host cores, on a bounded
  crop of the same volume;
* batched_windows: 2048 uneven windows (x,y,z in 24..64, t in 3..9) of 20
  steps each, batched preparation + batched mixed-precision steps, against
  plain per-job FP64 preparation and steps on a sample of the same jobs;
* serving: a Poisson stream of lognormal windows served by continuous
  batching against first-come-first-served plain FP64 jobs (jobs/s, p50/p99
  latency from arrival to the result on the host), each server warmed up
  first on another stream of the same law (untimed).
Both window sections report each form's largest relative error (max-abs over
a window / max |u|) against the converged solution of the same job (FP64 SOR
to relative residual 1e-12, untimed); each form runs at its fastest setting
that keeps this error within 1e-6.
"""
from __future__ import annotations

import argparse
import ctypes
from dataclasses import replace
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SOR voxel-updates/s + % HBM peak; jobs/s and p50/p99 latency vs plain GPU"
HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_UPDATE = 96.0   # 8 coefficients + rhs + own u read/write + amortised neighbour (FP64)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2111_11866_amd/csrc/ss4_sweep.hpp", "paper_2111_11866_amd/csrc/ss4_common.hpp")
COUNTER_SUMMARY = "profiles/k_sweep_config2_counters.md"


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    copy of known size), or None when the kernel sources changed since."""
    path = os.path.join(ROOT, COUNTER_SUMMARY)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    if "```json" not in txt:
        return None
    d = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d


def host_cpu_info():
    """CPU model, physical cores and logical CPUs of this host, and the CPUs
    this process may run on."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model == "unknown":
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                elif not key and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 0
    return {"model": model, "physical_cores": len(cores) or None, "logical_cpus": os.cpu_count(),
            "cpus_allowed": allowed}


def cpu_baseline(img, sp, seconds):
    """The oracle's red-black SOR timed on this host: a copy of the oracle built
    here (-O3 -march=native -ffp-contract=off, OpenMP over the host threads) on
    the first two frames of the same volume (512 x 512 x 96 x 2).  The system
    is one step's, assembled by the oracle from the multi-seed initial function
    with G = 1 (the cost of an SOR iteration does not depend on the coefficient
    values).  Two runs of K1 < K2 iterations test the residual only before the
    first and after the last iteration; their difference gives the time of
    K2 - K1 iterations without the residuals and the set-up."""
    import tempfile

    import numpy as np

    import oracle as orc
    from oracle.build import build_oracle_native

    orc.use_library(build_oracle_native(tempfile.mkdtemp(prefix="ss4_oracle_")))
    n = (512, 512, 96, 2)
    cs = img.centres[img.centres["frame"] < n[3]]
    w = orc.init_u(n, cs, 1.0, 8.0)
    G = np.ones((4,) + orc.padded_shape(n))
    coef, b = orc.assemble(n, G, w, 1.0, sp.eps, sp.tau)
    del G
    cells = n[0] * n[1] * n[2] * n[3]

    def run(k):
        t0 = time.perf_counter()
        orc.sor(n, coef, b, w, sp.omega, 0.0, k, orc.RB, check_every=k)
        return time.perf_counter() - t0

    k1 = 2
    t1 = run(k1)
    t_it = max((run(k1 + 2) - t1) / 2.0, 1e-3)
    k2 = k1 + max(4, int(seconds / t_it))
    t1 = run(k1)
    t2 = run(k2)
    dt = max(t2 - t1, 1e-6)
    host = host_cpu_info()
    return {"value": (k2 - k1) * cells / dt, "unit": "voxel-updates/s", "cores": orc.num_threads(),
            "kind": "oracle", "host": host,
            "sample": f"512x512x96x2 frames of the config-2 volume ({cells} cells), one step's system (G = 1), "
                      f"{k2 - k1} red-black iterations ({dt:.1f} s, the difference of runs of {k2} and {k1} "
                      f"iterations), oracle built with -march=native on this host, {orc.num_threads()} OpenMP "
                      f"threads on {host['cpus_allowed']} allowed CPUs"}


def bench_batch(n_windows, steps, plain_sample, log_steps=False):
    """Config 4: n_windows uneven windows (x,y,z in 24..64, t in 3..9), each a
    job of `steps` time steps.  Batched mixed-precision form (all windows in
    every launch, graph-replayed passes) against the plain per-job FP64 form
    timed on the first `plain_sample` windows."""
    import numpy as np
    import torch

    import synth
    from paper_2111_11866_amd import binding as B
    from paper_2111_11866_amd import serve as S

    pp, plain, mixed = S.default_params()
    t0 = time.perf_counter()
    imgs = synth.windows_cfg4(n_windows)
    cells = sum(im.cells for im in imgs)
    log(f"[batch] generated {n_windows} windows ({cells / 1e9:.2f} G cells) in {time.perf_counter() - t0:.1f}s")
    shared = S._Shared(n_windows)
    wins = [S.Window(jid=q, arrival=0.0, img=im) for q, im in enumerate(imgs)]
    jobs = S.admit_windows(wins, pp, 1.0, 0.0, mixed.ball_r, shared)    # untimed: allocations, warm-up
    B.step_batched(jobs, mixed, shared.table)          # one untimed step (tuning, warm caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = B.prepare_batched(jobs, pp, 1.0, 0.0, mixed.ball_r, shared.table)   # timed: every job from scratch
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    assert rc == 0, (rc, st)
    t0 = time.perf_counter()
    passes, mean_passes = [], []
    for st in range(steps):
        rc, res = B.step_batched(jobs, mixed, shared.table)
        passes.append(max(r["outer"] for r in res))
        mean_passes.append(sum(r["outer"] for r in res) / len(res))
        if log_steps:
            log(f"[batch] step {st}: max passes {passes[-1]}")
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    t_batch = t_prep + t_steps
    batched_u = [w.state.u.cpu().numpy() for w in wins[:plain_sample]]
    # the same batch in FP64 (FP64 red-black sweeps of every window in each
    # launch, stopping rule tested every 4 iterations), prepared again
    fp64b = replace(plain, inner_sweeps=4)
    B.step_batched(jobs, fp64b, shared.table)          # untimed: first FP64 batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = B.prepare_batched(jobs, pp, 1.0, 0.0, mixed.ball_r, shared.table)
    assert rc == 0, (rc, st)
    for _ in range(steps):
        B.step_batched(jobs, fp64b, shared.table)
    torch.cuda.synchronize()
    t_fp64b = time.perf_counter() - t0
    batched_fp64_u = [w.state.u.cpu().numpy() for w in wins[:plain_sample]]
    # plain per-job FP64 on a sample (same jobs, same initial function)
    for w in wins[plain_sample:]:
        w.state = None
    torch.cuda.empty_cache()
    def run_plain(sp):
        out = []
        for q in range(plain_sample):
            im = imgs[q]
            job = B.Job(im.n, im.image, im.centres, im.seeds, precision=B.FP64)
            job.prepare(pp)
            job.init(v=1.0, R=0.0, ball_r=sp.ball_r)
            for _ in range(steps):
                job.step(sp)
            out.append(job.u.cpu().numpy())
            del job
        return out

    t0 = time.perf_counter()
    plain_u = run_plain(plain)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_per_job = t_plain / plain_sample
    conv_u = run_plain(S.converged_params(plain))      # untimed reference

    def rel(a, ref):
        return max(float(np.abs(x - r).max() / max(np.abs(r).max(), 1e-300)) for x, r in zip(a, ref))
    return {
        "windows": n_windows, "cells": cells, "steps_per_job": steps,
        "batched_jobs_per_s": n_windows / t_batch,
        "batched_step_ms": t_steps * 1e3 / steps,
        "batched_voxel_steps_per_s": cells * steps / t_steps,
        "refinement_passes_per_step_max": passes,
        "refinement_passes_per_step_mean": mean_passes,
        "batched_fp64_jobs_per_s": n_windows / t_fp64b,
        "batched_fp64_note": "the same batch with FP64 sweeps (omega and tol of the plain form, stopping rule "
                             "tested every 4 iterations), preparation included",
        "mixed_vs_fp64_batched": t_fp64b / t_batch,
        "prepare_s_all_windows": t_prep,
        "plain_fp64_jobs_per_s": 1.0 / plain_per_job,
        "plain_sample_jobs": plain_sample,
        "speedup_jobs_per_s": (n_windows / t_batch) * plain_per_job,
        "max_rel_err_batched_vs_plain_fp64": rel(batched_u, plain_u),
        "max_rel_err_vs_converged": {"batched": rel(batched_u, conv_u), "plain_fp64": rel(plain_u, conv_u),
                                     "batched_fp64": rel(batched_fp64_u, conv_u),
                                     "reference": "plain FP64 SOR to relative residual 1e-12, sample jobs"},
        "note": "both forms include preparation (thresholding, presmoothing, G, initial function and "
                "rescale): one batched call for all windows, or one per job; device memory is allocated "
                "outside the timed region in the batched form and inside it in the plain form",
    }


def bench_serving(rates, count, plain_seconds, log=None, ref_jobs=40):
    """Config 5: Poisson arrivals of lognormal-size windows; continuous batching
    (mixed precision) against first-come-first-served plain FP64 per-job
    solves, at every arrival rate.  Job j's size and content do not depend on
    the rate (its own seeds), so one set of images serves every rate and only
    the arrival times change; the plain server is stopped after
    `plain_seconds` per rate (its p50/p99 are over the jobs it served)."""
    import numpy as np
    import torch

    import synth
    from paper_2111_11866_amd import serve as S

    pp, plain, mixed = S.default_params()
    t0 = time.perf_counter()
    _, sizes = synth.serving_stream(1.0, count)
    imgs = synth.serving_windows(sizes)
    if log:
        log(f"[serve] {count} job images in {time.perf_counter() - t0:.1f}s")

    def stream(rate):
        t, _ = synth.serving_stream(rate, count)
        return [S.Window(jid=q, arrival=float(t[q]), img=imgs[q]) for q in range(count)]

    def keep(wins):
        res = {w.jid: w.result for w in wins if w.result is not None and w.jid < ref_jobs}
        for w in wins:
            w.result = None
        return res

    def rel(a, ref):
        e = [float(np.abs(a[j] - ref[j]).max() / max(np.abs(ref[j]).max(), 1e-300)) for j in ref if j in a]
        return (max(e) if e else None), len(e)

    # converged reference of the first jobs (FP64 SOR to relative residual 1e-12; untimed)
    ref_wins = stream(1.0)[:ref_jobs]
    S.PlainServer(pp, S.converged_params(plain), steps=20).run(ref_wins, realtime=False)
    conv = keep(ref_wins)
    # untimed warm-up of both servers (shape tuning, device memory pool)
    batch_server = S.BatchServer(pp, mixed, steps=20, hbm_budget=96 << 30)
    warm = stream(max(rates))[: min(count, 600)]
    batch_server.run(warm, realtime=False)
    keep(warm)
    plain_server = S.PlainServer(pp, plain, steps=20)
    warm = stream(max(rates))[:8]
    plain_server.run(warm, realtime=False)
    keep(warm)
    torch.cuda.empty_cache()
    out = {}
    for rate in rates:
        wins = stream(rate)
        offered = count / max(w.arrival for w in wins)
        bs = batch_server.run(wins)
        got = keep(wins)
        del wins
        torch.cuda.empty_cache()
        wins = stream(rate)
        ps = plain_server.run(wins, max_seconds=plain_seconds)
        plain_res = keep(wins)
        del wins
        torch.cuda.empty_cache()
        bs["offered_jobs_per_s"] = ps["offered_jobs_per_s"] = offered
        bs["keeps_up"] = bool(bs["jobs_per_s"] >= 0.9 * offered)
        ps["keeps_up"] = bool(ps["jobs_per_s"] >= 0.9 * offered and ps.get("unserved", 0) == 0)
        bs["max_rel_err_vs_plain_fp64"], bs["jobs_compared_with_plain"] = rel(got, plain_res)
        bs["max_rel_err_vs_converged"], bs["jobs_compared_with_converged"] = rel(got, conv)
        ps["max_rel_err_vs_converged"], ps["jobs_compared_with_converged"] = rel(plain_res, conv)
        ps["stopped_after_s"] = plain_seconds
        out[str(rate)] = {"batched": bs, "plain_fp64": ps}
        del got, plain_res
        if log:
            log(f"[serve] rate {rate}/s (offered {offered:.0f}): batched {bs['jobs_per_s']:.1f} jobs/s "
                f"p50 {bs['p50_latency_s']:.3f}s p99 {bs['p99_latency_s']:.3f}s keeps up {bs['keeps_up']} | "
                f"plain {ps['jobs_per_s']:.1f} jobs/s p50 {ps['p50_latency_s']:.3f}s "
                f"p99 {ps['p99_latency_s']:.3f}s ({ps['jobs']} served, {ps.get('unserved', 0)} not)")
    out["jobs_per_rate"] = count
    out["note"] = ("latency from arrival to the result on the host; the plain FP64 server is stopped after "
                   f"{plain_seconds:.0f} s per rate, its jobs/s and latencies are over the jobs it served; "
                   "errors relative to max |u| of the job")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=16, help="t extent (16 = full workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-steps", type=int, default=-1,
                    help="also time this many steps with the mixed-precision solve (-1: same as --steps)")
    ap.add_argument("--inner", type=int, default=20, help="FP32 sweeps per refinement pass (mixed)")
    ap.add_argument("--inner-omega", type=float, default=0.0,
                    help="relaxation of the FP32 sweeps of the correction equation (mixed); "
                         "0: the FP64 solve's omega")
    ap.add_argument("--windows", type=int, default=2048, help="batched workload size (0: skip)")
    ap.add_argument("--window-steps", type=int, default=20)
    ap.add_argument("--plain-sample", type=int, default=24)
    ap.add_argument("--serving-rates", type=str, default="200,500,1000,2000,5000",
                    help="comma-separated arrival rates (jobs/s); empty: skip the serving run")
    ap.add_argument("--serving-jobs", type=int, default=2000, help="jobs per arrival rate")
    ap.add_argument("--plain-seconds", type=float, default=8.0,
                    help="the plain FP64 server is stopped after this many seconds per rate")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is a "
                                   "design note, not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2111_11866_amd import binding as B

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)

    n = (512, 512, 96, args.frames)
    t0 = time.perf_counter()
    img = synth.nuclei_cfg2(n=n)
    log(f"[bench] generated {n} with {len(img.centres)} centres in {time.perf_counter() - t0:.1f}s")
    pp = B.PrepareParams(image_scale=1.0 / 255.0)
    sp = B.StepParams(omega=1.8)
    if args.inner_omega <= 0.0:
        args.inner_omega = sp.omega

    job = B.Job(n, img.image, img.centres, img.seeds, precision=B.MIXED)
    t0 = time.perf_counter()
    rc = job.prepare(pp)
    job.init(v=1.0, R=8.0, ball_r=sp.ball_r)
    torch.cuda.synchronize()
    log(f"[bench] prepare rc={rc} in {time.perf_counter() - t0:.2f}s; "
        f"workspace {job.ws.numel() / 1e9:.1f} GB")
    # the preparation once more, warm (the first call also loads the code object)
    t0 = time.perf_counter()
    job.prepare(pp)
    torch.cuda.synchronize()
    t_prepare = time.perf_counter() - t0
    job.init(v=1.0, R=8.0, ball_r=sp.ball_r)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        r = job.step(sp)
        log(f"[bench] warmup step {w}: {r}")

    B.timing(1)
    B.timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for s in range(args.steps):
        r = job.step(sp)
        iters.append(r["iterations"])
        if r["status"] != 0:
            log(f"[bench] step {s} status {r['status']}")
        log(f"[bench] step {s}: {r['iterations']} iterations, rel_res {r['rel_res']:.3e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = B.timing(3)
    B.timing(0)

    cells = n[0] * n[1] * n[2] * n[3]
    updates = sum(iters) * cells
    value = updates / dt
    launch_ms = tm["sweep_ms"] / max(tm["sweep_launches"], 1)
    bytes_per_launch = SWEEP_BYTES_PER_UPDATE * cells / 2.0
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"config-2 nuclei volume {n[0]}x{n[1]}x{n[2]}x{n[3]} uint8, "
                               f"{len(img.centres) // n[3]} tracks, omega 1.8, tol 1e-8, FP64 red-black SOR",
                   "grid": list(n), "cells": cells, "parallelism": "single GPU"},
        "iterations_per_step": iters,
        "hbm_frac_sweeps": achieved / HBM_PEAK_GBS,
        "voxel_updates_per_s_kernel_time": updates / (tm["sweep_ms"] * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "red-black half-sweep (%s, red and black)" %
                               ("k_sweep_t2" if n[0] // 2 >= 64 else "k_sweep_tm"),
                     "avg_launch_ms": launch_ms, "launches": tm["sweep_launches"],
                     "bytes_per_launch": bytes_per_launch},
        "sweep_share_of_step_time": tm["sweep_ms"] / (dt * 1e3),
        "preparation_ms": t_prepare * 1e3,
        "preparation_note": "owner map, local thresholds, two presmoothing heat solves and face G of the whole volume; "
                            "once per job, outside the timed steps",
    }
    # cell tracking (Sec. 5) on the segmentation after the timed steps; its
    # label, distance and workspace buffers are allocated before the clock
    # starts, as the step's are
    cap = 1 << 20
    lab = torch.empty(B.interior_shape(n), dtype=torch.int32, device="cuda")
    d2 = torch.empty(B.interior_shape(n), dtype=torch.int32, device="cuda")
    tws = torch.empty(int(B.lib().subsurf4d_track_workspace_bytes(ctypes.byref(B.grid(n)), cap)),
                      dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tcells, lab, d2 = B.track(n, job.u, 0.5, capacity=cap, join_radius=3.0, label=lab, dist2=d2, ws=tws)
    torch.cuda.synchronize()
    t_track = time.perf_counter() - t0
    kinds = np.bincount(tcells["kind"], minlength=4) if len(tcells) else np.zeros(4, int)
    out["tracking"] = {"ms": t_track * 1e3, "cells": int(len(tcells)),
                       "cells_per_frame_mean": float(len(tcells)) / n[3],
                       "links": {"none": int(kinds[0]), "centre": int(kinds[1]), "overlap": int(kinds[2]),
                                 "joined": int(kinds[3])},
                       "note": "u >= 0.5 after the timed steps; labels, distances, centres, backward links on the GPU, "
                               "joining (radius 3 voxels) on the host; includes the copy of the cell records, "
                               "not the allocation of the label, distance and workspace buffers"}
    log(f"[bench] tracking: {len(tcells)} cells in {t_track * 1e3:.1f} ms, links {kinds.tolist()}")
    del lab, d2, tws, tcells
    torch.cuda.empty_cache()
    ct = counter_traffic()
    # the summary's counters hold for its own workload only (the full volume):
    # another grid (a --frames run) reports no traffic
    if ct is not None and ct.get("algorithmic_bytes_per_launch") == out["roofline"]["bytes_per_launch"]:
        out["roofline"]["traffic"] = ct["hbm_bytes_per_launch"]
        out["roofline"]["traffic_source"] = COUNTER_SUMMARY
    mixed_steps = args.steps if args.mixed_steps < 0 else args.mixed_steps
    if mixed_steps > 0:
        # same job from the same initial function: mixed-precision solve of every step
        # (FP32 red-black sweeps on BF16 coefficients, FP64 refinement to the FP64
        # stopping rule tol=1e-8, and to 1e-10 as configured for the mixed workload)
        from dataclasses import replace
        for tol_name, rtol in (("tol_1e-8", 1e-8), ("tol_1e-10", 1e-10)):
            # in the mixed form omega relaxes only the inner FP32 sweeps; the FP64
            # residual and refine_tol decide the result
            msp = replace(sp, precision=B.MIXED, refine_tol=rtol, inner_sweeps=args.inner,
                          omega=args.inner_omega, flags=B.FLAG_SHORT_LAST_PASS)
            job.init(v=1.0, R=8.0, ball_r=sp.ball_r)
            for w in range(args.warmup):
                job.step(msp)
            B.timing(1)
            B.timing(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = [job.step(msp) for _ in range(mixed_steps)]
            torch.cuda.synchronize()
            mdt = time.perf_counter() - t0
            mt = B.timing(3)
            B.timing(0)
            mlaunch = mt["sweep_ms"] / max(mt["sweep_launches"], 1)
            # 32 B per update, except the first iteration of each pass, which
            # starts from d = 0: red 8 B (r/D read, d written), black 28 B
            # (passes run inner_sweeps iterations, or fewer when the last one is shortened)
            n_it = max(sum(r["iterations"] for r in recs), 1)
            n_pass = sum(r["outer"] for r in recs)
            mbytes = cells / 2.0 * (64.0 * n_it - 28.0 * n_pass) / (2.0 * n_it)
            out.setdefault("mixed", {})[tol_name] = {
                "ms_per_step": mdt * 1e3 / mixed_steps,
                "speedup_vs_fp64_step": (dt / args.steps) / (mdt / mixed_steps),
                "refinement_passes": [r["outer"] for r in recs],
                "inner_sweeps_per_pass": args.inner,
                "inner_sweeps_per_step": [r["iterations"] for r in recs],
                "short_last_pass": True,
                "inner_omega": args.inner_omega,
                "final_rel_residual": [r["rel_res"] for r in recs],
                "inner_sweep_avg_launch_ms": mlaunch,
                "inner_sweep_GBs_algorithmic": mbytes / (mlaunch * 1e-3) / 1e9,
                "inner_bytes_per_update": 32,
                "inner_bytes_per_launch_avg": mbytes,
            }
            log(f"[bench] mixed {tol_name}: {mdt * 1e3 / mixed_steps:.1f} ms/step, passes "
                f"{[r['outer'] for r in recs]}, inner sweep {mbytes / (mlaunch * 1e-3) / 1e9:.0f} GB/s")
        # untimed: the error of each step against the converged FP64 step (relative
        # residual 1e-12) from the same u^{resc;n-1}, along the converged trajectory;
        # the FP64 step at its stopping rule 1e-8 is measured the same way
        conv = replace(sp, tol=1e-12, max_iter=100000)
        forms = {"fp64_tol_1e-8": sp}
        forms.update({k: replace(sp, precision=B.MIXED, refine_tol=float(k.split("_")[-1]),
                                 inner_sweeps=args.inner, omega=args.inner_omega) for k in out["mixed"]})
        errs = {k: ([], []) for k in forms}
        job.init(v=1.0, R=8.0, ball_r=sp.ball_r)
        for _ in range(mixed_steps):
            u_start = job.u.clone()
            job.step(conv)
            u_conv = job.u.clone()
            scale_max, scale_l2 = u_conv.abs().max(), torch.linalg.vector_norm(u_conv)
            for k, fsp in forms.items():
                job.u.copy_(u_start)
                job.step(fsp)
                d = job.u - u_conv
                errs[k][0].append(float(d.abs().max() / scale_max))
                errs[k][1].append(float(torch.linalg.vector_norm(d) / scale_l2))
                del d
            job.u.copy_(u_conv)
            del u_start, u_conv
        for k in out["mixed"]:
            out["mixed"][k]["max_abs_rel_err_vs_converged_per_step"] = errs[k][0]
            out["mixed"][k]["l2_rel_err_vs_converged_per_step"] = errs[k][1]
            log(f"[bench] mixed {k}: per-step max-abs rel err vs converged FP64 {max(errs[k][0]):.2e}")
        out["mixed"]["fp64_tol_1e-8_vs_converged"] = {
            "max_abs_rel_err_per_step": errs["fp64_tol_1e-8"][0],
            "l2_rel_err_per_step": errs["fp64_tol_1e-8"][1]}
        out["mixed"]["converged_reference"] = "FP64 red-black SOR to relative residual 1e-12, same u^{resc;n-1}"
    # practical HBM bandwidth of a plain 16-byte copy (4 GiB read + 4 GiB written)
    nb = 1 << 32
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nb, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    ms = B.copy_probe(src, dst, reps=5)
    out["copy_probe"] = {"bytes_moved": 2 * nb, "ms": ms, "GBs": 2 * nb / (ms * 1e-3) / 1e9,
                         "frac_of_peak": 2 * nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del src, dst
    # read-dominated probes: k streams of 1 GiB summed into one (k = 2: the
    # STREAM triad's mix; k = 11: about the FP64 sweep's 11 reads per write),
    # and the same 11 streams read with no write stream
    chunk = 1 << 30
    out["stream_probe"] = {}
    for k, w in ((2, 1), (11, 1), (11, 0)):
        src = torch.ones(k * chunk // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty(chunk // 8, dtype=torch.float64, device="cuda")
        ms = B.stream_probe(src, dst, k, writes=w, reps=5)
        moved = (k + w) * chunk
        key = f"reads_{k}_per_write" if w else f"reads_{k}_no_write"
        out["stream_probe"][key] = {"bytes_moved": moved, "ms": ms, "GBs": moved / (ms * 1e-3) / 1e9,
                                    "frac_of_peak": moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del src, dst
    out["stream_probe"]["sweep_vs_11_per_write"] = (
        achieved / out["stream_probe"]["reads_11_per_write"]["GBs"])
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(img, sp, args.cpu_seconds)
        log(f"[bench] cpu baseline in {time.perf_counter() - t0:.1f}s")
    del job
    torch.cuda.empty_cache()
    if args.windows > 0:
        t0 = time.perf_counter()
        out["batched_windows"] = bench_batch(args.windows, args.window_steps, args.plain_sample)
        log(f"[bench] batched windows in {time.perf_counter() - t0:.1f}s: {out['batched_windows']}")
        torch.cuda.empty_cache()
    rates = [float(r) for r in args.serving_rates.split(",") if r.strip()]
    if rates:
        t0 = time.perf_counter()
        out["serving"] = bench_serving(rates, args.serving_jobs, args.plain_seconds, log=log)
        log(f"[bench] serving sweep in {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
