"""Benchmark: TACAW hot path on the 512^2 x 32-slice x 1024-frame plane-wave workload.

One step = one whole pass of the hot path over the job: projected potentials
of every (frame, slice), the multislice of all 1024 frames, exit-wave capture,
FP64 frame mean and subtraction, time FFT and |.|^2.  Inputs (positions,
tables) are resident on the device before the timed region.

Prints one JSON line with the throughput in slice-steps/s (grid points x
slices x frames x probes per second), a roofline object for the dominant
kernel (HIP-event durations from inside the library) and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
WORKLOAD = ("12x12x8 diamond-cubic C/Si supercell (9216 atoms, 50/50 Z=6/14), 512x512 grid, "
            "32 slices of 1.3575 A, 100 kV plane wave, 1024 frames at 2 fs, seeded harmonic "
            "phonons (32 modes, 0.08 A rms), 512 one-sided energy bins")
WORKLOAD_C3 = ("hexagonal B/N layer stack (a=2.5 A, 40x20 orthohexagonal cells, 12 AA' layers, "
               "38400 atoms), 1000x866 full-cell potential grid, 256x256 probe windows, 20 slices, "
               "30 mrad probe at 60 kV, 32x32 probe positions over 20 A, 256 frames at 10 fs, "
               "seeded harmonic phonons, per-position I(k, w) with 128 bins")

# Algorithmic HBM bytes per slice-step of each kernel class (complex64 = 8 B):
#   row pass: read psi (8) + write psi (8) + read V (4)            = 20 B
#   col pass: read psi (8) + write psi (8)                         = 16 B
#   splat:    write V (4) per grid point per (frame, slice)        =  4 B
# time stage per (probe, frame, k): read psi (8) + write I (4 * M/F = 2) = 10 B
BYTES_PER_UNIT = {"row": 20.0, "col": 16.0, "splat": 4.0, "time": 10.0}


# Sources that decide what each launch reads and writes: the device code and
# the planner that sizes frame batches and builds the potential kernel's lists.
# Host orchestration (api, batch, serve, analysis) does not change a launch's
# traffic.
KERNEL_SOURCES = ("fft_engine.h", "kernels.hip", "planner.cpp", "runtime.h", "tacaw_internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2602_10064_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


# worker processes of the oracle baseline: the host CPUs this process may run
# on, capped at the 16 that a one-GPU share of the host provides
ORACLE_MAX_WORKERS = 16


def cpu_baseline(job, sample_frames: int, full_slice_steps: int, what: str = ""):
    """FP64 oracle on `sample_frames` frames of the workload, one frame per
    worker process, every worker busy (sample_frames is a multiple of the
    worker count).  The rate is the sample's; `extrapolated_s` scales the
    sample time linearly to the whole workload (work is linear in frames and
    probes)."""
    from tests.oracle_pool import exit_waves_parallel
    from oracle import tacaw_oracle
    host_cpus = len(os.sched_getaffinity(0))
    workers = max(1, min(sample_frames, ORACLE_MAX_WORKERS, host_cpus))
    frames = list(range(sample_frames))
    t0 = time.perf_counter()
    ex = exit_waves_parallel(job, frames=frames, workers=workers)
    tacaw_oracle.tacaw_spectrum(ex)
    dt = time.perf_counter() - t0
    steps = job.nx * job.ny * job.n_slices * sample_frames * job.n_probes
    return {"value": steps / dt, "unit": "slice-steps/s", "cores": workers, "kind": "oracle",
            "host_cpus": host_cpus, "sample_s": round(dt, 2), "sample_slice_steps": steps,
            "extrapolated_s": round(dt * full_slice_steps / steps, 1),
            "sample": (what or f"{sample_frames} of the 1024 frames (full 512^2 grid, all 32 slices, "
                               f"spectrum of the sample)") +
                      f", FP64 numpy, one frame per process on {workers} processes, {dt:.1f} s"}


def bench_c4(args):
    """64 seeded uneven jobs: plain per-job launches vs the batched executor.
    --workload c4small draws the same mix on small grids (64-128) with 16-96
    frames, where a job's launches are too small to fill the device alone."""
    import torch
    from paper_2602_10064_amd import tacaw, workloads
    small = args.workload == "c4small"
    ctx = tacaw.Context(0)
    handles, steps_total = [], 0
    t0 = time.perf_counter()
    for j in range(args.jobs):
        job = (workloads.c4_job(j, seed_base=4500, grids=(64, 96, 128), frames_range=(16, 96)) if small
               else workloads.c4_job(j))
        steps_total += job.slice_steps()
        handles.append(tacaw.TacawJob(ctx, job, keep_exit_waves=False))
        del job
        if j % 16 == 15:
            print(f"[bench] created {j + 1}/{args.jobs} jobs", file=sys.stderr, flush=True)
    print(f"[bench] {args.jobs} jobs generated and created in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    if args.autotune:
        seen = set()
        for h in handles:
            if h.nx not in seen:
                seen.add(h.nx)
                print(f"[bench] autotune {h.nx}: {h.autotune(stream)}", file=sys.stderr, flush=True)
    # warm-up: one batched pass (materialises every job)
    tacaw.run_batch(handles, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in handles:
        h.run(stream=stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    print(f"[bench] plain per-job launches: {t_plain:.3f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tacaw.run_batch(handles, stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[bench] batched: {t_batch:.3f} s", file=sys.stderr, flush=True)
    os.environ["TACAW_BATCH_STREAMS"] = "1"
    t0 = time.perf_counter()
    tacaw.run_batch(handles, stream)
    torch.cuda.synchronize()
    t_batch1 = time.perf_counter() - t0
    del os.environ["TACAW_BATCH_STREAMS"]
    print(f"[bench] batched on one stream: {t_batch1:.3f} s", file=sys.stderr, flush=True)
    # the batched launch sequence captured once as a HIP graph, then replayed
    with tacaw.Batch(handles) as graph:
        graph.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.launch(stream)
        torch.cuda.synchronize()
        t_graph = time.perf_counter() - t0
    print(f"[bench] batched, graph replay: {t_graph:.3f} s", file=sys.stderr, flush=True)
    for mb in os.environ.get("BENCH_LANE_MB_SWEEP", "").split():
        os.environ["TACAW_BATCH_LANE_MB"] = mb
        for ns in ("1", "4"):
            os.environ["TACAW_BATCH_STREAMS"] = ns
            t0 = time.perf_counter()
            tacaw.run_batch(handles, stream)
            torch.cuda.synchronize()
            print(f"[bench] lane cap {mb} MiB, {ns} streams: {time.perf_counter() - t0:.3f} s",
                  file=sys.stderr, flush=True)
        del os.environ["TACAW_BATCH_STREAMS"], os.environ["TACAW_BATCH_LANE_MB"]
    for h in handles:
        h.destroy()
    ctx.close()
    return {
        "metric": "slice-steps/sec (grid-pts*slices*frames/s), batched uneven jobs",
        "value": steps_total / t_batch, "unit": "slice-steps/s", "n_gpus": 1,
        "plain_value": steps_total / t_plain, "speedup_vs_plain": t_plain / t_batch,
        "ms_batched": t_batch * 1e3, "ms_plain": t_plain * 1e3, "ms_batched_one_stream": t_batch1 * 1e3,
        "ms_batched_graph_replay": t_graph * 1e3, "speedup_graph_vs_plain": t_plain / t_graph,
        "higher_is_better": True,
        "dtype": "fp32", "data": "synthetic",
        "config": {"workload": (f"{args.jobs} seeded uneven small jobs (grids 64-128, 8-48 slices, 16-96 "
                                f"frames, plane wave or probe)") if small else
                               (f"{args.jobs} seeded uneven jobs (grids 128-512, 8-48 slices, "
                                f"128-1024 frames, plane wave or probe)"), "slice_steps": steps_total},
    }


def c5_inputs(n_reg: int, with_big: bool):
    """Seeded request inputs of the serving workload: n_reg uneven jobs of the
    c4 generator (seeds 5000 + i) and, if asked, one 1024^2 x 2048-frame job
    (seed 5500).  Requests cycle over these inputs; every request still gets a
    job of its own (created, planned and uploaded inside its latency)."""
    from paper_2602_10064_amd import workloads
    reg = [workloads.c4_job(i, seed_base=5000) for i in range(n_reg)]
    big = workloads.c4_job(0, seed_base=5500, big=True) if with_big else None
    return reg, big


def bench_c5(args):
    """Serving loop: Poisson arrivals (4 req/s) of uneven jobs plus 10% 1024^2 x 2048-frame jobs.

    Latency of a request runs from its scheduled arrival to its spectrum in
    host memory: the job is created (host planning, encoding, device
    allocation at admission, uploads), served, and its spectrum copied to the
    host, all inside the clock."""
    import threading
    from paper_2602_10064_amd import tacaw, workloads
    times, big = workloads.c5_arrivals(args.requests, rate_per_s=args.rate)
    ctx = tacaw.Context(0)
    t0 = time.perf_counter()
    reg_inputs, big_input = c5_inputs(min(args.requests, 24), bool(big.any()))
    print(f"[bench] serving inputs ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    lat, lib_lat, create_ms, copy_ms, done_steps, finished_at = [], [], [], [], [0], []
    lock = threading.Lock()

    def request(job, arrival):
        tc = time.perf_counter()
        h = tacaw.TacawJob(ctx, job, keep_exit_waves=False, defer_alloc=True)
        tcreate = time.perf_counter() - tc
        h.submit()
        h.wait()
        tw = time.perf_counter()
        spec = h.spectrum()               # to host memory
        t_end = time.perf_counter()
        q, tot = h.latency_ms()
        h.destroy()
        del spec
        with lock:
            lat.append((t_end - arrival) * 1e3)
            lib_lat.append(tot)
            create_ms.append(tcreate * 1e3)
            copy_ms.append((t_end - tw) * 1e3)
            done_steps[0] += job.slice_steps()
            finished_at.append(t_end)

    threads = []
    start = time.perf_counter()
    ri = 0
    for k in range(args.requests):
        now = time.perf_counter() - start
        if times[k] > now:
            time.sleep(times[k] - now)
        if big[k]:
            job = big_input
        else:
            job = reg_inputs[ri % len(reg_inputs)]
            ri += 1
        th = threading.Thread(target=request, args=(job, start + times[k]))
        th.start()
        threads.append(th)
        if k % 20 == 0:
            print(f"[bench] arrived {k + 1}/{args.requests}", file=sys.stderr, flush=True)
    for th in threads:
        th.join()
    elapsed = max(finished_at) - start
    lat = np.array(lat)
    lib_lat = np.array(lib_lat)
    shared, grouped = ctx.serve_stats()
    ctx.close()
    return {
        "metric": "slice-steps/sec (grid-pts*slices*frames/s) + p50/p99 request latency",
        "value": done_steps[0] / elapsed, "unit": "slice-steps/s", "n_gpus": 1,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "p50_ms_from_submit_to_device_result": float(np.percentile(lib_lat, 50)),
        "p99_ms_from_submit_to_device_result": float(np.percentile(lib_lat, 99)),
        "p50_job_create_ms": float(np.percentile(create_ms, 50)),
        "p99_job_create_ms": float(np.percentile(create_ms, 99)),
        "p50_spectrum_to_host_ms": float(np.percentile(copy_ms, 50)),
        "p99_spectrum_to_host_ms": float(np.percentile(copy_ms, 99)),
        "requests": int(args.requests), "rate_per_s": args.rate, "elapsed_s": elapsed,
        "big_requests": int(big.sum()), "shared_pass_launches": int(shared), "requests_in_shared_launches": int(grouped),
        "higher_is_better": True, "dtype": "fp32", "data": "synthetic",
        "latency": "scheduled arrival -> spectrum in host memory, job creation (planning, uploads) included",
        "config": {"workload": "Poisson arrivals of seeded uneven jobs (90%) and 1024^2 x 2048-frame "
                               "jobs (10%), admission by device-memory footprint with backfill, continuous "
                               "batching"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c4small", "c5"],
                    help="c2: the 512^2 x 32 x 1024 plane-wave workload (default); c3: the spectrum "
                         "image; c4: uneven-job batch (c4small: the same on small grids); c5: serving")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=1024, help="frames (1024 = the named workload)")
    ap.add_argument("--cpu-sample", type=int, default=16, help="frames of the oracle baseline (0: skip)")
    ap.add_argument("--timing", default="passes", choices=["passes", "all", "none"],
                    help="kernel classes bracketed with HIP events in the timed region")
    ap.add_argument("--timing-every", type=int, default=7,
                    help="time one launch in this many of each timed class (7: coprime with the "
                         "slice count, so the sampled launches rotate over the slices)")
    ap.add_argument("--kspace", action="store_true",
                    help="c2 on the paper's reciprocal-space potential route (seeded 3 Lorentzian + 3 Gaussian "
                         "coefficients); the structure-factor kernel's MFMA roofline is reported")
    ap.add_argument("--no-host", action="store_true",
                    help="skip the host-transfer figures (profiling runs: they add copy kernels and a run)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding across GPUs (independent frames or "
                          "probes per GPU) is designed, not implemented"}))
        sys.exit(2)

    import torch
    from paper_2602_10064_amd import tacaw, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload in ("c4", "c4small"):
        print(json.dumps(bench_c4(args)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(bench_c5(args)), flush=True)
        return
    t_gen = time.perf_counter()
    if args.workload == "c3":
        job = workloads.c3_probe(n_frames=min(args.frames, 256))
    else:
        job = workloads.c2_plain(n_frames=args.frames)
    if args.kspace:      # the paper's reciprocal-space potential route, seeded coefficients
        job = workloads.with_kirkland(job, seed=2)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] inputs generated in {t_gen:.1f} s", file=sys.stderr, flush=True)

    ctx = tacaw.Context(0)
    torch.cuda.synchronize()
    t_create = time.perf_counter()
    j = tacaw.TacawJob(ctx, job, keep_exit_waves=True)   # plans, allocates, uploads (synchronous)
    t_create = time.perf_counter() - t_create
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        j.run(stream=stream)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # timed region: one launch in --timing-every of the two HBM passes (the
    # roofline candidates) records start/end events; the rest run without
    timed_classes = {"all": None, "passes": ("row", "col"), "none": ()}[args.timing]
    if args.kspace and timed_classes is not None and timed_classes:
        timed_classes = timed_classes + ("splat",)    # the structure-factor kernel is the candidate
    ctx.timing_select(timed_classes, args.timing_every)
    ctx.timing_enable(args.timing != "none")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        j.run(stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = {k: ctx.timing_get(k) for k in ("splat", "row", "col", "time")}
    ctx.timing_enable(False)
    print("[bench] timed steps done", file=sys.stderr, flush=True)
    # one more step, outside the timed region, with every class timed: the
    # per-class breakdown of a step
    ctx.timing_select(None)
    ctx.timing_enable(True)
    j.run(stream=stream)
    torch.cuda.synchronize()
    breakdown_full = {k: ctx.timing_get(k) for k in ("splat", "row", "col", "time")}
    breakdown = {k: round(v[0], 3) for k, v in breakdown_full.items()}
    ctx.timing_enable(False)

    # host transfers, outside the timed region (c2 only: the c3 spectrum is
    # 32 GiB): the spectrum to host memory, and a fresh job from host inputs
    # to the spectrum in host memory
    host = None
    if args.workload == "c2" and not args.no_host:
        t = time.perf_counter()
        spec_host = j.spectrum()
        d2h = time.perf_counter() - t
        d2h_bytes = spec_host.nbytes
        del spec_host
        torch.cuda.synchronize()
        t = time.perf_counter()
        j2 = tacaw.TacawJob(ctx, job, keep_exit_waves=False)
        j2.run(stream=stream)
        spec2 = j2.spectrum()
        h2h = time.perf_counter() - t
        j2.destroy()
        del spec2
        host = {"job_create_ms": round(t_create * 1e3, 1),
                "h2d_bytes": int(job.n_frames * job.n_atoms * 16),
                "d2h_spectrum_ms": round(d2h * 1e3, 1), "d2h_bytes": int(d2h_bytes),
                "d2h_GBps": round(d2h_bytes / d2h / 1e9, 2),
                "host_to_host_ms": round(h2h * 1e3, 1),
                "note": "job_create: planning on the host, device allocation, upload of the encoded positions "
                        "(16 B per frame and atom) and tables; host_to_host: a fresh job from host arrays to "
                        "the spectrum in host memory"}
        print(f"[bench] host transfers: {host}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    ms_per_step = elapsed / args.steps * 1e3
    slice_steps = job.nx * job.ny * job.n_slices * job.n_frames * job.n_probes
    value = slice_steps / (elapsed / args.steps)

    # roofline of the dominant kernel class: the timed class with the largest
    # total time in the timed region
    timed = {k: v for k, v in timing.items() if v[1] > 0 and k in ("row", "col", "splat")}
    roofline_kpot = None
    if args.kspace and "splat" in timed:
        # structure factors on MFMA: 8 real flops (one complex multiply-add)
        # per atom and computed k point (rows 0 .. ny/2 of the potential grid)
        # per frame, every atom lying in one slice; one launch covers a frame
        # batch and a group of slices (the breakdown step, with every launch
        # timed, counts the launches of a step)
        ms, n = timed.pop("splat")
        avg_ms = ms / n
        pnx, pny = job.pot_nx or job.nx, job.pot_ny or job.ny
        flops_step = 8.0 * (pny // 2 + 1) * pnx * job.n_atoms * job.n_frames
        flops_launch = flops_step / breakdown_full["splat"][1]
        tflops = flops_launch / (avg_ms * 1e-3) / 1e12
        roofline_kpot = {"bound": "mfma", "kernel": "structure factors (k_kpot)", "achieved": round(tflops, 2),
                         "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tflops / FP32_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                         "avg_launch_ms": round(avg_ms, 4), "launches": n,
                         "algorithmic_flops_per_launch": flops_launch}
    roofline = None
    if timed:
        dom = max(timed, key=lambda k: timed[k][0])
        ms, n = timed[dom]
        # every launch of a pass advances one frame batch by one slice; the
        # last batch may be shorter, so take the mean batch of the step
        fb = j.plan()[0]
        n_batches = -(-job.n_frames // fb)
        units = job.nx * job.ny * job.n_probes * job.n_frames / n_batches
        avg_ms = ms / n
        achieved = BYTES_PER_UNIT[dom] * units / (avg_ms * 1e-3) / 1e9
        # counter-measured HBM bytes per launch, when they were taken for this
        # grid and frame batch with the kernels as they are now
        traffic = None
        tpath = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tpath):
            tr = json.load(open(tpath))
            if (tr.get("source_hash") == kernel_source_hash() and dom in tr.get("per_launch_bytes", {})
                    and tr.get("grid") == [job.nx, job.ny] and tr.get("frame_batch") == fb
                    and tr.get("probes") == job.n_probes):
                # measured on full batches; scaled to the mean batch like `units`
                traffic = tr["per_launch_bytes"][dom] * (job.n_frames / n_batches) / fb
        roofline = {"bound": "hbm", "kernel": f"{dom} pass", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic, "avg_launch_ms": round(avg_ms, 4), "launches": n,
                    "algorithmic_bytes_per_launch": BYTES_PER_UNIT[dom] * units}
    # potentials are written once per (frame, slice) on the potential grid and
    # shared by all probes
    pot_pts = (job.pot_nx or job.nx) * (job.pot_ny or job.ny)
    model_bytes = (BYTES_PER_UNIT["row"] + BYTES_PER_UNIT["col"]) * slice_steps + \
        BYTES_PER_UNIT["splat"] * pot_pts * job.n_frames * job.n_slices + \
        BYTES_PER_UNIT["time"] * job.nx * job.ny * job.n_frames * job.n_probes
    kernel_ms = {k: round(v[0] / args.steps, 3) for k, v in timing.items() if v[1] > 0}

    cpu = None
    if args.cpu_sample > 0:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        if args.workload == "c3":
            # 4 probe positions x the sample frames, full windows and slices
            sub = job.replace(probe_xy=job.probe_xy[:4], positions=job.positions[:args.cpu_sample])
            cpu = cpu_baseline(sub, args.cpu_sample, slice_steps,
                               what="4 of the 1024 probe positions x %d of the "
                               "256 frames (256^2 windows, all 20 slices, potentials on the 1000x866 "
                               "grid, spectrum of the sample)" % args.cpu_sample)
        else:
            cpu = cpu_baseline(job, args.cpu_sample, slice_steps)

    out = {
        "metric": "slice-steps/sec (grid-pts*slices*frames/s) + %HBM peak",
        "value": value,
        "unit": "slice-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": (WORKLOAD_C3 if args.workload == "c3" else WORKLOAD) +
                               (", reciprocal-space potentials (paper's route)" if args.kspace else ""),
                   "grid": [job.nx, job.ny], "slices": job.n_slices,
                   "frames": job.n_frames, "probes": job.n_probes, "atoms": job.n_atoms,
                   "precision": "complex64 (FP32) multislice and time FFT, FP64 frame mean"},
        "hbm_effective_GBps": round(model_bytes / (elapsed / args.steps) / 1e9, 1),
        "hbm_frac": round(model_bytes / (elapsed / args.steps) / 1e9 / HBM_PEAK_GBPS, 4),
        "kernel_ms_per_step": breakdown,
        "timed_region_kernel_ms_per_step": kernel_ms,
        "host_transfers": host,
        "roofline": roofline,
        **({"roofline_kpot": roofline_kpot} if roofline_kpot else {}),
        "cpu_baseline": cpu,
        # the device code and planner this run was built from (counter runs
        # record it so that their bytes are used only while it holds)
        "kernel_source_hash": kernel_source_hash(),
    }
    j.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
