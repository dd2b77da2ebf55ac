"""Serving loop through the C ABI (needs an MI355X): admission by footprint,
continuous batching across requests, cancellation, and bitwise equality of
every result alone and in the mix."""
import time

import numpy as np
import pytest

from paper_2602_10064_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tacaw():
    import torch
    assert torch.cuda.is_available()
    from paper_2602_10064_amd import tacaw as t
    t.lib()
    return t


def mix():
    jobs = [
        w.c1_tiny(n_frames=32),
        w.random_small_job(31, nx=96, ny=64, n_slices=5, n_frames=10, cell=(12.0, 8.0, 6.0), n_atoms=12),
        w.random_small_job(32, nx=64, ny=64, n_slices=3, n_frames=8, cell=(8.0, 8.0, 4.0),
                           aperture_mrad=30.0, n_probes=3, voltage_V=60e3),
        w.random_small_job(33, nx=32, ny=32, n_slices=3, n_frames=12, cell=(10.0, 9.0, 4.0),
                           aperture_mrad=25.0, n_probes=4, pot_grid=(100, 90)),
        w.c2_plain(n_frames=6, grid=256, n_slices=8, reps=(6, 6, 2)),
        w.random_small_job(34, nx=128, ny=128, n_slices=4, n_frames=16, cell=(16.0, 16.0, 5.0),
                           n_atoms=30, two_sided=True),
    ]
    return jobs


def alone(tacaw, ctx, job):
    with tacaw.TacawJob(ctx, job) as j:
        j.run()
        return j.spectrum()


def test_alone_vs_mix_bitwise(tacaw):
    jobs = mix()
    with tacaw.Context(0) as ctx:
        ref = [alone(tacaw, ctx, j) for j in jobs]
    # a budget that holds about two of these jobs at once forces queueing
    fps = sorted(tacaw.footprint(j) for j in jobs)
    budget = fps[-1] + fps[-2] + (64 << 20)
    with tacaw.Context(0, hbm_budget_bytes=budget) as ctx:
        handles = [tacaw.TacawJob(ctx, j, defer_alloc=True) for j in jobs]
        for h in handles:
            h.submit()
        for h in handles:
            h.wait()
            assert h.poll()
        for h, r in zip(handles, ref):
            got = h.spectrum()
            assert np.array_equal(got.view(np.uint32), r.view(np.uint32)), h.job.name
            q, t = h.latency_ms()
            assert 0 <= q <= t
        for h in handles:
            h.destroy()


def test_cancel_and_reject(tacaw):
    jobs = mix()
    with tacaw.Context(0) as ctx:
        ref = [alone(tacaw, ctx, j) for j in jobs[:3]]
    big = w.c2_plain(n_frames=128)           # 256 MiB of exit waves alone
    with tacaw.Context(0, hbm_budget_bytes=200 << 20) as ctx:
        hb = tacaw.TacawJob(ctx, big, defer_alloc=True)
        with pytest.raises(tacaw.TacawError) as e:
            hb.submit()                       # can never fit 200 MiB: rejected
        assert e.value.status == 2
        hb.destroy()
        hs = [tacaw.TacawJob(ctx, j, defer_alloc=True) for j in jobs[:3]]
        victim = tacaw.TacawJob(ctx, w.c1_tiny(n_frames=64), defer_alloc=True)
        for h in hs[:2]:
            h.submit()
        victim.submit()
        victim.cancel()
        hs[2].submit()
        with pytest.raises(tacaw.TacawError) as e:
            victim.wait()
        assert e.value.status == 6
        for h, r in zip(hs, ref):
            h.wait()
            assert np.array_equal(h.spectrum().view(np.uint32), r.view(np.uint32))
        # a cancelled job can be submitted again and completes
        victim.submit()
        victim.wait()
        assert np.isfinite(victim.spectrum()).all()
        for h in hs + [victim]:
            h.destroy()


def test_streamed_arrivals_overlap(tacaw):
    # requests arrive while others run; all complete with latency recorded
    rng = np.random.default_rng(5)
    jobs = [w.c1_tiny(n_frames=32, seed=s) for s in range(1, 9)]
    with tacaw.Context(0) as ctx:
        hs = []
        for j in jobs:
            h = tacaw.TacawJob(ctx, j, defer_alloc=True)
            h.submit()
            hs.append(h)
            time.sleep(float(rng.exponential(0.002)))
        for h in hs:
            h.wait()
        lat = np.array([h.latency_ms()[1] for h in hs])
        assert np.all(lat > 0)
        for h in hs:
            h.destroy()


def test_cancelled_job_then_plain_run(tacaw):
    # a job cancelled in the serving loop and then run in the plain form
    # reports that run's spectrum, not the cancellation
    jobs = mix()
    victim_job = w.c1_tiny(n_frames=64)
    with tacaw.Context(0) as ctx:
        ref = alone(tacaw, ctx, victim_job)
    with tacaw.Context(0) as ctx:
        hs = [tacaw.TacawJob(ctx, j, defer_alloc=True) for j in jobs[:2]]
        victim = tacaw.TacawJob(ctx, victim_job, defer_alloc=True)
        for h in hs:
            h.submit()
        victim.submit()
        victim.cancel()
        with pytest.raises(tacaw.TacawError) as e:
            victim.wait()
        assert e.value.status == 6
        victim.run()
        assert np.array_equal(victim.spectrum().view(np.uint32), ref.view(np.uint32))
        for h in hs:
            h.wait()
        for h in hs + [victim]:
            h.destroy()


def test_c5_requests_alone_vs_mix(tacaw):
    """The first 16 requests of the serving workload (Poisson arrivals at
    4 req/s; 13 uneven jobs of the c4 generator and three 1024^2 x 2048-frame
    jobs), each run alone, then all submitted to the serving loop at once:
    every spectrum is the same bit for bit."""
    times, big = w.c5_arrivals(16)
    big_job = w.c4_job(0, seed_base=5500, big=True)
    jobs, ri = [], 0
    for k in range(16):
        if big[k]:
            jobs.append(big_job)
        else:
            jobs.append(w.c4_job(ri, seed_base=5000))
            ri += 1
    print(f"[gpu] c5 mix: {int(big.sum())} big jobs of {big_job.slice_steps():.3e} slice-steps, "
          f"{16 - int(big.sum())} uneven jobs", flush=True)
    with tacaw.Context(0) as ctx:
        handles = [tacaw.TacawJob(ctx, j, keep_exit_waves=False, defer_alloc=True) for j in jobs]
        ref = []
        for h in handles:
            h.run()
            ref.append(h.spectrum())
        print("[gpu] c5 mix: alone runs done", flush=True)
        for h in handles:
            h.submit()
        for h, r in zip(handles, ref):
            h.wait()
            got = h.spectrum()
            assert np.array_equal(got.view(np.uint32), r.view(np.uint32)), h.job.name
        for h in handles:
            h.destroy()


def test_shared_launches_across_requests(tacaw, monkeypatch):
    """Small requests of one grid size run in shared launches (one launch
    advances a frame batch of each by one slice, or through a slice group on
    the LDS-resident grids), with results bitwise those of each job alone; a
    second grid size forms a group of its own.  A batching window lets the
    requests submitted together start together, so the launches are shared
    whatever the host's timing."""
    monkeypatch.setenv("TACAW_SERVE_BATCH_WINDOW_MS", "500")
    jobs = [w.random_small_job(60 + i, nx=64, ny=64, n_slices=40 + 8 * (i % 3), n_frames=16 + 8 * (i % 2),
                               cell=(8.0, 8.0, 30.0), n_atoms=40) for i in range(6)]
    jobs += [w.random_small_job(70 + i, nx=96, ny=64, n_slices=40, n_frames=10, cell=(12.0, 8.0, 30.0), n_atoms=30,
                                aperture_mrad=25.0, n_probes=2, voltage_V=60e3) for i in range(3)]
    with tacaw.Context(0) as ctx:
        ref = [alone(tacaw, ctx, j) for j in jobs]
    with tacaw.Context(0) as ctx:
        hs = [tacaw.TacawJob(ctx, j, defer_alloc=True) for j in jobs]
        for h in hs:
            h.submit()
        for h in hs:
            h.wait()
        shared, grouped = ctx.serve_stats()
        print(f"[gpu] shared launches {shared}, grouped jobs {grouped}", flush=True)
        for h, r in zip(hs, ref):
            got = h.spectrum()
            assert np.array_equal(got.view(np.uint32), r.view(np.uint32)), h.job.name
            h.destroy()
    assert grouped == len(jobs)
    assert shared > 0


def test_lone_requests_share_nothing(tacaw):
    """Small requests served one after another (each waits for the previous)
    run in lane groups of their own: no pass launch serves two of them, and
    none counts as grouped; results are bitwise those of each job alone."""
    jobs = [w.random_small_job(80 + i, nx=64, ny=64, n_slices=6, n_frames=8, cell=(8.0, 8.0, 6.0), n_atoms=20)
            for i in range(3)]
    with tacaw.Context(0) as ctx:
        ref = [alone(tacaw, ctx, j) for j in jobs]
    with tacaw.Context(0) as ctx:
        for j, r in zip(jobs, ref):
            h = tacaw.TacawJob(ctx, j, defer_alloc=True)
            h.submit()
            h.wait()
            assert np.array_equal(h.spectrum().view(np.uint32), r.view(np.uint32)), j.name
            h.destroy()
        shared, grouped = ctx.serve_stats()
        print(f"[gpu] shared launches {shared}, grouped jobs {grouped}", flush=True)
    assert shared == 0 and grouped == 0
