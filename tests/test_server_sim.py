"""Admission and batching policy of the server, driven on the CPU through
the C ABI with the simulated executor (no device calls): budget accounting,
queue-full and too-large rejections, continuous batching, FIFO mode,
injected batch failures and memory release."""

import time
import types

import pytest

import synth

torch = pytest.importorskip("torch")
from paper_2605_11489_amd import abi  # noqa: E402
from paper_2605_11489_amd.serve import Server  # noqa: E402


def fake_scene(n, deg=3):
    return types.SimpleNamespace(n=n, sh_degree=deg)


def cam(W, H):
    return synth.look_at_camera((0.0, 0.0, -4.0), W, H)


def wait_all(srv, tickets, timeout=10.0, release=False):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
                    if release:
                        srv.release(t)
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.001)
    return res


def test_continuous_batching_groups_requests_arriving_during_a_batch():
    with Server(8 << 30, max_batch=16, n_streams=1, simulate=True, sim_batch_us=20000) as srv:
        sid = srv.register(fake_scene(100_000))
        first = srv.submit(sid, cam(320, 180))
        time.sleep(0.005)                      # first batch is now "on the GPU"
        rest = [srv.submit(sid, cam(640, 360)) for _ in range(10)]
        res = wait_all(srv, [first] + rest)
        assert res[first].batch_size == 1
        assert all(res[t].batch_size == 10 for t in rest)
        assert all(r.status == 0 for r in res.values())
        st = srv.stats()
        assert st["batches"] == 2 and st["max_batch"] == 10
        for t in [first] + rest:
            srv.release(t)


def test_work_queue_mode_batches_alike():
    """Work-queue mode changes only how a batch is composited on the device:
    in a dry run the batching is the same (frames of different sizes that
    arrive during a batch form the next one), and every frame completes at
    its batch's end (no device, so no completion words: flag_done stays 0)."""
    with Server(8 << 30, max_batch=16, n_streams=1, simulate=True, sim_batch_us=20000, work_queue=True) as srv:
        sid = srv.register(fake_scene(100_000))
        first = srv.submit(sid, cam(320, 180))
        time.sleep(0.005)
        big = [srv.submit(sid, cam(1920, 1080)) for _ in range(3)]
        small = srv.submit(sid, cam(320, 180))
        res = wait_all(srv, [first] + big + [small])
        assert all(r.status == 0 and r.flag_done == 0 for r in res.values())
        assert res[small].batch_size == 4 and all(res[t].batch_size == 4 for t in big)
        st = srv.stats()
        assert st["batches"] == 2 and st["flag_done"] == 0
        for t in [first] + big + [small]:
            srv.release(t)


def test_fifo_mode_runs_one_frame_per_launch_in_order():
    with Server(8 << 30, fifo=True, n_streams=2, simulate=True, sim_batch_us=2000) as srv:
        sid = srv.register(fake_scene(100_000))
        ts = [srv.submit(sid, cam(320, 180)) for _ in range(6)]
        res = wait_all(srv, ts)
        assert all(r.batch_size == 1 for r in res.values())
        starts = [res[t].t_start for t in ts]
        assert starts == sorted(starts)
        for a, b in zip(ts, ts[1:]):
            assert res[b].t_start >= res[a].t_done - 1e-3
        assert srv.stats()["batches"] == 6


def test_budget_bounds_memory_and_requests_queue_for_it():
    with Server(64 << 20, max_batch=64, n_streams=4, simulate=True, sim_batch_us=3000) as srv:
        sid = srv.register(fake_scene(50_000))
        ts = [srv.submit(sid, cam(960, 540)) for _ in range(12)]
        res = wait_all(srv, ts, release=True)
        st = srv.stats()
        assert st["bytes_peak"] <= 64 << 20
        assert all(r.status == 0 for r in res.values())
        # 960x540 outputs alone are 27 MB: at most two frames fit at once
        assert max(r.batch_size for r in res.values()) <= 2
        assert st["bytes_in_use"] < 14 << 20    # only the scene stays


def test_queue_full_returns_again():
    with Server(1 << 30, queue_depth=3, n_streams=1, simulate=True, sim_batch_us=50000) as srv:
        sid = srv.register(fake_scene(1000))
        codes = [srv.submit_rc(sid, cam(64, 64))[0] for _ in range(8)]
        assert abi.GS_ERR_AGAIN in codes
        assert codes[0] == 0
        assert srv.stats()["rejected"] >= 1


def test_too_large_and_unknown_scene():
    with Server(16 << 20, simulate=True) as srv:
        sid = srv.register(fake_scene(1000))
        rc, _ = srv.submit_rc(sid, cam(1920, 1080))       # 108 MB of outputs > 16 MB budget
        assert rc == abi.GS_ERR_TOO_LARGE
        rc, _ = srv.submit_rc(sid + 7, cam(64, 64))
        assert rc == abi.GS_ERR_NOT_FOUND


def test_scene_larger_than_budget_is_oom():
    with Server(8 << 20, simulate=True) as srv:
        with pytest.raises(abi.GsError) as e:
            srv.register(fake_scene(1_000_000))
        assert e.value.code == abi.GS_ERR_OOM


def test_injected_batch_failures_are_reported_and_serving_continues():
    with Server(1 << 30, max_batch=1, n_streams=1, simulate=True, sim_batch_us=500, sim_fail_every=3) as srv:
        sid = srv.register(fake_scene(1000))
        ts = [srv.submit(sid, cam(64, 64)) for _ in range(9)]
        res = wait_all(srv, ts)
        failed = [t for t in ts if res[t].status != 0]
        assert len(failed) == 3 and all(res[t].status == abi.GS_ERR_HIP for t in failed)
        ok = [t for t in ts if res[t].status == 0]
        assert len(ok) == 6
        st = srv.stats()
        assert st["failed"] == 3 and st["completed"] == 6
        # failed requests hold no memory; released ones give theirs back
        for t in ts:
            srv.release(t)
        more = srv.submit(sid, cam(64, 64))
        assert wait_all(srv, [more])[more].status in (0, abi.GS_ERR_HIP)


def test_poll_and_release_errors():
    with Server(1 << 30, n_streams=1, simulate=True, sim_batch_us=100000) as srv:
        sid = srv.register(fake_scene(1000))
        t = srv.submit(sid, cam(64, 64))
        assert srv.poll(t) is None
        with pytest.raises(abi.GsError) as e:
            srv.release(t)
        assert e.value.code == abi.GS_ERR_NOT_READY
        with pytest.raises(abi.GsError) as e:
            srv.poll(t + 100)
        assert e.value.code == abi.GS_ERR_NOT_FOUND


def test_bad_options():
    with pytest.raises(abi.GsError):
        Server(1 << 30, max_batch=0, simulate=True)
    with pytest.raises(abi.GsError):
        Server(1 << 30, key_factor=0.5, simulate=True)


def test_budget_left_by_resident_scenes_bounds_admission():
    """A request is judged against what the resident scenes leave of the
    budget, not the whole budget: with room for the scene plus a little,
    a 320x180 frame is admitted and rendered, a 1920x1080 frame (108 MB of
    outputs alone) is refused at submission."""
    n, deg = 100_000, 3
    scene_bytes = n * (12 + 12 + 16 + 4 + 12 * (deg + 1) ** 2)
    with Server(scene_bytes + (48 << 20), max_batch=4, n_streams=1, simulate=True, sim_batch_us=500) as srv:
        sid = srv.register(fake_scene(n, deg))
        rc, _ = srv.submit_rc(sid, cam(1920, 1080))
        assert rc == abi.GS_ERR_TOO_LARGE
        small = srv.submit(sid, cam(320, 180))
        res = wait_all(srv, [small])
        assert res[small].status == 0
        srv.release(small)
        assert srv.stats()["rejected"] == 1


def test_heavy_frames_run_alone_and_keep_arrival_order():
    """Cost-aware admission: a frame whose class is estimated at or above
    heavy_ms waits for the device to be free; beside it only tiny frames (a
    quarter of heavy_ms and below) start, the light frames queued behind it
    wait for it (arrival order), then batch together.  With heavy_ms = 0 the
    same heavy frame shares the device at once.  (Simulated estimates: 6M
    Gaussians at 1920x1080 ~0.43 ms, 1M at 320x180 ~0.11 ms, 100k ~0.06 ms.)"""
    for heavy_ms, alone in ((0.3, True), (0.0, False)):
        with Server(64 << 30, max_batch=8, n_streams=3, simulate=True, sim_batch_us=20000,
                    heavy_ms=heavy_ms) as srv:
            tiny_scene = srv.register(fake_scene(100_000))
            light_scene = srv.register(fake_scene(1_000_000))
            big = srv.register(fake_scene(6_000_000))
            l1 = srv.submit(light_scene, cam(320, 180))
            time.sleep(0.005)
            h = srv.submit(big, cam(1920, 1080))
            l2 = srv.submit(light_scene, cam(320, 180))
            l3 = srv.submit(light_scene, cam(640, 360))
            res = wait_all(srv, [l1, h, l2, l3])
            assert all(r.status == 0 for r in res.values())
            if alone:
                assert res[h].t_start >= res[l1].t_done - 1e-3 and res[h].batch_size == 1
                assert res[l2].t_start >= res[h].t_done - 1e-3 and res[l3].t_start >= res[h].t_done - 1e-3
                assert res[l2].batch_size == 2 and res[l3].batch_size == 2
                # a tiny frame submitted while the heavy one runs starts beside it
                h2 = srv.submit(big, cam(1920, 1080))
                time.sleep(0.005)
                t = srv.submit(tiny_scene, cam(320, 180))
                r2 = wait_all(srv, [h2, t])
                assert r2[t].t_start < r2[h2].t_done
                srv.release(h2)
                srv.release(t)
            else:
                assert res[h].t_start < res[l1].t_done
            for tk in (l1, h, l2, l3):
                srv.release(tk)
