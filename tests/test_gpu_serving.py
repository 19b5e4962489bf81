"""The continuous-batching server on the GPU: every request's outputs are
bit-identical alone (gs_render_forward of the same scene and camera) and in
the mix (batched with requests of other scenes and resolutions), in batched
and FIFO modes and after a key-capacity retry; served frames of every
resolution class match the FP64 oracle.  In work-queue mode the server
composites batches through the persistent work-queue kernel and reports
frames done from their completion words: frames read the moment they are
reported done (while a large frame of the same batch may still be
composited) are complete, and the wide list-position encoding that large
key capacities select is checked too."""

import time

import numpy as np
import pytest

import oracle
import synth
from tests.parity import compare_frame, gpu_outputs_numpy

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_11489_amd import render as R  # noqa: E402
from paper_2605_11489_amd.serve import Server  # noqa: E402

KEYS = ("rgb", "alpha", "depth", "dcdx", "dcdy", "final_T", "n_contrib")


def say(msg):
    print(msg, flush=True)


def wait(srv, tickets, timeout=60.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.0005)
    return res


def alone(ds, cam, bg):
    fr = R.render(ds, cam, bg=bg)
    assert R.forward_status(fr)[0] == 0
    return fr.outputs[0]


@pytest.fixture(scope="module")
def host_scenes():
    return [synth.gen_clustered(51, 20_000, 3), synth.gen_clustered(52, 60_000, 1)]


@pytest.fixture(scope="module")
def scenes(host_scenes):
    return [R.DeviceScene.from_host(s) for s in host_scenes]


@pytest.mark.parametrize("fifo,work_queue", [(False, False), (True, False), (False, True)])
def test_results_identical_alone_and_in_the_mix(scenes, fifo, work_queue):
    say(f"case: server fifo={fifo} work_queue={work_queue}, 24 mixed requests over 2 scenes and 4 resolutions")
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(24):
        s = int(rng.integers(2))
        W, H = synth.SERVING_RESOLUTIONS[int(rng.integers(4))]
        eye = synth.sphere_poses(rng, 1)[0]
        bg = tuple(float(x) for x in rng.uniform(0, 1, 3))
        reqs.append((s, synth.look_at_camera(eye, W, H), bg))
    with Server(4 << 30, max_batch=8, n_streams=2, fifo=fifo, work_queue=work_queue) as srv:
        ids = [srv.register(ds) for ds in scenes]
        tickets = [srv.submit(ids[s], cam, bg=bg) for s, cam, bg in reqs]
        res = wait(srv, tickets)
        sizes = [res[t].batch_size for t in tickets]
        say(f"  batch sizes: {sorted(set(sizes))}")
        if fifo:
            assert set(sizes) == {1}
        for t, (s, cam, bg) in zip(tickets, reqs):
            r = res[t]
            assert r.status == 0
            got = srv.outputs(r)
            ref = alone(scenes[s], cam, bg)
            for k in KEYS:
                assert torch.equal(got[k], ref[k]), (t, k)
            srv.release(t)
        st = srv.stats()
        say(f"  stats: {st}")
        assert st["completed"] == 24 and st["failed"] == 0
        # with the work queue, every frame but the last of each batch is
        # reported done from its completion word, written by the compositing
        # kernel (the last completes with its batch); without it, none
        assert st["flag_done"] == (24 - st["batches"] if work_queue else 0)


def test_capacity_retry_gives_identical_result(scenes):
    say("case: server key-capacity overflow and retry")
    with Server(4 << 30, max_batch=4, n_streams=1, key_factor=1.0) as srv:
        sid = srv.register(scenes[0])
        far = synth.look_at_camera((0.0, 0.0, -9.0), 320, 180)    # few pairs: sets the class estimate
        near = synth.look_at_camera((0.0, 0.0, -2.5), 320, 180)   # many more pairs, same class
        t1 = srv.submit(sid, far)
        wait(srv, [t1])
        t2 = srv.submit(sid, near)
        r = wait(srv, [t2])[t2]
        assert r.status == 0 and r.retries >= 1
        got = srv.outputs(r)
        ref = alone(scenes[0], near, (0.0, 0.0, 0.0))
        for k in KEYS:
            assert torch.equal(got[k], ref[k]), k
        srv.release(t1)
        srv.release(t2)


@pytest.mark.parametrize("work_queue", [False, True])
def test_capacity_retry_of_a_batch(scenes, work_queue):
    """Two frames whose pairs outgrow their class estimate (key factor 1),
    queued behind a blocker frame so that they usually share a batch: the
    overflowed batch composites nothing (in work-queue mode the queue kernel
    publishes nothing) and both frames are re-run with more room; both then
    equal the frames rendered alone, and at least one was retried."""
    say(f"case: server capacity overflow of a two-frame batch, work_queue={work_queue}")
    with Server(4 << 30, max_batch=2, n_streams=1, key_factor=1.0, heavy_ms=0.0, work_queue=work_queue) as srv:
        ids = [srv.register(ds) for ds in scenes]
        far = synth.look_at_camera((0.0, 0.0, -9.0), 480, 272)   # few pairs: sets the class estimate
        t = srv.submit(ids[0], far)
        wait(srv, [t])
        srv.release(t)
        near = [synth.look_at_camera((0.1, 0.0, -2.5), 480, 272), synth.look_at_camera((-0.1, 0.1, -2.6), 480, 272)]
        t_block = srv.submit(ids[1], synth.look_at_camera((0.0, 0.0, -3.0), 1920, 1080))
        tickets = [srv.submit(ids[0], cam) for cam in near]
        res = wait(srv, tickets + [t_block])
        assert res[t_block].status == 0
        assert max(res[t].retries for t in tickets) >= 1
        say(f"  batch sizes {[res[t].batch_size for t in tickets]}, retries {[res[t].retries for t in tickets]}")
        for t, cam in zip(tickets, near):
            r = res[t]
            assert r.status == 0
            got = srv.outputs(r)
            ref = alone(scenes[0], cam, (0.0, 0.0, 0.0))
            for k in KEYS:
                assert torch.equal(got[k], ref[k]), (t, k)
        for t in tickets + [t_block]:
            srv.release(t)


def test_served_frames_match_the_oracle(scenes, host_scenes):
    """One mixed batch with a frame of each resolution class (320x180 up to
    1920x1080) of both scenes: every served frame against the FP64 oracle
    on sampled tiles (the longest list, the last tile and six random ones),
    images and gradient buffers within 1e-4 and n_contrib exact."""
    say("case: served frames of all four resolution classes vs the FP64 oracle")
    rng = np.random.default_rng(13)
    reqs = []
    for k, (W, H) in enumerate(synth.SERVING_RESOLUTIONS):
        for s in range(2):
            eye = synth.sphere_poses(rng, 1)[0]
            bg = tuple(float(x) for x in rng.uniform(0, 1, 3))
            reqs.append((s, synth.look_at_camera(eye, W, H), bg))
    with Server(4 << 30, max_batch=8, n_streams=2) as srv:
        ids = [srv.register(ds) for ds in scenes]
        tickets = [srv.submit(ids[s], cam, bg=bg) for s, cam, bg in reqs]
        res = wait(srv, tickets)
        say(f"  batch sizes: {sorted(set(res[t].batch_size for t in tickets))}")
        for t, (s, cam, bg) in zip(tickets, reqs):
            r = res[t]
            assert r.status == 0
            got = gpu_outputs_numpy(srv.outputs(r))
            of = oracle.render_forward(host_scenes[s], cam, bg=bg, composite_all=False)
            nt = of.ranges.shape[0]
            lens = of.ranges[:, 1] - of.ranges[:, 0]
            tiles = sorted(set(rng.choice(nt, min(6, nt), replace=False).tolist())
                           | {int(np.argmax(lens)), nt - 1})
            of.image = oracle.composite.composite_image(of.proj, of.values, of.ranges, cam.width, cam.height,
                                                        of.bg, tiles=tiles)
            st = compare_frame(got, of, tiles=tiles)
            say(f"  scene {s} {cam.width}x{cam.height}: pixels={st['pixels']} "
                f"max err={st['clean_max_err']:.2e} flipped={st['flipped']}")
            assert not st["unresolved"], st["unresolved"][:3]
            assert st["clean_max_err"] <= 1e-4
            srv.release(t)


def test_frames_complete_from_their_words_while_the_batch_runs(scenes):
    """Work-queue mode: a tiny frame and a 1920x1080 frame queued behind a
    blocker frame (1M Gaussians at 1920x1080, about 0.6 ms, far longer than
    the two submissions behind it, and estimated above the 0.3-ms heavy
    threshold, so that it runs in a batch of its own), so that the two form
    the next batch together.  The frame first in the batch's work queue (shortest estimated
    first, so usually the tiny one) is reported done from its completion
    word, the other with its batch.  Whichever is reported first is read at
    once (a device copy on another stream), possibly while the other is still
    being composited; that copy, and later the other frame, equal the frames
    rendered alone, bit for bit.  Repeated until three shared batches (at
    most 24 rounds)."""
    say("case: work-queue early completion, 320x180 next to 1920x1080 in one batch")
    rng = np.random.default_rng(17)
    shared = early = rounds = 0
    heavy = R.DeviceScene.from_host(synth.gen_clustered(53, 1_000_000, 3))
    with Server(4 << 30, max_batch=2, n_streams=1, heavy_ms=0.3, work_queue=True) as srv:
        ids = [srv.register(ds) for ds in scenes]
        id_heavy = srv.register(heavy)
        while shared < 3 and rounds < 24:
            rounds += 1
            e_block, e_small, e_big = synth.sphere_poses(rng, 3)
            block = synth.look_at_camera(e_block, 1920, 1080)
            small = synth.look_at_camera(e_small, 320, 180)
            big = synth.look_at_camera(e_big, 1920, 1080)
            t_block = srv.submit(id_heavy, block)
            t_big = srv.submit(ids[1], big)
            t_small = srv.submit(ids[0], small)
            frames = {t_small: (scenes[0], small), t_big: (scenes[1], big)}
            # the first of the two frames reported done, read at once
            first = None
            t0 = time.time()
            while first is None:
                for t in (t_small, t_big):
                    r = srv.poll(t)
                    if r is not None:
                        first = (t, r)
                        break
                assert time.time() - t0 < 60.0, "server did not finish"
            t1, r1 = first
            snap = {k: v.clone() for k, v in srv.outputs(r1).items()}
            torch.cuda.synchronize()
            assert r1.status == 0
            t2 = t_big if t1 == t_small else t_small
            other_running = srv.poll(t2) is None
            res = wait(srv, [t2, t_block])
            r2 = res[t2]
            assert r2.status == 0 and res[t_block].status == 0
            # (arrival order: the blocker goes first, so a batch of two holding
            # the tiny frame, the last to arrive, pairs it with the large one)
            r_small = r1 if t1 == t_small else r2
            if r_small.batch_size == 2:
                assert r1.batch_size == 2 and r2.batch_size == 2
                # one frame of the pair was published by the kernel, the
                # other (last in the queue) completed with the batch
                assert sorted((r1.flag_done, r2.flag_done)) == [0, 1]
                shared += 1
                early += int(r1.flag_done == 1 and other_running)
            for t, got in ((t1, snap), (t2, srv.outputs(r2))):
                ds, cam = frames[t]
                ref = alone(ds, cam, (0.0, 0.0, 0.0))
                for k in KEYS:
                    assert torch.equal(got[k], ref[k]), (rounds, t == t_small, k)
            for t in (t_block, t_big, t_small):
                srv.release(t)
    say(f"  {shared} shared batches in {rounds} rounds; a frame read from its word while the other ran in {early}")
    assert shared >= 3


def test_wide_positions_in_the_work_queue_kernel(scenes):
    """Work-queue mode: a key factor that takes the capacity to 2^28 pairs or
    more selects the wide list-position encoding of the work-queue kernel;
    its frames (two poses of one class in one batch, the first published
    from its completion word) equal the same frames rendered alone."""
    cams = [synth.look_at_camera((0.3, -0.2, -3.0), 320, 180), synth.look_at_camera((-0.4, 0.1, -3.4), 320, 180)]
    jobs = R.make_jobs([(scenes[0], cams[0], R.opts_struct(), R.alloc_outputs(320, 180))])
    est = R.count_keys(jobs, 1)[0]
    factor = float((1 << 28) / est) * 1.01
    say(f"case: wide queue kernel, {est} pairs, key factor {factor:.0f}")
    with Server(16 << 30, max_batch=2, n_streams=1, key_factor=factor, work_queue=True) as srv:
        sid = srv.register(scenes[0])
        tickets = [srv.submit(sid, cam) for cam in cams]
        res = wait(srv, tickets)
        for t, cam in zip(tickets, cams):
            r = res[t]
            assert r.status == 0
            ref = alone(scenes[0], cam, (0.0, 0.0, 0.0))
            got = srv.outputs(r)
            for k in KEYS:
                assert torch.equal(got[k], ref[k]), (t, k)
            srv.release(t)
