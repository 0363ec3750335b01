"""GPU tests of the request loop (mpmx_server_* through the C ABI): scenes
admitted in arrival order within the device-memory budget, advanced in
shared batches, and returned with the oracle's final state."""
import time

import numpy as np
import pytest

import oracle
from paper_1909_13380_amd import scenes

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_server_runs_requests_to_the_oracle_state_within_budget():
    from paper_1909_13380_amd import mpmx
    steps = [7, 30, 0, 45, 12, 20, 33]
    scs = []
    for i, k in enumerate(steps):
        mat = scenes.drucker_prager() if i % 2 else scenes.elastic()
        sc = scenes.random_block(n_cells=(6, 5, 4), mesh_cells=(12, 10, 8), h=0.05, seed=60 + i, material=mat,
                                 stress_scale=2e3)
        scs.append(sc)
    bad = scenes.random_block(seed=70)
    bad["x"] = bad["x"].copy()
    bad["x"][3, 2] = -1.0                     # below the mesh
    per = mpmx.scene_bytes(scs[0], mpmx.FP64)
    ctx = mpmx.Context(0)
    srv = mpmx.Server(ctx, int(2.5 * per), max_tick_steps=16)
    try:
        ids = [srv.submit(sc, k, precision=mpmx.FP64, tag=100 + i) for i, (sc, k) in enumerate(zip(scs, steps))]
        bad_id = srv.submit(bad, 5, precision=mpmx.FP64, tag=999)
        done = {}
        for _ in range(200):
            r, q = srv.tick()
            assert r <= 2, "budget admits at most two of these scenes at a time"
            for c in srv.poll():
                done[c["request"]] = c
            if len(done) == len(ids) + 1:
                break
        assert len(done) == len(ids) + 1
        assert done[bad_id]["status"] == mpmx.E_OUT_OF_MESH and done[bad_id]["tag"] == 999
        admits = [done[i]["t_admit"] for i in ids]
        assert admits == sorted(admits), "admission in arrival order"
        for i, (sc, k) in enumerate(zip(scs, steps)):
            c = done[ids[i]]
            assert c["status"] == mpmx.OK and c["tag"] == 100 + i and c["steps_done"] == k
            assert c["t_submit"] <= c["t_admit"] <= c["t_done"]
            ref = oracle.run(sc, k) if k else {"x": sc["x"], "stress": sc["stress"], "v": sc["v"]}
            eu = _rel(c["x"] - sc["x"], ref["x"] - sc["x"]) if k else np.abs(c["x"] - sc["x"]).max()
            es = _rel(c["stress"], ref["stress"])
            print(f"[server/{i}/{k}] err_u={eu:.3e} err_sigma={es:.3e}", flush=True)
            assert eu <= 1e-9 and es <= 1e-9
    finally:
        srv.close()
        ctx.close()


def test_server_results_in_the_mix_equal_each_scene_alone():
    """FP32 requests of uneven size arriving while others are on the GPU:
    late arrivals are admitted before earlier requests finish, several
    scenes share the device at once, and every result equals the same scene
    run alone on the same context within the batch-versus-alone bar."""
    from paper_1909_13380_amd import mpmx
    plan = [((6, 5, 4), 40), ((3, 3, 2), 25), ((8, 6, 5), 33), ((2, 2, 2), 18), ((5, 4, 4), 29), ((7, 5, 3), 12)]
    scs = []
    for i, (cells, _) in enumerate(plan):
        mat = scenes.drucker_prager() if i % 2 else scenes.elastic()
        scs.append(scenes.random_block(n_cells=cells, mesh_cells=(12, 10, 8), h=0.05, seed=80 + i, material=mat,
                                       stress_scale=2e3))
    ctx = mpmx.Context(0)
    srv = mpmx.Server(ctx, 8 << 30, max_tick_steps=8)
    try:
        ids = [srv.submit(sc, k, tag=i) for i, (sc, (_, k)) in enumerate(zip(scs[:3], plan[:3]))]
        done, peak = {}, 0
        for t in range(400):
            if t == 2:   # the first three are resident and part-way through
                ids += [srv.submit(sc, k, tag=3 + i) for i, (sc, (_, k)) in enumerate(zip(scs[3:], plan[3:]))]
            r, q = srv.tick()
            peak = max(peak, r)
            for c in srv.poll():
                done[c["request"]] = c
            if len(done) == len(plan):
                break
        assert len(done) == len(plan)
        assert peak >= 4, "several scenes resident at once"
        first_done = min(done[i]["t_done"] for i in ids[:3])
        assert all(done[i]["t_admit"] < first_done for i in ids[3:]), "late arrivals admitted while others run"
        for i, (sc, (_, k)) in enumerate(zip(scs, plan)):
            c = done[ids[i]]
            assert c["status"] == mpmx.OK and c["steps_done"] == k
            s = ctx.create_scene(sc, precision=mpmx.FP32)
            s.step(k)
            alone = s.read()
            s.destroy()
            eu = _rel(c["x"] - sc["x"], alone["x"] - sc["x"])
            es = _rel(c["stress"], alone["stress"])
            ev = _rel(c["v"], alone["v"])
            print(f"[mix/{i}/{len(sc['x'])}/{k}] err_u={eu:.3e} err_sigma={es:.3e} err_v={ev:.3e}", flush=True)
            assert eu <= 1e-5 and es <= 1e-5 and ev <= 1e-5
    finally:
        srv.close()
        ctx.close()


def test_server_fill_limit_admits_one_filling_scene_at_a_time():
    """With the fill limit at one scene's particle count, a resident scene
    that still has steps to run holds back admission: the queue shrinks by
    at most one request per tick, at most two requests are resident (one
    stepping, one being read back), and results still equal each scene run
    alone."""
    from paper_1909_13380_amd import mpmx
    plan = [((6, 5, 4), 30), ((6, 5, 4), 20), ((6, 5, 4), 25), ((6, 5, 4), 17)]
    scs = [scenes.random_block(n_cells=cells, mesh_cells=(12, 10, 8), h=0.05, seed=120 + i,
                               material=scenes.drucker_prager(), stress_scale=2e3) for i, (cells, _) in enumerate(plan)]
    ctx = mpmx.Context(0)
    srv = mpmx.Server(ctx, 8 << 30, max_tick_steps=8, fill_particles=len(scs[0]["x"]))
    try:
        ids = [srv.submit(sc, k, tag=i) for i, (sc, (_, k)) in enumerate(zip(scs, plan))]
        done, last_q = {}, len(ids)
        for _ in range(400):
            r, q = srv.tick()
            assert r <= 2 and last_q - q <= 1, (r, q, last_q)
            last_q = q
            for c in srv.poll():
                done[c["request"]] = c
            if len(done) == len(plan):
                break
        assert len(done) == len(plan)
        admits = [done[i]["t_admit"] for i in ids]
        assert admits == sorted(admits)
        for i, (sc, (_, k)) in enumerate(zip(scs, plan)):
            c = done[ids[i]]
            assert c["status"] == mpmx.OK and c["steps_done"] == k
            s = ctx.create_scene(sc, precision=mpmx.FP32)
            s.step(k)
            alone = s.read()
            s.destroy()
            eu = _rel(c["x"] - sc["x"], alone["x"] - sc["x"])
            es = _rel(c["stress"], alone["stress"])
            print(f"[fill/{i}/{k}] err_u={eu:.3e} err_sigma={es:.3e}", flush=True)
            assert eu <= 1e-5 and es <= 1e-5
    finally:
        srv.close()
        ctx.close()


def test_fences_report_queued_steps_finished():
    """mpmx_fence_*: a fence recorded after queued steps reports finished
    once they are (a blocking wait returns done, the id is then freed), and
    a non-blocking query never claims done before the steps' results are
    readable."""
    from paper_1909_13380_amd import mpmx
    sc = scenes.random_block(n_cells=(6, 5, 4), mesh_cells=(12, 10, 8), h=0.05, seed=140, stress_scale=2e3)
    ctx = mpmx.Context(0)
    try:
        s = ctx.create_scene(sc, precision=mpmx.FP32)
        s.step(50)
        f = ctx.fence()
        t0 = time.monotonic()
        while not ctx.fence_done(f):
            assert time.monotonic() - t0 < 60.0, "fence never reported done"
            time.sleep(0.001)
        with pytest.raises(mpmx.MpmxError) as e:
            ctx.fence_done(f)
        assert e.value.code == mpmx.E_NOT_FOUND
        assert s.stats()["steps_done"] == 50
        s.step(20)
        g = ctx.fence()
        assert ctx.fence_done(g, block=True)
        h = ctx.fence()
        assert mpmx._lib.mpmx_fence_release(ctx._h, h) == mpmx.OK
        assert mpmx._lib.mpmx_fence_release(ctx._h, h) == mpmx.E_NOT_FOUND
        assert s.stats()["steps_done"] == 70
        s.destroy()
    finally:
        ctx.close()


def test_borrowed_inputs_and_caller_outputs_give_the_same_results():
    """MPMX_REQ_BORROW (the particle arrays kept by pointer) and caller-owned
    output buffers: the same final state as a copying request, written into
    the caller's arrays."""
    from paper_1909_13380_amd import mpmx
    scs = [scenes.random_block(n_cells=(5, 4, 4), mesh_cells=(12, 10, 8), h=0.05, seed=160 + i,
                               material=scenes.drucker_prager(), stress_scale=2e3) for i in range(3)]
    steps = [21, 9, 30]
    ctx = mpmx.Context(0)
    results = {}
    try:
        for mode in ("copy", "borrow_out", "borrow"):
            srv = mpmx.Server(ctx, 8 << 30, max_tick_steps=8)
            ids = [srv.submit(sc, k, tag=i, borrow=mode != "copy", out=mode == "borrow_out")
                   for i, (sc, k) in enumerate(zip(scs, steps))]
            done = {}
            for _ in range(200):
                srv.tick()
                for c in srv.poll():
                    done[c["tag"]] = c
                if len(done) == len(ids):
                    break
            srv.close()
            assert len(done) == len(ids)
            results[mode] = done
        for i, (sc, k) in enumerate(zip(scs, steps)):
            ref = results["copy"][i]
            assert ref["status"] == mpmx.OK and ref["steps_done"] == k
            for mode in ("borrow_out", "borrow"):
                got = results[mode][i]
                assert got["status"] == mpmx.OK and got["steps_done"] == k
                for f in ("x", "v", "stress", "vol"):
                    e = _rel(got[f], ref[f])
                    assert e <= 1e-5, (mode, i, f, e)
            np.testing.assert_array_equal(scs[i]["x"], scenes.random_block(
                n_cells=(5, 4, 4), mesh_cells=(12, 10, 8), h=0.05, seed=160 + i, material=scenes.drucker_prager(),
                stress_scale=2e3)["x"])   # borrowed inputs are read, never written
    finally:
        ctx.close()


def test_a_lone_request_of_zero_steps_completes():
    """A request of 0 steps, alone in the server (no round queues any GPU
    work), completes on the next tick with its input state."""
    from paper_1909_13380_amd import mpmx
    sc = scenes.random_block(n_cells=(3, 3, 2), mesh_cells=(8, 8, 6), h=0.05, seed=170, stress_scale=1e3)
    ctx = mpmx.Context(0)
    srv = mpmx.Server(ctx, 1 << 30, max_tick_steps=8)
    try:
        rid = srv.submit(sc, 0, precision=mpmx.FP64)
        done = []
        for _ in range(5):
            srv.tick()
            done += srv.poll()
            if done:
                break
        assert len(done) == 1 and done[0]["request"] == rid
        c = done[0]
        assert c["status"] == mpmx.OK and c["steps_done"] == 0
        np.testing.assert_array_equal(c["x"], sc["x"])
        assert srv.tick() == (0, 0)
    finally:
        srv.close()
        ctx.close()
