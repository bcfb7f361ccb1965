"""GPU tests of the serving runtime: jobs of mixed sizes and kinds arrive
while others run, are admitted under a small device-memory budget, run in
shared launches on several streams, and each result equals the result of
the same call made alone (stream bytes, and decompressed positions bit for
bit), and the oracle's stream for sampled jobs; a quarter of the jobs store
their references as original coordinates (ref_mode 1)."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from oracle import Oracle
from synth import cosmology, uniform_cube

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbx():
    import paper_2404_02826_amd as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    b.load()
    return b


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _jobs(nj, seed):
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(3.0, 5.3, size=nj)).astype(int)
    out = []
    for i in range(nj):
        gen = uniform_cube if i % 2 == 0 else cosmology
        pts = gen(int(sizes[i]), seed=100 + i)
        out.append(dict(pts=pts, kind="compress" if rng.random() < 0.5 else "decompress",
                        eb=1e-4 if i % 3 else 1e-3, ref_mode=1 if i % 4 == 3 else 0))
    return out


def test_served_results_equal_alone(bbx):
    jobs = _jobs(48, seed=11)
    for j in jobs:
        j["x"] = torch.from_numpy(j["pts"]).cuda()
        j["alone_stream"] = bbx.compress(j["x"], j["eb"], "rel", 32, ref_mode=j["ref_mode"])
        if j["kind"] == "decompress":
            j["header"] = j["alone_stream"][:128].cpu().numpy().tobytes()
            j["alone_pos"] = bbx.decompress(j["alone_stream"])
    torch.cuda.synchronize()
    need = max(bbx.compress_bound(len(j["pts"]), ref_mode=1) +
               bbx.compress_workspace_size(len(j["pts"]), ref_mode=1) for j in jobs)
    budget = (3 * need + (1 << 20)) // 256 * 256  # forces admission to wait for memory
    srv = bbx.Server(budget, max_jobs=64, max_batch=8, nstreams=3)
    _say(f"served: {len(jobs)} jobs, budget {budget} bytes")
    rng = np.random.default_rng(5)
    gaps = rng.exponential(2e-4, size=len(jobs))
    ids, done, max_inflight, t0 = {}, {}, 0, time.perf_counter()
    k, t_next = 0, 0.0
    while len(done) < len(jobs):
        now = time.perf_counter() - t0
        while k < len(jobs) and now >= t_next:
            j = jobs[k]
            jid = (srv.submit_compress(j["x"], j["eb"], "rel", 32, ref_mode=j["ref_mode"])
                   if j["kind"] == "compress"
                   else srv.submit_decompress(j["alone_stream"], j["header"]))
            ids[jid] = k
            t_next += gaps[k]
            k += 1
        srv.progress()
        c = srv.counts()
        max_inflight = max(max_inflight, c["inflight"])
        assert c["arena_used"] <= budget
        while True:
            jid = srv.pop_done()
            if not jid:
                break
            done[jid] = srv.info(jid)
        assert time.perf_counter() - t0 < 60, "served session did not finish"
    batched = [d["batch_jobs"] for d in done.values()]
    _say(f"launches {srv.counts()['launches']}, max jobs per launch {max(batched)}, "
         f"max launches in flight {max_inflight}")
    for jid, d in done.items():
        j = jobs[ids[jid]]
        assert d["status"] == 0, (ids[jid], d)
        got = srv.result(jid)
        if j["kind"] == "compress":
            assert torch.equal(got, j["alone_stream"]), f"job {ids[jid]}: stream differs"
        else:
            assert torch.equal(got.view(torch.uint8), j["alone_pos"].view(torch.uint8)), \
                f"job {ids[jid]}: positions differ"
    orc = Oracle()
    for jid, d in list(done.items())[:6]:
        j = jobs[ids[jid]]
        if j["kind"] == "compress":
            ref = orc.compress(j["pts"], j["eb"], "rel", 32, ref_mode=j["ref_mode"])
            assert srv.result(jid).cpu().numpy().tobytes() == ref
    for jid in done:
        srv.release(jid)
    assert srv.counts()["arena_used"] == 0
    assert max(batched) > 1, "no launch carried more than one job"
    srv.close()


def test_server_rejects_job_larger_than_budget(bbx):
    srv = bbx.Server(1 << 20, max_jobs=4, max_batch=4, nstreams=1)
    x = torch.from_numpy(uniform_cube(200000, seed=1)).cuda()
    with pytest.raises(bbx.BitboxError) as e:
        srv.submit_compress(x, 1e-3)
    assert e.value.name == "ENOMEM"
    srv.close()


def test_launches_overlap_on_the_device(bbx):
    """Continuous batching keeps several launches in flight: jobs submitted
    while earlier ones still run start on free streams at once, and a later
    launch starts before an earlier one has finished."""
    xs = [torch.from_numpy(cosmology(1 << 21, seed=40 + i)).cuda() for i in range(3)]
    alone = [bbx.compress(x, 1e-4, "rel", 32) for x in xs]
    torch.cuda.synchronize()
    srv = bbx.Server(4 << 30, max_jobs=8, max_batch=1, nstreams=3)
    ids, inflight = [], 0
    for x in xs:
        ids.append(srv.submit_compress(x, 1e-4, "rel", 32))
        srv.progress()
        inflight = max(inflight, srv.counts()["inflight"])
    done = {}
    t0 = time.perf_counter()
    while len(done) < len(ids):
        srv.progress()
        while True:
            jid = srv.pop_done()
            if not jid:
                break
            done[jid] = srv.info(jid)
        assert time.perf_counter() - t0 < 30, "jobs did not finish"
    _say(f"launches in flight after the submissions: {inflight}")
    assert inflight >= 2, "no two launches were in flight together"
    first = done[ids[0]]
    assert any(done[j]["t_launch"] < first["t_done"] for j in ids[1:]), \
        "no later launch started before the first one finished"
    for jid, a in zip(ids, alone):
        assert torch.equal(srv.result(jid), a)
        srv.release(jid)
    srv.close()

