"""Serving on the GPU: captured graphs replay to the eager result, and every
request's result is the same alone (plain form, one segment per launch) and
inside the continuous-batching mix."""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_graph_replays_match_eager(torch_dev):
    torch = torch_dev
    from paper_2603_29785_amd.serving import BucketKey, GpuExecutor
    ex = GpuExecutor(streams=1)
    key = BucketKey(4096.0, 16384, 8.0, 64, 10.0, 2048.0)
    res = ex.prepare(key, 4)
    x = torch.from_numpy(synthetic.batched_segments(4, 16384, 4096.0, workload=7)).cuda()
    p = res["plan"]
    eager = p.inverse(p.forward(x)).clone()
    assert len(res["sets"]) == 2
    for ss in res["sets"]:
        ss["x"].copy_(x)
        g, k = ex._graph(res, ss, 4)
        assert k == 4
        for rep in range(3):
            ss["xr"].zero_()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(ss["xr"], eager), rep
            # eager work between replays on the same buffers
            p.forward(x[:2].contiguous())
            torch.cuda.synchronize()


def test_alone_equals_mix(torch_dev):
    torch = torch_dev
    from paper_2603_29785_amd.serving import BucketKey, GpuExecutor, Request, Server, plain_run
    rng = np.random.default_rng(11)
    shapes = [(4096.0, 4096), (4096.0, 16384), (16384.0, 16384), (4096.0, 65536)]
    reqs = []
    for i in range(40):
        fs, n = shapes[rng.integers(len(shapes))]
        q = float(rng.choice([4.0, 8.0, 16.0]))
        rows = int(rng.choice([64, 128]))
        key = BucketKey(fs, n, q, rows, 10.0, 2048.0)
        data = synthetic.injected_segment(n, fs, synthetic.rng_for(8, i))[0].astype(np.float32)
        if i % 2:       # half the payloads in pinned host memory (copied by DMA), half staged
            data = torch.from_numpy(data).pin_memory()
        reqs.append(Request(i, key, data))
    srv = Server(GpuExecutor(streams=4), hbm_budget=8 << 30, streams=4)
    for r in reqs:
        srv.submit(r)
    srv.drain(timeout=120)
    srv.shutdown()
    assert all(r.status == "done" for r in reqs), [r.status for r in reqs]
    assert srv.launches < len(reqs)           # batched
    alone = [Request(r.rid, r.key, np.asarray(r.data)) for r in reqs]
    plain_run(alone)
    for r, a in zip(reqs, alone):
        assert np.array_equal(r.result, a.result), r.rid
    # and the mix matches the FP64 oracle
    for r in reqs[:4]:
        k = r.key
        op = o.OraclePlan(fs=k.fs, n=k.n, q=k.q, f_min=k.f_min, f_max=k.f_max, rows=k.rows)
        xm = op.project(np.asarray(r.data, dtype=np.float64))
        assert np.linalg.norm(r.result - xm) <= 1e-5 * np.linalg.norm(xm)
