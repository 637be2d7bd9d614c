"""The allocation-free batch (mapa_query_batch_noalloc) against the batch it
mirrors (mapa_query_batch with device pointers): every byte of every result
equal, on two calls in a row with the second smaller, with commits and the
busy masks they leave, plus the size limit."""
import numpy as np
import pytest

from paper_2110_03214_amd import binding as B
from paper_2110_03214_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return t


def _dev(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8).copy()).to("cuda:0")


def _res(t):
    return t.cpu().numpy().view(B.RESULT_DTYPE)


def test_noalloc_matches_batch_on_two_calls(torch):
    wl = synth.config2()
    stream = torch.cuda.current_stream()
    with B.Context(0) as ctx:
        q, ids = B.load_workload(ctx, wl)
        # call 1: the whole batched workload (65,536 queries), no commits
        q1 = q.copy()
        q1["commit"] = 0
        dq1 = _dev(torch, q1)
        ref1 = torch.zeros(len(q1) * 48, dtype=torch.uint8, device="cuda:0")
        got1 = torch.full_like(ref1, 0xAB)
        print(f"[noalloc] call 1: {len(q1)} queries", flush=True)
        ctx.query_batch(dq1, ref1, stream=stream)
        ctx.query_batch_noalloc(dq1, got1, stream=stream)
        torch.cuda.synchronize()
        r1, g1 = _res(ref1), _res(got1)
        assert int(r1["count"].sum()) > 0
        assert np.array_equal(r1.view(np.uint8), g1.view(np.uint8)), "call 1 results differ"
        assert np.array_equal(ctx.get_busy(ids), wl.busy)

        # call 2: a smaller batch (3,001 queries, ragged) whose queries commit
        q2 = q[:3001].copy()
        q2["commit"] = 1
        dq2 = _dev(torch, q2)
        ref2 = torch.zeros(len(q2) * 48, dtype=torch.uint8, device="cuda:0")
        got2 = torch.full_like(ref2, 0xCD)
        print(f"[noalloc] call 2: {len(q2)} queries with commit", flush=True)
        ctx.query_batch(dq2, ref2, stream=stream)
        torch.cuda.synchronize()
        busy_ref = ctx.get_busy(ids)
        ctx.release(ref2.view(torch.int64)[5:], stride=48, count=len(q2), stream=stream)
        torch.cuda.synchronize()
        assert np.array_equal(ctx.get_busy(ids), wl.busy), "release did not restore the busy masks"
        ctx.query_batch_noalloc(dq2, got2, stream=stream)
        torch.cuda.synchronize()
        r2, g2 = _res(ref2), _res(got2)
        assert (r2["alloc_handle"] >= 0).any()
        assert np.array_equal(r2.view(np.uint8), g2.view(np.uint8)), "call 2 results differ"
        assert np.array_equal(ctx.get_busy(ids), busy_ref), "commits differ"


def test_noalloc_size_limit(torch):
    wl = synth.config1(8)
    with B.Context(0) as ctx:
        B.load_workload(ctx, wl)
        n = B.NOALLOC_MAX_QUERIES + 1
        dq = torch.zeros(n * 16, dtype=torch.uint8, device="cuda:0")
        dr = torch.zeros(n * 48, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(B.MapaError) as e:
            ctx.query_batch_noalloc(dq, dr)
        assert e.value.code == B.ERR_ADMISSION
