"""GPU parity of the job-trace simulator (mapa_simulate, Sec. 5.2) against
the oracle's simulator: every job's status, start and finish cycles,
accelerators, mapping, AggBW, PreservedBW, predicted effective bandwidth and
link mix, under the Preserve, Greedy and lowest-id policies."""
import numpy as np
import pytest

import oracle
from oracle import simulate as osim
from paper_2110_03214_amd import binding as B
from paper_2110_03214_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return t


def assert_logs_equal(got, ref, jobs, label):
    assert len(got) == len(ref)
    for i, (g, r) in enumerate(zip(got, ref)):
        where = f"{label} job {i}"
        assert g["id"] == r["id"], where
        assert g["status"] == r["status"], where
        if r["status"] != oracle.OK:
            assert g["start"] == -1 and g["finish"] == -1, where
            continue
        k = int(jobs["k"][i])
        assert (g["start"], g["finish"], g["vertex_mask"]) == (r["start"], r["finish"], r["vertex_mask"]), \
            (where, g, r)
        assert tuple(int(v) for v in g["mapping"][:k]) == r["mapping"], where
        assert (g["mapping"][k:] == 0xFF).all(), where
        assert (g["agg"], g["pres"], g["effbw_milli"], g["links"]) == \
            (r["agg"], r["pres"], r["effbw_milli"], r["links"]), (where, g, r)


def run_both(jf, busy0=None):
    with B.Context(0) as ctx:
        ids = B.load_jobfiles(ctx, jf)
        if busy0 is not None:
            ctx.set_busy(ids, busy0)
        before = ctx.get_busy(ids)
        print(f"[sim] {jf.name}: {jf.nsim} simulations, {len(jf.jobs)} jobs", flush=True)
        logs, st = ctx.simulate(ids, jf.policy, jf.offsets, jf.jobs)
        assert np.array_equal(ctx.get_busy(ids), before), "servers not left as found"
    for i in range(jf.nsim):
        a, b = jf.offsets[i], jf.offsets[i + 1]
        W = jf.topologies[jf.sim_topo[i]]
        ref = osim.simulate(W, int(before[i]), jf.jobs[a:b], int(jf.policy[i]))
        assert_logs_equal(logs[a:b], ref, jf.jobs[a:b], f"simulation {i} (policy {jf.policy[i]})")
    return logs, st


def test_paper_job_files_on_dgx1v(torch):
    """The paper's setting: 300-job FIFO files (1-5 GPUs each) on the DGX-1
    V100, under all three policies."""
    jf = synth.config7(files_per_topology=2, njobs=300)
    dgx = np.nonzero(jf.sim_topo == 0)[0]
    logs, st = run_both(jf.subset(dgx))
    assert st["jobs_placed"] == 2 * 3 * 300 and st["rounds"] <= 300


def test_sixteen_gpu_topologies(torch):
    jf = synth.config7(files_per_topology=1, njobs=80)
    big = np.nonzero(jf.sim_topo != 0)[0]
    run_both(jf.subset(big))


def test_poisson_arrivals_reserved_gpus_and_unplaceable_jobs(torch):
    rng = np.random.default_rng(5)
    topos = [synth.dgx1v_topology(), synth.config2_topologies()[1]]
    parts, sim_topo, policy = [], [], []
    for t in range(2):
        for pol in (0, 1, 2):
            f = synth.job_file(rng, 120, kmax=8, dmin=5, dmax=60, mean_gap=6.0)
            parts.append(f)
            sim_topo.append(t)
            policy.append(pol)
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int32)
    jf = synth.JobFiles("poisson", topos, np.array(sim_topo, np.int32), np.array(policy, np.int32),
                        off, np.concatenate(parts))
    # two accelerators of every server stay reserved: 8-GPU jobs never fit
    busy0 = np.array([0b10000001, 0b00011000] * 3, dtype=np.uint32)
    logs, _ = run_both(jf, busy0)
    assert (logs["status"] == oracle.NOFIT).sum() == (jf.jobs["k"] > 6).sum()


def test_validation(torch):
    jf = synth.config7(files_per_topology=1, njobs=5)
    with B.Context(0) as ctx:
        ids = B.load_jobfiles(ctx, jf)
        sub = [0, 1]
        off = jf.offsets[:3]
        with pytest.raises(B.MapaError) as e:  # one server in two simulations
            ctx.simulate([ids[0], ids[0]], [0, 1], off, jf.jobs[:off[-1]])
        assert e.value.code == B.ERR_INVALID_ARG
        bad = jf.jobs[:off[-1]].copy()
        bad["duration"][1] = 0
        with pytest.raises(B.MapaError):
            ctx.simulate(ids[sub], jf.policy[sub], off, bad)
        with pytest.raises(B.MapaError) as e:  # weights above 2 have no Eq. 2 class
            W3 = np.array([[0, 3], [3, 0]], np.uint8)
            _, s3 = ctx.create_topology(W3, 1)
            ctx.simulate([s3], [0], [0, 1], jf.jobs[:1])
        assert e.value.code == B.ERR_UNSUPPORTED
