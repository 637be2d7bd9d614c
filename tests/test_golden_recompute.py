"""The stored oracle results (tests/golden/c3_expected.txt for the large
16-vertex workload, tests/golden/c6_expected.txt for the wide 32-vertex one)
still agree with the live oracle: a seeded sample of rows of each file is
recomputed here, field by field.  The GPU parity tests compare the GPU path
with every row of those files, so a stale file would otherwise go unnoticed."""
import os

import numpy as np
import pytest

from paper_2110_03214_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NTHREADS = min(8, os.cpu_count() or 1)


def read_rows(name, has_busy):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"tests/golden/{name} not generated")
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            v = [int(x) for x in line.split()]
            head = 4 if not has_busy else 5
            idx, server = v[0], v[1]
            busy = v[2] if has_busy else 0
            kind, k = v[head - 2], v[head - 1]
            count, status, key, agg, pres, mask = v[head:head + 6]
            mapping = tuple(v[head + 6:])
            rows.append(dict(idx=idx, server=server, busy=busy, kind=kind, k=k, count=count,
                             status=status, key=key, agg=agg, pres=pres, vertex_mask=mask,
                             mapping=mapping))
    return rows


def check_sample(orc, wl, rows, pick):
    sub = wl.subset(np.array([rows[i]["idx"] for i in pick]))
    res = orc.run_workload(sub, nthreads=NTHREADS)
    for j, i in enumerate(pick):
        row, r = rows[i], res[j]
        assert sub.queries["kind"][j] == row["kind"] and sub.queries["k"][j] == row["k"]
        for f in ("count", "status", "key", "agg", "pres", "vertex_mask"):
            assert int(r[f]) == row[f], (row["idx"], f, int(r[f]), row[f])
        assert tuple(int(x) for x in r["mapping"][:row["k"]]) == row["mapping"], row["idx"]


def test_large_config_rows_recomputed(orc):
    wl = synth.config3()
    rows = read_rows("c3_expected.txt", has_busy=False)
    assert len(rows) == wl.nq == 1536
    rng = np.random.default_rng(0x63_33)
    k6 = [i for i, r in enumerate(rows) if r["k"] == 6]
    k7 = [i for i, r in enumerate(rows) if r["k"] == 7]
    pick = list(rng.choice(k6, size=12, replace=False)) + list(rng.choice(k7, size=2, replace=False))
    check_sample(orc, wl, rows, sorted(int(i) for i in pick))


def test_wide_config_rows_recomputed(orc):
    wl = synth.config6()
    rows = read_rows("c6_expected.txt", has_busy=True)
    assert len(rows) == wl.nq == 96
    for r in rows:  # the file's busy masks are the generator's
        assert int(wl.busy[r["server"]]) == r["busy"]
    rng = np.random.default_rng(0x63_36)
    k9 = [i for i, r in enumerate(rows) if r["k"] == 9]
    pick = rng.choice(k9, size=6, replace=False)
    check_sample(orc, wl, rows, sorted(int(i) for i in pick))
