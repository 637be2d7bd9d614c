"""Write c6_expected.txt: the CPU oracle's result for every query of the wide
workload (16 seeded 32-vertex 5-cube-plus-chord topologies, 12 free
accelerators each, {ring, all-to-all, tree} x k in {9, 10}).

Calls only ``oracle`` and the seeded input generator.  Re-run it whenever the
oracle's arithmetic or the generator changes:

    python tests/golden/make_c6_expected.py [nthreads]

Takes about two minutes on 8 cores (1.53e10 embeddings).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2110_03214_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c6_expected.txt")


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.build()
    wl = synth.config6()
    t0 = time.time()
    res = oracle.run_workload(wl, nthreads=nthreads)
    dt = time.time() - t0
    q = wl.queries
    with open(OUT + ".tmp", "w") as f:
        f.write("# CPU oracle results, wide 32-vertex workload (seeded generator config 6)\n")
        f.write(f"# {wl.nq} queries, ALL mode, key weights (1,1); {dt:.0f} s on {nthreads} threads\n")
        f.write("# idx server busy kind k count status key agg pres vertex_mask mapping[0..k-1]\n")
        for i in range(wl.nq):
            r = res[i]
            k = int(q["k"][i])
            s = int(q["server"][i])
            mp = " ".join(str(int(x)) for x in r["mapping"][:k])
            f.write(f"{i} {s} {int(wl.busy[s])} {q['kind'][i]} {k} {r['count']} {r['status']} "
                    f"{r['key']} {r['agg']} {r['pres']} {r['vertex_mask']} {mp}\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} in {dt:.0f} s")


if __name__ == "__main__":
    main()
