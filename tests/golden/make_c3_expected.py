"""Write c3_expected.txt: the CPU oracle's result for every query of the large
16-vertex workload (256 topologies x {ring, all-to-all} x k in {6,7,8}).

Calls only ``oracle`` and the seeded input generator.  Re-run it whenever the
oracle's arithmetic or the generator changes:

    python tests/golden/make_c3_expected.py [nthreads]

Takes about 20 minutes on 8 cores (2.98e11 embeddings).
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2110_03214_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_expected.txt")


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    oracle.build()
    wl = synth.config3()
    t0 = time.time()
    res = oracle.run_workload(wl, nthreads=nthreads)
    dt = time.time() - t0
    q = wl.queries
    with open(OUT + ".tmp", "w") as f:
        f.write("# CPU oracle results, large 16-vertex workload (seeded generator config 3)\n")
        f.write(f"# {wl.nq} queries, ALL mode, key weights (1,1); {dt:.0f} s on {nthreads} threads\n")
        f.write("# idx server kind k count status key agg pres vertex_mask mapping[0..k-1]\n")
        for i in range(wl.nq):
            r = res[i]
            k = int(q["k"][i])
            mp = " ".join(str(int(x)) for x in r["mapping"][:k])
            f.write(f"{i} {q['server'][i]} {q['kind'][i]} {k} {r['count']} {r['status']} "
                    f"{r['key']} {r['agg']} {r['pres']} {r['vertex_mask']} {mp}\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} in {dt:.0f} s")


if __name__ == "__main__":
    main()
