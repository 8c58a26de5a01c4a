"""Writes the full-scan edge files under tests/golden/ from the oracle alone
(FP64, literal Eq. (1) for every pair i < j) on the seeded workloads:

  edges_n32768_l4096_thr0.8.txt    n = 32768, l = 4096 (the precision-sweep
                                   matrix), |r| >= 0.8
  edges_n65536_l2048_thr0.9.txt    n = 65536, l = 2048 (the large run of the
                                   uneven-batch workload), |r| >= 0.9

Each file lists every pair with |r| >= threshold - band, so a test knows the
exact edge set and which pairs lie within the band of the threshold (where
rounding may decide).  Run from the repository root:

  python tests/golden/make_edge_scans.py [name ...]

About 15 and 30 minutes on 8 cores.
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402

BAND = 1e-5
SCANS = {
    "edges_n32768_l4096_thr0.8": (lambda: workloads.config3()[0], 0.8,
                                  "workloads.config3(): n=32768 l=4096 FP32, planted"),
    "edges_n65536_l2048_thr0.9": (lambda: workloads.config5_big()[0], 0.9,
                                  "workloads.config5_big(): n=65536 l=2048 FP32, planted"),
}


def main(names):
    for name in names or list(SCANS):
        make, thr, desc = SCANS[name]
        X = make()
        t0 = time.time()
        I, J, R = oracle.edges(X, thr - BAND)
        dt = time.time() - t0
        path = os.path.join(ROOT, "tests", "golden", name + ".txt")
        with open(path, "w") as f:
            f.write(f"# full oracle scan (FP64, literal Eq. (1), every pair i < j) of {desc}\n")
            f.write(f"# threshold {thr} band {BAND}: every pair with |r| >= threshold - band\n")
            f.write(f"# {len(I)} pairs, scan took {dt:.0f} s on {oracle.num_threads()} threads\n")
            f.write("# columns: i j r\n")
            for i, j, r in zip(I.tolist(), J.tolist(), R.tolist()):
                f.write(f"{i} {j} {r:.17g}\n")
        print(name, len(I), f"{dt:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
