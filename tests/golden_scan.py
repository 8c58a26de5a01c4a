"""Reader of the full-scan edge files under tests/golden/ (written by
tests/golden/make_edge_scans.py from the oracle alone)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_scan(name):
    """(threshold, band, {(i, j): r}): every pair with |r| >= threshold - band."""
    thr = band = None
    pairs = {}
    for line in open(os.path.join(GOLDEN, name + ".txt")):
        if line.startswith("#"):
            w = line.replace(":", " ").split()
            if "threshold" in w and "band" in w:
                thr = float(w[w.index("threshold") + 1])
                band = float(w[w.index("band") + 1])
            continue
        i, j, r = line.split()
        pairs[(int(i), int(j))] = float(r)
    if thr is None:
        raise ValueError(f"{name}: no threshold line")
    return thr, band, pairs
