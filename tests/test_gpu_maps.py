"""The device job-map code the tile kernels run, against brute-force
enumeration (bit-exact)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 3, 64, 257, 1000, 2048, 4096])
def test_device_maps_exhaustive(n):
    import paper_1605_01584_amd as pcc
    for diag in (True, False):
        ys, xs = oracle.enumerate_upper(n, diag)
        if len(ys) == 0:
            continue
        y, x = pcc.cells_device(n, diag, 0, len(ys))
        assert np.array_equal(y.cpu().numpy(), ys) and np.array_equal(x.cpu().numpy(), xs)


@pytest.mark.parametrize("n", [65536, 131072, 1 << 20])
@pytest.mark.parametrize("diag", [True, False])
def test_device_row_boundaries(n, diag):
    """Ids around the ends of 512 seeded rows (and the first and last rows);
    the expected cells come from counting row lengths (cumulative sums)."""
    import paper_1605_01584_amd as pcc
    length = n - np.arange(n, dtype=np.int64) - (0 if diag else 1)
    start = np.concatenate([[0], np.cumsum(length)])
    total = int(start[-1])
    rows = np.unique(np.concatenate([[0, 1, n - 3, n - 2],
                                     np.random.default_rng(n).integers(1, n - 1, 512)]))
    for r in rows:
        J0 = max(0, int(start[r]) - 3)
        cnt = min(7, total - J0)
        if cnt <= 0:
            continue
        Js = np.arange(J0, J0 + cnt, dtype=np.int64)
        wy = np.searchsorted(start, Js, side="right") - 1
        wx = wy + (Js - start[wy]) + (0 if diag else 1)
        y, x = pcc.cells_device(n, diag, J0, cnt)
        assert np.array_equal(y.cpu().numpy(), wy), (n, r)
        assert np.array_equal(x.cpu().numpy(), wx), (n, r)
