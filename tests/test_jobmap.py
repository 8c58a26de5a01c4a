"""Job maps of the C ABI (Eq. (9)-(19) with the int64 correction, the
diagonal-free packed index, and the banded tile order) against brute-force
enumeration by the oracle: the paper's own bijection test (forward, then
inverse, compared with sequential numbering).  CPU only."""
import numpy as np
import pytest

import oracle


def _check_exhaustive(pcc, n, diag):
    ys, xs = oracle.enumerate_upper(n, diag)
    cnt = len(ys)
    if cnt == 0:
        return
    # inverse: id -> cell
    m = n if diag else n
    y, x = pcc.cells_host(m, diag, 0, cnt)
    assert np.array_equal(y, ys) and np.array_equal(x, xs)


@pytest.mark.parametrize("n", list(range(1, 130)) + [255, 256, 257, 300, 511, 512])
def test_exhaustive_small(n):
    import paper_1605_01584_amd as pcc
    _check_exhaustive(pcc, n, True)
    if n >= 2:
        _check_exhaustive(pcc, n, False)


@pytest.mark.parametrize("n", [1000, 2000, 2048, 4096])
def test_exhaustive_medium(n):
    import paper_1605_01584_amd as pcc
    _check_exhaustive(pcc, n, True)
    _check_exhaustive(pcc, n, False)


def test_forward_maps_scalar():
    import paper_1605_01584_amd as pcc
    for n in (1, 2, 5, 17, 64):
        ys, xs = oracle.enumerate_upper(n, True)
        for J, (y, x) in enumerate(zip(ys.tolist(), xs.tolist())):
            assert pcc.job_of_cell(n, y, x) == J
            assert pcc.cell_of_job(n, J) == (y, x)
        if n >= 2:
            ys, xs = oracle.enumerate_upper(n, False)
            for J, (y, x) in enumerate(zip(ys.tolist(), xs.tolist())):
                assert pcc.packed_index(n, y, x) == J
                assert pcc.packed_cell(n, J) == (y, x)


@pytest.mark.parametrize("n", [65536, 131072, 1 << 20, 46341, 3_000_000])
def test_row_boundaries_large(n):
    """First, middle and last id of every row (sampled rows for the largest n).
    Expected ids come from counting the cells of earlier rows (a cumulative
    sum of row lengths), not from the closed form."""
    import paper_1605_01584_amd as pcc
    rows = np.arange(n, dtype=np.int64)
    if n > (1 << 20):
        rng = np.random.default_rng(n)
        rows = np.unique(np.concatenate([rows[:2000], rows[-2000:], rng.integers(0, n, 20000)]))
    for diag in (True, False):
        length = (n - np.arange(n, dtype=np.int64)) - (0 if diag else 1)   # cells per row
        start = np.concatenate([[0], np.cumsum(length)[:-1]])
        for which in ("first", "mid", "last"):
            sel = rows[length[rows] > 0]
            off = {"first": 0 * sel, "mid": length[sel] // 2, "last": length[sel] - 1}[which]
            J = start[sel] + off
            want_y = sel
            want_x = sel + (0 if diag else 1) + off
            y = np.empty_like(J)
            x = np.empty_like(J)
            for k in range(len(J)):   # scalar C calls on a few thousand ids
                if k % max(1, len(J) // 3000) and which == "mid":
                    continue
                yy, xx = pcc.cell_of_job(n, int(J[k])) if diag else pcc.packed_cell(n, int(J[k]))
                assert (yy, xx) == (int(want_y[k]), int(want_x[k])), (n, diag, which, int(J[k]))


def test_largest_n_extremes():
    import paper_1605_01584_amd as pcc
    n = 2 ** 31 - 1
    total = n * (n + 1) // 2
    assert pcc.cell_of_job(n, 0) == (0, 0)
    assert pcc.cell_of_job(n, total - 1) == (n - 1, n - 1)
    assert pcc.cell_of_job(n, n - 1) == (0, n - 1)
    assert pcc.cell_of_job(n, n) == (1, 1)
    assert pcc.packed_cell(n, n * (n - 1) // 2 - 1) == (n - 2, n - 1)
    assert pcc.packed_index(n, n - 2, n - 1) == n * (n - 1) // 2 - 1


@pytest.mark.parametrize("m", [1, 2, 3, 7, 8, 9, 31, 64, 128, 129, 200])
@pytest.mark.parametrize("band", [1, 2, 4, 8, 16])
def test_banded_order_is_a_bijection(m, band):
    import paper_1605_01584_amd as pcc
    cfg = pcc.TileCfg(256, 1, band, 0)
    total = m * (m + 1) // 2
    y, x = pcc.tile_order_host(m, cfg, 0, total)
    ys, xs = oracle.enumerate_upper(m, True)
    got = set(zip(y.tolist(), x.tolist()))
    assert len(got) == total and got == set(zip(ys.tolist(), xs.tolist()))
    # bands are contiguous id ranges holding whole tile rows, walked by column
    b = y // band
    assert np.all(np.diff(b) >= 0)
    inside = np.diff(b) == 0
    assert np.all(np.diff(x)[inside] >= 0)


def test_paper_order_matches_enumeration():
    import paper_1605_01584_amd as pcc
    m = 150
    y, x = pcc.tile_order_host(m, pcc.TileCfg(256, 0, 1, 0), 0, m * (m + 1) // 2)
    ys, xs = oracle.enumerate_upper(m, True)
    assert np.array_equal(y, ys) and np.array_equal(x, xs)


def _rect_row_major(mr, mc):
    # Eq. (7)-(8) by counting: ids 0, 1, 2, ... over the rows of the job matrix
    ys, xs = [], []
    for y in range(mr):
        for x in range(mc):
            ys.append(y)
            xs.append(x)
    return np.array(ys), np.array(xs)


@pytest.mark.parametrize("mr,mc", [(1, 1), (1, 7), (7, 1), (5, 9), (33, 17), (128, 128), (3, 200)])
@pytest.mark.parametrize("order,band", [(0, 1), (1, 1), (1, 2), (1, 4), (1, 8), (1, 16)])
def test_rect_order(mr, mc, order, band):
    import paper_1605_01584_amd as pcc
    cfg = pcc.TileCfg(128, order, band, 0)
    yt, xt = pcc.rect_tile_order_host(mr, mc, cfg, 0, mr * mc)
    assert yt.min() >= 0 and yt.max() < mr and xt.min() >= 0 and xt.max() < mc
    ids = yt * mc + xt
    np.testing.assert_array_equal(np.sort(ids), np.arange(mr * mc))   # a bijection
    if order == 0 or band == 1:
        ry, rx = _rect_row_major(mr, mc)
        np.testing.assert_array_equal(yt, ry)
        np.testing.assert_array_equal(xt, rx)
    else:
        # bands of `band` tile rows, each walked column by column, top to bottom
        b = yt // band
        assert np.all(np.diff(b) >= 0)
        for bb in np.unique(b):
            sel = b == bb
            key = xt[sel] * band + (yt[sel] - bb * band)
            assert np.all(np.diff(key) > 0)
    # any window gives the same cells as the whole range
    if mr * mc > 3:
        y2, x2 = pcc.rect_tile_order_host(mr, mc, cfg, 2, mr * mc - 3)
        np.testing.assert_array_equal(y2, yt[2:mr * mc - 1])
        np.testing.assert_array_equal(x2, xt[2:mr * mc - 1])
