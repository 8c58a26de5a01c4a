"""pcc_threshold_edges on the GPU: the edge set against the oracle (pairs
within 1e-5 of the threshold excluded from the exact-set check), against the
same library's packed output, capacity overflow, and full-size runs, whose
edge lists are compared whole with the oracle's full scans stored under
tests/golden/."""
import numpy as np
import pytest

import oracle
import workloads
from golden_scan import read_scan
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu


def _edges(z, zd, thr, cap, cfg=None):
    import paper_1605_01584_amd as pcc
    ij, rv, cnt = pcc.threshold_edges(z, zd, thr, cap, cfg)
    return ij.cpu().numpy(), rv.cpu().numpy(), cnt


def _set(ij):
    return set(map(tuple, ij.tolist()))


@pytest.mark.parametrize("mode", ["fp32", "split"])
@pytest.mark.parametrize("thr", [0.8, 0.2])
def test_config1_vs_oracle(mode, thr):
    import paper_1605_01584_amd as pcc
    X, pl = workloads.config1()
    EI, EJ, ER = oracle.edges(X, thr, cap=1 << 22)
    ref_all = oracle.pearson_packed(X)
    z, zd = pcc.normalize(to_device(X), mode)
    ij, rv, cnt = _edges(z, zd, thr, 1 << 21)
    assert cnt == len(ij)
    got = _set(ij)
    assert all(i < j for i, j in got)
    near = np.abs(np.abs(ref_all) - thr) <= 1e-5
    I, J = np.triu_indices(2000, 1)
    near_set = set(zip(I[near].tolist(), J[near].tolist()))
    want = set(zip(EI.tolist(), EJ.tolist()))
    assert (got - near_set) == (want - near_set)
    # values
    pos = packed_pos(2000, ij[:, 0], ij[:, 1])
    assert np.max(np.abs(rv - ref_all[pos])) <= 1e-5
    if thr == 0.8:
        planted = set(zip(np.minimum(pl.u, pl.v).tolist(), np.maximum(pl.u, pl.v).tolist()))
        assert planted <= got


@pytest.mark.parametrize("mode", ["fp32", "split", "bf16", "fp16"])
def test_edges_equal_thresholded_allpairs(mode):
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(3)
    X = rng.standard_normal((700, 30)).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), mode)
    r = pcc.allpairs(z, zd).cpu().numpy()
    for thr in (0.5, 0.3):
        ij, rv, cnt = _edges(z, zd, thr, 1 << 20)
        I, J = np.triu_indices(700, 1)
        keep = np.abs(r) >= thr
        assert _set(ij) == set(zip(I[keep].tolist(), J[keep].tolist()))
        assert np.array_equal(rv, r[packed_pos(700, ij[:, 0], ij[:, 1])])


def test_capacity_overflow_reports_true_count():
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(4)
    X = rng.standard_normal((400, 20)).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), "fp32")
    ij_all, rv_all, total = _edges(z, zd, 0.4, 1 << 20)
    assert total > 100
    with pytest.raises(pcc.PccError) as e:
        pcc.threshold_edges(z, zd, 0.4, 50)
    assert e.value.status == pcc.PCC_E_CAPACITY
    ij, rv, cnt = pcc.threshold_edges(z, zd, 0.4, 50, sync=False)
    import torch
    torch.cuda.synchronize()
    assert int(cnt.item()) == total
    stored = _set(ij.cpu().numpy())
    assert len(stored) == 50 and stored <= _set(ij_all)


def test_threshold_zero_and_degenerate():
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(6)
    X = rng.standard_normal((130, 16)).astype(np.float32)
    X[7] = 2.0
    z, zd = pcc.normalize(to_device(X), "split")
    ij, rv, cnt = _edges(z, zd, 0.0, 1 << 16)
    assert cnt == 129 * 128 // 2          # every pair without row 7
    assert 7 not in set(ij.ravel().tolist())
    ij, rv, cnt = _edges(z, zd, 1.5, 16)
    assert cnt == 0


def _check_against_scan(ij, rv, cnt, thr, band, scan):
    """The edge set equals the full scan's outside the band around the
    threshold; every reported r is within 1e-5 of the oracle's."""
    got = _set(ij)
    assert cnt == len(got)
    near = {p for p, r in scan.items() if abs(abs(r) - thr) <= band}
    want = {p for p, r in scan.items() if abs(r) >= thr}
    assert (got - near) == (want - near)
    for (i, j), r in zip(map(tuple, ij.tolist()), rv.tolist()):
        if (i, j) in scan:
            assert abs(r - scan[(i, j)]) <= 1e-5, (i, j)
    return got, want


@pytest.mark.parametrize("mode", ["split", "fp32"])
def test_config3_edges_equal_full_scan(mode):
    """n = 32768, l = 4096, |r| >= 0.8: the whole edge list against the
    oracle's scan of all 536,854,528 pairs."""
    import paper_1605_01584_amd as pcc
    thr, band, scan = read_scan("edges_n32768_l4096_thr0.8")
    X, pl = workloads.config3()
    z, zd = pcc.normalize(to_device(X), mode)
    ij, rv, cnt = _edges(z, zd, thr, 1 << 16)
    got, want = _check_against_scan(ij, rv, cnt, thr, band, scan)
    planted = set(zip(np.minimum(pl.u, pl.v).tolist(), np.maximum(pl.u, pl.v).tolist()))
    assert planted <= want


def test_config5_big_edges_equal_full_scan():
    """n = 65536, l = 2048, split, |r| >= 0.9 (the large run of the
    uneven-batch workload, as the benchmark times it): the whole edge list
    against the oracle's scan of all 2,147,450,880 pairs, and r on 16 check
    blocks of the packed output."""
    import torch
    import paper_1605_01584_amd as pcc
    thr, band, scan = read_scan("edges_n65536_l2048_thr0.9")
    X, pl = workloads.config5_big()
    n = X.shape[0]
    z, zd = pcc.normalize(to_device(X), "split")
    ij, rv, cnt = _edges(z, zd, thr, 1 << 16)
    got, want = _check_against_scan(ij, rv, cnt, thr, band, scan)
    planted = set(zip(np.minimum(pl.u, pl.v).tolist(), np.maximum(pl.u, pl.v).tolist()))
    assert planted <= want
    r = pcc.allpairs(z, zd)
    blocks = workloads.check_blocks(n, nblocks=16, seed=65)
    I, J = workloads.block_pairs(n, blocks)
    ref = oracle.pearson_pairs(X, I, J)
    assert np.max(np.abs(r[torch.from_numpy(packed_pos(n, I, J)).to(r.device)].cpu().numpy() - ref)) <= 1e-5
    del r
    torch.cuda.empty_cache()


def test_config3_edges_full_size():
    """n = 32768, l = 4096, split, |r| >= 0.8: every planted pair found with
    the oracle's r, and on 16 check blocks the edge set equals the oracle's."""
    import torch
    import paper_1605_01584_amd as pcc
    X, pl = workloads.config3()
    n = X.shape[0]
    z, zd = pcc.normalize(to_device(X), "split")
    ij, rv, cnt = _edges(z, zd, 0.8, 1 << 16)
    got = _set(ij)
    planted = set(zip(np.minimum(pl.u, pl.v).tolist(), np.maximum(pl.u, pl.v).tolist()))
    assert planted <= got
    ref = oracle.pearson_pairs(X, ij[:, 0], ij[:, 1])
    assert np.max(np.abs(rv - ref)) <= 1e-5
    blocks = workloads.check_blocks(n, nblocks=16, seed=44)
    I, J = workloads.block_pairs(n, blocks)
    rr = oracle.pearson_pairs(X, I, J)
    inblk = {(i, j) for i, j in got
             if any(by * 128 <= i < by * 128 + 128 and bx * 128 <= j < bx * 128 + 128
                    for by, bx in blocks)}
    near = set(zip(I[np.abs(np.abs(rr) - 0.8) <= 1e-5].tolist(),
                   J[np.abs(np.abs(rr) - 0.8) <= 1e-5].tolist()))
    want = set(zip(I[np.abs(rr) >= 0.8].tolist(), J[np.abs(rr) >= 0.8].tolist()))
    assert (inblk - near) == (want - near)
    torch.cuda.synchronize()
