"""Non-symmetric all pairs (two variable sets, Eq. (7)-(8)) on the GPU
against the oracle's literal Eq. (1) over the whole nx x ny job matrix:
ragged shapes in every mode, schedules, a wider output pitch, X x X against
the symmetric path, edges, and a sampled full-size run."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import to_device

pytestmark = pytest.mark.gpu

LOOSE = {"bf16": 6e-3, "fp16": 1.5e-3}


def tol_for(mode, l):
    if mode == "fp64":
        return (2 * l + 64) * 2.0 ** -53 + 2.0 ** -24      # FP32 output
    return LOOSE.get(mode, 1e-5)


def _xy(X, Y, mode, cfg=None, out=None):
    import torch
    import paper_1605_01584_amd as pcc
    zx, zdx = pcc.normalize(to_device(X), mode)
    zy, zdy = pcc.normalize(to_device(Y), mode)
    r = pcc.allpairs_xy(zx, zdx, zy, zdy, cfg, out=out)
    torch.cuda.synchronize()
    return r


def _data(nx, ny, l, seed):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((nx, l)) + rng.uniform(-2, 2, (nx, 1))).astype(np.float32)
    Y = (rng.standard_normal((ny, l)) * 2).astype(np.float32)
    k = min(nx, ny, 5)
    Y[:k] = 0.7 * X[:k] + 0.3 * Y[:k]          # a few strongly correlated cross pairs
    return X, Y


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 300), (129, 7), (257, 383), (600, 129)])
@pytest.mark.parametrize("l", [2, 17, 65, 300])
@pytest.mark.parametrize("mode", ["fp32", "split", "fp64"])
def test_ragged(nx, ny, l, mode):
    import paper_1605_01584_amd as pcc
    X, Y = _data(nx, ny, l, nx * 7 + ny * 3 + l)
    ref = oracle.pearson_xy(X, Y)
    tiles = (128,) if mode == "fp64" else (128, 256)
    for tile in tiles:
        r = _xy(X, Y, mode, pcc.TileCfg(tile, 1, 2, 0)).cpu().numpy()
        assert r.shape == (nx, ny)
        assert np.max(np.abs(r - ref)) <= tol_for(mode, l), (nx, ny, l, tile)


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
def test_16bit_modes(mode):
    X, Y = _data(300, 500, 256, 5)
    ref = oracle.pearson_xy(X, Y)
    r = _xy(X, Y, mode).cpu().numpy()
    err = np.max(np.abs(r - ref))
    print(f"xy {mode}: max|dr| = {err:.3e}")
    assert err <= LOOSE[mode]


def test_schedules_identical_and_pitch():
    import torch
    import paper_1605_01584_amd as pcc
    X, Y = _data(700, 530, 100, 21)
    outs = [_xy(X, Y, "split", c).cpu().numpy()
            for c in (pcc.TileCfg(256, 0, 1, 0), pcc.TileCfg(256, 1, 4, 0), pcc.TileCfg(256, 1, 3, 5))]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # a wider output matrix: columns ny.. are left untouched
    big = torch.full((700, 600), 7.0, dtype=torch.float32, device="cuda")
    _xy(X, Y, "split", pcc.TileCfg(256, 0, 1, 0), out=big)
    b = big.cpu().numpy()
    assert np.array_equal(b[:, :530], outs[0])
    assert np.all(b[:, 530:] == 7.0)


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_x_with_itself_matches_symmetric_path(mode):
    import torch
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(8)
    X = rng.standard_normal((513, 96)).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), mode)
    cfg = pcc.TileCfg(128, 0, 1, 0)
    full = pcc.allpairs_xy(z, zd, z, zd, cfg).cpu().numpy()
    packed = pcc.allpairs(z, zd, cfg).cpu().numpy()
    torch.cuda.synchronize()
    iu = np.triu_indices(513, 1)
    # the tiles above the diagonal are the same computations, bit for bit
    assert np.array_equal(full[iu], packed)
    # below the diagonal the operand roles swap: equal within the mode's error
    assert np.max(np.abs(full.T[iu] - packed)) <= 1e-5
    assert np.max(np.abs(np.diag(full) - 1.0)) <= 1e-5


def test_edges_xy():
    import paper_1605_01584_amd as pcc
    X, Y = _data(900, 700, 128, 44)
    ref = oracle.pearson_xy(X, Y)
    zx, zdx = pcc.normalize(to_device(X), "fp32")
    zy, zdy = pcc.normalize(to_device(Y), "fp32")
    thr = 0.3
    ij, rv, c = pcc.threshold_edges_xy(zx, zdx, zy, zdy, thr, 1 << 16)
    got = set(zip(ij[:, 0].cpu().tolist(), ij[:, 1].cpu().tolist()))
    wy, wx = np.nonzero(np.abs(ref) >= thr)
    want = set(zip(wy.tolist(), wx.tolist()))
    assert len(got) == c > 5
    for (y, x) in got ^ want:                    # only pairs at the threshold may differ
        assert abs(abs(ref[y, x]) - thr) <= 1e-5
    g = {p: k for k, p in enumerate(zip(ij[:, 0].cpu().tolist(), ij[:, 1].cpu().tolist()))}
    both = sorted(got & want)
    gv = rv.cpu().numpy()[[g[p] for p in both]]
    assert np.max(np.abs(gv - np.array([ref[p] for p in both]))) <= 1e-5
    # capacity overflow reports the true count
    with pytest.raises(pcc.PccError) as e:
        pcc.threshold_edges_xy(zx, zdx, zy, zdy, thr, 3)
    assert e.value.status == pcc.PCC_E_CAPACITY


def test_full_size_sampled():
    """16384 x 16384 cross pairs of l = 4096 (the benchmark's non-symmetric
    leg: the two halves of the n = 32768 matrix), split tiles: every cell
    written and identical under four schedules, sampled against the
    oracle."""
    import torch
    import paper_1605_01584_amd as pcc
    Xall, _ = workloads.config3()
    h = Xall.shape[0] // 2
    X, Y = Xall[:h], Xall[h:]
    zx, zdx = pcc.normalize(to_device(X), "split")
    zy, zdy = pcc.normalize(to_device(Y), "split")
    # every cell is written (the output starts as NaN), the same by every schedule
    r = torch.full((h, h), float("nan"), dtype=torch.float32, device="cuda")
    pcc.allpairs_xy(zx, zdx, zy, zdy, out=r)
    assert not bool(r.isnan().any())
    for cfg in (pcc.TileCfg(256, 0, 1, 0), pcc.TileCfg(128, 1, 8, 0), pcc.TileCfg(256, 1, 8, 7)):
        r2 = torch.full_like(r, float("nan"))
        pcc.allpairs_xy(zx, zdx, zy, zdy, cfg, out=r2)
        assert torch.equal(r2, r), cfg
        del r2
    torch.cuda.synchronize()
    I, J = workloads.random_pairs(2 * h, 20000, seed=5)
    I, J = I % h, J % h
    ref = oracle.pearson_pairs(Xall, I, J + h)
    got = r[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()
    err = np.max(np.abs(got - ref))
    print(f"xy full size sampled: max|dr| = {err:.3e}")
    assert err <= 1e-5
    # the planted cross pairs are found
    del r
