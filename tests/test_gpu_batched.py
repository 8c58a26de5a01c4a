"""Uneven batches in one graph launch: every dataset's packed triangle equals
the single-dataset call with the same tile size, bit for bit, and the oracle
within 1e-5; graph replays with eager work between them agree."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu


def _datasets(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, (n, l) in enumerate(shapes):
        X, _ = workloads.planted(n, l, seed * 100 + k, n_planted=3, dtype=np.float32)
        out.append(X.astype(np.float64) if k % 3 == 1 else X)
    return out


def _late_waits(plan):
    """The kernel's count of bounded waits that expired (the fourth job counter
    of the plan's workspace); must stay 0."""
    return int(plan.workspace[384:392].view(__import__("torch").int64).item())


@pytest.mark.parametrize("mode", ["split", "fp32"])
def test_small_batch_vs_single_and_oracle(mode):
    import torch
    import paper_1605_01584_amd as pcc
    shapes = [(130, 17), (900, 300), (2, 2), (257, 64), (513, 129), (1000, 33)]
    Xs = _datasets(shapes, 7)
    xs = [to_device(X) for X in Xs]
    tiles = [128, 256, 128, 256, 128, 0]
    plan = pcc.BatchPlan(xs, mode, tiles=tiles)
    plan.launch()
    torch.cuda.synchronize()
    assert _late_waits(plan) == 0
    for d, X in enumerate(Xs):
        n = X.shape[0]
        got = plan.r[d].cpu().numpy()
        ref = oracle.pearson_packed(X)
        assert np.max(np.abs(got - ref)) <= 1e-5, d
        tile = tiles[d] or pcc.default_cfg(plan.zd[d]).tile
        z, zd = pcc.normalize(xs[d], mode)
        single = pcc.allpairs(z, zd, pcc.TileCfg(tile, 0, 1, 0)).cpu().numpy()
        assert np.array_equal(got, single), d
    plan.close()


@pytest.mark.parametrize("mode", ["split", "fp32"])
def test_long_rows_batch_vs_single_and_oracle(mode):
    """Rows past the registers' share (2048 samples per wave), partly staged in
    LDS (up to 6144 FP32 or 4096 FP64 samples) and partly read again: every
    set bit-identical to the single-set call and within 1e-5 of the oracle."""
    import torch
    import paper_1605_01584_amd as pcc
    shapes = [(300, 4500), (130, 9000), (257, 2049), (70, 6144), (90, 5000)]
    Xs = _datasets(shapes, 13)          # sets 1 and 4 are FP64
    xs = [to_device(X) for X in Xs]
    plan = pcc.BatchPlan(xs, mode, tiles=[256, 128, 0, 128, 256])
    for r in plan.r:
        r.fill_(float("nan"))
    plan.launch()
    torch.cuda.synchronize()
    assert _late_waits(plan) == 0
    for d, X in enumerate(Xs):
        got = plan.r[d].cpu().numpy()
        assert np.max(np.abs(got - oracle.pearson_packed(X))) <= 1e-5, d
        tile = [256, 128, 0, 128, 256][d] or pcc.default_cfg(plan.zd[d]).tile
        z, zd = pcc.normalize(xs[d], mode)
        assert torch.equal(plan.z[d], z), d
        single = pcc.allpairs(z, zd, pcc.TileCfg(tile, 0, 1, 0)).cpu().numpy()
        assert np.array_equal(got, single), d
    plan.close()


def test_graph_replays_agree():
    import torch
    import paper_1605_01584_amd as pcc
    Xs = _datasets([(400, 50), (700, 90), (1200, 40)], 9)
    xs = [to_device(X) for X in Xs]
    plan = pcc.BatchPlan(xs, "split")
    plan.launch()
    torch.cuda.synchronize()
    first = [r.clone() for r in plan.r]
    for rep in range(3):
        for r in plan.r:
            r.fill_(7.0)                       # eager work between replays
        _ = (xs[0] * 2).sum().item()
        plan.launch()
        torch.cuda.synchronize()
        for a, b in zip(first, plan.r):
            assert torch.equal(a, b), rep
    plan.close()


def test_config5_batch_sampled():
    """64 datasets, n ~ U[500, 8000], l ~ U[50, 2000], split, one graph:
    per dataset 4 seeded 128 x 128 check blocks, 300 random pairs and the
    planted pairs against the oracle."""
    import torch
    import paper_1605_01584_amd as pcc
    batch = workloads.config5_batch()
    xs = [to_device(X) for X, _ in batch]
    plan = pcc.BatchPlan(xs, "split")
    for r in plan.r:
        r.fill_(float("nan"))
    plan.launch()
    torch.cuda.synchronize()
    assert _late_waits(plan) == 0
    total = 0
    for d, (X, pl) in enumerate(batch):
        n = X.shape[0]
        # every element of each triangle was written (they start as NaN)
        assert bool(torch.isfinite(plan.r[d]).all()), d
        BI, BJ = workloads.block_pairs(n, workloads.check_blocks(n, nblocks=4, seed=500 + d))
        I, J = workloads.random_pairs(n, 300, seed=d)
        I = np.concatenate([BI, I, np.minimum(pl.u, pl.v)])
        J = np.concatenate([BJ, J, np.maximum(pl.u, pl.v)])
        got = plan.r[d][torch.from_numpy(packed_pos(n, I, J)).cuda()].cpu().numpy()
        ref = oracle.pearson_pairs(X, I, J)
        assert np.max(np.abs(got - ref)) <= 1e-5, d
        total += n * (n - 1) // 2
    assert plan.jobs > 64
    plan.close()


def test_autotuned_batch_matches_single(tmp_path, monkeypatch):
    """The tuner's tile choice changes speed, never results."""
    import torch
    import paper_1605_01584_amd as pcc
    from paper_1605_01584_amd import tune
    monkeypatch.setenv("PCC_TUNE_CACHE", str(tmp_path / "tune.json"))
    Xs = _datasets([(300, 40), (1500, 64), (2600, 20)], 13)
    xs = [to_device(X) for X in Xs]
    tiles, times = tune.tune_batch(xs, "split", reps=2)
    assert set(tiles) <= {128, 256} and len(tiles) == 3 and len(times) >= 3
    again, _ = tune.tune_batch(xs, "split")       # served from the cache
    assert again == tiles
    plan = pcc.BatchPlan(xs, "split", tiles=tiles)
    plan.launch()
    torch.cuda.synchronize()
    for d, X in enumerate(Xs):
        z, zd = pcc.normalize(xs[d], "split")
        single = pcc.allpairs(z, zd, pcc.TileCfg(tiles[d], 0, 1, 0))
        assert torch.equal(plan.r[d], single)
    plan.close()
    cfg = tune.best_cfg(700, 50, "split", reps=1)
    assert cfg.tile in (128, 256)
