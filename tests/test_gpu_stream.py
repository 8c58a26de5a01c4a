"""Multi-pass all pairs into host memory (double-buffered passes of whole
tile rows, each copied to its place in a host triangle, pinned or pageable):
the host triangle equals the single-launch device result bit for bit, passes
arrive in order and have landed when reported, and the full-size run matches
the oracle on sampled pairs."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu


def _device_ref(z, zd, cfg):
    import torch
    import paper_1605_01584_amd as pcc
    r = pcc.allpairs(z, zd, cfg)
    torch.cuda.synchronize()
    return r.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp32", "split", "fp64"])
@pytest.mark.parametrize("tile,order,band,rpp", [
    (128, 0, 1, 1),      # one tile row per pass, the paper's order
    (128, 1, 4, 8),      # banded, two bands per pass
    (256, 1, 2, 2),      # 256-wide tiles
    (128, 1, 2, 100),    # one pass holds everything
    (256, 0, 1, 3),      # ragged last pass
])
def test_matches_device_allpairs(mode, tile, order, band, rpp):
    import paper_1605_01584_amd as pcc
    if mode == "fp64" and tile != 128:
        pytest.skip("FP64 tiles are 128 wide")
    rng = np.random.default_rng(tile + rpp)
    X = (rng.standard_normal((3001, 70)) + 1).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), mode)
    cfg = pcc.TileCfg(tile, order, band, 0)
    ref = _device_ref(z, zd, cfg)
    host = pcc.allpairs_to_host(z, zd, rpp, cfg).numpy()
    assert np.array_equal(host, ref)


@pytest.mark.parametrize("mode", ["split", "fp32"])
@pytest.mark.parametrize("tile,order,band,rpp", [(128, 1, 4, 8), (256, 0, 1, 3)])
def test_pageable_host_memory(mode, tile, order, band, rpp):
    """Pageable host memory (the copies cannot run asynchronously to it): the
    same triangle, every pass reported."""
    import torch
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(rpp)
    X = rng.standard_normal((2100, 90)).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), mode)
    cfg = pcc.TileCfg(tile, order, band, 0)
    ref = _device_ref(z, zd, cfg)
    out = torch.full((zd.n * (zd.n - 1) // 2,), float("nan"), dtype=torch.float32)
    assert not out.is_pinned()
    seen = []
    pcc.allpairs_to_host(z, zd, rpp, cfg, out=out, on_pass=lambda f, c: seen.append((f, c)))
    assert np.array_equal(out.numpy(), ref)
    assert sum(c for _, c in seen) == len(ref)


def test_passes_in_order_and_landed():
    import torch
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(3)
    n = 2500
    X = rng.standard_normal((n, 96)).astype(np.float32)
    z, zd = pcc.normalize(to_device(X), "split")
    cfg = pcc.TileCfg(128, 1, 2, 0)
    ref = _device_ref(z, zd, cfg)
    out = torch.full((n * (n - 1) // 2,), float("nan"), dtype=torch.float32, pin_memory=True)
    seen = []

    def on_pass(first, count):
        # the slice is complete when reported
        landed = np.array_equal(out[first:first + count].numpy(), ref[first:first + count])
        seen.append((first, count, landed))

    pcc.allpairs_to_host(z, zd, 2, cfg, out=out, on_pass=on_pass)
    m = (n + 127) // 128
    assert len(seen) == (m + 1) // 2
    pos = 0
    for first, count, landed in seen:
        assert first == pos and count > 0 and landed
        pos += count
    assert pos == n * (n - 1) // 2
    np.testing.assert_array_equal(out.numpy(), ref)
    # rows of the triangle start where counting says
    rows = 2 * 128
    assert seen[1][0] == packed_pos(n, [rows], [rows + 1])[0]


def test_against_oracle_small():
    import paper_1605_01584_amd as pcc
    X, _ = workloads.config1()
    z, zd = pcc.normalize(to_device(X), "fp32")
    host = pcc.allpairs_to_host(z, zd, 1, pcc.TileCfg(128, 0, 1, 0)).numpy()
    ref = oracle.pearson_packed(X)
    assert np.max(np.abs(host - ref)) <= 1e-5


def test_full_size_sampled():
    """n = 32768, l = 4096, split, 8 tile rows per pass (16 passes): the
    benchmark's streaming leg, sampled against the oracle."""
    import paper_1605_01584_amd as pcc
    import torch
    X, _ = workloads.config3()
    n = X.shape[0]
    z, zd = pcc.normalize(to_device(X), "split")
    out = torch.full((n * (n - 1) // 2,), float("nan"), dtype=torch.float32, pin_memory=True)
    host = pcc.allpairs_to_host(z, zd, 8, out=out).numpy()
    # every element of the host triangle was written (it starts as NaN)
    assert np.isfinite(host).all()
    blocks = workloads.check_blocks(n, nblocks=16, seed=91)
    I, J = workloads.block_pairs(n, blocks)
    ref = oracle.pearson_pairs(X, I, J)
    got = host[packed_pos(n, I, J)]
    assert np.max(np.abs(got - ref)) <= 1e-5
    # first and last elements of the triangle
    ends = oracle.pearson_pairs(X, [0, n - 2], [1, n - 1])
    assert np.max(np.abs(host[[0, -1]] - ends)) <= 1e-5
