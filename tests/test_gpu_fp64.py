"""The FP64 tile path (v_mfma_f64_16x16x4_f64, the paper's own precision)
against the FP64 oracle: every pair of config 1 (FP64 input), ragged shapes,
schedules, degenerate rows, edges and a sampled full-size run."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu


def fp64_tol(l):
    """|dr| bound of two FP64 evaluations of r: each is a dot product of l
    terms of unit-norm rows (error <= l 2^-53 sum|z_i z_j| <= l 2^-53 by
    Cauchy-Schwarz) after a transformation of a few roundings per sample."""
    return (2 * l + 64) * 2.0 ** -53


def _run(X, cfg=None, f64_out=True, dtype=None):
    import torch
    import paper_1605_01584_amd as pcc
    z, zd = pcc.normalize(to_device(X, dtype), "fp64")
    r = pcc.allpairs_f64(z, zd, cfg) if f64_out else pcc.allpairs(z, zd, cfg)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def test_config1_every_pair():
    X, _ = workloads.config1()            # FP64 input, as the paper computes
    ref = oracle.pearson_packed(X)
    r = _run(X)
    assert r.dtype == np.float64 and r.shape == ref.shape == (1999000,)
    err = np.abs(r - ref)
    print(f"config1 fp64: max|dr| = {err.max():.3e} (bound {fp64_tol(256):.1e})")
    assert err.max() <= fp64_tol(256)
    r32 = _run(X, f64_out=False)          # FP32 output of the same tiles
    assert r32.dtype == np.float32
    assert np.max(np.abs(r32 - ref)) <= 2.0 ** -24 + fp64_tol(256)
    np.testing.assert_array_equal(r32, r.astype(np.float32))


@pytest.mark.parametrize("n", [2, 3, 16, 17, 127, 128, 129, 257, 773])
@pytest.mark.parametrize("l", [2, 3, 15, 16, 17, 1000])
def test_ragged_shapes(n, l):
    rng = np.random.default_rng(9000 + n * 10 + l)
    X = rng.standard_normal((n, l)) * rng.uniform(0.5, 4, (n, 1)) + rng.uniform(-3, 3, (n, 1))
    ref = oracle.pearson_packed(X)
    r = _run(X)
    assert r.shape == ref.shape
    assert np.max(np.abs(r - ref)) <= fp64_tol(l), (n, l)


def test_fp32_input_and_schedules_identical():
    import paper_1605_01584_amd as pcc
    rng = np.random.default_rng(31)
    X = (rng.standard_normal((900, 333)) + 2).astype(np.float32)
    ref = oracle.pearson_packed(X)
    outs = [_run(X, c) for c in (pcc.TileCfg(128, 0, 1, 0), pcc.TileCfg(128, 1, 4, 0),
                                 pcc.TileCfg(128, 1, 8, 5))]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.max(np.abs(outs[0] - ref)) <= fp64_tol(333)


def test_degenerate_rows_and_exact_values():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 64))
    X[7] = 3.0                     # constant: NaN
    X[9] = X[1]                    # duplicate: r = 1
    X[11] = -2.0 * X[1] + 1.0      # negative affine: r = -1
    r = _run(X)
    ref = oracle.pearson_packed(X)
    nanmask = np.isnan(ref)
    assert np.array_equal(np.isnan(r), nanmask)
    assert np.max(np.abs(r[~nanmask] - ref[~nanmask])) <= fp64_tol(64)
    pos = packed_pos(300, [1, 1], [9, 11])
    np.testing.assert_allclose(r[pos], [1.0, -1.0], rtol=0, atol=1e-15)
    assert np.all(np.abs(r[~nanmask]) <= 1.0)


def test_edges_fp64():
    import paper_1605_01584_amd as pcc
    X, _ = workloads.config1()
    z, zd = pcc.normalize(to_device(X), "fp64")
    thr = 0.5
    ij, rv, c = pcc.threshold_edges(z, zd, thr, 1 << 16)
    EI, EJ, ER = oracle.edges(X, thr)
    got = set(zip(ij[:, 0].cpu().tolist(), ij[:, 1].cpu().tolist()))
    want = set(zip(EI.tolist(), EJ.tolist()))
    assert len(got) == c
    # pairs whose oracle |r| lies within the FP64 bound of thr may go either way
    diff = sorted(got ^ want)
    if diff:
        I, J = np.array(diff).T
        assert np.all(np.abs(np.abs(oracle.pearson_pairs(X, I, J)) - thr) <= fp64_tol(256))
    both = sorted(got & want)
    gi = {p: k for k, p in enumerate(zip(ij[:, 0].cpu().tolist(), ij[:, 1].cpu().tolist()))}
    wi = {p: k for k, p in enumerate(zip(EI.tolist(), EJ.tolist()))}
    gv = rv.cpu().numpy()[[gi[p] for p in both]].astype(np.float64)
    np.testing.assert_allclose(gv, ER[[wi[p] for p in both]], rtol=0, atol=2.0 ** -24)


def test_config3_shape_sampled():
    """n = 32768, l = 4096 in FP64 (the benchmark's FP64 leg): the 128-wide
    tile grid at full size writes every element of the triangle (the output
    starts as NaN); sampled blocks against the oracle."""
    import torch
    import paper_1605_01584_amd as pcc
    X, _ = workloads.config3()
    n = X.shape[0]
    z, zd = pcc.normalize(to_device(X), "fp64")
    r = torch.full((n * (n - 1) // 2,), float("nan"), dtype=torch.float64, device="cuda")
    pcc.allpairs_f64(z, zd, out=r)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(r).all())
    blocks = workloads.check_blocks(n, nblocks=8, seed=77)
    I, J = workloads.block_pairs(n, blocks)
    ref = oracle.pearson_pairs(X, I, J)
    got = r[torch.from_numpy(packed_pos(n, I, J)).cuda()].cpu().numpy()
    err = np.abs(got - ref)
    print(f"config3 fp64 sampled: {len(I)} pairs, max|dr| = {err.max():.3e}")
    assert err.max() <= fp64_tol(4096)


def test_paper_table1_16k_sampled():
    """The paper's smallest Table I workload (16,000 profiles of 5,000
    uniform samples) in FP64 end to end, 2048 seeded pairs and the triangle's
    first and last pairs against the oracle."""
    import paper_1605_01584_amd as pcc
    X = workloads.table1(16000)
    n, l = X.shape
    z, zd = pcc.normalize(to_device(X), "fp64")
    r = pcc.allpairs_f64(z, zd).cpu().numpy()
    I, J = workloads.random_pairs(n, 2048, seed=1600)
    I = np.concatenate([I, [0, n - 2]])
    J = np.concatenate([J, [1, n - 1]])
    ref = oracle.pearson_pairs(X, I, J)
    err = np.abs(r[packed_pos(n, I, J)] - ref)
    print(f"Table I 16K fp64: max|dr| = {err.max():.3e} (bound {fp64_tol(l):.1e})")
    assert err.max() <= fp64_tol(l)
