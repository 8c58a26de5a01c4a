"""The tiled permutation test (rows of any length) against the oracle's
permutation counts, with the same rules as the LDS kernel's tests: FP32
bit-exact except pairs whose nearest |r_p| lies within 1e-6 of |r_obs|;
split-BF16x3 inside the oracle's [c_lo, c_hi] for a band of twice split's r
tolerance, and exact wherever that range is one value.  Outputs start at -7
(a value no count takes), so every count is shown written."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu

BAND = 1e-6
SPLIT_BAND = 2e-5


def _perms(l, P, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)


def _gpu(X, perms, mode, tiles=True, cfg=None):
    import torch
    import paper_1605_01584_amd as pcc
    z, zd = pcc.normalize(to_device(X), mode)
    n = X.shape[0]
    c = torch.full((n * (n - 1) // 2,), -7, dtype=torch.int32, device="cuda")
    p = torch.from_numpy(perms).cuda()
    if tiles:
        pcc.permtest_tiles(z, zd, p, cfg=cfg, out=c)
    else:
        pcc.permtest(z, zd, p, out=c)
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    assert not np.any(got == -7)
    return got


def _check(got, X, perms, I, J, mode):
    if mode == "fp32":
        want, gap = oracle.permcounts(X, perms, I, J)
        sure = gap > BAND
        assert np.array_equal(got[sure], want[sure])
        return int((~sure).sum())
    want, _, lo, hi = oracle.permcounts(X, perms, I, J, band=SPLIT_BAND)
    assert np.all((lo <= got) & (got <= hi))
    sure = lo == hi
    assert np.array_equal(got[sure], want[sure])
    return int((~sure).sum())


@pytest.mark.parametrize("mode", ["fp32", "split"])
@pytest.mark.parametrize("n,l,P", [(200, 5000, 24), (300, 609, 25), (257, 1000, 33),
                                   (130, 2049, 7), (2, 700, 5), (50, 20000, 4), (40, 33000, 3)])
def test_long_rows_all_pairs(mode, n, l, P):
    """Long rows on every pair: through pcc_permtest where the rows are past
    the LDS kernel's limit (it takes the tiled form for them), through
    pcc_permtest_tiles where that kernel would still hold them (the split
    kernel holds rows of up to 992 samples, the FP32 one up to 608).  The
    gather of permuted copies stages 8 rows in LDS up to 4096 samples, one
    row up to 32768 samples, and reads longer rows from memory (l = 33000)."""
    import paper_1605_01584_amd as pcc
    zd = pcc.z_layout(n, l, mode)
    direct = zd.l_pad <= pcc.permtest_max_l(mode)
    X, _ = workloads.planted(n, l, n + l, n_planted=min(5, n // 2), dtype=np.float32)
    perms = _perms(l, P, n * 7 + l)
    print(f"[permtest tiles] {mode} n={n} l={l} P={P} direct={direct}", flush=True)
    got = _gpu(X, perms, mode, tiles=direct)
    I, J = np.triu_indices(n, 1)
    loose = _check(got, X, perms, I, J, mode)
    assert np.all((got >= 0) & (got <= P))
    print(f"{mode} n={n} l={l} P={P}: {loose} undecided")


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_tiles_and_lds_kernel_agree_with_oracle(mode):
    """Where both forms apply, both meet the oracle by the same rule, and they
    agree on every pair whose count the oracle decides."""
    n, l, P = 400, 300, 30
    X, _ = workloads.planted(n, l, 5, n_planted=5, dtype=np.float32)
    perms = _perms(l, P, 6)
    a = _gpu(X, perms, mode, tiles=True)
    b = _gpu(X, perms, mode, tiles=False)
    I, J = np.triu_indices(n, 1)
    _check(a, X, perms, I, J, mode)
    _check(b, X, perms, I, J, mode)
    if mode == "fp32":
        _, gap = oracle.permcounts(X, perms, I, J)
        sure = gap > BAND
    else:
        _, _, lo, hi = oracle.permcounts(X, perms, I, J, band=SPLIT_BAND)
        sure = lo == hi
    assert np.array_equal(a[sure], b[sure])


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_schedules_give_identical_counts(mode):
    import paper_1605_01584_amd as pcc
    n, l, P = 700, 900, 19
    X, _ = workloads.planted(n, l, 8, n_planted=4, dtype=np.float32)
    perms = _perms(l, P, 9)
    ref = _gpu(X, perms, mode, cfg=pcc.TileCfg(256, 1, 8, 0))
    for cfg in [pcc.TileCfg(128, 0, 1, 0), pcc.TileCfg(128, 1, 4, 0), pcc.TileCfg(256, 0, 1, 7)]:
        assert np.array_equal(_gpu(X, perms, mode, cfg=cfg), ref), cfg


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_identity_repeated_zero_and_degenerate(mode):
    rng = np.random.default_rng(3)
    n, l, P = 290, 1100, 9
    X = rng.standard_normal((n, l)).astype(np.float32)
    ident = np.tile(np.arange(l, dtype=np.int32), (P, 1))
    assert np.all(_gpu(X, ident, mode) == P)       # r_p reproduces r_obs bit for bit
    one = rng.permutation(l).astype(np.int32)
    c = _gpu(X, np.tile(one, (P, 1)), mode)
    assert set(np.unique(c).tolist()) <= {0, P}
    X[3] = 0.25
    perms = _perms(l, 5, 4)
    c = _gpu(X, perms, mode)
    I, J = np.triu_indices(n, 1)
    bad = (I == 3) | (J == 3)
    assert np.all(c[bad] == -1) and np.all(c[~bad] >= 0)
    c0 = _gpu(X, perms[:0], mode)
    assert np.all(c0[~bad] == 0) and np.all(c0[bad] == -1)


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_n4096_l5000_sampled(mode):
    """n = 4096 profiles of l = 5000 samples (the evaluation's profile length),
    P = 100: 4096 seeded pairs and the planted ones against the oracle."""
    n, l, P = 4096, 5000, 100
    X, pl = workloads.planted(n, l, 4242, dtype=np.float32)
    perms = _perms(l, P, 4243)
    print(f"[permtest tiles] {mode} n={n} l={l} P={P}", flush=True)
    got = _gpu(X, perms, mode, tiles=False)
    I, J = workloads.random_pairs(n, 4096, seed=4244)
    I = np.concatenate([I, np.minimum(pl.u, pl.v)])
    J = np.concatenate([J, np.maximum(pl.u, pl.v)])
    g = got[packed_pos(n, I, J)]
    loose = _check(g, X, perms, I, J, mode)
    assert np.all(g[-len(pl.u):] == 0)
    assert np.all((got >= 0) & (got <= P))
    print(f"{mode}: {loose} of {len(I)} sampled pairs undecided")
