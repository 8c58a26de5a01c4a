"""pcc_permtest on the GPU against the oracle's permutation counts.

FP32: bit-exact except pairs whose nearest |r_p| is within 1e-6 of |r_obs|
(there FP32 and FP64 may decide differently).  Split-BF16x3: every count lies
in the range the oracle gives for |r| values each off by at most split's r
tolerance (c_lo <= count <= c_hi, band = twice that tolerance), and is exact
wherever that range is a single value."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu

BAND = 1e-6
# split's tolerance on r, 1e-5 at every l (rows of at most 64 samples are
# computed in FP32 arithmetic in the split layout)
SPLIT_TOL = 1e-5


def split_band(l):
    return 2 * SPLIT_TOL


def _gpu_counts(X, perms, mode="fp32"):
    """Counts of every pair; the output starts at -7, a value no count takes,
    so a pair that kept it was never written."""
    import torch
    import paper_1605_01584_amd as pcc
    z, zd = pcc.normalize(to_device(X), mode)
    n = X.shape[0]
    c = torch.full((n * (n - 1) // 2,), -7, dtype=torch.int32, device="cuda")
    pcc.permtest(z, zd, torch.from_numpy(perms).cuda(), out=c)
    torch.cuda.synchronize()
    got = c.cpu().numpy()
    assert not np.any(got == -7)
    return got


def _check(got, X, perms, I, J, mode):
    l = X.shape[1]
    if mode == "fp32":
        want, gap = oracle.permcounts(X, perms, I, J)
        sure = gap > BAND
        assert np.array_equal(got[sure], want[sure])
        return int((~sure).sum())
    want, _, lo, hi = oracle.permcounts(X, perms, I, J, band=split_band(l))
    assert np.all((lo <= got) & (got <= hi))
    sure = lo == hi
    assert np.array_equal(got[sure], want[sure])
    return int((~sure).sum())


@pytest.mark.parametrize("mode", ["fp32", "split"])
@pytest.mark.parametrize("n,l,P", [(300, 50, 40), (33, 7, 25), (600, 129, 12), (200, 96, 33),
                                   (150, 64, 5), (97, 512, 17), (2, 10, 7), (40, 64, 1),
                                   (120, 300, 9), (150, 131, 60)])
def test_small_all_pairs(mode, n, l, P):
    """Every pair against the oracle.  In split the kernel streams the
    unpermuted rows in segments of 1, 2, 3 or 4 chunks of 32 samples, the
    most that divide the row's chunks: l = 129, 300, 96 and 512 take each.
    Rows with l % 4 != 0 load their permutation indices one by one; l = 131
    with P = 60 does so over three passes."""
    rng = np.random.default_rng(n + l + P)
    X, _ = workloads.planted(n, l, n, n_planted=5, dtype=np.float32)
    perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
    got = _gpu_counts(X, perms, mode)
    I, J = np.triu_indices(n, 1)
    loose = _check(got, X, perms, I, J, mode)
    assert np.all((got >= 0) & (got <= P))
    print(f"{mode} n={n} l={l} P={P}: {loose} pairs with an undecided count")


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_longest_rows(mode):
    """Rows of the longest length the LDS holds (both 32-profile panels and
    the count block fill the workgroup's LDS), and rows one sample past it,
    which take the tiled form, both against the oracle."""
    import paper_1605_01584_amd as pcc
    lmax = pcc.permtest_max_l(mode)
    rng = np.random.default_rng(lmax)
    n, P = 70, 9
    for l in (lmax, lmax + 1):
        X, _ = workloads.planted(n, l, 11, n_planted=3, dtype=np.float32)
        perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
        assert (pcc.workspace_size(pcc.z_layout(n, l, mode), 2) > 0) == (l > lmax)
        got = _gpu_counts(X, perms, mode)
        I, J = np.triu_indices(n, 1)
        _check(got, X, perms, I, J, mode)


@pytest.mark.parametrize("mode", ["fp32", "split"])
@pytest.mark.parametrize("l", [64, 160, 512])
def test_identity_and_repeated_permutations(mode, l):
    """An identity permutation reproduces the observed r bit for bit, so it
    always counts; P copies of one permutation give 0 or P.  (Split rows of
    at most 64 samples are computed in FP32; l = 160 and 512 run the split
    kernel, whose observed r goes through an identity index table.  P = 50
    spreads the slots over three passes of the split kernel and two of the
    FP32 one.)"""
    rng = np.random.default_rng(1)
    n, P = 290, 50
    X = rng.standard_normal((n, l)).astype(np.float32)
    ident = np.tile(np.arange(l, dtype=np.int32), (P, 1))
    assert np.all(_gpu_counts(X, ident, mode) == P)
    one = rng.permutation(l).astype(np.int32)
    c = _gpu_counts(X, np.tile(one, (P, 1)), mode)
    assert set(np.unique(c).tolist()) <= {0, P}


@pytest.mark.parametrize("mode", ["fp32", "split"])
@pytest.mark.parametrize("l", [20, 100])
def test_zero_permutations_and_degenerate_rows(mode, l):
    rng = np.random.default_rng(2)
    n = 100
    X = rng.standard_normal((n, l)).astype(np.float32)
    X[3] = 0.5
    perms = np.stack([rng.permutation(l) for _ in range(4)]).astype(np.int32)
    c = _gpu_counts(X, perms, mode)
    I, J = np.triu_indices(n, 1)
    bad = (I == 3) | (J == 3)
    assert np.all(c[bad] == -1) and np.all(c[~bad] >= 0)
    c0 = _gpu_counts(X, perms[:0], mode)
    assert np.all(c0[~bad] == 0) and np.all(c0[bad] == -1)


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_config4_full_size_sampled(mode):
    """n = 8192, l = 512, P = 1000 in one launch; 65,536 seeded pairs plus
    the planted pairs against the oracle (each pair's 1000 permutations)."""
    X, pl, perms = workloads.config4()
    got = _gpu_counts(X, perms, mode)
    n = X.shape[0]
    I, J = workloads.random_pairs(n, 65536, seed=404)
    I = np.concatenate([I, np.minimum(pl.u, pl.v)])
    J = np.concatenate([J, np.maximum(pl.u, pl.v)])
    g = got[packed_pos(n, I, J)]
    loose = _check(g, X, perms, I, J, mode)
    # planted pairs (|r| ~ 0.99) are never reached by a permutation
    assert np.all(g[-len(pl.u):] == 0)
    assert np.all((got >= 0) & (got <= 1000))
    print(f"{mode}: {loose} of {len(I)} sampled pairs with an undecided count")


@pytest.mark.parametrize("mode", ["fp32", "split"])
def test_ragged_n_full_P_sampled(mode):
    """n = 1000 (not a multiple of the 64-row or 32-row jobs), l = 512,
    P = 1000: every job runs all passes and the last tile row and column are
    partial; 3000 seeded pairs against the oracle."""
    rng = np.random.default_rng(77)
    n, l, P = 1000, 512, 1000
    X, pl = workloads.planted(n, l, 77, n_planted=6, dtype=np.float32)
    perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
    got = _gpu_counts(X, perms, mode)
    I, J = workloads.random_pairs(n, 3000, seed=78)
    I = np.concatenate([I, np.minimum(pl.u, pl.v), [n - 2, 0]])
    J = np.concatenate([J, np.maximum(pl.u, pl.v), [n - 1, n - 1]])
    loose = _check(got[packed_pos(n, I, J)], X, perms, I, J, mode)
    assert np.all((got >= 0) & (got <= P))
    print(f"{mode}: {loose} of {len(I)} sampled pairs with an undecided count")
