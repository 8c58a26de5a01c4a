"""pcc_permtest on the GPU against the oracle's permutation counts: bit-exact
except pairs whose nearest |r_p| is within 1e-6 of |r_obs| (there FP32 and
FP64 may decide differently)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import packed_pos, to_device

pytestmark = pytest.mark.gpu

BAND = 1e-6


def _gpu_counts(X, perms):
    import torch
    import paper_1605_01584_amd as pcc
    z, zd = pcc.normalize(to_device(X), "fp32")
    c = pcc.permtest(z, zd, torch.from_numpy(perms).cuda())
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("n,l,P", [(300, 50, 40), (33, 7, 25), (600, 129, 12)])
def test_small_all_pairs(n, l, P):
    rng = np.random.default_rng(n + l + P)
    X, _ = workloads.planted(n, l, n, n_planted=5, dtype=np.float32)
    perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
    got = _gpu_counts(X, perms)
    I, J = np.triu_indices(n, 1)
    want, gap = oracle.permcounts(X, perms, I, J)
    sure = gap > BAND
    assert np.array_equal(got[sure], want[sure])
    assert np.all((got >= 0) & (got <= P))
    print(f"n={n} l={l} P={P}: {int((~sure).sum())} pairs inside the 1e-6 band")


def test_identity_and_repeated_permutations():
    rng = np.random.default_rng(1)
    n, l, P = 290, 64, 9
    X = rng.standard_normal((n, l)).astype(np.float32)
    ident = np.tile(np.arange(l, dtype=np.int32), (P, 1))
    assert np.all(_gpu_counts(X, ident) == P)
    one = rng.permutation(l).astype(np.int32)
    c = _gpu_counts(X, np.tile(one, (P, 1)))
    assert set(np.unique(c).tolist()) <= {0, P}


def test_zero_permutations_and_degenerate_rows():
    rng = np.random.default_rng(2)
    n, l = 100, 20
    X = rng.standard_normal((n, l)).astype(np.float32)
    X[3] = 0.5
    perms = np.stack([rng.permutation(l) for _ in range(4)]).astype(np.int32)
    c = _gpu_counts(X, perms)
    I, J = np.triu_indices(n, 1)
    bad = (I == 3) | (J == 3)
    assert np.all(c[bad] == -1) and np.all(c[~bad] >= 0)
    c0 = _gpu_counts(X, perms[:0])
    assert np.all(c0[~bad] == 0) and np.all(c0[bad] == -1)


def test_config4_full_size_sampled():
    """n = 8192, l = 512, P = 1000 in one launch; 2048 seeded pairs plus the
    planted pairs against the oracle."""
    X, pl, perms = workloads.config4()
    got = _gpu_counts(X, perms)
    n = X.shape[0]
    I, J = workloads.random_pairs(n, 2048, seed=404)
    I = np.concatenate([I, np.minimum(pl.u, pl.v)])
    J = np.concatenate([J, np.maximum(pl.u, pl.v)])
    want, gap = oracle.permcounts(X, perms, I, J)
    g = got[packed_pos(n, I, J)]
    sure = gap > BAND
    assert np.array_equal(g[sure], want[sure])
    # planted pairs (|r| ~ 0.99) are never reached by a permutation
    assert np.all(g[-len(pl.u):] == 0)
    assert np.all((got >= 0) & (got <= 1000))
