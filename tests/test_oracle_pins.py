"""Pins of the FP64 oracle against facts that do not come from the oracle:
a library routine (numpy.corrcoef), closed forms, invariants of Eq. (1),
hand-worked fixtures, and brute force.  CPU only."""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_textbook():
    vals = {}
    with open(os.path.join(GOLDEN, "pearson_textbook.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *rest = line.split()
            vals[k] = np.array([float(t) for t in rest])
    return vals


def test_textbook_example(oracle_mod):
    v = _read_textbook()
    X = np.stack([v["u"], v["v"]])
    r = oracle_mod.pearson_packed(X)
    assert r.shape == (1,)
    assert abs(r[0] - v["r"][0]) <= 1e-15
    assert abs(r[0] - np.sqrt(0.6)) <= 1e-15


@pytest.mark.parametrize("l", [2, 3, 17, 256])
@pytest.mark.parametrize("n", [2, 5, 64])
def test_vs_numpy_corrcoef(oracle_mod, n, l):
    rng = np.random.default_rng(100 + n * 7 + l)
    X = rng.standard_normal((n, l)) * rng.uniform(0.1, 10, (n, 1)) + rng.uniform(-5, 5, (n, 1))
    r = oracle_mod.pearson_packed(X)
    C = np.corrcoef(X)
    iu = np.triu_indices(n, 1)
    assert r.shape == (n * (n - 1) // 2,)
    np.testing.assert_allclose(r, C[iu], rtol=0, atol=1e-12)


def test_packed_order_matches_row_major_upper(oracle_mod):
    # a permutation-free check of the output order: distinct rows give
    # distinct r, and position t must hold the pair of the t-th cell
    rng = np.random.default_rng(5)
    X = rng.standard_normal((9, 40))
    r = oracle_mod.pearson_packed(X)
    t = 0
    for i in range(9):
        for j in range(i + 1, 9):
            assert r[t] == oracle_mod.pearson_pairs(X, [i], [j])[0]
            t += 1


def test_invariants(oracle_mod):
    rng = np.random.default_rng(11)
    l = 300
    u = rng.standard_normal(l)
    v = rng.standard_normal(l)
    X = np.stack([u, u.copy(), -u, 2.5 * u - 7.0, -0.3 * u + 1.0, v, 4.0 * v + 3.0])
    r = oracle_mod.pearson_pairs
    assert r(X, [0], [1])[0] == 1.0                       # r(u,u) = 1
    assert abs(r(X, [0], [2])[0] + 1.0) <= 1e-15          # r(u,-u) = -1
    assert abs(r(X, [0], [3])[0] - 1.0) <= 1e-13          # positive affine
    assert abs(r(X, [0], [4])[0] + 1.0) <= 1e-13          # negative slope
    # symmetry, bit for bit
    assert r(X, [0], [5])[0] == r(X, [5], [0])[0]
    # invariance of r(u, v) under a positive affine map of v
    assert abs(r(X, [0], [5])[0] - r(X, [0], [6])[0]) <= 1e-13
    # bounded
    Y = rng.standard_normal((40, 8))
    assert np.all(np.abs(oracle_mod.pearson_packed(Y)) <= 1.0)


def test_constant_and_nonfinite_rows_give_nan(oracle_mod):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 10))
    X[1] = 3.25
    X[3, 4] = np.nan
    r = oracle_mod.pearson_packed(X)
    # pairs: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    assert np.isnan(r[0]) and np.isnan(r[2]) and np.isnan(r[3]) and np.isnan(r[4])
    assert np.isnan(r[5])
    assert np.isfinite(r[1])


@pytest.mark.parametrize("a,c", [(1.0, 0.0), (0.6, 0.8), (-2.0, 1.0), (0.1, 3.0), (-0.5, -0.5)])
def test_closed_form_planted_pair(oracle_mod, a, c):
    # u and w centred, unit length and orthogonal; v = a*u + c*w + b has
    # r(u, v) = a / sqrt(a^2 + c^2) exactly.
    rng = np.random.default_rng(21)
    l = 257
    u = rng.standard_normal(l)
    u -= u.mean()
    u /= np.linalg.norm(u)
    w = rng.standard_normal(l)
    w -= w.mean()
    w -= (w @ u) * u
    w -= w.mean()
    w /= np.linalg.norm(w)
    v = a * u + c * w + 0.37
    r = oracle_mod.pearson_pairs(np.stack([u, v]), [0], [1])[0]
    assert abs(r - a / np.hypot(a, c)) <= 1e-13


def test_transform_pins(oracle_mod):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((30, 101)) * 3.0 + 11.0
    U, mean, m2 = oracle_mod.transform(X)
    np.testing.assert_allclose(mean, X.mean(axis=1), rtol=0, atol=1e-13)
    np.testing.assert_allclose(m2, ((X - X.mean(axis=1, keepdims=True)) ** 2).sum(axis=1),
                               rtol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(U, axis=1), 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(U.sum(axis=1), 0.0, rtol=0, atol=1e-13)
    # Eq. (5): after Eq. (4) the dot product of two rows is Eq. (1)
    G = U @ U.T
    iu = np.triu_indices(30, 1)
    np.testing.assert_allclose(G[iu], oracle_mod.pearson_packed(X), rtol=0, atol=1e-14)


def test_transform_degenerate_row_is_nan(oracle_mod):
    X = np.ones((2, 5))
    X[1] = [1, 2, 3, 4, 5]
    U, mean, m2 = oracle_mod.transform(X)
    assert m2[0] == 0.0 and np.all(np.isnan(U[0]))
    assert np.all(np.isfinite(U[1]))


def _golden_jobmap():
    tab = {}
    cur = None
    with open(os.path.join(GOLDEN, "jobmap_n4.txt")) as f:
        for line in f:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            if s in ("inclusive", "exclusive"):
                cur = s
                tab[cur] = []
                continue
            tab[cur].append(tuple(int(t) for t in s.split()))
    return tab


def test_enumeration_golden(oracle_mod):
    tab = _golden_jobmap()
    for name, diag in (("inclusive", True), ("exclusive", False)):
        ys, xs = oracle_mod.enumerate_upper(4, diag)
        got = [(i, int(y), int(x)) for i, (y, x) in enumerate(zip(ys, xs))]
        assert got == tab[name]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257])
def test_enumeration_brute_force(oracle_mod, n):
    for diag in (True, False):
        ys, xs = oracle_mod.enumerate_upper(n, diag)
        want = [(y, x) for y in range(n) for x in range(y if diag else y + 1, n)]
        assert list(zip(ys.tolist(), xs.tolist())) == want
        # F_n(n) = n(n+1)/2 cells with the diagonal, n(n-1)/2 without
        assert len(ys) == (n * (n + 1) // 2 if diag else n * (n - 1) // 2)


def test_permcounts_identity_and_repeated(oracle_mod):
    rng = np.random.default_rng(4)
    n, l, P = 12, 33, 20
    X = rng.standard_normal((n, l))
    I, J = np.triu_indices(n, 1)
    ident = np.tile(np.arange(l, dtype=np.int32), (P, 1))
    counts, gap = oracle_mod.permcounts(X, ident, I, J)
    assert np.all(counts == P) and np.all(gap == 0.0)
    one = rng.permutation(l).astype(np.int32)
    counts, _ = oracle_mod.permcounts(X, np.tile(one, (P, 1)), I, J)
    assert set(np.unique(counts).tolist()) <= {0, P}


def test_permcounts_vs_numpy(oracle_mod):
    rng = np.random.default_rng(9)
    n, l, P = 10, 24, 50
    X = rng.standard_normal((n, l))
    perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
    I, J = np.triu_indices(n, 1)
    counts, gap = oracle_mod.permcounts(X, perms, I, J)
    for q, (i, j) in enumerate(zip(I, J)):
        robs = abs(np.corrcoef(X[i], X[j])[0, 1])
        rp = np.array([abs(np.corrcoef(X[i], X[j][perms[p]])[0, 1]) for p in range(P)])
        want = int(np.sum(rp >= robs))
        if gap[q] > 1e-10:
            assert counts[q] == want
        assert abs(gap[q] - np.min(np.abs(rp - robs))) <= 1e-12


def test_permcounts_band_bounds(oracle_mod):
    """c_lo / c_hi against numpy corrcoef; band 0 collapses both onto the
    count, a band of 2 (wider than any |r| difference) opens them to 0 and P."""
    rng = np.random.default_rng(19)
    n, l, P = 9, 20, 40
    X = rng.standard_normal((n, l))
    perms = np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)
    I, J = np.triu_indices(n, 1)
    c, _, lo, hi = oracle_mod.permcounts(X, perms, I, J, band=0.0)
    assert np.array_equal(lo, c) and np.array_equal(hi, c)
    c, _, lo, hi = oracle_mod.permcounts(X, perms, I, J, band=2.0)
    assert np.all(lo == 0) and np.all(hi == P)
    band = 0.03
    c, _, lo, hi = oracle_mod.permcounts(X, perms, I, J, band=band)
    for q, (i, j) in enumerate(zip(I, J)):
        robs = abs(np.corrcoef(X[i], X[j])[0, 1])
        rp = np.array([abs(np.corrcoef(X[i], X[j][perms[p]])[0, 1]) for p in range(P)])
        d = rp - robs
        # decisions within 1e-12 of an edge may go either way in rounding
        if np.all(np.abs(np.abs(d) - band) > 1e-12):
            assert lo[q] == int(np.sum(d >= band)) and hi[q] == int(np.sum(d >= -band))
    assert np.all(lo <= c) and np.all(c <= hi) and np.any(lo < hi)
    X[4] = 2.0
    c, _, lo, hi = oracle_mod.permcounts(X, perms, [4, 0], [5, 4], band=band)
    assert np.all(lo == -1) and np.all(hi == -1) and np.all(c == -1)


def test_permcounts_nan_pair(oracle_mod):
    X = np.random.default_rng(1).standard_normal((3, 8))
    X[2] = 1.0
    perms = np.stack([np.arange(8), np.arange(8)[::-1]]).astype(np.int32)
    counts, _ = oracle_mod.permcounts(X, perms, [0, 0, 1], [1, 2, 2])
    assert counts[1] == -1 and counts[2] == -1 and counts[0] >= 1


def test_edges_vs_numpy(oracle_mod):
    rng = np.random.default_rng(12)
    X = rng.standard_normal((60, 20))
    X[7] = 0.9 * X[3] + 0.1 * rng.standard_normal(20)
    X[40] = -X[11] + 0.05 * rng.standard_normal(20)
    thr = 0.6
    EI, EJ, ER = oracle_mod.edges(X, thr)
    C = np.corrcoef(X)
    iu = np.triu_indices(60, 1)
    keep = np.abs(C[iu]) >= thr
    near = np.abs(np.abs(C[iu]) - thr) <= 1e-12
    want = set(zip(iu[0][keep & ~near].tolist(), iu[1][keep & ~near].tolist()))
    got = set(zip(EI.tolist(), EJ.tolist()))
    assert want <= got and len(got - want) <= int(near.sum())
    assert (3, 7) in got and (11, 40) in got
    # (i, j) order
    order = np.lexsort((EJ, EI))
    assert np.all(order == np.arange(len(EI)))


def test_planted_pairs_follow_model(oracle_mod):
    X, pl = workloads.config1()
    assert X.shape == (2000, 256) and X.dtype == np.float64
    r = oracle_mod.pearson_pairs(X, pl.u, pl.v)
    rho = pl.a / np.sqrt(pl.a ** 2 + 0.01)
    # sampling error of r around rho is about (1 - rho^2)/sqrt(l)
    assert np.all(np.abs(r - rho) <= 6 * (1 - rho ** 2) / np.sqrt(256) + 1e-3)
    assert len(set(pl.u.tolist()) | set(pl.v.tolist())) == 40


@pytest.mark.parametrize("nx,ny,l", [(1, 1, 2), (3, 7, 5), (17, 9, 33), (40, 64, 256)])
def test_xy_vs_numpy_corrcoef(oracle_mod, nx, ny, l):
    # non-symmetric job matrix (two variable sets): the cross block of
    # numpy's correlation matrix of the stacked rows, in (X row, Y row) order
    rng = np.random.default_rng(300 + nx + 5 * ny + l)
    X = rng.standard_normal((nx, l)) * rng.uniform(0.1, 10, (nx, 1))
    Y = rng.standard_normal((ny, l)) + rng.uniform(-5, 5, (ny, 1))
    r = oracle_mod.pearson_xy(X, Y)
    C = np.corrcoef(np.vstack([X, Y]))
    assert r.shape == (nx, ny)
    np.testing.assert_allclose(r, C[:nx, nx:], rtol=0, atol=1e-12)


def test_xy_closed_form_and_orientation(oracle_mod):
    # Y_j = a_j u + c_j w with u, w centred and orthogonal of equal norm:
    # r(u, Y_j) = a_j / sqrt(a_j^2 + c_j^2) exactly; row 1 of X is -u.
    l = 64
    k = np.arange(l)
    u = np.cos(2 * np.pi * 3 * k / l)
    w = np.sin(2 * np.pi * 5 * k / l)
    a = np.array([1.0, -2.0, 0.5, 3.0])
    c = np.array([1.0, 1.0, 2.0, 0.0])
    Y = a[:, None] * u + c[:, None] * w
    r = oracle_mod.pearson_xy(np.stack([u, -u]), Y)
    ref = a / np.sqrt(a * a + c * c)
    np.testing.assert_allclose(r[0], ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r[1], -ref, rtol=0, atol=1e-14)


def test_xy_with_itself_is_the_symmetric_matrix(oracle_mod):
    rng = np.random.default_rng(17)
    X = rng.standard_normal((23, 41))
    X[5] = 2.0                                   # constant row: NaN everywhere
    r = oracle_mod.pearson_xy(X, X)
    packed = oracle_mod.pearson_packed(X)
    iu = np.triu_indices(23, 1)
    np.testing.assert_array_equal(r[iu], packed)          # same arithmetic, bit for bit
    np.testing.assert_array_equal(r.T[iu], packed)        # Eq. (1) is symmetric
    d = np.diag(r).copy()
    assert np.isnan(d[5]) and np.all(np.isnan(r[5])) and np.all(np.isnan(r[:, 5]))
    np.testing.assert_allclose(np.delete(d, 5), 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,n,l", [("edges_n32768_l4096_thr0.8", 32768, 4096),
                                      ("edges_n65536_l2048_thr0.9", 65536, 2048)])
def test_stored_full_scans(oracle_mod, name, n, l):
    """The stored full scans (tests/golden/make_edge_scans.py, oracle only)
    parse, list pairs i < j in scan order with |r| >= threshold - band, hold
    every planted pair of their workload, and agree with the oracle
    recomputed on the listed pairs."""
    import os
    import workloads
    from golden_scan import GOLDEN, read_scan
    if not os.path.exists(os.path.join(GOLDEN, name + ".txt")):
        pytest.fail(f"{name}.txt missing: run tests/golden/make_edge_scans.py")
    thr, band, scan = read_scan(name)
    assert band == 1e-5 and thr in (0.8, 0.9)
    keys = list(scan)
    assert keys == sorted(keys)
    assert all(0 <= i < j < n for i, j in keys)
    assert all(abs(r) >= thr - band for r in scan.values())
    X, pl = (workloads.config3() if n == 32768 else workloads.config5_big())
    assert X.shape == (n, l)
    planted = set(zip(np.minimum(pl.u, pl.v).tolist(), np.maximum(pl.u, pl.v).tolist()))
    strong = {p for p, r in scan.items() if abs(r) >= thr}
    assert planted <= strong
    I = np.array([i for i, _ in keys], dtype=np.int64)
    J = np.array([j for _, j in keys], dtype=np.int64)
    np.testing.assert_allclose(oracle_mod.pearson_pairs(X, I, J), [scan[k] for k in keys],
                               rtol=0, atol=1e-15)
