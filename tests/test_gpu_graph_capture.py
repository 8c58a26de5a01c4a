"""Entry points recorded under stream capture (kernels only: no memcpy or
memset nodes) and replayed several times, with the program's own eager work
and synchronisations between the replays: every replay equals the eager
result bit for bit."""
import numpy as np
import pytest

import workloads
from gpu_util import to_device

pytestmark = pytest.mark.gpu


def _datasets(shapes, seed):
    return [workloads.planted(n, l, seed * 100 + k, n_planted=3, dtype=np.float32)[0]
            for k, (n, l) in enumerate(shapes)]


def test_batch_noalloc_captured_and_replayed():
    import torch
    import paper_1605_01584_amd as pcc
    Xs = _datasets([(700, 90), (300, 40), (1100, 330), (260, 65)], 31)
    xs = [to_device(X) for X in Xs]
    zd, z0, r0 = pcc.batch_run_noalloc(xs, "split")          # eager; also the first call on the device
    torch.cuda.synchronize()
    ref = [r.clone() for r in r0]
    zs = [torch.empty_like(z) for z in z0]
    rs = [torch.empty_like(r) for r in r0]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pcc.batch_run_noalloc(xs, "split", zs=zs, rs=rs, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for r in rs:
            r.fill_(float("nan"))                              # eager work between replays
        _ = (xs[0] * 3).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for d, (a, b) in enumerate(zip(ref, rs)):
            assert torch.equal(a, b), (rep, d)


@pytest.mark.parametrize("mode", ["split", "fp32"])
def test_normalize_allpairs_edges_captured_and_replayed(mode):
    import torch
    import paper_1605_01584_amd as pcc
    X, _ = workloads.planted(900, 300, 32, n_planted=5, dtype=np.float32)
    x = to_device(X)
    z, zd = pcc.normalize(x, mode)
    r_ref = pcc.allpairs(z, zd)
    ij_ref, rv_ref, c_ref = pcc.threshold_edges(z, zd, 0.8, 64)
    assert c_ref >= 5                                          # the planted pairs
    torch.cuda.synchronize()
    z2 = torch.empty_like(z)
    r2 = torch.empty_like(r_ref)
    ij = torch.empty(2 * 64, dtype=torch.int32, device="cuda")
    rv = torch.empty(64, dtype=torch.float32, device="cuda")
    cnt = torch.empty((), dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pcc.normalize(x, mode, z=z2, stream=s)
            pcc.allpairs(z2, zd, out=r2, stream=s)
            pcc._check(pcc._lib.pcc_threshold_edges(
                pcc.ctypes.byref(zd), pcc._dev_ptr(z2, "z"), 0.8, pcc._dev_ptr(ij, "ij"),
                pcc._dev_ptr(rv, "rv"), 64, pcc._dev_ptr(cnt, "count"), None, None,
                pcc._stream(torch, s)), "pcc_threshold_edges")
    torch.cuda.synchronize()
    for rep in range(3):
        r2.fill_(float("nan"))
        cnt.fill_(-5)
        _ = (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r2, r_ref), rep
        assert int(cnt.item()) == c_ref, rep
        got = sorted(zip(ij.view(-1, 2)[:c_ref].cpu().numpy().tolist(), rv[:c_ref].cpu().numpy().tolist()))
        want = sorted(zip(ij_ref.cpu().numpy().reshape(-1, 2).tolist(), rv_ref.cpu().numpy().tolist()))
        assert got == want, rep


@pytest.mark.parametrize("mode,l,tiles", [("split", 200, False), ("fp32", 200, False),
                                          ("split", 1100, True)])
def test_permtest_captured_and_replayed(mode, l, tiles):
    """The permutation test recorded as one graph (the persistent LDS kernel,
    or the tiled form's fills, observed r, gathers, tile launches and final
    sum) and replayed: every replay gives the eager counts."""
    import torch
    import paper_1605_01584_amd as pcc
    n, P = 300, 40
    X, _ = workloads.planted(n, l, 33, n_planted=4, dtype=np.float32)
    rng = np.random.default_rng(l)
    perms = torch.from_numpy(np.stack([rng.permutation(l) for _ in range(P)]).astype(np.int32)).cuda()
    z, zd = pcc.normalize(to_device(X), mode)
    assert (zd.l_pad > pcc.permtest_max_l(mode)) == tiles
    ws = torch.empty(max(pcc.workspace_size(zd, 2), 256), dtype=torch.uint8, device="cuda")
    ref = pcc.permtest(z, zd, perms, workspace=ws)            # eager, rows checked
    torch.cuda.synchronize()
    c = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pcc.permtest(z, zd, perms, out=c, stream=s, validate=False, workspace=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        c.fill_(-7)
        ws.fill_(0x5a)                                           # the tiled form refills its slots
        _ = (z.float() * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(c, ref), rep
