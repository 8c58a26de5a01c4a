"""pcc_batch_run_noalloc (the uneven batch with its descriptor table and job
counters in the library's static scratch) against a batch plan of the same
items: z and r bit-identical, and r within 1e-5 of the oracle.  Two calls in
a row, the second with fewer and smaller datasets, so the second runs on the
scratch the first left behind."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import to_device

pytestmark = pytest.mark.gpu


def _datasets(shapes, seed):
    out = []
    for k, (n, l) in enumerate(shapes):
        X, _ = workloads.planted(n, l, seed * 100 + k, n_planted=3, dtype=np.float32)
        out.append(X.astype(np.float64) if k % 3 == 1 else X)
    return out


def _check_against_plan(Xs, tiles, mode):
    import torch
    import paper_1605_01584_amd as pcc
    xs = [to_device(X) for X in Xs]
    plan = pcc.BatchPlan(xs, mode, tiles=tiles)
    plan.launch()
    torch.cuda.synchronize()
    zs = [torch.full_like(z, 0x5A) for z in plan.z]          # stale bytes everywhere
    rs = [torch.full_like(r, float("nan")) for r in plan.r]   # every r shown written
    zd, z, r = pcc.batch_run_noalloc(xs, mode, tiles=tiles, zs=zs, rs=rs)
    torch.cuda.synchronize()
    for d, X in enumerate(Xs):
        print(f"[no-alloc] mode={mode} dataset {d} n={X.shape[0]} l={X.shape[1]}", flush=True)
        assert zd[d].bytes == plan.zd[d].bytes
        assert torch.equal(z[d][: zd[d].bytes], plan.z[d][: zd[d].bytes]), d
        assert torch.equal(r[d], plan.r[d]), d
        got = r[d].cpu().numpy()
        assert np.max(np.abs(got - oracle.pearson_packed(X))) <= 1e-5, d
    plan.close()


@pytest.mark.parametrize("mode", ["split", "fp32"])
def test_noalloc_matches_plan_twice(mode):
    big = [(900, 300), (130, 17), (1100, 600), (257, 64), (513, 129), (2, 2), (700, 2100),
           (1000, 33), (300, 40), (640, 95)]
    small = [(200, 70), (3, 5), (450, 31)]
    _check_against_plan(_datasets(big, 21), [256, 128, 0, 256, 128, 0, 0, 128, 256, 0], mode)
    _check_against_plan(_datasets(small, 22), [128, 0, 256], mode)

