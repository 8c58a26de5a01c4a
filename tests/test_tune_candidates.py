"""The batch autotuner's candidate tile assignments, on the CPU: the pair
slots a tiling computes, and the candidate rules on the uneven batch's
shapes (distinct assignments only)."""
import math

import workloads


def test_tile_slots():
    from paper_1605_01584_amd import tune
    # whole tiles of the inclusive triangle: m(m+1)/2 tiles of t x t slots
    for n, t in [(1, 128), (256, 256), (257, 256), (500, 128), (8000, 256)]:
        m = math.ceil(n / t)
        assert tune._tile_slots(n, t) == m * (m + 1) // 2 * t * t
    assert tune._tile_slots(500, 256) / tune._tile_slots(500, 128) - 1.0 > 0.1


def test_batch_candidates():
    from paper_1605_01584_amd import tune
    shapes = workloads.config5_shapes()
    cands = tune._assignments(shapes)
    assert cands["all256"] == [256] * len(shapes) and cands["all128"] == [128] * len(shapes)
    assert cands["128_below_2048"] == [128 if n < 2048 else 256 for n, _ in shapes]
    ex = cands["128_over_0.1_excess"]
    for (n, _), t in zip(shapes, ex):
        excess = tune._tile_slots(n, 256) / tune._tile_slots(n, 128) - 1.0
        assert t == (128 if excess > 0.1 else 256)
    # every candidate is a distinct assignment of 128 or 256 per dataset
    seen = set()
    for tiles in cands.values():
        assert len(tiles) == len(shapes) and set(tiles) <= {128, 256}
        assert tuple(tiles) not in seen
        seen.add(tuple(tiles))
