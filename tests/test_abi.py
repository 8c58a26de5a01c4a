"""The C-ABI library loads, exports every symbol include/pcc.h declares, and
rejects bad arguments on the host before launching anything.  CPU only: no
call here reaches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pcc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pcc_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    import paper_1605_01584_amd as pcc
    lib = ctypes.CDLL(pcc.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pcc.EXPORTED) == names


def test_status_strings_and_version():
    import paper_1605_01584_amd as pcc
    for s in range(-7, 1):
        assert pcc.status_string(s).startswith("PCC_")
    assert pcc.version() >= 10000


@pytest.mark.parametrize("mode,kchunk,elem", [("fp32", 32, 4), ("split", 32, 4), ("bf16", 64, 2),
                                              ("fp16", 64, 2), ("fp64", 16, 8)])
@pytest.mark.parametrize("n,l", [(2, 2), (2000, 256), (257, 65), (32768, 4096), (65536, 2048)])
def test_layout(mode, kchunk, elem, n, l):
    import paper_1605_01584_amd as pcc
    zd = pcc.z_layout(n, l, mode)
    assert zd.n == n and zd.l == l and zd.kchunk == kchunk
    assert zd.n_pad % 256 == 0 and n <= zd.n_pad < n + 256
    assert zd.l_pad % kchunk == 0 and l <= zd.l_pad < l + kchunk
    assert zd.row_bytes == zd.l_pad * elem and zd.row_bytes % 128 == 0
    assert zd.bytes == zd.n_pad * zd.row_bytes


def test_layout_rejects():
    import paper_1605_01584_amd as pcc
    for n, l in [(0, 10), (-1, 10), (10, 1), (10, 0), (2 ** 31, 10), (10, 2 ** 21 + 1)]:
        with pytest.raises(pcc.PccError) as e:
            pcc.z_layout(n, l)
        assert e.value.status == pcc.PCC_E_SHAPE
    # one profile is a valid layout (a query against a set), but not a pair set
    one = pcc.z_layout(1, 10)
    fake = ctypes.c_void_p(0x1000)
    assert pcc._lib.pcc_allpairs(ctypes.byref(one), fake, fake, None, None, None) == pcc.PCC_E_SHAPE
    assert pcc._lib.pcc_threshold_edges(ctypes.byref(one), fake, 0.5, fake, fake, 1, fake, None,
                                        None, None) == pcc.PCC_E_SHAPE
    assert pcc._lib.pcc_permtest(ctypes.byref(one), fake, fake, 1, fake, None, None) == pcc.PCC_E_SHAPE
    # the largest accepted l keeps a 256-row panel within 2 GiB (32-bit loads)
    for mode in ("fp32", "split", "bf16", "fp16", "fp64"):
        zd = pcc.z_layout(10, 2 ** 21, mode)
        tile = 128 if mode == "fp64" else 256
        assert tile * zd.row_bytes <= 2 ** 31
    with pytest.raises(pcc.PccError) as e:
        pcc.z_layout(10, 10, 7)
    assert e.value.status == pcc.PCC_E_MODE


def test_host_argument_errors_return_before_launch():
    import paper_1605_01584_amd as pcc
    lib = pcc._lib
    zd = pcc.z_layout(100, 50, "fp32")
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    # null pointers
    assert lib.pcc_normalize(None, 0, 50, ctypes.byref(zd), fake, None, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_normalize(fake, 0, 50, ctypes.byref(zd), None, None, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_normalize(fake, 0, 50, None, fake, None, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_allpairs(ctypes.byref(zd), None, fake, None, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_allpairs(ctypes.byref(zd), fake, None, None, None, None) == pcc.PCC_E_ARG
    # ld < l, bad input type
    assert lib.pcc_normalize(fake, 0, 49, ctypes.byref(zd), fake, None, None, None) == pcc.PCC_E_SHAPE
    assert lib.pcc_normalize(fake, 5, 50, ctypes.byref(zd), fake, None, None, None) == pcc.PCC_E_ARG
    # inconsistent descriptor
    bad = pcc.z_layout(100, 50, "fp32")
    bad.row_bytes += 128
    assert lib.pcc_allpairs(ctypes.byref(bad), fake, fake, None, None, None) == pcc.PCC_E_SHAPE
    bad = pcc.z_layout(100, 50, "fp32")
    bad.mode = 9
    assert lib.pcc_allpairs(ctypes.byref(bad), fake, fake, None, None, None) == pcc.PCC_E_MODE
    # bad schedules
    for cfg in [pcc.TileCfg(64, 0, 1, 0), pcc.TileCfg(256, 2, 1, 0), pcc.TileCfg(256, 1, 0, 0),
                pcc.TileCfg(128, 0, 1, -1)]:
        assert lib.pcc_allpairs(ctypes.byref(zd), fake, fake, ctypes.byref(cfg), None,
                                None) == pcc.PCC_E_ARG
    # edges: null count, negative cap, NaN threshold, cap>0 without arrays
    assert lib.pcc_threshold_edges(ctypes.byref(zd), fake, 0.5, fake, fake, 10, None, None, None,
                                   None) == pcc.PCC_E_ARG
    assert lib.pcc_threshold_edges(ctypes.byref(zd), fake, 0.5, fake, fake, -1, fake, None, None,
                                   None) == pcc.PCC_E_ARG
    assert lib.pcc_threshold_edges(ctypes.byref(zd), fake, float("nan"), fake, fake, 10, fake,
                                   None, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_threshold_edges(ctypes.byref(zd), fake, 0.5, None, None, 10, fake, None, None,
                                   None) == pcc.PCC_E_ARG
    # capacity helper
    assert lib.pcc_edges_status(5, 10) == pcc.PCC_OK
    assert lib.pcc_edges_status(11, 10) == pcc.PCC_E_CAPACITY
    assert lib.pcc_edges_status(-1, 10) == pcc.PCC_E_ARG
    # permtest: unsupported mode, too long rows, null perms with P > 0
    zs = pcc.z_layout(100, 50, "bf16")
    assert lib.pcc_permtest(ctypes.byref(zs), fake, fake, 3, fake, None, None) == pcc.PCC_E_MODE
    # rows past the LDS form take the tiled form, which needs a workspace
    zl = pcc.z_layout(100, 100000, "fp32")
    assert lib.pcc_permtest(ctypes.byref(zl), fake, fake, 3, fake, None, None) == pcc.PCC_E_WORKSPACE
    # tiled form: mode, workspace, schedule
    need = lib.pcc_workspace_size(ctypes.byref(zl), 3)
    assert lib.pcc_permtest_tiles(ctypes.byref(zs), fake, fake, 3, fake, None, fake, 1 << 40,
                                  None) == pcc.PCC_E_MODE
    assert lib.pcc_permtest_tiles(ctypes.byref(zl), fake, fake, 3, fake, None, fake, need - 1,
                                  None) == pcc.PCC_E_WORKSPACE
    assert lib.pcc_permtest_tiles(ctypes.byref(zl), fake, fake, 3, fake, None, None, need,
                                  None) == pcc.PCC_E_WORKSPACE
    odd = ctypes.c_void_p(0x1000 + 64)   # not 256-byte aligned
    assert lib.pcc_permtest_tiles(ctypes.byref(zl), fake, fake, 3, fake, None, odd, need,
                                  None) == pcc.PCC_E_WORKSPACE
    assert lib.pcc_permtest(ctypes.byref(zl), fake, fake, 3, fake, odd, None) == pcc.PCC_E_WORKSPACE
    bad = pcc.TileCfg(64, 0, 1, 0)
    assert lib.pcc_permtest_tiles(ctypes.byref(zl), fake, fake, 3, fake, ctypes.byref(bad), fake,
                                  need, None) == pcc.PCC_E_ARG
    assert lib.pcc_permtest_tiles(ctypes.byref(zl), fake, None, 3, fake, None, fake, need,
                                  None) == pcc.PCC_E_ARG
    assert lib.pcc_permtest(ctypes.byref(zd), fake, None, 3, fake, None, None) == pcc.PCC_E_ARG
    assert lib.pcc_permtest(ctypes.byref(zd), fake, fake, -1, fake, None, None) == pcc.PCC_E_ARG
    # batch plan: bad counts / missing workspace
    plan = ctypes.c_void_p()
    items = (pcc.BatchItem * 1)()
    assert lib.pcc_batch_plan_create(0, items, 1, fake, 1 << 20, None, ctypes.byref(plan)) == pcc.PCC_E_ARG
    assert lib.pcc_batch_plan_create(1, items, 1, None, 1 << 20, None, ctypes.byref(plan)) == pcc.PCC_E_WORKSPACE
    assert lib.pcc_batch_plan_create(1, items, 1, ctypes.c_void_p(0x1000 + 8), 1 << 20, None,
                                     ctypes.byref(plan)) == pcc.PCC_E_WORKSPACE
    assert lib.pcc_batch_plan_create(1, items, 1, fake, 1 << 20, None, ctypes.byref(plan)) == pcc.PCC_E_ARG
    assert lib.pcc_batch_plan_create(1, items, 9, fake, 1 << 20, None, ctypes.byref(plan)) == pcc.PCC_E_MODE
    assert lib.pcc_batch_plan_launch(None, None) == pcc.PCC_E_ARG
    assert lib.pcc_batch_plan_destroy(None) == pcc.PCC_E_ARG
    # batch without allocation: too many datasets, none, a bad mode, a null item
    big = (pcc.BatchItem * (pcc.BATCH_NOALLOC_MAX_D + 1))()
    assert lib.pcc_batch_run_noalloc(pcc.BATCH_NOALLOC_MAX_D + 1, big, 1, None) == pcc.PCC_E_SHAPE
    assert lib.pcc_batch_run_noalloc(0, items, 1, None) == pcc.PCC_E_ARG
    assert lib.pcc_batch_run_noalloc(1, items, pcc.FP64, None) == pcc.PCC_E_MODE
    assert lib.pcc_batch_run_noalloc(1, items, 1, None) == pcc.PCC_E_ARG
    # maps
    assert lib.pcc_cells_host(10, 1, 50, 10, fake, fake) == pcc.PCC_E_SHAPE
    assert lib.pcc_cells_device(10, 1, 0, 5, None, fake, None) == pcc.PCC_E_ARG


def _perm_ws(n, l, mode):
    """The tiled permutation test's workspace, from its definition: observed r,
    S count slots when S > 1, S copies of Z; 256-byte aligned parts."""
    import paper_1605_01584_amd as pcc
    zd = pcc.z_layout(n, l, mode)
    np_ = n * (n - 1) // 2
    S = min(32, max(1, (1 << 27) // np_))
    rb = (np_ * 4 + 255) // 256 * 256
    return rb + (S * rb if S > 1 else 0) + S * zd.bytes


def test_workspace_sizes():
    import paper_1605_01584_amd as pcc
    zd = pcc.z_layout(1000, 100, "split")
    for op in range(3):
        assert pcc._lib.pcc_workspace_size(ctypes.byref(zd), op) == 0
    for n, l, mode in [(1000, 100, "split"), (600, 5000, "fp32"), (4096, 5000, "split"),
                       (32768, 4096, "split"), (2, 700, "fp32")]:
        zd = pcc.z_layout(n, l, mode)
        assert pcc.workspace_size(zd, 3) == _perm_ws(n, l, mode)
        long_rows = zd.l_pad > pcc.permtest_max_l(mode)
        assert pcc.workspace_size(zd, 2) == (_perm_ws(n, l, mode) if long_rows else 0)
    assert pcc.workspace_size(pcc.z_layout(600, 5000, "bf16"), 2) == 0
    assert pcc._lib.pcc_batch_workspace_size(64) >= 256 + 64 * 64
    assert pcc._lib.pcc_batch_workspace_size(64) % 256 == 0


def test_default_cfg():
    import paper_1605_01584_amd as pcc
    big = pcc.default_cfg(pcc.z_layout(32768, 4096, "split"))
    assert big.tile == 256 and big.order in (0, 1)
    small = pcc.default_cfg(pcc.z_layout(600, 100, "split"))
    assert small.tile == 128


def test_permtest_limit_is_lds_bound():
    import paper_1605_01584_amd as pcc
    # without a device the library assumes gfx950's 160 KiB per workgroup (with
    # one it uses the device's limit): the largest multiple of 32 whose LDS
    # footprint fits.  FP32 holds two 32-row panels (rows padded by 16 and 4
    # bytes) and 32 x 32 counts; split holds the 32 permuted rows, a ring of
    # two 64-row chunks at 144 bytes a row, and 64 x 32 observed |r| and
    # counts, and its identity table caps it at 1024 samples.
    cap = 160 * 1024

    def fp32_bytes(lp):
        return 32 * (lp + 4) * 4 + (32 * (lp + 1) * 4 + 15) // 16 * 16 + 32 * 32 * 4

    def split_bytes(lp):
        return (32 * (lp + 1) * 4 + 15) // 16 * 16 + 2 * 64 * 144 + 2 * 64 * 32 * 4

    def largest(f, top):
        return max(lp for lp in range(32, top + 1, 32) if f(lp) <= cap)

    assert pcc.permtest_max_l("fp32") == largest(fp32_bytes, 4096) == 608
    assert pcc.permtest_max_l("split") == largest(split_bytes, 1024) == 992
    assert pcc.permtest_max_l("bf16") == 0 and pcc.permtest_max_l("fp16") == 0
    assert pcc.permtest_max_l("fp64") == 0


def test_fp64_and_xy_argument_errors():
    import paper_1605_01584_amd as pcc
    lib = pcc._lib
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    z64 = pcc.z_layout(100, 50, "fp64")
    z32 = pcc.z_layout(100, 50, "fp32")
    # FP64 tiles are 128 wide only; the FP64-output entry point needs FP64 Z
    c256 = pcc.TileCfg(256, 0, 1, 0)
    assert lib.pcc_allpairs(ctypes.byref(z64), fake, fake, ctypes.byref(c256), None,
                            None) == pcc.PCC_E_ARG
    assert lib.pcc_allpairs_f64(ctypes.byref(z32), fake, fake, None, None, None) == pcc.PCC_E_MODE
    assert lib.pcc_allpairs_f64(ctypes.byref(z64), fake, None, None, None, None) == pcc.PCC_E_ARG
    assert pcc.default_cfg(z64).tile == 128
    assert pcc.default_cfg(pcc.z_layout(40000, 300, "fp64")).tile == 128
    # FP64 is not a permutation-test or batch mode
    assert lib.pcc_permtest(ctypes.byref(z64), fake, fake, 3, fake, None, None) == pcc.PCC_E_MODE
    plan = ctypes.c_void_p()
    items = (pcc.BatchItem * 1)()
    items[0] = pcc.BatchItem(0x1000, 50, 100, 50, 0, 0, 0x1000, 0x1000)
    assert lib.pcc_batch_plan_create(1, items, pcc.FP64, fake, 1 << 20, None,
                                     ctypes.byref(plan)) == pcc.PCC_E_MODE
    # non-symmetric: same mode and samples, output pitch >= ny, pointers
    zy = pcc.z_layout(70, 50, "fp32")
    zy_l = pcc.z_layout(70, 51, "fp32")
    zy_m = pcc.z_layout(70, 50, "split")
    xy = lib.pcc_allpairs_xy
    assert xy(ctypes.byref(z32), fake, ctypes.byref(zy_m), fake, fake, 70, None, None,
              None) == pcc.PCC_E_MODE
    assert xy(ctypes.byref(z32), fake, ctypes.byref(zy_l), fake, fake, 70, None, None,
              None) == pcc.PCC_E_SHAPE
    assert xy(ctypes.byref(z32), fake, ctypes.byref(zy), fake, fake, 69, None, None,
              None) == pcc.PCC_E_SHAPE
    assert xy(ctypes.byref(z32), fake, ctypes.byref(zy), None, fake, 70, None, None,
              None) == pcc.PCC_E_ARG
    assert xy(ctypes.byref(z32), fake, ctypes.byref(zy), fake, None, 70, None, None,
              None) == pcc.PCC_E_ARG
    assert xy(ctypes.byref(z32), fake, None, fake, fake, 70, None, None, None) == pcc.PCC_E_ARG
    ex = lib.pcc_threshold_edges_xy
    assert ex(ctypes.byref(z32), fake, ctypes.byref(zy), fake, float("nan"), fake, fake, 10, fake,
              None, None, None) == pcc.PCC_E_ARG
    assert ex(ctypes.byref(z32), fake, ctypes.byref(zy), fake, 0.5, fake, fake, 10, None,
              None, None, None) == pcc.PCC_E_ARG
    assert ex(ctypes.byref(z32), fake, ctypes.byref(zy_m), fake, 0.5, fake, fake, 10, fake,
              None, None, None) == pcc.PCC_E_MODE
    # rectangle order helper
    cfg = pcc.TileCfg(128, 1, 4, 0)
    assert lib.pcc_rect_tile_order_host(3, 4, ctypes.byref(cfg), 10, 5, fake, fake) == pcc.PCC_E_SHAPE
    assert lib.pcc_rect_tile_order_host(0, 4, ctypes.byref(cfg), 0, 1, fake, fake) == pcc.PCC_E_ARG


def test_stream_to_host_argument_errors():
    import paper_1605_01584_amd as pcc
    lib = pcc._lib
    fake = ctypes.c_void_p(0x1000)
    zd = pcc.z_layout(3000, 100, "split")
    cfg = pcc.TileCfg(128, 1, 4, 0)
    need = pcc.stream_buffer_bytes(zd, cfg, 8)
    # the first pass is the largest: rows 0 .. 8*128-1 of the triangle, two buffers
    first_rows = 8 * 128
    assert need == 2 * 4 * sum(3000 - 1 - y for y in range(first_rows))
    assert pcc.stream_buffer_bytes(zd, cfg, 0) == 0
    nofn = pcc.PASS_FN()
    call = lib.pcc_allpairs_to_host
    # a pass must be a whole number of bands
    assert call(ctypes.byref(zd), fake, fake, 6, fake, need, ctypes.byref(cfg), nofn, None, None,
                None) == pcc.PCC_E_ARG
    # too small a device buffer, missing buffer
    assert call(ctypes.byref(zd), fake, fake, 8, fake, need - 1, ctypes.byref(cfg), nofn, None,
                None, None) == pcc.PCC_E_WORKSPACE
    assert call(ctypes.byref(zd), fake, fake, 8, None, need, ctypes.byref(cfg), nofn, None, None,
                None) == pcc.PCC_E_WORKSPACE
    assert call(ctypes.byref(zd), fake, None, 8, fake, need, ctypes.byref(cfg), nofn, None, None,
                None) == pcc.PCC_E_ARG
    one = pcc.z_layout(1, 100, "split")
    assert call(ctypes.byref(one), fake, fake, 8, fake, need, ctypes.byref(cfg), nofn, None, None,
                None) == pcc.PCC_E_SHAPE


def test_one_hip_runtime_whatever_the_import_order():
    # importing the package before torch must not load a second HIP runtime
    import subprocess
    import sys
    code = ("import paper_1605_01584_amd, torch\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_tile_arith_routes_short_split_rows_to_fp32():
    """Split layouts of rows of one or two chunks (l_pad <= 64) compute in
    FP32; every other layout computes in its own mode."""
    import paper_1605_01584_amd as pcc
    for l, want in [(2, pcc.FP32), (32, pcc.FP32), (33, pcc.FP32), (64, pcc.FP32),
                    (65, pcc.SPLIT_BF16X3), (4096, pcc.SPLIT_BF16X3)]:
        assert pcc.tile_arith(pcc.z_layout(100, l, "split")) == want, l
    for mode in ("fp32", "bf16", "fp16", "fp64"):
        for l in (2, 64, 65, 4096):
            assert pcc.tile_arith(pcc.z_layout(100, l, mode)) == pcc.MODES[mode]
    # the split layout of short rows is byte-compatible with the FP32 one
    for l in (2, 33, 64):
        a, b = pcc.z_layout(300, l, "split"), pcc.z_layout(300, l, "fp32")
        assert (a.row_bytes, a.l_pad, a.bytes) == (b.row_bytes, b.l_pad, b.bytes)
    bad = pcc.z_layout(10, 10, "fp32")
    bad.row_bytes += 128
    assert pcc._lib.pcc_tile_arith(ctypes.byref(bad)) == -1


def test_autotune_default_count():
    import paper_1605_01584_amd as pcc
    from paper_1605_01584_amd import tune
    assert pcc.AUTOTUNE_DEFAULT_CANDIDATES == pcc._lib.pcc_autotune_default_count() == 10
    assert len(tune.candidates()) == 10
