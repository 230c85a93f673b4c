"""Host logic of the library on a machine without a GPU: the launch geometry a
context plans (fftnk_describe), checked against what the kernels assume.

* Radix plans multiply to the length; the register engine takes exactly the
  lengths it is compiled for (8 points: powers of two 8..256; 12 points:
  3 * 2^k, 12..192), everything else the LDS engine.
* a2 work-groups: pass 1 holds one voxel per thread (rt1 * n2 <= 256); the
  tiles of passes 1 and 5 cover every grid line exactly once.
* Column passes: the tiles cover every pencil; LDS-engine tiles hold at most
  4 points per thread (M pencils consecutive in k2-fastest order, across k2
  lines where h < M); every kernel family's LDS fits its budget.
* Batched contexts: per-cell offsets are cumulative, the launch sizes are the
  sums of the cells' work-groups, the engine bits cover every cell's engine.
* The GMRES basis adds m + 1 fields (padded to 64 elements) to the workspace;
  unsupported lengths are refused.
"""
import math
import os

import numpy as np
import pytest

THREADS = 256
LDS_LIMIT = 61440


def _lib_or_skip():
    from paper_1603_08893_amd import fftnk
    import os
    if not os.path.exists(fftnk._LIB_PATH):
        pytest.skip("libfftnk.so not built")
    return fftnk


def _reg_engine(n):
    if n >= 8 and n <= 256 and n & (n - 1) == 0:
        return 8
    k = n // 3
    if n % 3 == 0 and 12 <= n <= 192 and k & (k - 1) == 0:
        return 12
    return 0


def _pairs32(c, axis):
    """FP32 column passes over a 256-long axis take k2-adjacent pencil pairs
    (one 16-byte access per element) where h and the spectrum offset are even."""
    ax = c["axes"][axis]
    return axis < 2 and ax["reg"] == 8 and THREADS // (ax["n"] // 8) < 16 and c["h"] % 2 == 0 and \
        c["spec_off"] % 2 == 0


def _eng_bit(c, axis):
    return 8 if _pairs32(c, axis) else {8: 2, 12: 4, 0: 1}[c["axes"][axis]["reg"]]


def _check_cell(c, prec, policy=0):
    n0, n1, n2 = c["n"]
    h = n2 // 2 if n2 % 2 == 0 else (n2 + 1) // 2
    assert c["h"] == h and c["rows"] == n0 * n1
    for d, (ax, n) in enumerate(zip(c["axes"], (n0, n1, n2))):
        assert ax["n"] == n and math.prod(ax["radix"]) == n, ax
        assert ax["reg"] == (0 if policy >> d & 1 else _reg_engine(n)), (ax, policy)
    b = c["blocks"]
    # a2 passes: every grid line in exactly one tile; pass 1 one voxel per thread
    for key, rt in (("row", c["rt"]), ("row1", c["rt1"])):
        assert rt >= 1 and b[key] * rt >= c["rows"] > (b[key] - 1) * rt, (key, c)
    assert c["rt1"] * n2 <= THREADS
    # column passes (a1: 9 n0 h pencils, a0: 3 n1 h pencils of three components)
    for axis, npen, k64, k32 in ((1, 9 * n0 * h, "col1_64", "col1_32"), (0, 3 * n1 * h, "col0_64", "col0_32")):
        ax = c["axes"][axis]
        for key, M in ((k64, c["m64"]), (k32, c["m32"])):
            if ax["reg"]:
                per = THREADS // (ax["n"] // ax["reg"])
                if key.endswith("_32") and _pairs32(c, axis):
                    per *= 2
                assert b[key] * per >= npen > (b[key] - 1) * per, (key, c)
            else:
                # M consecutive pencils in k2-fastest order (across k2 lines where h < M)
                assert M >= 1 and ax["n"] * M <= 4 * THREADS
                groups = 1 if axis == 1 else 3  # a1: one range over all pencils; a0: one per tensor row
                assert b[key] == groups * math.ceil(npen // groups / M), (key, c)
    assert b["elem9"] >= 1 and b["vox"] >= 1


SHAPES = [(8, 8, 8), (31, 31, 31), (128, 128, 128), (96, 96, 96), (192, 192, 192), (256, 256, 256),
          (24, 24, 24), (12, 10, 16), (7, 6, 9), (3, 64, 4), (10, 48, 12), (6, 12, 96), (4, 6, 192),
          (451, 451, 2), (512, 512, 8), (257, 3, 256), (2, 2, 2), (5, 451, 2), (300, 7, 5), (9, 384, 6),
          (48, 40, 36), (17, 13, 11)] + [(n, 5, m) for n in (2, 3, 13, 37, 64, 100, 243) for m in (2, 9, 24, 128, 255)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_cell_geometry(prec):
    fftnk = _lib_or_skip()
    for shape in SHAPES:
        d = fftnk.describe(shape, prec)
        assert d["nrve"] == 1
        c = d["cells"][0]
        _check_cell(c, prec)
        assert max(d["lds"]) <= LDS_LIMIT
        b = c["blocks"]
        assert d["nblk"] == [b["row"], b["row1"], b["col1_64"], b["col1_32"], b["col0_64"], b["col0_32"],
                             b["elem9"], b["vox"]]
        for axis in range(3):
            assert d["eng"][axis] == _eng_bit(c, axis), (shape, d["eng"])
        esz = 8 if prec == "fp64" else 4
        assert d["workspace_bytes"] >= 9 * math.prod(shape) * (3 * 8 + 4 * esz)


def test_batched_geometry():
    fftnk = _lib_or_skip()
    dims = [(32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (7, 9, 11), (451, 5, 2), (12, 24, 48)]
    d = fftnk.describe(dims)
    vox = spec = rows = 0
    sums = np.zeros(8, dtype=np.int64)
    eng = [0, 0, 0]
    for c, shape in zip(d["cells"], dims):
        assert c["n"] == list(shape)
        _check_cell(c, "fp64")
        assert (c["vox_off"], c["spec_off"], c["row_off"]) == (vox, spec, rows)
        vox += math.prod(shape)
        spec += 9 * c["rows"] * c["h"]
        rows += c["rows"]
        b = c["blocks"]
        sums += [b["row"], b["row1"], b["col1_64"], b["col1_32"], b["col0_64"], b["col0_32"], b["elem9"], b["vox"]]
        for axis in range(3):
            eng[axis] |= _eng_bit(c, axis)
    assert d["nblk"] == sums.tolist() and d["eng"] == eng
    assert max(d["lds"]) <= LDS_LIMIT
    # one twiddle table per distinct length
    lengths = {n for shape in dims for n in shape}
    assert d["tw_total"] == sum(lengths)


def test_gmres_basis_and_refused_lengths():
    fftnk = _lib_or_skip()
    shape = (24, 20, 16)
    for prec, esz in (("fp64", 8), ("fp32", 4)):
        d = fftnk.describe(shape, prec, gmres_restart=12)
        extra = d["workspace_bytes"] - d["workspace_base_bytes"]
        stride = -(-9 * math.prod(shape) // 64) * 64  # basis vectors start on even element counts
        need = 13 * stride * esz
        # and the CG directions of the windowed x update (slots of 256-byte aligned fields)
        W = d["x_window"]
        assert 1 <= W <= 8
        need += W * (-(-9 * math.prod(shape) * esz // 256) * 256) if W > 1 else 0
        assert need <= extra < need + 512
    for bad in ((513, 4, 4), (4, 600, 4), (4, 4, 257), (1, 4, 4)):
        with pytest.raises(fftnk.FftnkError):
            fftnk.describe(bad)


POLICY_SHAPES = [(16, 16, 16), (24, 20, 12), (31, 9, 7), (128, 128, 128), (96, 96, 96), (256, 256, 256),
                 (192, 192, 192), (451, 451, 2), (12, 10, 16), (3, 64, 4), (6, 12, 96), (512, 512, 8), (9, 384, 6)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_policy_geometry(prec):
    """Under every valid plan policy: engines as the policy bits say, the tiles
    of every pass cover the grid lines and pencils exactly, LDS within budget,
    and the partial-sum stride (sized at creation for all policies) covers
    every launch; M and rt follow the policy's caps."""
    fftnk = _lib_or_skip()
    for shape in POLICY_SHAPES:
        base = fftnk.describe(shape, prec)
        for pol in range(64):
            if (pol >> 3) & 3 == 3:
                with pytest.raises(fftnk.FftnkError):
                    fftnk.describe(shape, prec, policy=pol)
                continue
            try:
                d = fftnk.describe(shape, prec, policy=pol)
            except fftnk.FftnkError as e:
                assert e.status == fftnk.EUNSUPPORTED, (shape, pol)
                continue
            c = d["cells"][0]
            assert d["policy"] == pol
            _check_cell(c, prec, pol)
            assert max(d["lds"]) <= LDS_LIMIT
            assert d["pstride"] == base["pstride"] >= max(d["nblk"])
            b0 = base["cells"][0]
            s = (pol >> 3) & 3
            assert c["m64"] <= max(1, 8 >> s) and c["m32"] <= max(1, 16 >> s)
            if c["axes"][2]["reg"] and b0["axes"][2]["reg"] and pol & 32:
                assert c["rt"] == max(1, b0["rt"] // 2)
    with pytest.raises(fftnk.FftnkError):
        fftnk.describe((8, 8, 8), prec, policy=64)


def test_x_window_option():
    """FFTNK_OPT_X_WINDOW: 1..8 (default 8) CG directions in the workspace,
    refused outside that range and once the workspace is bound."""
    import ctypes
    fftnk = _lib_or_skip()
    L = fftnk.lib()
    shape = (24, 20, 16)
    for prec, esz in ((fftnk.FP64, 8), (fftnk.FP32_MIXED, 4)):
        ctx = ctypes.c_void_p()
        assert L.fftnk_create(ctypes.byref(ctx), *shape, prec, None) == fftnk.OK
        try:
            assert fftnk._describe_ctx(ctx)["x_window"] == 8
            slot = -(-9 * math.prod(shape) * esz // 256) * 256
            base = L.fftnk_workspace_bytes(ctx)
            for bad in (0, 9, -1):
                assert L.fftnk_set_option(ctx, fftnk.OPT_X_WINDOW, bad) == fftnk.EINVAL
            assert L.fftnk_set_option(ctx, fftnk.OPT_X_WINDOW, 1) == fftnk.OK
            assert base - L.fftnk_workspace_bytes(ctx) == 8 * slot  # W = 1 uses the p vector itself
            assert L.fftnk_set_option(ctx, fftnk.OPT_X_WINDOW, 3) == fftnk.OK
            assert base - L.fftnk_workspace_bytes(ctx) == 5 * slot
            assert fftnk._describe_ctx(ctx)["x_window"] == 3
        finally:
            L.fftnk_destroy(ctx)


def test_dynamic_lds_declared_aligned():
    """Kernels that also hold static LDS (block reductions) start their dynamic
    LDS right after it: every dynamic LDS declaration is 16-byte aligned so
    that the 16-byte complex accesses of the transforms stay aligned."""
    import glob
    import re
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1603_08893_amd", "csrc")
    decls = []
    for f in glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h")):
        decls += [(f, l) for l in open(f) if re.search(r"extern\s+__shared__", l)]
    assert decls
    for f, l in decls:
        assert "aligned(16)" in l, (f, l)
