"""CPU checks of the HIP library: it builds, loads and exports the C ABI.

No compute call is made here (there is no GPU in the build container).
"""
import ctypes as C
import os
import re

import pytest

import paper_1811_01604_amd as mpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "mpr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpr_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mpr.load()
    declared = header_symbols()
    assert declared == sorted(mpr.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_library_is_gfx950_code_object():
    data = open(mpr.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_struct_layouts_match_header():
    # sizes implied by the header's field order (natural alignment)
    assert C.sizeof(mpr.Image) == 24
    assert C.sizeof(mpr.Params) == 128
    assert mpr.Params.sweep_limit.offset == 116 and mpr.Params.resume.offset == 120
    assert mpr.Params.barrier_timeout_us.offset == 124
    assert C.sizeof(mpr.ChainStats) == 32


def test_default_params_and_workspace_size():
    p = mpr.default_params()
    assert (p.q, p.R, p.K, p.n_f, p.n_fit, p.sg_degree) == (0.5, 1, 100, 5, 20, 1)
    assert (p.a_targ, p.k_a, p.i_max, p.fixed_relax, p.eq_a_mode) == (0.3, 3.0, 20000, -1, 0)
    assert (p.table_nT, p.table_burn, p.table_meas) == (32, 200, 400)
    lib = mpr.load()
    imgs = mpr.images([(64, 64)])
    ws1 = lib.mpr_workspace_size(imgs, 1, C.byref(p))
    p.R = 64
    ws64 = lib.mpr_workspace_size(imgs, 1, C.byref(p))
    assert 0 < ws1 < ws64
    # each chain holds two 64 x 64 half-grids (stride 64) and their sum arrays
    assert ws64 >= 64 * 2 * 2 * 64 * 64 * 4
    p.R = 0
    assert lib.mpr_workspace_size(imgs, 1, C.byref(p)) < 0
    p.R = 1
    p.n_fit = 65
    assert lib.mpr_workspace_size(imgs, 1, C.byref(p)) < 0


def test_calls_without_device_fail_cleanly():
    lib = mpr.load()
    if os.environ.get("HIP_VISIBLE_DEVICES", None) is None:
        try:
            import torch
            if torch.cuda.is_available():
                pytest.skip("a GPU is present")
        except ImportError:
            pass
    h = C.c_void_p()
    rc = lib.mpr_create(C.byref(h), 0)
    assert rc == mpr.MPR_ERR_HIP and not h
    assert lib.mpr_map_to_angles(None, None, 0, None, None, None, None, None) == mpr.MPR_ERR_ARG
    assert lib.mpr_last_error(None) == b"null context"


def test_size_limits_and_q_validation():
    """Host checks: at most 2^31 sites per image, and a single-precision
    half-grid (rows of ceil(nx/2) rounded up to 64 floats) below 4 GiB, the
    limit of the sweep kernels' 32-bit offsets; q in (0, 1/2], below 1/2
    only with double-precision chains."""
    lib = mpr.load()
    p = mpr.default_params(R=1, K=1)
    ws = lambda shape, prm: lib.mpr_workspace_size(mpr.images([shape]), 1, C.byref(prm))
    assert ws((46000, 46000), p) > 0          # 46000 x 23040 x 4 B = 3.95 GiB
    assert ws((46340, 46340), p) < 0          # 46340 x 23232 x 4 B = 4.01 GiB
    assert ws((65536, 32768), p) < 0          # 2^31 sites, half-grid 4 GiB
    assert ws((46341, 46341), p) < 0          # more than 2^31 sites
    for q, fp64, ok in ((0.5, 0, True), (0.5, 1, True), (0.3, 1, True), (0.3, 0, False), (0.0, 1, False),
                        (0.6, 1, False)):
        prm = mpr.default_params(R=1, K=1, q=q, fp64=fp64)
        assert (ws((64, 64), prm) > 0) == ok, (q, fp64)
    qs = (C.c_double * 2)(0.25, 0.5)
    assert lib.mpr_select_q_workspace_size(mpr.images([(64, 64)]), C.byref(p), qs, 2) > 0
    bad = (C.c_double * 2)(0.25, 0.75)
    assert lib.mpr_select_q_workspace_size(mpr.images([(64, 64)]), C.byref(p), bad, 2) < 0


def test_table_side_cap_bounds_the_table_workspace():
    """With table_side_cap the e(T, L) table chains of a large image run on a
    cap x cap grid: the workspace is then the chains' own (one chain of one
    state: two half-grids and the two of the fused sweep's second buffer),
    not 32 table chains' half-grids; 1 is invalid."""
    lib = mpr.load()
    imgs = mpr.images([(2048, 2048)])
    ws = lambda prm: lib.mpr_workspace_size(imgs, 1, C.byref(prm))
    full = ws(mpr.default_params(R=1, K=1))
    capped = ws(mpr.default_params(R=1, K=1, table_side_cap=256))
    half_grid = 2048 * 1024 * 4
    assert full >= 32 * 2 * half_grid
    assert 4 * half_grid <= capped < 5 * half_grid
    assert ws(mpr.default_params(R=1, K=1, table_side_cap=1)) < 0
    assert ws(mpr.default_params(R=1, K=1, table_side_cap=2)) > 0
    assert mpr.default_params().table_side_cap == 0


def test_binding_rejects_host_tensors_and_short_buffers():
    """The binding checks every tensor before the C call: a host tensor, a
    wrong dtype or a buffer shorter than the images would reach a kernel as a
    bad device pointer.  The checks run without a device (the context is made
    without calling mpr_create)."""
    torch = pytest.importorskip("torch")
    ctx = mpr.Context.__new__(mpr.Context)
    ctx.lib = mpr.load()
    ctx._h = C.c_void_p()
    ctx.device = 0
    imgs = mpr.images([(8, 8), (4, 6)])
    assert mpr.sites_of(imgs) == 88
    z = torch.zeros(88)
    with pytest.raises(ValueError, match="z: must be a tensor on cuda:0"):
        ctx.map_to_angles(imgs, z, z, z)
    with pytest.raises(ValueError, match="a tensor is required"):
        ctx._t(None, "phi_sum", torch.float32, 88)
    assert ctx._t(None, "phi_init", torch.float32, 88, optional=True) is None
    fake = torch.empty(0, device="meta")  # not on cuda: refused like a host tensor
    with pytest.raises(ValueError, match="must be a tensor on cuda:0"):
        ctx._t(fake, "phi", torch.float32, 88)
    ctx._h = C.c_void_p()  # nothing to destroy


def test_batch_validation():
    """An empty batch, a negative offset and an image id in the range the
    temperature tables use for their random streams (>= 0x80000000) are
    refused by the host checks."""
    lib = mpr.load()
    p = mpr.default_params(R=1, K=1)
    ws = lambda imgs, n: lib.mpr_workspace_size(imgs, n, C.byref(p))
    good = mpr.images([(8, 8), (4, 6)])
    assert ws(good, 2) > 0
    assert ws(good, 0) < 0
    bad = mpr.images([(8, 8)], ids=[0x80000000])
    assert ws(bad, 1) < 0
    ok = mpr.images([(8, 8)], ids=[0x7FFFFFFF])
    assert ws(ok, 1) > 0
    neg = mpr.images([(8, 8)])
    neg[0].offset = -1
    assert ws(neg, 1) < 0
    zero = mpr.images([(8, 8)])
    zero[0].nx = 0
    assert ws(zero, 1) < 0
