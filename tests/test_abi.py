"""Host-side checks of the C ABI that run without a GPU: the library loads,
exports every entry point declared in include/*.h, and rejects invalid
arguments on the host before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stkde_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1705_09366_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libstkde.so is not built (run __graft_entry__.build())")
    return m


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    decl = _declared_symbols()
    assert "stkde_compute" in decl and "stkde_plan" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(L.EXPORTED)


def test_status_strings_and_version(L):
    assert L.status_string(0) == "ok"
    assert "workspace" in L.status_string(L.STKDE_ERR_WORKSPACE)
    assert L.lib().stkde_version() >= 100


def _plan_status(L, **kw):
    base = dict(gx=16, gy=16, gt=16, hs=2.0, ht=2.0)
    base.update(kw)
    d = L.Desc(**base)
    h = ctypes.c_void_p()
    st = L.lib().stkde_plan(ctypes.byref(d._c()), None, ctypes.byref(h))
    if st == 0:
        L.lib().stkde_plan_destroy(h)
    return st


@pytest.mark.parametrize("kw,expect", [
    (dict(), 0),
    (dict(gx=0), -1), (dict(gy=-3), -1), (dict(gt=0), -1),
    (dict(gx=70000), -2),
    (dict(hs=0.0), -1), (dict(ht=-1.0), -1), (dict(hs=float("nan")), -1),
    (dict(sres=0.0), -1), (dict(tres=float("inf")), -1),
    (dict(x0=float("nan")), -1),
    (dict(flags=1 << 10), -1),
    (dict(hs=1e12), -2),
])
def test_plan_validation(L, kw, expect):
    assert _plan_status(L, **kw) == expect


def test_tuning_validation(L):
    d = L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0)
    for bad in (L.Tuning(tile_t=8), L.Tuning(cell_xy=2), L.Tuning(cell_t=2), L.Tuning(cell_xy=512),
                L.Tuning(split_share=63), L.Tuning(split_share=65537), L.Tuning(split_share=-1),
                L.Tuning(kahan_mode=3), L.Tuning(kahan_mode=-1), L.Tuning(operand_form=2),
                L.Tuning(operand_form=-1)):
        with pytest.raises(L.StkdeError):
            L.Plan(d, bad)
    L.Plan(d, L.Tuning(tile_t=16, cell_xy=32, cell_t=8)).close()
    L.Plan(d, L.Tuning(split_share=64)).close()
    L.Plan(d, L.Tuning(kahan_mode=2)).close()
    L.Plan(d, L.Tuning(operand_form=1)).close()
    L.Plan(d, L.Tuning(split_share=65536)).close()


def test_workspace_bytes_monotone(L):
    p = L.Plan(L.Desc(gx=100, gy=90, gt=70, hs=5.0, ht=4.0))
    a, b = p.workspace_bytes(1000), p.workspace_bytes(100000)
    assert 0 < a < b
    with pytest.raises(L.StkdeError):
        p.workspace_bytes(0)


def test_compute_rejects_before_launch(L):
    """Every one of these fails host-side validation, so no HIP call is made
    and the test is safe without a GPU."""
    lib = L.lib()
    p = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0))
    need = p.workspace_bytes(10)
    fake = ctypes.c_void_p(0x10000)
    h = p.handle
    assert lib.stkde_compute(None, fake, 10, fake, fake, need, None, None) == -1
    assert lib.stkde_compute(h, None, 10, fake, fake, need, None, None) == -1
    assert lib.stkde_compute(h, fake, 10, None, fake, need, None, None) == -1
    assert lib.stkde_compute(h, fake, 0, fake, fake, need, None, None) == -1
    assert lib.stkde_compute(h, fake, 1 << 31, fake, fake, need, None, None) == -2
    assert lib.stkde_compute(h, fake, 10, fake, None, need, None, None) == -3
    assert lib.stkde_compute(h, fake, 10, fake, fake, need - 1, None, None) == -3
    assert lib.stkde_compute(h, fake, 10, fake, ctypes.c_void_p(0x10010), need, None, None) == -3


def test_compute_noalloc_rejects_before_launch(L):
    """The entry point without allocation validates like stkde_compute and
    refuses a computation whose workspace exceeds the static scratch, all on
    the host (no HIP call)."""
    lib = L.lib()
    p = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0))
    fake = ctypes.c_void_p(0x10000)
    h = p.handle
    assert lib.stkde_compute_noalloc(None, fake, 10, fake, None, None) == -1
    assert lib.stkde_compute_noalloc(h, None, 10, fake, None, None) == -1
    assert lib.stkde_compute_noalloc(h, fake, 10, None, None, None) == -1
    assert lib.stkde_compute_noalloc(h, fake, 0, fake, None, None) == -1
    assert lib.stkde_compute_noalloc(h, fake, 1 << 31, fake, None, None) == -2
    big = L.Plan(L.Desc(gx=1024, gy=1024, gt=256, hs=10.0, ht=7.0))
    n = 4_000_000
    assert big.workspace_bytes(n) > L.STATIC_SCRATCH_BYTES
    assert lib.stkde_compute_noalloc(big.handle, fake, n, fake, None, None) == -3
    ad = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.FLAG_ADAPTIVE))
    assert lib.stkde_compute_noalloc(ad.handle, fake, 10, fake, None, None) == -1


def test_ablation_rejects_before_launch(L):
    """The baselines validate like stkde_compute, and reject unknown methods."""
    lib = L.lib()
    p = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0))
    need = p.workspace_bytes(10)
    fake = ctypes.c_void_p(0x10000)
    h = p.handle
    for m in (0, 3, -1):
        assert lib.stkde_ablation_compute(h, m, fake, 10, fake, fake, need, None) == -1
        assert lib.stkde_ablation_accumulate(h, m, 10, fake, fake, need, None) == -1
    for m in (L.ABLATION_SCATTER, L.ABLATION_VOXEL):
        assert lib.stkde_ablation_compute(None, m, fake, 10, fake, fake, need, None) == -1
        assert lib.stkde_ablation_compute(h, m, None, 10, fake, fake, need, None) == -1
        assert lib.stkde_ablation_compute(h, m, fake, 10, None, fake, need, None) == -1
        assert lib.stkde_ablation_compute(h, m, fake, 0, fake, fake, need, None) == -1
        assert lib.stkde_ablation_compute(h, m, fake, 1 << 31, fake, fake, need, None) == -2
        assert lib.stkde_ablation_compute(h, m, fake, 10, fake, fake, need - 1, None) == -3
        assert lib.stkde_ablation_accumulate(h, m, 10, None, fake, need, None) == -1
        assert lib.stkde_ablation_accumulate(h, m, 10, fake, None, need, None) == -3
        assert lib.stkde_ablation_accumulate(h, m, 10, fake, fake, need - 1, None) == -3


def test_oracle_and_library_share_no_code():
    """The oracle and the GPU path are independent: neither source tree
    includes or imports the other."""
    for dp, _, files in os.walk(os.path.join(ROOT, "paper_1705_09366_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                s = open(os.path.join(dp, f)).read()
                assert "oracle" not in s.lower().replace("oracles", ""), os.path.join(dp, f)
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            s = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1705_09366_amd" not in s and "stkde.h" not in s, f


# ------------------------------------------------------- sets and batches (host)
def _set(L, n=100, **kw):
    base = dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0)
    base.update(kw)
    return L.BinnedSet(L.Desc(**base), n)


def _item_status(L, s, plan_kw, ox=0, oy=0, ot=0, d_set=0x10000, count=1):
    plan = L.Plan(L.Desc(**plan_kw))
    arr = (L._Item * count)()
    for k in range(count):
        arr[k] = L._Item(plan.handle.value, s.handle.value, d_set, ox, oy, ot, 0x20000, None)
    h = ctypes.c_void_p()
    st = L.lib().stkde_batch_plan(arr, count, ctypes.byref(h))
    if st == 0:
        b = ctypes.c_size_t(0)
        assert L.lib().stkde_batch_workspace_bytes(h, ctypes.byref(b)) == 0 and b.value > 0
        # nothing recorded yet: replay is refused without touching the device
        assert L.lib().stkde_batch_replay(h, None) == L.STKDE_ERR_UNSUPPORTED
        L.lib().stkde_batch_destroy(h)
    plan.close()
    return st


def test_set_plan_validation(L):
    s = _set(L)
    assert s.set_bytes > 100 * 32 and s.scratch_bytes > 100 * 16
    with pytest.raises(L.StkdeError):
        L.BinnedSet(L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0), 0)
    with pytest.raises(ValueError):
        L.BinnedSet(L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0, flags=1), 10)
    h = ctypes.c_void_p()
    d = L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0)
    assert L.lib().stkde_set_plan(ctypes.byref(d._c()), None, 2**31, ctypes.byref(h)) == L.STKDE_ERR_TOO_LARGE
    # build refuses missing or small buffers before any launch
    assert L.lib().stkde_set_build(s.handle, ctypes.c_void_p(0x1000), None, 0, None, 0, None) == \
        L.STKDE_ERR_WORKSPACE
    assert L.lib().stkde_set_build(s.handle, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x10000),
                                   s.set_bytes - 1, ctypes.c_void_p(0x100000), s.scratch_bytes,
                                   None) == L.STKDE_ERR_WORKSPACE
    s.close()


@pytest.mark.parametrize("plan_kw,off,expect", [
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0), (0, 0, 0), 0),
    (dict(gx=32, gy=16, gt=16, hs=3.0, ht=2.5, x0=10.0, y0=20.0, t0=5.0), (10, 20, 5), 0),
    (dict(gx=32, gy=16, gt=16, hs=3.0, ht=2.5, x0=10.0, y0=20.0, t0=5.0, flags=1 | 4), (10, 20, 5), 0),
    # origin does not match the window offset
    (dict(gx=32, gy=16, gt=16, hs=3.0, ht=2.5, x0=10.5), (10, 0, 0), -1),
    # window leaves the base grid
    (dict(gx=32, gy=16, gt=16, hs=3.0, ht=2.5, x0=70.0), (70, 0, 0), -1),
    (dict(gx=32, gy=16, gt=16, hs=3.0, ht=2.5, x0=-1.0), (-1, 0, 0), -1),
    # bandwidth above the set's
    (dict(gx=96, gy=80, gt=48, hs=6.5, ht=4.0), (0, 0, 0), -1),
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.5), (0, 0, 0), -1),
    # another resolution
    (dict(gx=48, gy=40, gt=48, hs=6.0, ht=4.0, sres=2.0), (0, 0, 0), -1),
    # point statistics are computed only by stkde_compute
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0, flags=8), (0, 0, 0), -5),
    # per-point bandwidths need their own binning
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0, flags=16), (0, 0, 0), -5),
    # corner sampling and kernel pairs other than the default: single grids only
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0, flags=32), (0, 0, 0), -5),
    (dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0, flags=1 << 8), (0, 0, 0), -5),
])
def test_batch_plan_validation(L, plan_kw, off, expect):
    s = _set(L)
    assert _item_status(L, s, plan_kw, *off) == expect
    s.close()


def test_batch_plan_rejects_bad_items(L):
    s = _set(L)
    kw = dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0)
    assert _item_status(L, s, kw, d_set=0x10001) == L.STKDE_ERR_INVALID_ARG  # unaligned set memory
    assert _item_status(L, s, kw, d_set=0) == L.STKDE_ERR_INVALID_ARG
    assert _item_status(L, s, kw, count=4096) == 0
    assert _item_status(L, s, kw, count=4097) == L.STKDE_ERR_TOO_LARGE
    h = ctypes.c_void_p()
    assert L.lib().stkde_batch_plan(None, 1, ctypes.byref(h)) == L.STKDE_ERR_INVALID_ARG
    s.close()


def test_batch_plan_refuses_too_many_bin_rows(L):
    # a set binned with small cells cannot serve the same bandwidth with
    # 64-row tiles: a tile would read more bin rows than the gather holds
    d = L.Desc(gx=512, gy=512, gt=256, hs=40.0, ht=40.0)
    s = L.BinnedSet(d, 1000, L.Tuning(tile_t=16, cell_xy=16, cell_t=16))
    ok = _item_status(L, s, dict(gx=512, gy=512, gt=256, hs=40.0, ht=40.0))
    plan_kw = dict(gx=512, gy=512, gt=256, hs=40.0, ht=40.0)
    plan = L.Plan(L.Desc(**plan_kw), L.Tuning(tile_t=64))
    arr = (L._Item * 1)()
    arr[0] = L._Item(plan.handle.value, s.handle.value, 0x10000, 0, 0, 0, 0x20000, None)
    h = ctypes.c_void_p()
    assert L.lib().stkde_batch_plan(arr, 1, ctypes.byref(h)) == L.STKDE_ERR_UNSUPPORTED
    assert ok in (0, L.STKDE_ERR_UNSUPPORTED)
    plan.close()
    s.close()


def _passes(L, s, plans):
    arr = (L._Item * len(plans))()
    for k, plan in enumerate(plans):
        arr[k] = L._Item(plan.handle.value, s.handle.value, 0x10000, 0, 0, 0, 0x20000 + 0x100000 * k, None)
    h = ctypes.c_void_p()
    assert L.lib().stkde_batch_plan(arr, len(plans), ctypes.byref(h)) == 0
    v = ctypes.c_int32(0)
    assert L.lib().stkde_batch_passes(h, ctypes.byref(v)) == 0
    assert L.lib().stkde_batch_passes(h, None) == L.STKDE_ERR_INVALID_ARG
    L.lib().stkde_batch_destroy(h)
    return v.value


def test_batch_passes(L):
    """Grids that are all compensated (or all plain) with 16- and 32-row
    tiles, two-term and FP32 operands, small and full-cover bandwidths share
    one pass; mixing plain and compensated grids, or 64-row tiles, does not."""
    base = dict(gx=192, gy=160, gt=96, hs=20.0, ht=6.0)
    s = L.BinnedSet(L.Desc(**base), 100, L.Tuning(tile_t=32))

    def plan(hs, tt, flags, form=0):
        return L.Plan(L.Desc(**{**base, "hs": hs, "flags": flags}), L.Tuning(tile_t=tt, operand_form=form))
    for flags in (1, 0):
        mixed = [plan(4.0, 16, flags), plan(4.0, 32, flags), plan(18.0, 16, flags), plan(18.0, 32, flags),
                 plan(6.0, 32, flags, form=1)]
        assert _passes(L, s, mixed) == 1
        assert _passes(L, s, mixed[:1]) == 1
        for p in mixed:
            p.close()
    two = [plan(4.0, 16, 1), plan(4.0, 16, 0)]
    assert _passes(L, s, two) == 2
    rows64 = [plan(4.0, 64, 0), plan(4.0, 16, 0)]
    assert _passes(L, s, rows64) == 2
    with pytest.raises(L.StkdeError):
        b = L.Batch.__new__(L.Batch)
        b._h = ctypes.c_void_p()
        b.passes()
    for p in two + rows64:
        p.close()
    s.close()


def test_profile_api_host_checks(L):
    plan = L.Plan(L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0))
    assert L.lib().stkde_plan_profile(plan.handle, -1) == L.STKDE_ERR_INVALID_ARG
    assert L.lib().stkde_plan_profile(plan.handle, 0) == 0
    cnt = ctypes.c_int32(7)
    assert L.lib().stkde_plan_profile_read(plan.handle, None, 0, ctypes.byref(cnt)) == 0
    assert cnt.value == 0
    plan.close()


def test_adaptive_entry_points_host_checks(L):
    """Adaptive plans take the adaptive entry points only, and vice versa;
    their workspace holds the per-point terms."""
    lib = L.lib()
    fixed = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0))
    ad = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.FLAG_ADAPTIVE))
    n = 1000
    assert ad.workspace_bytes(n) >= fixed.workspace_bytes(n) + 16 * n
    need = ad.workspace_bytes(n)
    fake = ctypes.c_void_p(0x10000)
    h, hf = ad.handle, fixed.handle
    assert lib.stkde_compute(h, fake, n, fake, fake, need, None, None) == -1
    assert lib.stkde_bin(h, fake, n, fake, need, None) == -1
    assert lib.stkde_compute_adaptive(hf, fake, fake, n, fake, fake, need, None, None) == -1
    assert lib.stkde_bin_adaptive(hf, fake, fake, n, fake, need, None) == -1
    assert lib.stkde_compute_adaptive(h, fake, None, n, fake, fake, need, None, None) == -1
    assert lib.stkde_compute_adaptive(h, None, fake, n, fake, fake, need, None, None) == -1
    assert lib.stkde_compute_adaptive(h, fake, fake, n, None, fake, need, None, None) == -1
    assert lib.stkde_compute_adaptive(h, fake, fake, 0, fake, fake, need, None, None) == -1
    assert lib.stkde_compute_adaptive(h, fake, fake, 1 << 31, fake, fake, need, None, None) == -2
    assert lib.stkde_compute_adaptive(h, fake, fake, n, fake, fake, need - 1, None, None) == -3
    assert lib.stkde_bin_adaptive(h, fake, None, n, fake, need, None) == -1
    assert lib.stkde_bin_adaptive(h, fake, fake, n, fake, need - 1, None) == -3
    assert lib.stkde_ablation_compute(h, L.ABLATION_VOXEL, fake, n, fake, fake, need, None) == -5
    assert lib.stkde_ablation_accumulate(h, L.ABLATION_SCATTER, n, fake, fake, need, None) == -5
    # a set's base carries no flags
    hs = ctypes.c_void_p()
    d = L.Desc(gx=16, gy=16, gt=16, hs=2.0, ht=2.0, flags=L.FLAG_ADAPTIVE)
    assert lib.stkde_set_plan(ctypes.byref(d._c()), None, 10, ctypes.byref(hs)) == -1
    fixed.close()
    ad.close()


def test_kernel_pair_and_corner_host_checks(L):
    lib = L.lib()
    for k in range(4):
        p = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.kernel_flag(k) | L.FLAG_CORNER))
        p.close()
    for k in (4, 9, 15):
        with pytest.raises(L.StkdeError) as e:
            L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.kernel_flag(k)))
        assert e.value.status == L.STKDE_ERR_INVALID_ARG
    with pytest.raises(L.StkdeError) as e:
        L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.kernel_flag(L.KERNEL_QUARTIC) | L.FLAG_ADAPTIVE))
    assert e.value.status == L.STKDE_ERR_UNSUPPORTED
    # corner sampling with per-point bandwidths is fine
    L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.FLAG_CORNER | L.FLAG_ADAPTIVE)).close()
    p = L.Plan(L.Desc(gx=32, gy=32, gt=32, hs=3.0, ht=3.0, flags=L.kernel_flag(L.KERNEL_GAUSSIAN)))
    need = p.workspace_bytes(10)
    fake = ctypes.c_void_p(0x10000)
    assert lib.stkde_ablation_compute(p.handle, L.ABLATION_SCATTER, fake, 10, fake, fake, need, None) == -5
    p.close()
