"""Host-side checks of the C ABI (no device work): the library loads and exports
every symbol declared in include/sharp.h, argument validation, the tile ->
frame incidence lists and the workspace size."""
import ctypes
import os
import re

import numpy as np
import pytest

from sharp_data import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sharp.h")


@pytest.fixture(scope="module")
def L():
    from paper_1602_01448_amd._lib import load
    return load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sharp_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    from paper_1602_01448_amd._lib import SIGNATURES
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert sorted(n for n, _, _ in SIGNATURES) == names


def _create(L, n, m, pos, **kw):
    from paper_1602_01448_amd._lib import SharpOptions
    h = ctypes.c_void_p()
    pos = np.ascontiguousarray(pos, dtype=np.int32)
    opts = SharpOptions(kw.get("periodic", 0), kw.get("probe_every", 0), kw.get("probe_start", 1),
                        kw.get("eps_D", 0.0), kw.get("tile", 0), kw.get("merge_split", 0), kw.get("grad_groups", 0),
                        kw.get("frame_launch", 0), kw.get("fft_block", 0), kw.get("strip_rows", 0),
                        kw.get("probe_center", 0))
    if "reserved" in kw:
        opts.reserved[0] = kw["reserved"]
    st = L.sharp_plan_create(ctypes.byref(h), n, n, m, len(pos), pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             ctypes.byref(opts))
    return st, h


def test_read_reference_rejects_bad_arguments(L):
    # every case returns before any device work
    vp = ctypes.c_void_p
    assert L.sharp_read_reference(None, 16, vp(256), None) == -1
    assert L.sharp_read_reference(vp(256), 16, None, None) == -1
    assert L.sharp_read_reference(vp(256), 0, vp(256), None) == -1
    assert L.sharp_read_reference(vp(256), 24, vp(256), None) == -1
    assert L.sharp_read_reference(vp(264), 32, vp(256), None) == -1


def test_status_strings(L):
    for s in range(-9, 1):
        assert len(L.sharp_status_string(s)) > 0 and L.sharp_status_string(s) != b"unknown status"
    assert L.sharp_status_string(-99) == b"unknown status"
    assert L.sharp_status_string(-10) == b"unknown status"


@pytest.mark.parametrize("m,expect", [(16, 0), (32, 0), (64, 0), (128, 0), (256, 0), (48, -2), (8, -2), (512, -2)])
def test_supported_sizes(L, m, expect):
    n = max(m, 16) + 8
    st, h = _create(L, n, m, [(0, 0)])
    assert st == expect
    L.sharp_plan_destroy(h)


def test_validation(L):
    assert _create(L, 64, 32, [(0, 0), (33, 0)])[0] == -3      # leaves the object
    assert _create(L, 64, 32, [(0, -1)])[0] == -3
    assert _create(L, 64, 32, [(32, 32)])[0] == 0               # last valid corner
    assert _create(L, 64, 32, [(63, 63)], periodic=1)[0] == 0   # wraps
    assert _create(L, 64, 32, [(64, 0)], periodic=1)[0] == -3
    assert _create(L, 16, 32, [(0, 0)])[0] == -2                # m > n
    assert _create(L, 64, 32, [(0, 0)], tile=24)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], reserved=1)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], eps_D=-1.0)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], frame_launch=3)[0] == 0     # taken as the small-frame form
    assert _create(L, 64, 32, [(0, 0)], fft_block=64)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], strip_rows=3)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], probe_center=2)[0] == -1
    assert _create(L, 64, 32, [(0, 0)], frame_launch=4)[0] == -1
    assert _create(L, 300, 256, [(0, 0)], fft_block=512)[0] == 0
    h = ctypes.c_void_p()
    assert L.sharp_plan_create(ctypes.byref(h), 64, 64, 32, 0, None, None) == -1
    assert L.sharp_plan_create(None, 64, 64, 32, 1, None, None) == -1


@pytest.mark.parametrize("n,kw,form,rows", [(300, {}, 2, 1), (300, {"strip_rows": 2}, 2, 2),
                                           (5000, {"strip_rows": 2}, 2, 1), (9000, {}, 1, 0),
                                           (300, {"frame_launch": 1}, 1, 0), (300, {"frame_launch": 3}, 3, 1),
                                           (300, {"frame_launch": 3, "strip_rows": 2}, 3, 2),
                                           (9000, {"frame_launch": 3}, 1, 0), (-300, {}, 3, 1),
                                           (-300, {"frame_launch": 2}, 2, 1), (-9000, {}, 1, 0)])
def test_large_frame_form_selection(L, n, kw, form, rows):
    """m = 256: Fourier-carry form with 1-row strips by default, 2-row strips
    on request while a 2-row strip fits in LDS, frame-space form beyond 8192;
    the form whose column pass forms its own row transform on request, and
    by default from 400 frames on (n < 0: 800 frames)."""
    from paper_1602_01448_amd._lib import SharpPlanInfo
    K = 800 if n < 0 else 2
    n = abs(n)
    pos = [(0, 0)] * (K - 1) + [(n - 256, n - 256)]
    st, h = _create(L, n, 256, pos, **kw)
    assert st == 0
    info = SharpPlanInfo()
    assert L.sharp_get_plan_info(h, ctypes.byref(info)) == 0
    assert (info.frame_launch, info.strip_rows) == (form, rows)
    L.sharp_plan_destroy(h)


@pytest.mark.parametrize("m,kw,form", [(128, {}, 2), (128, {"frame_launch": 1}, 1), (64, {}, 1),
                                       (64, {"frame_launch": 2}, 1), (32, {}, 1), (128, {"frame_launch": 3}, 2),
                                       (64, {"frame_launch": 3}, 1)])
def test_small_frame_form_selection(L, m, kw, form):
    """m = 128 keeps the carry in the Fourier domain by default; smaller
    frames always keep it in frame space."""
    from paper_1602_01448_amd._lib import SharpPlanInfo
    st, h = _create(L, 300, m, [(0, 0), (300 - m, 300 - m)], **kw)
    assert st == 0
    info = SharpPlanInfo()
    assert L.sharp_get_plan_info(h, ctypes.byref(info)) == 0
    assert (info.frame_launch, info.strip_rows) == (form, 0)
    L.sharp_plan_destroy(h)


@pytest.mark.parametrize("n,tile", [(300, 16), (512, 16), (992, 16), (993, 32), (2048, 32)])
def test_default_merge_tile(L, n, tile):
    """Merge tiles of 32 while that still gives >= 1024 tiles, else 16."""
    from paper_1602_01448_amd._lib import SharpPlanInfo
    st, h = _create(L, n, 64, [(0, 0), (n - 64, n - 64)])
    assert st == 0
    info = SharpPlanInfo()
    assert L.sharp_get_plan_info(h, ctypes.byref(info)) == 0
    assert info.tile == tile
    assert info.tiles_x == -(-n // tile)
    L.sharp_plan_destroy(h)


@pytest.mark.parametrize("m,K,stream", [(128, 2048, 0), (128, 2049, 1), (256, 512, 0), (256, 513, 1), (64, 5000, 0)])
def test_streaming_threshold(L, m, K, stream):
    """Frame arrays of K m^2 complex values above 256 MiB (the last-level
    cache) are moved with streaming accesses; at or below it, cached ones."""
    from paper_1602_01448_amd._lib import SharpPlanInfo
    n = m + 64
    pos = [(i % 65, (i // 65) % 65) for i in range(K)]
    st, h = _create(L, n, m, pos)
    assert st == 0
    info = SharpPlanInfo()
    assert L.sharp_get_plan_info(h, ctypes.byref(info)) == 0
    assert info.streaming == stream
    assert info.csr_nnz > 0 and info.strip_rows == (1 if m == 256 else 0)   # fields after it read correctly
    L.sharp_plan_destroy(h)


def test_calls_before_workspace_are_not_ready(L):
    st, h = _create(L, 64, 32, [(0, 0), (8, 8)])
    assert st == 0
    assert L.sharp_set_data(h, ctypes.c_void_p(16)) == -4
    assert L.sharp_set_probe_constraint(h, 1, ctypes.c_void_p(16)) == -4
    assert L.sharp_set_probe_constraint(h, 3, ctypes.c_void_p(16)) == -1
    assert L.sharp_set_probe_constraint(h, 2, None) == -1
    assert L.sharp_raar_iterate(h, 1, ctypes.c_float(1.5)) == -1          # beta outside (0, 1]
    assert L.sharp_raar_iterate(h, 1, ctypes.c_float(0.0)) == -1
    assert L.sharp_raar_iterate(h, 1, ctypes.c_float(0.75)) == -4
    assert L.sharp_set_workspace(h, ctypes.c_void_p(256), 16) == -5       # too small (checked first)
    assert L.sharp_set_workspace(h, ctypes.c_void_p(3), 1 << 40) == -1    # misaligned
    L.sharp_plan_destroy(h)


def _brute_csr(n, m, T, pos, periodic):
    tiles = (n + T - 1) // T
    lists = [[] for _ in range(tiles * tiles)]
    for i, (py, px) in enumerate(pos):
        hit = set()
        for ry in range(m):
            for rx in range(m):
                y, x = py + ry, px + rx
                if periodic:
                    y, x = y % n, x % n
                hit.add((y // T) * tiles + x // T)
        for t in sorted(hit):
            lists[t].append(i)
    ptr = np.zeros(len(lists) + 1, np.int32)
    ptr[1:] = np.cumsum([len(l) for l in lists])
    return ptr, np.array([f for l in lists for f in l], np.int32)


@pytest.mark.parametrize("n,m,T,periodic,jit", [(128, 32, 16, 0, 0), (100, 32, 32, 0, 2), (96, 16, 16, 1, 3),
                                                (200, 64, 64, 1, 5)])
def test_csr_matches_brute_force(L, n, m, T, periodic, jit):
    rng = np.random.default_rng(n + m)
    if periodic:
        pos = rng.integers(0, n, size=(40, 2)).astype(np.int32)
    else:
        pos = gen.raster_positions(5, (n - m) / 4, n, m, jitter=jit, rng=rng)
    st, h = _create(L, n, m, pos, periodic=periodic, tile=T)
    assert st == 0
    from paper_1602_01448_amd._lib import SharpPlanInfo
    info = SharpPlanInfo()
    assert L.sharp_get_plan_info(h, ctypes.byref(info)) == 0
    ptr = np.zeros(info.tiles_x * info.tiles_y + 1, np.int32)
    fr = np.zeros(info.csr_nnz, np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    assert L.sharp_get_plan_csr(h, ptr.ctypes.data_as(P), fr.ctypes.data_as(P)) == 0
    bptr, bfr = _brute_csr(n, m, T, pos, periodic)
    assert np.array_equal(ptr, bptr) and np.array_equal(fr, bfr)
    L.sharp_plan_destroy(h)


def test_workspace_grows_with_frames(L):
    sizes = []
    for K in (10, 20, 40):
        pos = np.zeros((K, 2), np.int32)
        st, h = _create(L, 256, 64, pos)
        sizes.append(L.sharp_workspace_bytes(h))
        # frame stacks a (4 B), u (8 B), v (8 B) per pixel at least
        assert sizes[-1] >= K * 64 * 64 * 20
        assert sizes[-1] % 256 == 0
        L.sharp_plan_destroy(h)
    assert sizes[0] < sizes[1] < sizes[2]


def test_noalloc_scratch_limit_checked_before_device_work(L):
    """sharp_apply_noalloc refuses an operator whose scratch exceeds its fixed
    array (64 MiB): 200 frames of 256^2 need a 100 MiB stage buffer for F.
    The check comes before any device call (no workspace is set here); an
    operator that fits gets the plan's usual NOT_READY instead."""
    pos = [(0, 0)] * 200
    st, h = _create(L, 256, 256, pos)
    assert st == 0
    dummy = ctypes.c_void_p(256)
    assert L.sharp_apply_noalloc(h, 0, dummy, ctypes.c_void_p(512)) == -9    # F: stage 200 x 512 KiB
    assert L.sharp_apply_noalloc(h, 4, dummy, ctypes.c_void_p(512)) == -9    # P_a likewise
    assert L.sharp_apply_noalloc(h, 7, dummy, ctypes.c_void_p(512)) == -1    # no such operator
    assert L.sharp_apply_noalloc(None, 0, dummy, ctypes.c_void_p(512)) == -1
    L.sharp_plan_destroy(h)
    st, h = _create(L, 64, 32, [(0, 0), (8, 8)])
    assert L.sharp_apply_noalloc(h, 5, dummy, ctypes.c_void_p(512)) == -4    # fits; no workspace yet
    L.sharp_plan_destroy(h)
