"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
entry point include/mpv.h declares, and rejects bad arguments before enqueueing work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2001_09678_amd import build, _lib
    build.build(force=False)
    return _lib


def header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mpv_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert "mpv_pyramid" in names and "mpv_cost" in names and "mpv_aggregate" in names
    assert "mpv_disparity" in names and "mpv_lb_conv" in names and "mpv_batch_run_graph" in names
    raw = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_status_strings(L):
    lib = L.lib()
    for s, name in enumerate(["MPV_OK", "MPV_ERR_INVALID_ARG", "MPV_ERR_UNSUPPORTED",
                              "MPV_ERR_WORKSPACE", "MPV_ERR_OVERFLOW", "MPV_ERR_DEVICE"]):
        assert lib.mpv_status_string(s).decode() == name
    assert lib.mpv_status_string(99).decode() == "MPV_ERR_UNKNOWN"


def _params(L, **kw):
    d = dict(num_disp=64, census_radius=2, num_paths=4, lambda_=8, tau=4, lr_max_diff=1, agg_type=0)
    d.update(kw)
    return L.Params(**d)


def test_validation_before_enqueue(L):
    lib = L.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    img = L.Image(fake, 32, 16, 32)
    bad_img = L.Image(fake, 32, 16, 8)  # pitch < width
    assert lib.mpv_census(None, fake, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_census(C.byref(bad_img), fake, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_cost(None, C.byref(img), C.byref(img), None, fake, None) == L.MPV_ERR_INVALID_ARG
    for kw, st in [(dict(num_disp=0), L.MPV_ERR_INVALID_ARG), (dict(num_disp=257), L.MPV_ERR_INVALID_ARG),
                   (dict(num_paths=3), L.MPV_ERR_INVALID_ARG), (dict(census_radius=3), L.MPV_ERR_UNSUPPORTED),
                   (dict(tau=0), L.MPV_ERR_INVALID_ARG), (dict(lambda_=-1), L.MPV_ERR_INVALID_ARG),
                   (dict(agg_type=7), L.MPV_ERR_INVALID_ARG)]:
        p = _params(L, **kw)
        assert lib.mpv_cost(C.byref(p), C.byref(img), C.byref(img), None, fake, None) == st, kw
    # mismatched pair shapes
    other = L.Image(fake, 31, 16, 32)
    p = _params(L)
    assert lib.mpv_cost(C.byref(p), C.byref(img), C.byref(other), None, fake, None) == L.MPV_ERR_INVALID_ARG
    # a band wider than the range
    band = L.Band(fake, None, 65)
    assert lib.mpv_cost(C.byref(p), C.byref(img), C.byref(img), C.byref(band), fake, None) == L.MPV_ERR_INVALID_ARG


def test_overflow_detected(L):
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    # 8 paths * 24 * 1280 > 65535: uint16 sums cannot hold 1280-wide lines
    p = _params(L, num_disp=128, num_paths=8, agg_type=L.MPV_AGG_U16)
    assert lib.mpv_aggregate(C.byref(p), fake, 1280, 720, None, 0, fake, None) == L.MPV_ERR_OVERFLOW
    # the 320x240, 4-path workload fits uint16
    p = _params(L, num_disp=64, num_paths=4, agg_type=L.MPV_AGG_U16)
    assert lib.mpv_aggregate(C.byref(p), None, 320, 240, None, 0, fake, None) == L.MPV_ERR_INVALID_ARG


def test_fused_limits(L):
    lib = L.lib()
    # 24 + lambda*min(tau, D-1) must fit the uint8 partial energies of the fused path
    ok = L.PyramidParams(_params(L, num_disp=128, num_paths=8), 3, 4)
    big = L.PyramidParams(_params(L, num_disp=128, num_paths=8, lambda_=60, tau=4), 3, 4)
    assert lib.mpv_pyramid_workspace_bytes(C.byref(ok), 1280, 720) > 0
    assert lib.mpv_pyramid_workspace_bytes(C.byref(big), 1280, 720) == 0
    # too many levels for the image
    deep = L.PyramidParams(_params(L, num_disp=128, num_paths=8), 4, 4)
    assert lib.mpv_pyramid_workspace_bytes(C.byref(deep), 6, 6) == 0
    # height limit (unnormalised 32-bit line energies) and the 2^31-byte partial volume
    one = L.PyramidParams(_params(L, num_disp=64, num_paths=8), 1, 4)
    assert lib.mpv_pyramid_workspace_bytes(C.byref(one), 16, 65536) > 0
    assert lib.mpv_pyramid_workspace_bytes(C.byref(one), 16, 65537) == 0
    p256 = _params(L, num_disp=256, num_paths=8)
    assert lib.mpv_match_workspace_bytes(C.byref(p256), 4096, 2047, None) > 0
    assert lib.mpv_match_workspace_bytes(C.byref(p256), 4096, 2049, None) == 0
    # workspace too small is reported before any launch
    fake = C.c_void_p(0x1000)
    img = L.Image(fake, 1280, 720, 1280)
    out = L.PyramidOut(fake, None, None)
    assert lib.mpv_pyramid(C.byref(ok), C.byref(img), C.byref(img), C.byref(out), fake, 16, None) == L.MPV_ERR_WORKSPACE


def test_workspace_model(L):
    """Workspace = images of the coarse levels + per-level raw maps + band map + census of both
    views + one uint8 energy volume per path (the largest level)."""
    lib = L.lib()
    pp = L.PyramidParams(_params(L, num_disp=128, num_paths=8), 1, 4)
    ws = lib.mpv_pyramid_workspace_bytes(C.byref(pp), 1280, 720)
    assert ws >= 8 * 1280 * 720 * 128
    assert ws < 8 * 1280 * 720 * 128 + 32 * 2**20


def test_layered_merge_limits(L):
    """The layered merge (Section 3.2, Table alg) needs pairs of directions and merged
    energies that fit a byte: 24 + (layers) * lambda * min(tau, D-1) <= 255; only the fused
    entry points run it."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    lay = L.MPV_MERGE_LAYERED
    ok = _params(L, num_disp=128, num_paths=8, merge=lay)  # 24 + 4 * 32 = 152
    assert lib.mpv_match_workspace_bytes(C.byref(ok), 320, 240, None) > 0
    pp = L.PyramidParams(ok, 3, 4)
    assert lib.mpv_pyramid_workspace_bytes(C.byref(pp), 1280, 720) > 0
    # one path is no pair; an unknown merge is an argument error
    for kw in (dict(num_paths=1, merge=lay), dict(merge=3), dict(merge=-1)):
        p = _params(L, **kw)
        assert lib.mpv_match_workspace_bytes(C.byref(p), 320, 240, None) == 0, kw
        assert lib.mpv_cost(C.byref(p), None, None, None, fake, None) == L.MPV_ERR_INVALID_ARG, kw
    # 24 + 4 * 8 * 8 = 280 > 255 with four layers, but 24 + 2 * 64 = 152 fits two
    big = _params(L, num_disp=128, num_paths=8, tau=8, merge=lay)
    assert lib.mpv_match_workspace_bytes(C.byref(big), 320, 240, None) == 0
    two = _params(L, num_disp=128, num_paths=4, tau=8, merge=lay)
    assert lib.mpv_match_workspace_bytes(C.byref(two), 320, 240, None) > 0
    img = L.Image(fake, 320, 240, 320)
    assert lib.mpv_match(C.byref(big), C.byref(img), C.byref(img), None, fake, None, None, fake,
                         1 << 40, None) == L.MPV_ERR_UNSUPPORTED
    # the unfused export and the learned coarse level sum the paths
    assert lib.mpv_aggregate(C.byref(ok), fake, 320, 240, None, 0, fake, None) == L.MPV_ERR_UNSUPPORTED
    assert lib.mpv_lb_coarse_workspace_bytes(C.byref(ok), 320, 180) == 0
    # batches plan the layers (host only: no launch before bind)
    item = L.BatchItem(img, img, 128, fake, None, None)
    handle = C.c_void_p()
    assert lib.mpv_batch_create(C.byref(pp), C.byref(item), 1, C.byref(handle)) == L.MPV_OK
    assert lib.mpv_batch_workspace_bytes(handle) > 0
    lib.mpv_batch_destroy(handle)
    bad = L.PyramidParams(big, 3, 4)
    assert lib.mpv_batch_create(C.byref(bad), C.byref(item), 1, C.byref(handle)) != L.MPV_OK


def test_layered_occlusion_limit(L):
    """With the occlusion strategy the left-to-right pass stores energies up to
    24 + 2 * lambda * tau even when there is one layer."""
    lib = L.lib()
    one = _params(L, num_disp=128, num_paths=2, tau=16, merge=L.MPV_MERGE_LAYERED)       # 24 + 128
    occ = _params(L, num_disp=128, num_paths=2, tau=16, merge=L.MPV_MERGE_LAYERED_OCC)   # 24 + 256
    assert lib.mpv_match_workspace_bytes(C.byref(one), 320, 240, None) > 0
    assert lib.mpv_match_workspace_bytes(C.byref(occ), 320, 240, None) == 0
    occ8 = _params(L, num_disp=128, num_paths=8, merge=L.MPV_MERGE_LAYERED_OCC)
    assert lib.mpv_match_workspace_bytes(C.byref(occ8), 320, 240, None) > 0


def test_gradient_weight_limits(L):
    """grad_sigma is 0 (constant lambda) or 1..255; the entry points that see the left
    images (mpv_match, mpv_pyramid, batches) take gradient weights."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    ok = _params(L, num_disp=128, num_paths=8, grad_sigma=16)
    assert lib.mpv_match_workspace_bytes(C.byref(ok), 320, 240, None) > 0
    pp = L.PyramidParams(ok, 3, 4)
    plain = L.PyramidParams(_params(L, num_disp=128, num_paths=8), 3, 4)
    # the pyramid keeps the coarse levels' left images for the weights
    assert lib.mpv_pyramid_workspace_bytes(C.byref(pp), 1280, 720) >= \
        lib.mpv_pyramid_workspace_bytes(C.byref(plain), 1280, 720) + 640 * 360 + 320 * 180
    for sigma in (-1, 256):
        p = _params(L, grad_sigma=sigma)
        assert lib.mpv_match_workspace_bytes(C.byref(p), 320, 240, None) == 0
        assert lib.mpv_cost(C.byref(p), None, None, None, fake, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_aggregate(C.byref(ok), fake, 320, 240, None, 0, fake, None) == L.MPV_ERR_UNSUPPORTED
    img = L.Image(fake, 320, 240, 320)
    item = L.BatchItem(img, img, 128, fake, None, None)
    handle = C.c_void_p()
    assert lib.mpv_batch_create(C.byref(pp), C.byref(item), 1, C.byref(handle)) == L.MPV_OK
    lib.mpv_batch_destroy(handle)
    assert lib.mpv_lb_coarse_workspace_bytes(C.byref(ok), 320, 180) == 0


def test_road_limits(L):
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    assert lib.mpv_road_workspace_bytes(128, 720) >= 128 * 720
    for D, H in [(0, 720), (257, 720), (128, 0), (128, L.MPV_ROAD_MAX_HEIGHT + 1)]:
        assert lib.mpv_road_workspace_bytes(D, H) == 0
        assert lib.mpv_road(fake, D, H, 8, fake, fake, fake, 1 << 30, None) == L.MPV_ERR_INVALID_ARG
    for eta in (1, 0, 257):
        assert lib.mpv_road(fake, 128, 720, eta, fake, fake, fake, 1 << 30, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_road(fake, 128, 720, 8, fake, fake, fake, 16, None) == L.MPV_ERR_WORKSPACE
    assert lib.mpv_vdisparity(fake, 32, 16, 31, 64, fake, None) == L.MPV_ERR_INVALID_ARG  # pitch < width
    assert lib.mpv_vdisparity(fake, 32, 16, 32, 257, fake, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_udisparity(fake, 32, 16, 31, 64, fake, None) == L.MPV_ERR_INVALID_ARG  # pitch < width
    assert lib.mpv_udisparity(fake, 32, 16, 32, 257, fake, None) == L.MPV_ERR_INVALID_ARG
    assert lib.mpv_udisparity(fake, 0, 16, 32, 64, fake, None) == L.MPV_ERR_INVALID_ARG


def test_noalloc_limits_before_any_device_call(L):
    """mpv_pyramid_noalloc checks its arguments and the size of its fixed array before it
    touches a device: oversize shapes and bad parameters are rejected here, without a GPU."""
    from paper_2001_09678_amd import mpv
    lib = L.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced
    out = L.PyramidOut(fake, None, None, (C.c_void_p * L.MPV_MAX_LEVELS)())
    big = mpv.pyramid_params(mpv.MPVParams(num_disp=256, num_paths=8), 3, 4)
    img = L.Image(fake, 1920, 1080, 1920)
    need = lib.mpv_pyramid_workspace_bytes(C.byref(big), 1920, 1080)
    assert need > L.MPV_PYRAMID_NOALLOC_MAX_BYTES
    assert lib.mpv_pyramid_noalloc(C.byref(big), C.byref(img), C.byref(img), C.byref(out), None) == \
        L.MPV_ERR_WORKSPACE
    # the measured 1280x720, D=128, 3-level frame fits the array
    fits = mpv.pyramid_params(mpv.MPVParams(num_disp=128, num_paths=8), 3, 4)
    assert 0 < lib.mpv_pyramid_workspace_bytes(C.byref(fits), 1280, 720) <= L.MPV_PYRAMID_NOALLOC_MAX_BYTES
    bad = mpv.pyramid_params(mpv.MPVParams(num_disp=300, num_paths=8), 3, 4)
    small = L.Image(fake, 64, 48, 64)
    assert lib.mpv_pyramid_noalloc(C.byref(bad), C.byref(small), C.byref(small), C.byref(out), None) == \
        L.MPV_ERR_INVALID_ARG
    assert lib.mpv_pyramid_noalloc(None, C.byref(small), C.byref(small), C.byref(out), None) == \
        L.MPV_ERR_INVALID_ARG


def test_propagation_arguments_checked(L):
    lib = L.lib()
    for prop, block, ok in [(0, 0, True), (1, 0, True), (1, 8, True), (1, 32, True), (2, 0, False),
                            (1, 7, False), (1, 34, False), (1, -2, False)]:
        pp = L.PyramidParams(_params(L, num_disp=128, num_paths=8), 3, 4)
        pp.propagation, pp.block = prop, block
        n = lib.mpv_pyramid_workspace_bytes(C.byref(pp), 640, 480)
        assert (n > 0) == ok, (prop, block)


def test_ssim_combinations_checked(L):
    """The SSIM data term runs with the sum of the paths and constant weights on the fused
    path; other combinations, batches and unknown data terms are rejected up front."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    for kw, ok in [(dict(data_term=1), True), (dict(data_term=1, merge=1), False),
                   (dict(data_term=1, grad_sigma=16), False), (dict(data_term=2), False)]:
        pp = L.PyramidParams(_params(L, num_disp=64, num_paths=8, **kw), 3, 4)
        assert (lib.mpv_pyramid_workspace_bytes(C.byref(pp), 320, 240) > 0) == ok, kw
    pp = L.PyramidParams(_params(L, num_disp=64, num_paths=8, data_term=1), 3, 4)
    item = (L.BatchItem * 1)()
    item[0] = L.BatchItem(L.Image(fake, 64, 48, 64), L.Image(fake, 64, 48, 64), 32, fake, None, None)
    h = C.c_void_p()
    assert lib.mpv_batch_create(C.byref(pp), item, 1, C.byref(h)) == L.MPV_ERR_UNSUPPORTED
