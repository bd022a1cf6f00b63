"""mpv_pyramid_noalloc (the allocation-free variant of mpv_pyramid) through the C ABI: two
calls in a row on the library's own device array, the second with a smaller input, each
bit-identical to mpv_pyramid with a caller workspace; sizes beyond the array are rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run_both(L, torch, left, right, num_disp, levels):
    from paper_2001_09678_amd import mpv
    lib = L.lib()
    h, w = left.shape
    params = mpv.MPVParams(num_disp=num_disp, num_paths=8)
    pp = mpv.pyramid_params(params, levels, 4)
    li = L.Image(left.data_ptr(), w, h, left.stride(0))
    ri = L.Image(right.data_ptr(), w, h, right.stride(0))
    outs = []
    for variant in ("noalloc", "workspace"):
        disp = torch.full((h, w), -7, dtype=torch.int16, device="cuda")
        raw = torch.full((h, w), -7, dtype=torch.int16, device="cuda")
        rgt = torch.full((h, w), -7, dtype=torch.int16, device="cuda")
        out = L.PyramidOut(disp.data_ptr(), raw.data_ptr(), rgt.data_ptr(), (C.c_void_p * L.MPV_MAX_LEVELS)())
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if variant == "noalloc":
            rc = lib.mpv_pyramid_noalloc(C.byref(pp), C.byref(li), C.byref(ri), C.byref(out), st)
        else:
            nbytes = lib.mpv_pyramid_workspace_bytes(C.byref(pp), w, h)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            rc = lib.mpv_pyramid(C.byref(pp), C.byref(li), C.byref(ri), C.byref(out), ws.data_ptr(),
                                 nbytes, st)
        assert rc == L.MPV_OK, (variant, L.lib().mpv_status_string(rc))
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (disp, raw, rgt)])
    return outs


def test_noalloc_equals_workspace_twice():
    import torch
    from paper_2001_09678_amd import _lib as L
    from paper_2001_09678_amd.scene import config_scene, make_scene
    assert torch.cuda.is_available()
    L.lib()
    sc, _ = config_scene("c2")
    small = make_scene(77, 333, 191, 63, 8, ground=True)
    for name, s, D, levels in (("1280x720 D=128", sc, 128, 3), ("333x191 D=64", small, 64, 3)):
        print("noalloc vs workspace:", name, flush=True)
        left = torch.from_numpy(s.left).cuda()
        right = torch.from_numpy(s.right).cuda()
        (a, b) = _run_both(L, torch, left, right, D, levels)
        for x, y, what in zip(a, b, ("disp", "raw", "right")):
            np.testing.assert_array_equal(x, y, err_msg=f"{name} {what}")
        assert (a[0] >= 0).mean() > 0.5


def test_noalloc_rejects_oversize():
    import torch
    from paper_2001_09678_amd import _lib as L, mpv
    lib = L.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: the size check comes first
    pp = mpv.pyramid_params(mpv.MPVParams(num_disp=256, num_paths=8), 3, 4)
    img = L.Image(fake, 1920, 1080, 1920)
    out = L.PyramidOut(fake, None, None, (C.c_void_p * L.MPV_MAX_LEVELS)())
    assert lib.mpv_pyramid_workspace_bytes(C.byref(pp), 1920, 1080) > L.MPV_PYRAMID_NOALLOC_MAX_BYTES
    assert lib.mpv_pyramid_noalloc(C.byref(pp), C.byref(img), C.byref(img), C.byref(out), None) == \
        L.MPV_ERR_WORKSPACE
