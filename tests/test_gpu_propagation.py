"""The paper's propagation (Section 3.4: block modes at intermediate levels, linear
interpolation at the last level) on the GPU through mpv_pyramid, against the oracle bit for
bit: every level's raw winners, the finest right disparity and LR-checked map. Shapes with
ragged blocks and odd sizes (coarse images one pixel short of the finer ones), every block
size, 2 to 4 levels, the +/-4 band and the paper's d/4 scope, the layered merge, and the
1280x720, D=128 workload at full size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_09678_amd import mpv as m, _lib
    _lib.lib()
    return m


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _log(*a):
    print(*a, flush=True)


def _check(mpv, orc, L, R, D, levels, radius, P, block, **kw):
    p = mpv.MPVParams(num_disp=D, num_paths=P, **{k: v for k, v in kw.items() if k in ("merge", "grad_sigma")})
    pyr = mpv.pyramid(_cuda(L), _cuda(R), p, levels=levels, radius=radius, keep_levels=True,
                      propagation="paper", block=block)
    okw = {}
    if kw.get("merge", "sum") != "sum":
        okw = dict(merge="layered", occ=kw["merge"] == "layered_occ")
    ref = orc.pyramid(L, R, D, levels=levels, radius=radius, num_paths=P, propagation="paper",
                      block=block or 8, grad_sigma=kw.get("grad_sigma", 0), **okw)
    for l in range(levels):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.raw), ref[-1].dl)
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)
    return ref


@pytest.mark.parametrize("w,h,D,levels,R,P,block", [
    (160, 96, 64, 3, 4, 8, 8), (163, 99, 64, 3, 4, 8, 8), (97, 61, 48, 3, 6, 4, 4),
    (130, 70, 128, 3, 16, 8, 0), (200, 120, 128, 4, 4, 8, 16), (201, 123, 64, 4, 8, 4, 32),
    (90, 50, 32, 2, 4, 8, 8), (33, 17, 16, 3, 2, 2, 2), (8, 8, 8, 3, 1, 1, 2),
])
def test_paper_propagation_small(mpv, orc, w, h, D, levels, R, P, block):
    from paper_2001_09678_amd.scene import make_scene
    _log("paper propagation", w, h, D, levels, R, P, block)
    sc = make_scene(w * 3 + h + D, w, h, D - 1, 6, ground=True)
    _check(mpv, orc, sc.left, sc.right, D, levels, R, P, block)


def test_paper_propagation_layered_merge(mpv, orc):
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(4242, 150, 90, 63, 6, ground=True)
    _check(mpv, orc, sc.left, sc.right, 64, 3, 8, 8, 8, merge="layered_occ", grad_sigma=16)


@pytest.mark.parametrize("radius", [4, 16])
def test_paper_propagation_full_size(mpv, orc, radius):
    """1280x720, D=128, 3 levels, 8 paths with the paper's propagation (blocks of 8 at the
    middle level), the +/-4 band and the paper's d/4 scope (radius 16)."""
    from paper_2001_09678_amd.scene import config_scene
    sc, _ = config_scene("c2")
    _log("paper propagation full size, radius", radius)
    _check(mpv, orc, sc.left, sc.right, 128, 3, radius, 8, 8)


def test_paper_propagation_rejected_by_batches(mpv):
    from paper_2001_09678_amd import _lib as L
    from paper_2001_09678_amd.scene import make_scene
    import ctypes as C
    sc = make_scene(1, 64, 48, 31, 4)
    l, r = _cuda(sc.left), _cuda(sc.right)
    item = (L.BatchItem * 1)()
    out = _cuda(np.zeros((48, 64), np.int16))
    item[0] = L.BatchItem(L.Image(l.data_ptr(), 64, 48, 64), L.Image(r.data_ptr(), 64, 48, 64), 32,
                          out.data_ptr(), None, None)
    pp = mpv.pyramid_params(mpv.MPVParams(num_disp=32, num_paths=4), 3, 4, propagation="paper")
    h = C.c_void_p()
    assert L.lib().mpv_batch_create(C.byref(pp), item, 1, C.byref(h)) == L.MPV_ERR_UNSUPPORTED
