"""Quality smoke test (a sanity check, not parity): on seeded synthetic scenes with known
ground truth, the matcher's error stays below loose bounds.

Error = non-occluded pixels whose disparity is invalid or more than 1 from the ground truth.
Plain full-range MPV and the +/-4 px pyramid are both checked; the pyramid may lose a little
against plain (the paper's multi-scale scheme trades accuracy for work, Section 3.4)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _err(disp, sc):
    m = ~sc.occluded
    bad = m & ((disp < 0) | (np.abs(disp.astype(np.int64) - sc.disp) > 1))
    return bad.sum() / max(m.sum(), 1)


@pytest.mark.parametrize("w,h,d", [(640, 360, 64), (1280, 720, 128)])
def test_error_vs_ground_truth(w, h, d):
    import torch
    from paper_2001_09678_amd import mpv
    from paper_2001_09678_amd.scene import make_scene
    print("quality", w, h, d, flush=True)
    params = mpv.MPVParams(num_disp=d, num_paths=8)
    errs = {"plain": [], "pyramid": []}
    for seed in (7001, 7002, 7003):
        sc = make_scene(seed, w, h, d - 1, 30, ground=True)
        L, R = torch.from_numpy(sc.left).cuda(), torch.from_numpy(sc.right).cuda()
        plain = mpv.pyramid(L, R, params, levels=1).disp.cpu().numpy()
        pyr = mpv.pyramid(L, R, params, levels=3, radius=4).disp.cpu().numpy()
        errs["plain"].append(_err(plain, sc))
        errs["pyramid"].append(_err(pyr, sc))
    e_plain, e_pyr = float(np.mean(errs["plain"])), float(np.mean(errs["pyramid"]))
    print(f"error vs ground truth: plain {e_plain:.4f}, pyramid {e_pyr:.4f}", flush=True)
    assert e_plain < 0.15
    assert e_pyr < 0.15
    assert e_pyr < e_plain + 0.03
