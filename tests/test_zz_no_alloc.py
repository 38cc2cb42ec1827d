"""The allocation-free forward entry point (mb_render_forward_noalloc)
against the entry point it stands for (mb_prepare with a count, then
mb_render_forward on caller workspaces): bit-identical images and saved state
on two calls in a row, the second with a smaller scene and image (the
library's scratch keeps the first call's contents), and a frame too large
for the scratch is rejected before anything is rendered."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _both(scene, cams, opts):
    import paper_2512_11800_amd as M
    g = M.Gaussians.from_scene(scene)
    ref_img, ref_saved, st = M.render_forward(g, cams, opts)
    img, saved, n_entries = M.render_forward_noalloc(g, cams, opts)
    torch.cuda.synchronize()
    return ref_img, ref_saved, st, img, saved, n_entries


def test_noalloc_matches_the_workspace_path_twice():
    scene, cams, opts = W.w1_small()
    a = _both(scene, cams, opts)
    small = scene.subset(np.arange(0, scene.n, 3))
    cams2 = [W.camera_look_at((2.0, 1.0, -2.5), (0, 0, 0), (0, 1, 0), 100, 75)]
    opts2 = W.Options(n_moments=6)
    b = _both(small, cams2, opts2)
    for label, (ref_img, ref_saved, st, img, saved, n_entries) in (("first", a), ("second, smaller", b)):
        log(f"[noalloc] {label}: entries {n_entries} (workspace path {st.n_entries}), image {tuple(img.shape)}")
        assert n_entries == st.n_entries > 0
        assert torch.isfinite(img).all()
        assert torch.equal(img, ref_img)
        assert torch.equal(saved, ref_saved)


def test_noalloc_rejects_a_frame_beyond_its_scratch():
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w2_clusters()
    g = M.Gaussians.from_scene(scene)
    with pytest.raises(M.MbError, match="scratch"):
        M.render_forward_noalloc(g, cams, opts)
    # a normal frame still renders after the rejection
    scene1, cams1, opts1 = W.w1_small()
    ref_img, _, _, img, _, _ = _both(scene1, cams1, opts1)
    assert torch.equal(img, ref_img)
