"""Renders with the list count kept on the device (MB_ENTRIES_ON_DEVICE): no
host round trip inside a frame, the pair workspace laid out for a capacity.

Bars: image, saved state and gradients bit-identical to the counted path (the
same kernels on the same lists; only launch sizes differ). A frame with more
entries than the capacity is reported by ``state.check()``, its kernels stay
inside the workspace (finite outputs), and the frame rendered again after
the capacity grows is bit-identical to the counted one."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _frame(g, cams, opts, ws, on_device, gi):
    import paper_2512_11800_amd as M
    img, saved, st = M.render_forward(g, cams, opts, ws=ws, on_device=on_device)
    grads = M.render_backward(g, cams, opts, st, saved, gi)
    torch.cuda.synchronize()
    return img.clone(), saved.clone(), {k: v.clone() for k, v in grads.items()}, st


def _upstream(cams, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return 1e-3 * torch.randn(len(cams), cams[0].height, cams[0].width, 3, generator=gen, device="cuda")


def _case(name):
    if name == "w1_two_cameras_ragged":
        scene, _, opts = W.w1_small()
        cams = [W.camera_on_axis(3.0, 100, 75),
                W.camera_look_at((2.0, 1.0, -2.5), (0, 0, 0), (0, 1, 0), 100, 75)]
        return scene, cams, opts
    scene, cams, opts = W.w2_clusters(n=100_000)
    return scene, cams, opts


@pytest.mark.parametrize("case", ["w1_two_cameras_ragged", "w2_100k"])
def test_device_count_matches_counted_path(case):
    import paper_2512_11800_amd as M
    scene, cams, opts = _case(case)
    g = M.Gaussians.from_scene(scene)
    gi = _upstream(cams, 5)
    ref = _frame(g, cams, opts, M.Workspace(), False, gi)
    ws = M.Workspace()
    first = _frame(g, cams, opts, ws, True, gi)   # sizes the capacity from its count (one wait)
    second = _frame(g, cams, opts, ws, True, gi)  # nothing waits
    n = ref[3].n_entries
    log(f"[device count] {case}: {n} entries, capacity {ws.capacity}")
    for label, out in (("first", first), ("second", second)):
        st = out[3]
        assert st.n_entries == -1
        st.check()
        assert st.entry_count() == n
        assert torch.equal(out[0], ref[0]), label
        assert torch.equal(out[1], ref[1]), label
        for k, v in ref[2].items():
            assert torch.equal(out[2][k], v), (label, k)


def test_overflow_is_reported_and_stays_in_bounds():
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w1_small()
    g = M.Gaussians.from_scene(scene)
    gi = _upstream(cams, 6)
    ref = _frame(g, cams, opts, M.Workspace(), False, gi)
    n = ref[3].n_entries
    ws = M.Workspace()
    ws.capacity = n // 4
    img, saved, grads, st = _frame(g, cams, opts, ws, True, gi)
    cap = int(M._lib.load().mb_pair_capacity(ws.pws.numel(), len(cams), cams[0].width, cams[0].height))
    log(f"[device count] overflow: {n} entries, workspace holds {cap}")
    assert cap < n
    assert bool(torch.isfinite(img).all())
    for k, v in grads.items():
        assert bool(torch.isfinite(v).all()), k
    assert not torch.equal(img, ref[0])  # entries were dropped
    with pytest.raises(RuntimeError):
        st.check()
    assert ws.capacity > n
    again = _frame(g, cams, opts, ws, True, gi)
    again[3].check()
    assert torch.equal(again[0], ref[0]) and torch.equal(again[1], ref[1])
    for k, v in ref[2].items():
        assert torch.equal(again[2][k], v), k


@pytest.mark.parametrize("n_keep", [0, 1])
def test_device_count_empty_and_single(n_keep):
    """No Gaussians (no emit launch, the capacity's default slack) and one
    Gaussian: the device-count frame equals the counted one."""
    import paper_2512_11800_amd as M
    scene, cams, opts = W.w1_small()
    scene = scene.subset(np.arange(5, 5 + n_keep))
    g = M.Gaussians.from_scene(scene)
    gi = _upstream(cams, 7)
    ref = _frame(g, cams, opts, M.Workspace(), False, gi)
    ws = M.Workspace()
    for _ in range(2):
        out = _frame(g, cams, opts, ws, True, gi)
        out[3].check()
        assert out[3].entry_count() == ref[3].n_entries
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
        for k, v in ref[2].items():
            assert torch.equal(out[2][k], v), k
