"""A whole frame (forward + backward, list count on the device) captured in a
HIP graph through torch.cuda.graph: no host round trip inside the frame makes
it capturable. Every replay, with eager frames and synchronisations between
the replays, must equal the eager frame bit for bit (image, saved state,
gradients)."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "w1":
        return W.w1_small()
    return W.w2_clusters(n=100_000)


@pytest.mark.parametrize("case", ["w1", "w2_100k"])
def test_graph_replays_equal_the_eager_frame(case):
    import paper_2512_11800_amd as M
    scene, cams, opts = _case(case)
    g = M.Gaussians.from_scene(scene)
    gen = torch.Generator(device="cuda").manual_seed(3)
    gi = 1e-3 * torch.randn(len(cams), cams[0].height, cams[0].width, 3, generator=gen, device="cuda")
    ws = M.Workspace()

    def frame():
        img, saved, st = M.render_forward(g, cams, opts, ws=ws, on_device=True)
        grads = M.render_backward(g, cams, opts, st, saved, gi)
        return img, saved, grads, st

    ref = frame()  # sizes the capacity (one wait)
    torch.cuda.synchronize()
    ref[3].check()
    ref = (ref[0].clone(), ref[1].clone(), {k: v.clone() for k, v in ref[2].items()})

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            frame()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = frame()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        out[3].check()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), r
        for k, v in ref[2].items():
            assert torch.equal(out[2][k], v), (r, k)
        eager = frame()  # the program's own eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(eager[0], ref[0]), r
    log(f"[graph] {case}: 3 replays equal the eager frame")
