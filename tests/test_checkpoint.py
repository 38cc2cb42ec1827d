"""Surrogate checkpoints (host logic, CPU): weights and harvested samples
round-trip bit-exactly with their manifest, and the cached harvest/train
reuse a file only when everything in the manifest matches."""
import types

import numpy as np
import pytest
import torch

import workloads as W
from paper_2512_11800_amd import checkpoint as C


def _g(scene):
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32))
    return types.SimpleNamespace(means=t(scene.means), scales=t(scene.scales), quats=t(scene.quats),
                                 densities=t(scene.densities), colors=t(scene.colors),
                                 sh_degree=int(scene.sh_degree), n=int(scene.n))


def test_weights_and_samples_round_trip(tmp_path):
    scene, cams, opts = W.w1_small()
    g = _g(scene)
    man = C.harvest_manifest(g, cams, opts, 1000, 7)
    x = torch.randn(1000, 8)
    t = torch.rand(1000)
    C.save_samples(str(tmp_path / "s.safetensors"), x, t, man, {"rate": 0.5})
    x2, t2, man2, info = C.load_samples(str(tmp_path / "s.safetensors"))
    assert torch.equal(x, x2) and torch.equal(t, t2) and info == {"rate": 0.5}
    assert man2 == C.harvest_manifest(g, cams, opts, 1000, 7)
    theta = torch.randn(4737)
    wm = C.train_manifest(man, 100, 4096, 1e-3, 1e-4, 3)
    C.save_weights(str(tmp_path / "w.safetensors"), theta, wm, [(100, 0.5)])
    th2, wm2, winfo = C.load_weights(str(tmp_path / "w.safetensors"), expect_params=4737)
    assert torch.equal(theta, th2) and wm2 == wm and winfo["losses"] == [[100, 0.5]]
    with pytest.raises(ValueError, match="parameters"):
        C.load_weights(str(tmp_path / "w.safetensors"), expect_params=10)
    with pytest.raises(ValueError, match="not a weights file"):
        C.load_weights(str(tmp_path / "s.safetensors"))


def test_manifest_names_scene_cameras_options_and_seed():
    scene, cams, opts = W.w1_small()
    g = _g(scene)
    base = C.harvest_manifest(g, cams, opts, 1000, 7)
    g2 = _g(scene)
    g2.densities = g2.densities.clone()
    g2.densities[5] *= 1.0001
    assert C.harvest_manifest(g2, cams, opts, 1000, 7)["scene_sha256"] != base["scene_sha256"]
    assert C.harvest_manifest(g, cams, opts, 1000, 8) != base
    assert C.harvest_manifest(g, cams, opts, 1001, 7) != base
    cams2 = W.random_cameras(1, 3.0, 128, 128, seed=1)
    assert C.harvest_manifest(g, cams2, opts, 1000, 7) != base
    opts.n_intervals = 5
    assert C.harvest_manifest(g, cams, opts, 1000, 7) != base


def test_cached_harvest_and_train_reuse_only_matching_files(tmp_path, monkeypatch):
    from paper_2512_11800_amd import surrogate as S
    calls = {"harvest": 0, "train": 0}

    def fake_harvest(g, cams, opts, n_target, seed=0, ws=None):
        calls["harvest"] += 1
        gen = torch.Generator().manual_seed(seed)
        return torch.randn(n_target, 8, generator=gen), torch.rand(n_target, generator=gen), {"rate": 1.0}

    def fake_train(x, t, steps, batch=65536, lr=1e-3, lr_final=None, seed=0, log_every=0, theta=None):
        calls["train"] += 1
        return torch.full((4737,), float(seed)), None, [(steps, 0.25)]

    monkeypatch.setattr(S, "harvest", fake_harvest)
    monkeypatch.setattr(S, "train", fake_train)
    monkeypatch.setattr(S, "mlp_pack", lambda theta: theta)
    monkeypatch.setattr(S, "param_count", lambda: 4737)
    scene, cams, opts = W.w1_small()
    g = _g(scene)
    p = str(tmp_path / "samples.safetensors")
    x1, t1, _, hit1 = C.harvest_cached(p, g, cams, opts, 500, seed=3)
    x2, t2, _, hit2 = C.harvest_cached(p, g, cams, opts, 500, seed=3)
    assert (hit1, hit2) == (False, True) and calls["harvest"] == 1
    assert torch.equal(x1, x2) and torch.equal(t1, t2)
    _, _, _, hit3 = C.harvest_cached(p, g, cams, opts, 500, seed=4)  # another seed: recomputed
    assert not hit3 and calls["harvest"] == 2
    man = C.harvest_manifest(g, cams, opts, 500, 4)
    w = str(tmp_path / "weights.safetensors")
    th1, _, l1, h1 = C.train_cached(w, man, x1, t1, steps=50, seed=2)
    th2, _, l2, h2 = C.train_cached(w, man, x1, t1, steps=50, seed=2)
    assert (h1, h2) == (False, True) and calls["train"] == 1
    assert torch.equal(th1, th2) and l2 == [(50, 0.25)]
    _, _, _, h3 = C.train_cached(w, man, x1, t1, steps=60, seed=2)
    assert not h3 and calls["train"] == 2
