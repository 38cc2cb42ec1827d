"""Checkpoints of the learned surrogate: its weights, the harvested training
samples, and a manifest of everything that determined them (the scene's
content hash, the cameras, the render options, the seeds and the training
schedule), in safetensors files (tensors plus string metadata; loading runs
nothing from the file).

``harvest_cached`` and ``train_cached`` return the stored result when the
manifest of the file at the given path matches the request, and otherwise
compute it (on the GPU, through ``surrogate.harvest`` / ``surrogate.train``)
and store it there. Host-side bookkeeping only: no arithmetic of the method
happens here.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional, Sequence

import numpy as np
import torch

FORMAT = "mb3dgs-surrogate/1"


def scene_hash(g) -> str:
    """SHA-256 over the Gaussians' float32 bytes (means, scales, quats,
    densities, colors, in that order) and the SH degree."""
    h = hashlib.sha256()
    for t in (g.means, g.scales, g.quats, g.densities, g.colors):
        h.update(np.ascontiguousarray(torch.as_tensor(t).detach().to("cpu", torch.float32).numpy()).tobytes())
    h.update(str(int(g.sh_degree)).encode())
    return h.hexdigest()


def camera_record(cam) -> dict:
    return {"world_to_cam": [float(v) for v in np.asarray(cam.world_to_cam, np.float64).reshape(-1)],
            "fx": float(cam.fx), "fy": float(cam.fy), "cx": float(cam.cx), "cy": float(cam.cy),
            "width": int(cam.width), "height": int(cam.height), "t_near": float(cam.t_near),
            "background": [float(v) for v in cam.background]}


def options_record(opts) -> dict:
    keys = ("n_moments", "n_intervals", "kappa", "conf_c", "beta", "eps", "basis")
    return {k: (getattr(opts, k) if isinstance(getattr(opts, k), str) else float(getattr(opts, k)))
            for k in keys if hasattr(opts, k)}


def harvest_manifest(g, cams: Sequence, opts, n_target: int, seed: int) -> dict:
    return {"format": FORMAT, "kind": "harvest", "scene_sha256": scene_hash(g), "n_gaussians": int(g.n),
            "cameras": [camera_record(c) for c in cams], "options": options_record(opts),
            "n_target": int(n_target), "seed": int(seed)}


def train_manifest(samples_manifest: dict, steps: int, batch: int, lr: float, lr_final: Optional[float],
                   seed: int) -> dict:
    return {"format": FORMAT, "kind": "weights", "samples": samples_manifest, "steps": int(steps),
            "batch": int(batch), "lr": float(lr), "lr_final": None if lr_final is None else float(lr_final),
            "seed": int(seed)}


def _save(path: str, tensors: dict, manifest: dict, extra: Optional[dict] = None) -> None:
    from safetensors.torch import save_file
    meta = {"manifest": json.dumps(manifest, sort_keys=True)}
    if extra:
        meta["info"] = json.dumps(extra, sort_keys=True)
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    save_file({k: v.detach().contiguous().cpu() for k, v in tensors.items()}, tmp, metadata=meta)
    os.replace(tmp, path)  # a reader never sees a half-written file


def _load(path: str):
    from safetensors import safe_open
    with safe_open(path, framework="pt", device="cpu") as f:
        meta = f.metadata() or {}
        tensors = {k: f.get_tensor(k) for k in f.keys()}
    if "manifest" not in meta:
        raise ValueError(f"{path}: no manifest")
    manifest = json.loads(meta["manifest"])
    if manifest.get("format") != FORMAT:
        raise ValueError(f"{path}: format {manifest.get('format')!r}, expected {FORMAT!r}")
    info = json.loads(meta["info"]) if "info" in meta else {}
    return tensors, manifest, info


def save_samples(path: str, x: torch.Tensor, t: torch.Tensor, manifest: dict, info: Optional[dict] = None):
    _save(path, {"x": x, "t": t}, manifest, info)


def load_samples(path: str, device="cpu"):
    """(x, t, manifest, info) of a harvested-sample file."""
    ts, manifest, info = _load(path)
    if manifest.get("kind") != "harvest":
        raise ValueError(f"{path}: not a harvested-sample file")
    return ts["x"].to(device), ts["t"].to(device), manifest, info


def save_weights(path: str, theta: torch.Tensor, manifest: dict, losses=None):
    _save(path, {"theta": theta}, manifest, {"losses": losses or []})


def load_weights(path: str, device="cpu", expect_params: Optional[int] = None):
    """(theta, manifest, info) of a weights file; ``expect_params`` checks the
    parameter count against the library's layout."""
    ts, manifest, info = _load(path)
    if manifest.get("kind") != "weights":
        raise ValueError(f"{path}: not a weights file")
    theta = ts["theta"]
    if theta.dtype != torch.float32 or theta.dim() != 1:
        raise ValueError(f"{path}: theta must be a float32 vector")
    if expect_params is not None and theta.numel() != expect_params:
        raise ValueError(f"{path}: {theta.numel()} parameters, the network has {expect_params}")
    return theta.to(device), manifest, info


def _matches(path: str, manifest: dict) -> bool:
    if not os.path.exists(path):
        return False
    try:
        _, stored, _ = _load(path)
    except (ValueError, OSError):
        return False
    return stored == json.loads(json.dumps(manifest, sort_keys=True))


def harvest_cached(path: str, g, cams: Sequence, opts, n_target: int, seed: int = 0, ws=None):
    """surrogate.harvest, stored at ``path`` and reused when the file's
    manifest matches. Returns (x, t, info, hit) with x, t on g's device."""
    man = harvest_manifest(g, cams, opts, n_target, seed)
    dev = g.means.device
    if _matches(path, man):
        x, t, _, info = load_samples(path, dev)
        return x, t, info, True
    from .surrogate import harvest
    x, t, info = harvest(g, cams, opts, n_target, seed=seed, ws=ws)
    save_samples(path, x, t, man, info)
    return x, t, info, False


def train_cached(path: str, samples_manifest: dict, x: torch.Tensor, t: torch.Tensor, steps: int,
                 batch: int = 65536, lr: float = 1e-3, lr_final: Optional[float] = None, seed: int = 0,
                 log_every: int = 0):
    """surrogate.train, stored at ``path`` and reused when the file's manifest
    (which embeds the samples' manifest) matches. Returns (theta, packed,
    losses, hit)."""
    from .surrogate import mlp_pack, param_count, train
    man = train_manifest(samples_manifest, steps, batch, lr, lr_final, seed)
    if _matches(path, man):
        theta, _, info = load_weights(path, x.device, expect_params=param_count())
        return theta, mlp_pack(theta), [tuple(v) for v in info.get("losses", [])], True
    theta, packed, losses = train(x, t, steps=steps, batch=batch, lr=lr, lr_final=lr_final, seed=seed,
                                  log_every=log_every)
    save_weights(path, theta, man, losses)
    return theta, packed, losses, False
