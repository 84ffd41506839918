"""Autotuner of the blend launch configuration for a mapping workload.

The blend kernels have knobs that leave the images unchanged (bit-identical)
and the gradients equal up to float rounding order: the screen tile (16x16,
16x8, 32x8, 8x8), pixels per thread (1, or 2 for tiles of at least 128
pixels), the backward's batch depth (Gaussians staged in LDS per round: 16,
32 or 64) and its work unit (chunks of a tile list: length and count). The
tuner times the graph-replayed mapping iteration under each candidate on the
caller's workload and keeps the fastest. Results are cached per (device,
workload shape) in a JSON file.
"""
from __future__ import annotations

import json
import os

import torch

from .rasterize import Rasterizer

CANDIDATES = [
    # tile_w, tile_h, pixels_per_thread, batch_depth, chunk_len (0 automatic, -1 whole list), max_chunks
    (16, 16, 1, 0, 0, 0), (16, 16, 1, 0, -1, 0), (16, 16, 1, 0, 128, 4), (16, 16, 1, 0, 64, 8),
    (16, 16, 1, 16, 0, 0), (16, 16, 1, 64, 0, 0), (16, 16, 2, 0, 0, 0),
    (16, 8, 1, 0, 0, 0), (16, 8, 2, 0, 0, 0), (32, 8, 1, 0, 0, 0), (32, 8, 2, 0, 0, 0), (8, 8, 1, 0, 0, 0),
]
FIELDS = ("tile_w", "tile_h", "pixels_per_thread", "batch_depth", "chunk_len", "max_chunks")


def _cache_path():
    p = os.environ.get("GSR_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2509_06433_amd", "autotune.json")


def signature(params, sh_degree, cams, adam):
    dev = torch.cuda.get_device_name(params.device)
    res = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"v2|{dev}|N={params.shape[1]}|deg={sh_degree}|views={len(cams)}|{res}|adam={int(adam)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    except OSError:
        pass


def time_config(params, sh_degree, cams, targets, cfg, depth_weight=0.5, adam_lrs=None, warmup=2, steps=5):
    """Milliseconds per graph-replayed mapping iteration under one candidate.
    The parameters are not modified (Adam, if timed, updates a copy)."""
    tw, th, ppt, depth, chunk, nchunks = cfg
    R = Rasterizer(tile_w=tw, tile_h=th, pixels_per_thread=ppt, batch_depth=depth, chunk_len=chunk,
                   max_chunks=nchunks)
    p = params.clone() if adam_lrs is not None else params
    outs = R.alloc_images(cams, params.device)
    grad = torch.empty_like(p)
    loss = torch.empty(1, device=params.device)
    adam = None
    if adam_lrs is not None:
        adam = dict(m=torch.zeros_like(p), v=torch.zeros_like(p), lr=adam_lrs, step=1)
    for i in range(warmup):
        R.mapping_iteration(p, sh_degree, cams, outs, targets, grad, depth_weight, loss, adam)
        if adam is not None:
            adam["step"] = 0
    st = R.mapping_status()
    if st["skipped"]:
        # the first replays sized the capacity; time a clean set
        R.mapping_iteration(p, sh_degree, cams, outs, targets, grad, depth_weight, loss, adam)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        R.mapping_iteration(p, sh_degree, cams, outs, targets, grad, depth_weight, loss, adam)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    R.close()
    return ms


def tune(params, sh_degree, cams, targets, depth_weight=0.5, adam_lrs=None, candidates=None, use_cache=True,
         warmup=2, steps=5, log=None):
    """Returns dict(tile_w, tile_h, pixels_per_thread, batch_depth, chunk_len, max_chunks, ms, table) for the
    fastest candidate."""
    path = _cache_path()
    key = signature(params, sh_degree, cams, adam_lrs is not None)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    table = []
    for cfg in candidates or CANDIDATES:
        ms = time_config(params, sh_degree, cams, targets, cfg, depth_weight, adam_lrs, warmup, steps)
        table.append([*cfg, round(ms, 4)])
        if log:
            log(f"autotune {cfg}: {ms:.4f} ms")
    best = min(table, key=lambda r: r[-1])
    out = dict(zip(FIELDS, best[:-1]), ms=best[-1], table=table)
    if use_cache:
        cache[key] = out
        _store(path, cache)
    return dict(out, cached=False)
