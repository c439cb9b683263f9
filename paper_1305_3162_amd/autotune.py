"""Timing autotuner for the choices the library leaves open without
changing the result beyond rounding order or the stated tolerance:

* the gridding split (``slp_params.seg_share``): how many sources one gridding
  workgroup takes before a tile is cut into pieces, each with its own padded
  block. Fewer, fuller pieces store and sum fewer blocks; more pieces balance
  the compute units better. The automatic rule shares the chip's workgroup
  slots out evenly; the tuner times the candidates around it on the device.
* the block-sum form (``slp_params.reduce_cells``): one cell per thread in
  workgroups of 512 or two in workgroups of 256. Two share a thread's
  neighbour tests and keep two load chains in flight; one keeps twice the
  waves, which small regions need. Both are timed at the tuned split (the
  result is the same bit for bit).
* the window and cut-off m at a requested tolerance (the paper's Gaussian or
  Kaiser-Bessel window, Sec. 3.2): every window whose smallest predicted m
  meets the tolerance (``choose_cutoff``) is timed, the fastest is kept and its
  split is tuned.

A step is the timed unit of the library: ``set_density`` + ``eval`` of one
density on the current stream. Results are cached in a JSON file keyed by the
device name, precision, window, m, grid, source count, tile counts and target
count, so a workload of the same shape reuses them without timing.
"""
import json
import os

import numpy as np

from . import FP32, FP64, WINDOW_GAUSS, WINDOW_KB, Geometry, SlpError, choose_cutoff

# multiples of the automatic share that are timed
SHARE_FACTORS = (0.25, 0.5, 0.75, 1.0, 1.5, 2.0)
MIN_SHARE, MAX_SHARE = 64, 1 << 24


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace("|", "/")


def cache_key(info, grid, m, window, precision, device, kind="split"):
    """Key of one tuning result: everything the split and the timings depend on."""
    return "|".join([kind, device, "fp64" if precision == FP64 else "fp32",
                     "kb" if window == WINDOW_KB else "gauss", f"m{int(m)}",
                     "g%dx%dx%d" % tuple(int(v) for v in grid), f"src{int(info['n_src'])}",
                     "t%dx%dx%d" % tuple(int(v) for v in info["tiles"]),
                     f"tgt{int(info['n_targets'])}"])


def load_cache(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a tuning cache")
    return data


def store_cache(path, data):
    if not path:
        return
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def share_candidates(auto_share, n_src):
    """Shares timed around the automatic one, plus one that never splits."""
    c = {int(min(MAX_SHARE, max(MIN_SHARE, round(auto_share * f)))) for f in SHARE_FACTORS}
    c.add(int(min(MAX_SHARE, max(MIN_SHARE, n_src))))
    return sorted(c)


def time_steps(G, dens, reps=30, warmup=3, rounds=3):
    """Mean microseconds of one step (set_density + eval), the best of `rounds`
    windows of `reps` steps bracketed by events on the current stream."""
    import torch
    phi = torch.empty(G.info["n_targets"], dtype=torch.float64, device=dens.device)
    for _ in range(warmup):
        G.set_density(dens)
        G.eval(phi)
    best = float("inf")
    for _ in range(rounds):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            G.set_density(dens)
            G.eval(phi)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e3 / reps)
    return best


def _density(n_src, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.normal(size=n_src)).cuda()


def tune_share(nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64, eta2=37.0,
               window=WINDOW_GAUSS, targets=None, cache=None, reps=30, force=False):
    """Times the gridding split candidates of one workload, then both block-sum
    forms at the fastest split; returns {"seg_share", "reduce_cells", "us",
    "auto_share", "auto_cells", "candidates": [...], "cached"}. Splits giving
    the same segment count as one already timed are skipped."""
    G = Geometry(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2,
                 window=window, targets=targets)
    info = dict(G.info)
    key = cache_key(info, grid, m, window, precision, _device_name())
    data = load_cache(cache)
    if not force and key in data:
        G.close()
        return dict(data[key], cached=True)
    auto = int(info["seg_share"])
    auto_cells = int(info["reduce_cells"])
    dens = _density(int(info["n_src"]))
    results, seen = [], {}
    try:
        for share in share_candidates(auto, int(info["n_src"])):
            H = G if share == auto else Geometry(nodes, tris, grid, m, es_w, es_gamma, alpha,
                                                 precision, eta2, window=window, targets=targets,
                                                 seg_share=share)
            try:
                nseg = int(H.info["n_segments"])
                if nseg in seen and share != auto:
                    continue
                us = time_steps(H, dens, reps=reps)
                seen[nseg] = share
                results.append({"seg_share": share, "reduce_cells": auto_cells,
                                "n_segments": nseg, "us": us})
            finally:
                if H is not G:
                    H.close()
        best = min(results, key=lambda r: r["us"])
        for cells in (1, 2):
            if cells == auto_cells:
                continue
            H = Geometry(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2,
                         window=window, targets=targets, seg_share=best["seg_share"],
                         reduce_cells=cells)
            try:
                results.append({"seg_share": best["seg_share"], "reduce_cells": cells,
                                "n_segments": int(H.info["n_segments"]),
                                "us": time_steps(H, dens, reps=reps)})
            finally:
                H.close()
    finally:
        G.close()
    best = min(results, key=lambda r: r["us"])
    out = {"seg_share": best["seg_share"], "reduce_cells": best["reduce_cells"], "us": best["us"],
           "auto_share": auto, "auto_cells": auto_cells, "candidates": results}
    data = load_cache(cache)
    data[key] = out
    store_cache(cache, data)
    return dict(out, cached=False)


def tune_cutoff(tol, nodes, tris, grid, es_w, es_gamma, alpha=2, precision=FP64, eta2=37.0,
                targets=None, cache=None, reps=30, force=False):
    """Fastest (window, m) predicted to meet `tol`, with its tuned split;
    returns {"window", "m", "seg_share", "reduce_cells", "us", "candidates": [...],
    "cached"}."""
    cands = []
    for w in (WINDOW_GAUSS, WINDOW_KB):
        try:
            cands.append(choose_cutoff(tol, precision, w))
        except SlpError:
            pass
    if not cands:
        raise SlpError(-1, f"no window and cut-off m <= 8 is predicted to reach {tol:g}")
    timed = []
    for w, m in cands:
        r = tune_share(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2, window=w,
                       targets=targets, cache=cache, reps=reps, force=force)
        timed.append({"window": w, "m": m, "seg_share": r["seg_share"],
                      "reduce_cells": r.get("reduce_cells", 0), "us": r["us"],
                      "cached": r["cached"]})
    best = min(timed, key=lambda r: r["us"])
    return dict(best, candidates=timed, cached=all(t["cached"] for t in timed))


def tuned_geometry(nodes, tris, grid, m, es_w, es_gamma, alpha=2, precision=FP64, eta2=37.0,
                   window=WINDOW_GAUSS, targets=None, cache=None):
    """Geometry with the tuned gridding split and block-sum form (timed now or
    read from `cache`)."""
    r = tune_share(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2, window=window,
                   targets=targets, cache=cache)
    G = Geometry(nodes, tris, grid, m, es_w, es_gamma, alpha, precision, eta2, window=window,
                 targets=targets, seg_share=r["seg_share"], reduce_cells=r.get("reduce_cells", 0))
    return G, r


__all__ = ["cache_key", "load_cache", "store_cache", "share_candidates", "time_steps",
           "tune_share", "tune_cutoff", "tuned_geometry", "FP32", "FP64"]
