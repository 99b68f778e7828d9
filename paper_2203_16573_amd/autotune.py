"""Tile-shape autotuner for the fused time-step kernel.

For a problem shape (padded grid, stencil order, storage type, shots) it
times the candidate tile heights of the fused step on a short copy of the
problem (same grid, same shots, few time steps) for the full grid and for
the thin slab separately, also times the split two-launch step on the full
grid, and applies the fastest choice to a context.  Results are cached in a
JSON file keyed by shape, never by the data or the mix of other work, so a
given shape always runs the same kernels (results do not depend on the
choice: every variant evaluates the same expressions).
"""
from __future__ import annotations

import json
import os
import threading

from . import (OPT_STEP_KERNEL, OPT_STEPS_PER_LAUNCH, OPT_STEPS_PER_LAUNCH_SLAB, OPT_TILE_Z,
               OPT_TILE_Z_SLAB, Context)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ssx", "autotune-v2.json")
_lock = threading.Lock()


def shape_key(prob, nshots: int, field_dtype: str) -> str:
    NZ, NX = prob.nz + 2 * prob.npml, prob.nx + 2 * prob.npml
    k = prob.order // 2
    nzs = abs(prob.slab_dz) + 1 + 2 * k + 2 * prob.npml
    return f"{NZ}x{NX}|slab{nzs}|o{prob.order}|{field_dtype}|s{nshots}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(fn, reps=2):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(prob, kappa, rho, xs=None, field_dtype="f32", nt_tune: int = 60,
         stream=None) -> dict:
    """Measure the candidates and return {"step_kernel", "tile_z", "tile_z_slab",
    "us": {...}} (per-step times in microseconds)."""
    import torch
    xs = tuple(prob.xs) if xs is None else tuple(xs)
    short = prob.replace(nt=min(int(nt_tune), int(prob.nt))) if hasattr(prob, "replace") else prob
    ctx = Context(short, kappa, rho, xs=xs, field_dtype=field_dtype, stream=stream)
    ctx.set_graphs(False)
    nt = short.nt
    vdt = ctx.vdtype
    h = torch.randn((len(xs), nt, short.ns), dtype=vdt, device="cuda")
    d = ctx.empty_r()
    g = ctx.empty_s()
    P, V = ctx.empty_s(), ctx.empty_s()
    # candidates: (steps per launch, tile height)
    if field_dtype == "f64":
        cands = [(1, 8), (1, 16)]
    elif field_dtype == "f32":
        cands = [(1, 8), (1, 16), (1, 32), (2, 8)]
    else:  # two steps per launch are FP32-only
        cands = [(1, 8), (1, 16), (1, 32)]
    us = {}
    ctx.set_option(OPT_STEP_KERNEL, 1)
    for spl, tz in cands:
        ctx.set_option(OPT_TILE_Z, tz)
        ctx.set_option(OPT_STEPS_PER_LAUNCH, spl)
        tag = f"s{spl}_tz{tz}"
        us[f"full_{tag}"] = 1e3 * _time_ms(lambda: (ctx.fwd(h, d), ctx.adj(d, g))) / (2 * nt)
        us[f"slab_{tag}"] = 1e3 * _time_ms(
            lambda: (ctx.slab_fwd(h, P, V), ctx.slab_adj(V, P, g))) / (2 * nt)
    ctx.set_option(OPT_STEPS_PER_LAUNCH, 1)
    ctx.set_option(OPT_STEP_KERNEL, 0)
    us["full_split"] = 1e3 * _time_ms(lambda: (ctx.fwd(h, d), ctx.adj(d, g))) / (2 * nt)
    us["slab_split"] = 1e3 * _time_ms(
        lambda: (ctx.slab_fwd(h, P, V), ctx.slab_adj(V, P, g))) / (2 * nt)
    ctx.close()
    best_full = min(cands, key=lambda c: us[f"full_s{c[0]}_tz{c[1]}"])
    best_slab = min(cands, key=lambda c: us[f"slab_s{c[0]}_tz{c[1]}"])
    fused_total = us[f"full_s{best_full[0]}_tz{best_full[1]}"] + \
        us[f"slab_s{best_slab[0]}_tz{best_slab[1]}"]
    split_total = us["full_split"] + us["slab_split"]
    return {"step_kernel": 1 if fused_total <= split_total else 0,
            "steps_per_launch": best_full[0], "tile_z": best_full[1],
            "steps_per_launch_slab": best_slab[0], "tile_z_slab": best_slab[1], "us": us}


def choose(prob, kappa, rho, xs=None, field_dtype="f32", cache_path: str | None = DEFAULT_CACHE,
           retune: bool = False, **kw) -> dict:
    """Cached :func:`tune` keyed by :func:`shape_key`."""
    xs = tuple(prob.xs) if xs is None else tuple(xs)
    key = shape_key(prob, len(xs), field_dtype)
    if cache_path and not retune:
        with _lock:
            hit = _load(cache_path).get(key)
        if hit:
            return hit
    res = tune(prob, kappa, rho, xs=xs, field_dtype=field_dtype, **kw)
    if cache_path:
        with _lock:
            table = _load(cache_path)
            table[key] = res
            _store(cache_path, table)
    return res


def apply(ctx: Context, choice: dict) -> None:
    """Set a context's step kernel and tile heights from a tuning result."""
    ctx.set_option(OPT_STEP_KERNEL, int(choice["step_kernel"]))
    ctx.set_option(OPT_TILE_Z, int(choice["tile_z"]))
    ctx.set_option(OPT_TILE_Z_SLAB, int(choice["tile_z_slab"]))
    ctx.set_option(OPT_STEPS_PER_LAUNCH, int(choice.get("steps_per_launch", 1)))
    ctx.set_option(OPT_STEPS_PER_LAUNCH_SLAB, int(choice.get("steps_per_launch_slab", 1)))
