"""Execution-shape autotuner for the time-step kernels.

For a problem shape (padded grid, stencil order, storage type, shots) it
times, on a short copy of the problem (same grid, same shots, few time
steps) and under captured graphs as the solver runs them, first the
launch forms of each grid -- the fused one-step kernel at each tile height,
with and without the tile loop, the multi-step kernel at each (steps per
launch, strip width) it runs on that grid, and the split two-launch step --
then the number of shots advanced per launch, for the full grid and the
thin slab separately, and applies the fastest choice to a context.  Results are cached in a JSON file keyed by shape, never by
the data or the mix of other work, so a given shape always runs the same
kernels (results do not depend on the choice: every variant evaluates the
same expressions).
"""
from __future__ import annotations

import json
import os
import threading

import numpy as np

from . import (OPT_SHOT_GROUP, OPT_SHOT_GROUP_SLAB, OPT_SLAB_STRIP, OPT_STEP_KERNEL,
               OPT_STEPS_PER_LAUNCH, OPT_STEPS_PER_LAUNCH_SLAB, OPT_STRIP, OPT_TILE_LOOP,
               OPT_TILE_Z, OPT_TILE_Z_SLAB,
               Context)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ssx", "autotune-v8.json")
SLAB_MAXZ = 56  # rows of one region of the multi-step kernel


def multi_shapes(order: int, field_dtype: str, nz_rows: int,
                 variable_density: bool = False) -> list:
    """(steps per launch, strip width) pairs of the multi-step kernel that
    can run on a grid of nz_rows rows: owned columns left after the halo of
    ns stencil reaches (rounded up to 4) on each side, 64-column strips for
    F64 fields and density arrays, and owned rows left in each window of a
    taller grid."""
    out = []
    for ns in (2, 4, 8):
        for wr in (64, 128):
            if (field_dtype == "f64" or variable_density) and wr != 64:
                continue
            halo = -(-ns * (order - 1) // 4) * 4
            if wr - 2 * halo <= 0:
                continue
            if nz_rows > SLAB_MAXZ and SLAB_MAXZ - 2 * ns * (order - 1) <= 0:
                continue
            out.append((ns, wr))
    return out
_lock = threading.Lock()


def shape_key(prob, nshots: int, field_dtype: str, variable_density: bool = False) -> str:
    NZ, NX = prob.nz + 2 * prob.npml, prob.nx + 2 * prob.npml
    k = prob.order // 2
    nzs = abs(prob.slab_dz) + 1 + 2 * k + 2 * prob.npml
    key = f"{NZ}x{NX}|slab{nzs}|o{prob.order}|{field_dtype}|s{nshots}"
    rdz = int(getattr(prob, "rslab_dz", 0))
    if rdz:  # the receiver-side slab shares the slab options
        key += f"|rslab{abs(rdz) + 1 + 2 * k + 2 * prob.npml}"
    if variable_density:  # other kernel instances, fewer launch forms
        key += "|vrho"
    return key


def tallest_slab(prob) -> int:
    """Rows of the taller thin slab (one more than the count for a line
    between rows), which must fit the multi-step slab kernel."""
    rows = abs(prob.slab_dz) + 1 + prob.order + 2 * prob.npml + 1
    rdz = int(getattr(prob, "rslab_dz", 0))
    if rdz:
        rows = max(rows, abs(rdz) + 1 + prob.order + 2 * prob.npml + 1)
    return rows


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


def _time_ms(fn, stream, reps=3):
    """Milliseconds per call of fn, timed with events on `stream` (the
    stream the context issues its work on)."""
    import torch
    fn()  # first call captures the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _group_candidates(auto: int, nshots: int) -> list:
    c = {auto, nshots, max(1, auto // 2), min(nshots, 2 * auto)}
    return sorted(c)


def tune(prob, kappa, rho, xs=None, field_dtype="f32", nt_tune: int = 60,
         stream=None, rounds: int = 2) -> dict:
    """Measure the candidates and return {"step_kernel", "steps_per_launch",
    "tile_z", "shot_group", "steps_per_launch_slab", "tile_z_slab",
    "slab_strip", "shot_group_slab", "us": {...}} (per-step times in
    microseconds)."""
    import torch
    xs = tuple(prob.xs) if xs is None else tuple(xs)
    short = prob.replace(nt=min(int(nt_tune), int(prob.nt))) if hasattr(prob, "replace") else prob
    ctx = Context(short, kappa, rho, xs=xs, field_dtype=field_dtype, stream=stream)
    ctx.set_graphs(True)
    nt, ns = short.nt, len(xs)
    NZ, NX = short.nz + 2 * short.npml, short.nx + 2 * short.npml
    vdt = ctx.vdtype
    h = torch.randn((ns, nt, short.ns), dtype=vdt, device="cuda")
    d = ctx.empty_r()
    g = ctx.empty_s()
    P, V = ctx.empty_s(), ctx.empty_s()
    full = lambda: (ctx.fwd(h, d), ctx.adj(d, g))          # noqa: E731
    slab = lambda: (ctx.slab_fwd(h, P, V), ctx.slab_adj(V, P, g))  # noqa: E731
    # candidates: (steps per launch, tile height)
    if field_dtype == "f64":
        cands = [(1, 8), (1, 16)]
    else:
        cands = [(1, 8), (1, 16), (1, 32)]
    # candidates on each grid: (steps per launch, tile height, tile loop,
    # strip width).  One-step launches at every tile height, on the full
    # grid also with workgroups looping over the interior tiles; the
    # multi-step kernel at each (steps, strip width) it runs on that grid,
    # with tile height 8 for the one-step remainder (the tile loop: constant
    # density only)
    vrho = np.ndim(rho) != 0
    full_cands = [(1, tz, 0, 0) for _, tz in cands]
    slab_cands = [(1, tz, 0, 0) for _, tz in cands]
    if not vrho:
        full_cands += [(1, tz, 1, 0) for _, tz in cands]
    full_cands += [(ns, 8, 0, wr) for ns, wr in multi_shapes(short.order, field_dtype, NZ, vrho)]
    slab_cands += [(ns, 8, 0, wr)
                   for ns, wr in multi_shapes(short.order, field_dtype, tallest_slab(short), vrho)]
    key_f = lambda c: f"full_s{c[0]}_tz{c[1]}_l{c[2]}_w{c[3]}"  # noqa: E731
    key_s = lambda c: f"slab_s{c[0]}_tz{c[1]}_w{c[3]}"          # noqa: E731

    def set_full(c):
        # strip back to its default first: steps and strip are checked together
        ctx.set_option(OPT_STRIP, 0)
        ctx.set_option(OPT_TILE_Z, c[1])
        ctx.set_option(OPT_STEPS_PER_LAUNCH, c[0])
        ctx.set_option(OPT_STRIP, c[3])
        ctx.set_option(OPT_TILE_LOOP, c[2])

    def set_slab(c):
        ctx.set_option(OPT_SLAB_STRIP, 0)
        ctx.set_option(OPT_TILE_Z_SLAB, c[1])
        ctx.set_option(OPT_STEPS_PER_LAUNCH_SLAB, c[0])
        ctx.set_option(OPT_SLAB_STRIP, c[3])

    us = {}
    ctx.set_option(OPT_STEP_KERNEL, 1)
    ctx.set_option(OPT_SHOT_GROUP, 0)
    auto_group = max(1, ctx.cells_per_launch() // (NZ * NX))
    # every candidate is timed in each of `rounds` passes over the list and
    # keeps its fastest time, so that a slow moment of the device does not
    # decide between close candidates
    for _ in range(rounds):
        ctx.set_option(OPT_STEP_KERNEL, 1)
        for c in full_cands:
            set_full(c)
            t = 1e3 * _time_ms(full, ctx.stream) / (2 * nt)
            us[key_f(c)] = min(t, us.get(key_f(c), t))
        set_full((1, 8, 0, 0))
        for c in slab_cands:
            set_slab(c)
            t = 1e3 * _time_ms(slab, ctx.stream) / (2 * nt)
            us[key_s(c)] = min(t, us.get(key_s(c), t))
        set_slab((1, 8, 0, 0))
        ctx.set_option(OPT_STEP_KERNEL, 0)
        for k, fn in (("full_split", full), ("slab_split", slab)):
            t = 1e3 * _time_ms(fn, ctx.stream) / (2 * nt)
            us[k] = min(t, us.get(k, t))
    best_full = min(full_cands, key=lambda c: us[key_f(c)])
    best_slab = min(slab_cands, key=lambda c: us[key_s(c)])
    fused_total = us[key_f(best_full)] + us[key_s(best_slab)]
    split_total = us["full_split"] + us["slab_split"]
    step_kernel = 1 if fused_total <= split_total else 0
    ctx.set_option(OPT_STEP_KERNEL, step_kernel)
    set_full(best_full)
    set_slab(best_slab)
    group, group_slab = auto_group, 0
    if ns > 1:
        for _ in range(rounds):
            for gsz in _group_candidates(auto_group, ns):
                ctx.set_option(OPT_SHOT_GROUP, gsz)
                ctx.set_option(OPT_SHOT_GROUP_SLAB, 0)
                t = 1e3 * _time_ms(full, ctx.stream) / (2 * nt)
                us[f"full_group{gsz}"] = min(t, us.get(f"full_group{gsz}", t))
        group = min(_group_candidates(auto_group, ns), key=lambda x: us[f"full_group{x}"])
    ctx.close()
    return {"step_kernel": step_kernel,
            "steps_per_launch": best_full[0], "tile_z": best_full[1], "tile_loop": best_full[2],
            "strip": best_full[3], "shot_group": group,
            "steps_per_launch_slab": best_slab[0], "tile_z_slab": best_slab[1],
            "slab_strip": best_slab[3], "shot_group_slab": group_slab, "us": us}


def choose(prob, kappa, rho, xs=None, field_dtype="f32", cache_path: str | None = DEFAULT_CACHE,
           retune: bool = False, **kw) -> dict:
    """Cached :func:`tune` keyed by :func:`shape_key`."""
    xs = tuple(prob.xs) if xs is None else tuple(xs)
    key = shape_key(prob, len(xs), field_dtype, np.ndim(rho) != 0)
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
    """Set a context's step kernel, tile heights, steps per launch and shot
    groups from a tuning result."""
    ctx.set_option(OPT_STEP_KERNEL, int(choice["step_kernel"]))
    ctx.set_option(OPT_TILE_Z, int(choice["tile_z"]))
    ctx.set_option(OPT_TILE_Z_SLAB, int(choice["tile_z_slab"]))
    # steps per launch and strip width are checked together: strips back to
    # their defaults first
    ctx.set_option(OPT_STRIP, 0)
    ctx.set_option(OPT_SLAB_STRIP, 0)
    ctx.set_option(OPT_STEPS_PER_LAUNCH, int(choice.get("steps_per_launch", 1)))
    ctx.set_option(OPT_STEPS_PER_LAUNCH_SLAB, int(choice.get("steps_per_launch_slab", 1)))
    ctx.set_option(OPT_STRIP, int(choice.get("strip", 0)))
    ctx.set_option(OPT_SLAB_STRIP, int(choice.get("slab_strip", 0)))
    ctx.set_option(OPT_SHOT_GROUP, int(choice.get("shot_group", 0)))
    ctx.set_option(OPT_SHOT_GROUP_SLAB, int(choice.get("shot_group_slab", 0)))
    ctx.set_option(OPT_TILE_LOOP, int(choice.get("tile_loop", 0)))
