"""Autotuner for the build's launch options.

The knobs change only speed, never results (every cell is certified by its security radius
whatever the search does):
  * ``k_init`` -- the first search shell, as the number of particles it holds on average (the
    paper's equivalent is the buffer thickness, section 2: too thin needs more passes, too thick
    wastes work);
  * ``pts_per_grid_cell`` -- the resolution of the uniform-grid (Morton level) table the kNN
    search walks: about this many particles per finest cell;
  * ``waves_per_cu`` -- how many wavefronts (one cell each) the persistent clipping kernel keeps
    resident per compute unit;
  * ``cell_mapping`` -- the wavefront-to-cell mapping: each XCD (its own L2) takes a contiguous
    eighth of the cells in Morton order and then helps the others (``VT_MAP_XCD``), or one queue
    deals consecutive cells to wavefronts on every XCD in turn (``VT_MAP_GLOBAL``).

``tune`` times ``vt_build`` with device events for each candidate on the caller's inputs (or a
representative subset of items), keeps the fastest, and caches the choice per input signature
for the life of the process.
"""
from __future__ import annotations

import itertools

K_INITS = (24, 34, 50)
PTS_PER_GRID_CELL = (1.0, 0.125, 1.0 / 64)
WAVES_PER_CU = (12, 16)
CELL_MAPPINGS = (0, 1)  # VT_MAP_XCD, VT_MAP_GLOBAL

_cache = {}


def candidates(k_inits=K_INITS, pts_per_grid_cell=PTS_PER_GRID_CELL, waves_per_cu=WAVES_PER_CU,
               cell_mappings=CELL_MAPPINGS):
    return [dict(k_init=int(k), pts_per_grid_cell=float(g), waves_per_cu=int(w), cell_mapping=int(m))
            for k, g, w, m in itertools.product(k_inits, pts_per_grid_cell, waves_per_cu, cell_mappings)]


def signature(device_name, dtype, n_total, n_items, precision):
    """Inputs that share a signature share tuned options (sizes bucketed to powers of two)."""
    return (str(device_name), str(dtype), max(int(n_total), 1).bit_length(), max(int(n_items), 1).bit_length(),
            int(precision))


def pick(timings):
    """The fastest candidate: ``timings`` is a list of (options, milliseconds); ties keep the
    earlier candidate."""
    if not timings:
        raise ValueError("no timings")
    best = min(range(len(timings)), key=lambda k: (timings[k][1], k))
    return dict(timings[best][0])


def tune(ctx_factory, pos, items, global_id=None, precision=0, reps=2, cands=None, use_cache=True):
    """Time each candidate with ``reps`` builds after one warm-up; return (options, timings).

    ``ctx_factory`` makes a fresh ``Context``; builds are timed with events on the current
    stream, so the result reflects device time only.
    """
    import torch

    key = signature(torch.cuda.get_device_name(pos.device), pos.dtype, pos.shape[0], len(items), precision)
    if use_cache and key in _cache:
        return dict(_cache[key]), []
    timings = []
    for opts in (cands or candidates()):
        ctx = ctx_factory()
        ctx.vt_build(pos, items, global_id=global_id, precision=precision, **opts)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            ctx.vt_build(pos, items, global_id=global_id, precision=precision, **opts)
        stop.record()
        stop.synchronize()
        code = ctx.vt_query()[0]
        if code == 0:
            timings.append((opts, start.elapsed_time(stop) / reps))
        del ctx
    best = pick(timings)
    _cache[key] = best
    return dict(best), timings
