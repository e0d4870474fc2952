"""Tile-shape autotuner for the two stencil kernel classes.

For a grid and precision, every compiled tile shape of the reverse-stage kernel (timed through
``vjp``) and of the primal-stage kernel (timed through whole RK steps, ``primal_step``: the
residual alone can rank the tiles otherwise than the stage launches a step makes, whose stage
updates and final combination change the kernel's registers and stores) is run on the device
with HIP events, and the fastest is installed with ``set_tile``.  Results are cached in a JSON file
keyed by library build, kernel class, precision, grid shape and boundary type, so a process pays
for the search once per configuration.
"""
import json
import os

import torch

from . import (F64, PROF_ADJOINT_STAGE, PROF_PRIMAL_STAGE, SSPRK3, TILES, get_tile, primal_step, set_tile,
               tile_launched, vjp, workspace)

CACHE = os.environ.get("ADJNS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "adjns_tiles.json"))


def _build_id():
    """Size and modification time of the loaded library: a rebuilt library re-tunes."""
    from . import LIB_PATH
    st = os.stat(LIB_PATH)
    return f"{st.st_size}-{int(st.st_mtime)}"


def _key(g, kclass):
    # the cache is per machine: no device name (a profiler-wrapped process may not see it)
    return f"{_build_id()}|{'adjoint' if kclass == PROF_ADJOINT_STAGE else 'primal'}|" \
           f"{'f64' if g.precision == F64 else 'f32'}|{g.n[0]}x{g.n[1]}x{g.n[2]}|bc{g.bc_x}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _state(g, seed):
    """A smooth positive-density state and a random adjoint field of the grid's shape."""
    gen = torch.Generator(device="cuda").manual_seed(seed)
    N = g.ncells
    w = torch.empty(5, N, dtype=g.dtype, device="cuda")
    w[0] = 1.0 + 0.05 * torch.rand(N, generator=gen, device="cuda", dtype=g.dtype)
    w[1:4] = 0.1 * torch.randn(3, N, generator=gen, device="cuda", dtype=g.dtype)
    w[4] = 2.5 + 0.05 * torch.rand(N, generator=gen, device="cuda", dtype=g.dtype)
    kh = torch.randn(5 * N, generator=gen, device="cuda", dtype=g.dtype)
    return w.reshape(-1).contiguous(), kh


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(g, reps=20, use_cache=True, verbose=False, rounds=3, margin=0.03):
    """Pick and install the fastest tile of both kernel classes for grid g; returns
    {kernel_class: (tile_id, {tile_id: ms})} (primal class: ms per stage of an RK step).  Every tile is timed in `rounds` interleaved rounds
    (best round kept); the tile installed before tuning stays unless another is faster by more
    than `margin`, so that near-ties do not flip between runs."""
    db = _load() if use_cache else {}
    out = {}
    w, kh = _state(g, 0)
    buf = torch.empty_like(w)
    ws = None
    for kclass in (PROF_ADJOINT_STAGE, PROF_PRIMAL_STAGE):
        key = _key(g, kclass)
        if use_cache and key in db:
            set_tile(kclass, g.precision, db[key]["tile"])
            out[kclass] = (db[key]["tile"], {int(k): v for k, v in db[key]["ms"].items()})
            continue
        prev = get_tile(kclass, g.precision)
        # only tiles that launch as themselves (the others run as a smaller tile already timed)
        cands = [t for t in TILES if tile_launched(kclass, g.precision, g.bc_x, False, t) == t]
        times = {}
        for _ in range(rounds):
            for t in cands:
                set_tile(kclass, g.precision, t)
                if kclass == PROF_ADJOINT_STAGE:
                    ms = _time(lambda: vjp(g, w, kh, buf), reps)
                else:
                    ws = workspace(g) if ws is None else ws
                    # time per stage of an RK step (one stage-kernel launch each)
                    nst = 3 if g.time_scheme == SSPRK3 else 4
                    ms = _time(lambda: primal_step(g, w, None, buf, ws), max(1, reps // nst)) / nst
                times[t] = min(times.get(t, ms), ms)
        best = min(times, key=times.get) if times else prev
        if prev in times and times[prev] <= (1.0 + margin) * times[best]:
            best = prev
        set_tile(kclass, g.precision, best)
        out[kclass] = (best, times)
        db[key] = {"tile": best, "ms": times}
        if verbose:
            print(f"[autotune] {key}: " + ", ".join(f"{TILES[t]} {ms * 1e3:.1f} us" for t, ms in times.items()),
                  flush=True)
    if use_cache:
        _store(db)
    # the timing buffers go back to the device, so that a plan sized from free memory sees them
    del w, kh, buf, ws
    torch.cuda.empty_cache()
    return out
