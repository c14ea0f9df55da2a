"""Launch-configuration tuner of the step kernel and of the batch engine.

The step has five kernel variants: plain (one site per thread over the flat
site index), rows (a block covers tile_x consecutive x of tile_rows rows),
flat (256 tile_rows consecutive sites of the x-fastest order per block),
resident (a whole small lattice in one workgroup's LDS) and two (two steps
per pass over row tiles with a one-site halo).
All variants compute every site with the same arithmetic in the same order,
so their results are bit-identical; the tuner times each candidate on the
GPU, keeps only candidates whose state after a few steps is bit-identical
to the plain variant's, and stores the fastest per (model, precision,
size class) in a JSON cache next to this file (or FLB_TUNE_CACHE).
"""

import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("FLB_TUNE_CACHE", os.path.join(HERE, "tuned.json"))

DEFAULTS = {1: dict(kernel="rows", tile_x=256, tile_rows=1, nt_store=0),
            2: dict(kernel="rows", tile_x=256, tile_rows=4, nt_store=0),
            3: dict(kernel="rows", tile_x=256, tile_rows=4, nt_store=0)}

CANDIDATES = ([("plain", 0, 0, 0, 0), ("resident", 0, 0, 0, 0)] +
              [("two", 0, ty, nt, 0) for ty in (4, 8, 16) for nt in (0, 1)] +
              [("flat", 0, ry, nt, 0) for ry in (1, 2, 4, 8) for nt in (0, 1)] +
              [("rows", tx, ry, nt, 0) for tx in (64, 128, 256, 512, 1024) for ry in (1, 2, 4, 8, 16)
               for nt in (0, 1)] +
              [("rows", tx, ry, nt, 1) for tx in (128, 256, 512) for ry in (2, 4, 8, 16) for nt in (0, 1)])
QUICK = ([("plain", 0, 0, 0, 0), ("resident", 0, 0, 0, 0), ("two", 0, 8, 1, 0), ("two", 0, 16, 1, 0)] +
         [("flat", 0, ry, nt, 0) for ry in (1, 2, 4) for nt in (0, 1)] +
         [("rows", tx, ry, 1, 0) for tx in (256, 512) for ry in (1, 2, 4)])


def size_class(dims):
    """tiny lattices (up to 4096 sites) may be resident in one workgroup's LDS"""
    n = int(np.prod(dims))
    if n <= 4096:
        return "tiny"
    return "small" if n < (1 << 16) else ("medium" if n < (1 << 22) else "large")


def _key(d, precision, dims):
    return f"D{d}-fp{8 * precision}-{size_class(dims)}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def best_config(d, precision, dims, layout="two"):
    """Kernel keyword arguments for a lattice: the cached tuning result, or
    the defaults.  The two-step and flat kernels address a population plane
    with 32-bit byte offsets and accept only Q N precision < 2^32; larger
    lattices of a size class tuned to one of them take the defaults.  The
    single-buffer AA layout steps with the flat kernel (resident when tiny):
    its tiles follow a tuned flat entry, else the flat defaults."""
    ent = _load().get(_key(d, precision, dims))
    if layout == "aa":
        if size_class(dims) == "tiny":
            return dict(kernel="auto", layout="aa")
        ry = ent["tile_rows"] if ent and ent["kernel"] == "flat" else (2 if d == 2 else 1)
        return dict(kernel="flat", tile_rows=ry, nt_store=1, layout="aa")
    if size_class(dims) == "tiny" and (not ent or ent["kernel"] == "resident"):
        return dict(kernel="auto")      # resident when the lattice fits the LDS, else rows
    if ent and ent["kernel"] in ("two", "flat") and (2 * d + 1) * int(np.prod(dims)) * precision >= 1 << 32:
        ent = None
    if ent:
        return dict(kernel=ent["kernel"], tile_x=ent["tile_x"], tile_rows=ent["tile_rows"],
                    nt_store=ent.get("nt_store", 0), pipeline=ent.get("pipeline", 0))
    return dict(DEFAULTS[d])


def tune(d, precision, dims, steps=100, candidates=None, write=True, verbose=True):
    """Time every candidate on `dims` and cache the fastest bit-identical one
    (candidates "quick" = a short list of the shapes that have won before)."""
    if candidates == "quick":
        candidates = QUICK
    import torch
    from . import flb, inputs

    w, _ = flb.constants(d)
    f0 = inputs.poisson_counts(dims, 10.0 * w, seed=0).astype(np.float32 if precision == 4 else np.float64)
    ref = None
    results = []
    for cand in (candidates or CANDIDATES):
        kern, tx, ry, nt = cand[:4]
        pp = cand[4] if len(cand) > 4 else 0
        if d == 1 and ry > 1:
            continue
        try:
            L = flb.Lattice(d, dims, precision=precision, omega=1.0, seed=0, kernel=kern, tile_x=tx,
                            tile_rows=ry, nt_store=nt, pipeline=pp)
        except flb.FlbError:          # the resident kernel on a lattice that does not fit
            continue
        L.set_populations(f0)
        L.step(3)
        state = L.get_populations()
        if ref is None:
            ref = state
        same = np.array_equal(state.view(np.uint8), ref.view(np.uint8))
        st = L.stream
        L.step(max(steps // 2, 5))                  # let clocks settle
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        L.step(steps)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        L.close()
        results.append(dict(kernel=kern, tile_x=tx, tile_rows=ry, nt_store=nt, pipeline=pp, ms=ms,
                            identical=bool(same)))
        if verbose:
            print(f"[tune] D{d} fp{8 * precision} {dims} {kern} {tx}x{ry} nt={nt} pipe={pp}: {ms * 1e3:.1f} us/step"
                  f"{'' if same else '  (NOT bit-identical: rejected)'}", flush=True)
    ok = [r for r in results if r["identical"]]
    best = min(ok, key=lambda r: r["ms"])
    if write:
        cache = _load()
        cache[_key(d, precision, dims)] = dict(best, dims=list(dims), when=time.strftime("%Y-%m-%d %H:%M"))
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best, results


BATCH_DEFAULT = {"depth": 2, "tiling": 0, "chunk": 16, "width": 256}


def batch_config():
    """Options of flb.Batch for ensembles: the cached batch tuning result
    (temporal-blocking depth of the D2Q5 members and the width of their
    two-step tiles, work-item tiling, graph chunk), or the defaults."""
    ent = _load().get("batch")
    return {k: int(ent.get(k, v)) for k, v in BATCH_DEFAULT.items()} if ent else dict(BATCH_DEFAULT)


def pick_batch(results, within=0.01):
    """The batch option to cache from timed results: among those within
    `within` of the fastest, whole-member tiles (tiling 0) first, then the
    fastest.  The tuning ensemble may not hold every lattice kind a batch
    later serves, and row tiles lose on D3Q7 members, so a near-tie is not
    allowed to pick them."""
    fastest = min(r["ms"] for r in results)
    near = [r for r in results if r["ms"] <= fastest * (1 + within)]
    return min(near, key=lambda r: (r["tiling"] != 0, r["ms"]))


def _time_batch(make_members, steps, opts):
    """ms per step of a batch of make_members() with options opts."""
    from . import flb

    lats = make_members()
    B = flb.Batch(**opts)
    for L in lats:
        B.admit(L)
    B.step(2 * opts["chunk"])
    B.sync()
    t0 = time.perf_counter()
    B.step(steps)
    B.sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for L in lats:
        B.retire(L)
        L.close()
    B.close()
    return ms


def tune_batch(make_members, steps=400, depths=(1, 2), tilings=(0, 1), chunks=(8, 16, 32),
               widths=(256, 128, 64), write=True, verbose=True):
    """Time the batch options on the ensemble make_members() builds (a list
    of lattices with their state set) and cache the fastest.  Members are
    bit-identical under every option, so only the time decides.  The
    two-step tile width only matters at depth 2."""
    results = []
    for depth in depths:
        for width in (widths if depth == 2 else (256,)):
            for tiling in tilings:
                for chunk in chunks:
                    ms = _time_batch(make_members, steps, dict(chunk=chunk, tiling=tiling, depth=depth,
                                                               width=width))
                    results.append(dict(depth=depth, width=width, tiling=tiling, chunk=chunk, ms=ms))
                    if verbose:
                        print(f"[tune] batch depth={depth} width={width} tiling={tiling} chunk={chunk}: "
                              f"{ms * 1e3:.1f} us/step", flush=True)
    best = pick_batch(results)
    if write:
        cache = _load()
        cache["batch"] = dict(best, when=time.strftime("%Y-%m-%d %H:%M"))
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best, results
