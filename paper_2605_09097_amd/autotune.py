"""Tile-shape autotuner.

The tile shape of a domain (cells per workgroup tile) sets the LDS region of
the P2G, tangent and CG kernels, the number of workgroups per launch and the
halo overhead: small tiles give more workgroups (latency hiding when a domain
is small), large tiles fewer and fuller ones (better when many scenes share a
launch).  The best shape depends on the workload, so it is measured: each
candidate runs the same frames on fresh domains and the fastest wins.  The
timed frames are whole Schwarz frames through the C ABI; only the tile shape
differs between candidates.  Each candidate's domains can first be advanced
a few untimed frames (`advance`), so that the timed frames are past the
start-up transient of the scene.

Results can be kept in a JSON file (`cache`, or the file named by the
environment variable OSMPM_TILE_CACHE) keyed by a signature of the problem:
the device, the library build, the precision and Schwarz options, and every
domain's dimension, particle count and grid.  A later call with the same
signature returns the stored choice without measuring.
"""
import hashlib
import json
import os
import time

from . import binding

CANDIDATES_2D = [(4, 4), (8, 4), (8, 8), (16, 8), (16, 16)]
CANDIDATES_3D = [(4, 4, 2), (4, 4, 4), (8, 4, 4), (8, 8, 4)]


def _frames(run_frame, warmup, frames, torch):
    for _ in range(warmup):
        run_frame()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(frames):
        run_frame()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / frames


def _lib_digest():
    try:
        st = os.stat(binding.LIB_PATH)
        return "%d-%d" % (st.st_size, int(st.st_mtime))
    except OSError:
        return "none"


def signature(kind, scenes, opts, precision, candidates, advance):
    """Key of a tuning problem (see the module docstring)."""
    import torch

    # the device by compute-unit count and memory size (its name string is
    # not reported the same way under every tool)
    dev = "cpu"
    if torch.cuda.is_available():
        pr = torch.cuda.get_device_properties(0)
        dev = "%d-%d" % (pr.multi_processor_count, pr.total_memory)
    parts = [kind, dev, _lib_digest(),
             "prec%d" % precision, "M%d" % opts.M, "warm%d" % getattr(opts, "warm_start", 0),
             "adv%d" % advance, repr([tuple(c) for c in candidates])]
    for sc in scenes:
        for spec in (sc.B, sc.S):
            parts.append("%d:%d:%s:%d" % (spec.dim, len(spec.x), list(spec.n_nodes), spec.dx_q))
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:24]


def _cache_file(cache):
    return cache if cache is not None else os.environ.get("OSMPM_TILE_CACHE")


def _cache_get(path, key):
    if not path or not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def _cache_put(path, key, value):
    if not path:
        return
    data = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
    data[key] = value
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_pair(ctx, scene, opts, precision=binding.OSMPM_FP64, candidates=None, warmup=1, frames=2, advance=0,
              cache=None):
    """Best (tile_B, tile_S) for one coarse/fine pair, searching the two sides
    one after the other (coarse with the default fine tile, then fine with the
    chosen coarse tile).  Returns (tile_B, tile_S, {description: seconds});
    the timings are empty when the choice came from the cache."""
    import torch

    cands = candidates or (CANDIDATES_2D if scene.B.dim == 2 else CANDIDATES_3D)
    path = _cache_file(cache)
    key = signature("pair", [scene], opts, precision, cands, advance)
    hit = _cache_get(path, key)
    if hit is not None:
        return tuple(hit["tile_B"]), tuple(hit["tile_S"]), {}
    timings = {}

    def measure(tB, tS):
        k = "B%s S%s" % (tB, tS)
        if k not in timings:
            pair = binding.SchwarzPair(ctx, scene, precision, tile_B=tB, tile_S=tS)
            try:
                for _ in range(advance):
                    pair.frame(opts)
                timings[k] = _frames(lambda: pair.frame(opts), warmup, frames, torch)
            finally:
                pair.close()
        return timings[k]

    default = cands[len(cands) // 2]
    tB = min(cands, key=lambda t: measure(t, default))
    tS = min(cands, key=lambda t: measure(tB, t))
    _cache_put(path, key, {"tile_B": list(tB), "tile_S": list(tS), "timings": timings})
    return tB, tS, timings


def tune_batch(ctx, scenes, opts, precision=binding.OSMPM_FP64, candidates=None, warmup=1, frames=1, advance=0,
               cache=None):
    """Best single tile shape for every domain of a Schwarz batch of the
    given scenes.  Returns (tile, {tile: seconds per frame}); the timings are
    empty when the choice came from the cache."""
    import torch

    cands = candidates or (CANDIDATES_2D if scenes[0].B.dim == 2 else CANDIDATES_3D)
    path = _cache_file(cache)
    key = signature("batch", scenes, opts, precision, cands, advance)
    hit = _cache_get(path, key)
    if hit is not None:
        return tuple(hit["tile"]), {}
    timings = {}
    for t in cands:
        sb = binding.SchwarzBatch(ctx, scenes, precision=precision, tile=t)
        try:
            for _ in range(advance):
                sb.frame(opts)
            timings[t] = _frames(lambda: sb.frame(opts), warmup, frames, torch)
        finally:
            sb.close()
    best = min(timings, key=timings.get)
    _cache_put(path, key, {"tile": list(best), "timings": {"%s" % (k,): v for k, v in timings.items()}})
    return best, timings
