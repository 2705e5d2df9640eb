"""Autotuner for the decoders' result-invariant launch knobs.

Knobs that cannot change any output bit:

* workgroup size of the flooding and layered decoders,
* for the mixed-shape persistent decoder, the workgroup size and the number
  of codewords of each shape that share one workgroup (tile),
* persistent work list vs one workgroup per tile.

Every candidate is timed with HIP events on the current stream and its
output is compared bit for bit with the first (reference) candidate; a
candidate that disagrees is rejected (it would mean a kernel bug).  The
winner is cached in a JSON file keyed by the code shapes, counts and
decoder parameters.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import MixedPlan, decode, params as make_params  # noqa: F401

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _key(parts) -> str:
    return hashlib.sha1(json.dumps(parts, sort_keys=True).encode()).hexdigest()[:16]


def _load(path):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, cache):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, reps=3):
    fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _tile_options(Z, threads):
    g = max(1, threads // Z)
    opts = sorted({g, max(1, g // 2), 1})
    return opts


def tune_mixed(codes, counts, p, llr_concat, cache_path: str | None = DEFAULT_CACHE,
               threads_options=(384, 512, 768, 1024), reps: int = 3, verbose: bool = False):
    """Best (threads, codewords_per_tile, persistent) for a mixed batch.
    For the int8 offset min-sum decoder the tile is always a codeword pair
    and the workgroup sizes are 256, 512 and 1024."""
    from . import OMS_I8
    oms = p.algo == OMS_I8
    if oms:
        threads_options = (256, 512, 1024)
    zmax = max(c.Z for c in codes)
    key = _key(["mixed", [(c.Z, c.rows, c.cols, c.E, c.e_tx) for c in codes], list(counts),
                [p.algo, p.iters, p.alpha, p.offset, p.sat]])
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        return cache[key]
    ref_bits = None
    best = None
    n_bits = sum(int(k) * c.k for c, k in zip(codes, counts))
    for threads in threads_options:
        if not oms and threads < zmax:
            continue
        # uniform tile shrink factors keep the search small
        for shrink in ((1,) if oms else (1, 2)):
            cpt = ([2] * len(codes) if oms
                   else [max(1, (threads // c.Z) // shrink) for c in codes])
            try:
                plan = MixedPlan(codes, counts, p, codewords_per_tile=cpt, threads=threads)
            except Exception:
                continue
            work = plan.workspace(llr_concat.device)
            for persistent in (True, False):
                bits = torch.zeros(n_bits, dtype=torch.uint8, device=llr_concat.device)
                ms = _time(lambda: plan.decode(llr_concat, bits=bits, work=work,
                                               persistent=persistent), reps)
                if ref_bits is None:
                    ref_bits = bits.clone()
                elif not torch.equal(bits, ref_bits):
                    raise RuntimeError(f"result changed under threads={threads} tiles={cpt}")
                cand = {"threads": threads, "codewords_per_tile": cpt, "persistent": persistent,
                        "ms": ms}
                if verbose:
                    print(cand, flush=True)
                if best is None or ms < best["ms"]:
                    best = cand
    if cache_path:
        cache[key] = best
        _store(cache_path, cache)
    return best


def tune_decode(code, llr, p, cache_path: str | None = DEFAULT_CACHE, reps: int = 3,
                verbose: bool = False):
    """Best workgroup size for lsim_decode of one code."""
    from . import NMS_F32, params, decode_workspace
    key = _key(["decode", code.Z, code.rows, code.cols, code.E, int(llr.shape[0]), p.algo, p.iters])
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        return cache[key]
    opts = (256, 384, 512, 768, 1024) if p.algo == NMS_F32 else (256, 512, 1024)
    best, ref = None, None
    for t in opts:
        if p.algo == NMS_F32 and t < code.Z:
            continue
        q = params(p.algo, p.iters, p.offset, p.alpha, p.llr_max, p.sat, t)
        work = None
        nb = decode_workspace(code, q, llr.shape[0])
        if nb:
            work = torch.empty(nb, dtype=torch.uint8, device=llr.device)
        bits = torch.empty((llr.shape[0], code.k), dtype=torch.uint8, device=llr.device)
        try:
            ms = _time(lambda: decode(code, llr, q, bits=bits, work=work), reps)
        except Exception:
            continue
        if ref is None:
            ref = bits.clone()
        elif not torch.equal(ref, bits):
            raise RuntimeError(f"result changed under threads={t}")
        if verbose:
            print({"threads": t, "ms": ms}, flush=True)
        if best is None or ms < best["ms"]:
            best = {"threads": t, "ms": ms}
    if cache_path:
        cache[key] = best
        _store(cache_path, cache)
    return best
