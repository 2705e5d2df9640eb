"""Autotuner for the decoders' launch knobs and schedules.

Knobs that cannot change any output bit (``tune_mixed``, ``tune_decode``):

* workgroup size of the flooding and layered decoders,
* for the mixed-shape persistent decoder, the workgroup size and the number
  of codewords of each shape that share one workgroup (tile),
* persistent work list vs one workgroup per tile.

Every candidate is timed with HIP events on the current stream and its
output is compared bit for bit with the first (reference) candidate; a
candidate that disagrees is rejected (it would mean a kernel bug).  The
winner is cached in a JSON file keyed by the code shapes, counts and
decoder parameters (no cache unless a path is given).

``tune_schedule`` also tunes knobs that change results: per shape of a
mixed batch, the layered normalized min-sum decoder (FP32, the default) or
the flooding int8 offset min-sum decoder; and where the layered decoder
keeps its check records (LDS or device memory, result-invariant).  A shape
may move to offset min-sum only if its block error rate on the plan's data
lies inside the default decoder's Wilson 95% interval on the same data.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import MixedPlan, decode, params as make_params  # noqa: F401



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


def tune_mixed(codes, counts, p, llr_concat, cache_path: str | None = None,
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


def tune_decode(code, llr, p, cache_path: str | None = None, reps: int = 3,
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
        q = params(p.algo, p.iters, p.offset, p.alpha, p.llr_max, p.sat, t, p.lds_rows)
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


def wilson(k: int, n: int, z: float = 1.959963984540054):
    """Wilson score interval of a binomial proportion k / n."""
    if n <= 0:
        return 0.0, 1.0
    p = k / n
    den = 1.0 + z * z / n
    mid = (p + z * z / (2 * n)) / den
    half = z * ((p * (1 - p) / n + z * z / (4 * n * n)) ** 0.5) / den
    return max(0.0, mid - half), min(1.0, mid + half)


def oms_fits(code) -> bool:
    """The flooding int8 decoder keeps a tile's whole state in LDS: 2 bytes
    per edge and per variable node for one codeword (4 for a pair)."""
    return 2 * (code.E + code.n_dec) <= 160 * 1024 - 96


class ScheduledMixed:
    """A mixed batch decoded under a schedule: the shapes marked "nms" in one
    persistent layered-NMS launch, the shapes marked "oms" quantized and
    decoded in one persistent int8 offset min-sum launch.  LLRs come per
    shape (f32 [count][e_tx]); bits go out per shape."""

    def __init__(self, codes, counts, schedule, p_nms, p_oms, threads: int = 0):
        from . import MixedPlan
        self.codes, self.counts, self.schedule = list(codes), list(counts), list(schedule)
        self.nms_idx = [s for s, a in enumerate(schedule) if a == "nms"]
        self.oms_idx = [s for s, a in enumerate(schedule) if a == "oms"]
        self.nplan = (MixedPlan([codes[s] for s in self.nms_idx], [counts[s] for s in self.nms_idx],
                                p_nms, threads=threads) if self.nms_idx else None)
        self.oplan = (MixedPlan([codes[s] for s in self.oms_idx], [counts[s] for s in self.oms_idx],
                                p_oms) if self.oms_idx else None)
        self.p_oms = p_oms
        self.nwork = self.nplan.workspace() if self.nplan else None
        self.owork = self.oplan.workspace() if self.oplan else None

    def inputs(self, parts):
        """The launches' concatenated inputs from per-shape f32 LLRs (the int8
        ones are filled by ``decode``)."""
        f = torch.cat([parts[s].reshape(-1) for s in self.nms_idx]) if self.nms_idx else None
        o = torch.cat([parts[s].reshape(-1) for s in self.oms_idx]) if self.oms_idx else None
        q = torch.empty(o.shape, dtype=torch.int8, device=o.device) if o is not None else None
        nb = (torch.empty(self.nplan.n_bits, dtype=torch.uint8, device=parts[0].device)
              if self.nplan else None)
        ob = (torch.empty(self.oplan.n_bits, dtype=torch.uint8, device=parts[0].device)
              if self.oplan else None)
        return {"f32": f, "oms_f32": o, "oms_q": q, "nms_bits": nb, "oms_bits": ob}

    def decode(self, io, persistent=True):
        from . import quantize
        if self.nplan:
            self.nplan.decode(io["f32"], bits=io["nms_bits"], work=self.nwork, persistent=persistent)
        if self.oplan:
            quantize(io["oms_f32"], 2.0, self.p_oms.sat, out=io["oms_q"])
            self.oplan.decode(io["oms_q"], bits=io["oms_bits"], work=self.owork,
                              persistent=persistent)

    def bits(self, io):
        """Per-shape views of the decoded bits."""
        out = [None] * len(self.codes)
        for plan, idx, key in ((self.nplan, self.nms_idx, "nms_bits"),
                               (self.oplan, self.oms_idx, "oms_bits")):
            if plan is None:
                continue
            for j, s in enumerate(idx):
                o = plan.bits_offsets[j]
                out[s] = io[key][o:o + self.counts[s] * self.codes[s].k].view(self.counts[s], -1)
        return out


def _block_errors(ref, hat):
    return int((ref != hat).any(dim=1).sum().item())


def tune_layer_order(code, llr, ref_bits, p, reps: int = 5, rounds: int = 3):
    """Layer order of one code for the layered decoder: natural (the
    default) or grouped.  The grouped order is accepted only if its block
    error rate on (llr, ref_bits) lies inside the natural order's Wilson 95%
    interval on the same frames, and taken only if it decodes faster (median
    over `rounds` interleaved timings of `reps` launches).  Leaves the chosen
    order set on the code and returns both orders' block errors, barriers
    per iteration and times."""
    from . import decode, decode_workspace
    n = int(llr.shape[0])
    work = torch.empty(max(1, decode_workspace(code, p, n)), dtype=torch.uint8, device=llr.device)
    bits = torch.empty((n, code.k), dtype=torch.uint8, device=llr.device)
    out = {"codewords": n}
    times = {"natural": [], "grouped": []}
    for r in range(rounds):
        for order in ("natural", "grouped"):
            code.set_layer_order(order)
            if r == 0:
                b, _ = decode(code, llr, p, bits=bits, work=work)
                out[order] = {"block_errors": _block_errors(ref_bits, b),
                              "barriers_per_iteration": code.layer_order()[1]}
            times[order].append(_time(lambda: decode(code, llr, p, bits=bits, work=work), reps))
    for order in times:
        out[order]["ms"] = round(sorted(times[order])[len(times[order]) // 2], 4)
    lo, hi = wilson(out["natural"]["block_errors"], n)
    acc = bool(lo - 1e-12 <= out["grouped"]["block_errors"] / n <= hi + 1e-12)
    out["natural_ci95"] = [round(lo, 5), round(hi, 5)]
    out["grouped_accepted"] = acc
    out["chosen"] = "grouped" if acc and out["grouped"]["ms"] < out["natural"]["ms"] else "natural"
    code.set_layer_order(out["chosen"])
    return out


def tune_schedule(codes, counts, parts, ref_bits, p_nms, p_oms=None, reps: int = 3,
                  verbose: bool = False):
    """Schedule (decoder and layer order per shape) and placement for a
    mixed batch.

    parts: per-shape f32 LLRs [count][e_tx]; ref_bits: per-shape transmitted
    information bits [count][k].  Returns the chosen schedule, the layer
    order of every shape ("natural" or "grouped", left set on the codes),
    the NMS plan's lds_rows setting, per-shape block errors of every
    candidate decoder with the default's (natural-order NMS) Wilson
    interval, and the time of every candidate timed.  Candidates start from
    every shape on natural-order layered NMS; shapes whose grouped-order or
    offset min-sum BLER is accepted are changed one knob at a time, heaviest
    first, and a change is kept when the schedule gets faster."""
    from . import OMS_I8, decode, decode_workspace, params, quantize
    if p_oms is None:
        p_oms = params(OMS_I8, iters=p_nms.iters, offset=1, sat=31)
    dev = parts[0].device
    for code in codes:
        code.set_layer_order("natural")
    per_shape = []
    for s, (code, x, u) in enumerate(zip(codes, parts, ref_bits)):
        n = int(counts[s])
        work = torch.empty(max(1, decode_workspace(code, p_nms, n)), dtype=torch.uint8, device=dev)
        bn, _ = decode(code, x, p_nms, work=work)
        en = _block_errors(u, bn)
        lo, hi = wilson(en, n)
        info = {"shape": s, "Z": code.Z, "codewords": n, "nms_block_errors": en,
                "nms_ci95": [round(lo, 5), round(hi, 5)], "oms_fits": oms_fits(code)}
        code.set_layer_order("grouped")
        info["grouped_barriers"] = code.layer_order()[1]
        bg, _ = decode(code, x, p_nms, work=work)
        code.set_layer_order("natural")
        info["natural_barriers"] = code.layer_order()[1]
        eg = _block_errors(u, bg)
        info["grouped_block_errors"] = eg
        info["grouped_accepted"] = bool(lo - 1e-12 <= eg / n <= hi + 1e-12)
        if info["oms_fits"]:
            bo, _ = decode(code, quantize(x, 2.0, p_oms.sat), p_oms)
            eo = _block_errors(u, bo)
            info["oms_block_errors"] = eo
            info["oms_accepted"] = bool(lo - 1e-12 <= eo / n <= hi + 1e-12)
        else:
            info["oms_accepted"] = False
        per_shape.append(info)

    def timed(schedule, lds_rows):
        pn = params(p_nms.algo, p_nms.iters, p_nms.offset, p_nms.alpha, p_nms.llr_max, p_nms.sat,
                    p_nms.threads, lds_rows)
        sm = ScheduledMixed(codes, counts, schedule, pn, p_oms)
        io = sm.inputs(parts)
        return _time(lambda: sm.decode(io), reps), sm, io

    tried = []
    best_lds, best_t = 0, None
    base = ["nms"] * len(codes)
    orders = ["natural"] * len(codes)
    for lds_rows in (0, -1):
        t, _, _ = timed(base, lds_rows)
        tried.append({"schedule": list(base), "layer_order": list(orders), "lds_rows": lds_rows,
                      "ms": round(t, 4)})
        if best_t is None or t < best_t:
            best_t, best_lds = t, lds_rows
    schedule = list(base)
    # one knob at a time, heaviest shape first: the grouped layer order
    # (for a shape still on NMS), then offset min-sum
    heavy = sorted(per_shape, key=lambda i: -i["codewords"] * codes[i["shape"]].E)
    moves = [(i["shape"], "grouped") for i in heavy if i["grouped_accepted"]]
    moves += [(i["shape"], "oms") for i in heavy if i["oms_accepted"]]
    for sh, knob in moves:
        cand, cord = list(schedule), list(orders)
        if knob == "grouped":
            if cand[sh] != "nms" or cord[sh] == "grouped":
                continue
            cord[sh] = "grouped"
            codes[sh].set_layer_order("grouped")
        else:
            cand[sh] = "oms"          # the layer order applies to NMS only
            cord[sh] = "natural"
            codes[sh].set_layer_order("natural")
        t, _, _ = timed(cand, best_lds)
        tried.append({"schedule": cand, "layer_order": cord, "lds_rows": best_lds,
                      "ms": round(t, 4)})
        if verbose:
            print(tried[-1], flush=True)
        if t < best_t:
            best_t, schedule, orders = t, cand, cord
        else:
            codes[sh].set_layer_order(orders[sh])
    return {"schedule": schedule, "layer_order": orders, "lds_rows": best_lds,
            "ms": round(best_t, 4), "shapes": per_shape, "tried": tried}
