"""Throughput of the LDPC link hot path on one MI355X.

One step = one batch of the BG2-shaped workload through the whole link:
Philox information bits -> QC encoder -> Gray 16-QAM + AWGN -> max-log
demapper -> flooding FP32 sum-product decoder (20 iterations) -> error count
binned by Eb/N0.  The batch is 4096 codewords (k = 1280, n = 6656 mother,
3840 transmitted); codeword b sits at Eb/N0 point b mod 9 of 0:0.5:4 dB, so
every step covers the whole BLER curve.  Inputs are synthetic (counter-based
Philox in-kernel), resident in HBM before the timed region.

Printed: one JSON line with the decoded-information throughput (Gbit/s),
the decoder kernel's roofline position, the oracle's CPU baseline on a
bounded sample, and secondary legs (int8 offset min-sum, layered NMS on the
BG1-shaped code, mixed-shape persistent batch, weighted BP fwd/fwd+bwd).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
N_CU = 256
CLOCK_GHZ = 2.4
VALU_LANES_PER_CU_CLK = 64          # 4 SIMDs x 16 lanes
VALU_PEAK_TOPS = N_CU * VALU_LANES_PER_CU_CLK * CLOCK_GHZ / 1e3   # 39.32 T lane-ops/s

# Algorithmic VALU work per edge and round ("Roofline"):
# sum-product: check side 12 simple ops + 4 transcendentals (quarter rate,
# 4 issue slots each), variable side 3 ops -> 31 issue slots.
SPA_SLOTS_PER_EDGE = 12 + 4 * 4 + 3
# offset min-sum: check side 9 ops, variable side 3 ops.
OMS_SLOTS_PER_EDGE = 9 + 3
# layered normalized min-sum: 12 ops per edge and layer visit.
NMS_SLOTS_PER_EDGE = 12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="codewords of the oracle CPU baseline sample (0 = skip)")
    ap.add_argument("--legs", default="oms,nms",
                    help="secondary legs to time: oms,nms (empty = none)")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every lsim call uses)."""

    def __init__(self, torch):
        self.torch = torch
        self.total = 0.0
        self.n = 0

    def __enter__(self):
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.b = self.torch.cuda.Event(enable_timing=True)
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.pending = (self.a, self.b)
        return False

    def collect(self):
        self.torch.cuda.synchronize()
        self.total += self.pending[0].elapsed_time(self.pending[1])
        self.n += 1


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2203_11854_amd as lsim
    from inputs.workloads import BG1, BG2, data_seed

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda:0"

    # ---------------- workload: BG2-shaped code, 16-QAM, batch 4096
    qb = BG2.load()
    code = lsim.Code.from_qcbase(qb, 3840)
    B, k, m, S = 4096, code.k, 4, 3840 // 4
    pts = np.arange(9) * 0.5
    rate = k / code.e_tx
    n0_pts = lsim.ebn0_to_n0(pts, rate, m)
    bins = np.arange(B) % 9
    no = torch.tensor(n0_pts[bins], dtype=torch.float32, device=dev)
    tbins = torch.tensor(bins, dtype=torch.int32, device=dev)
    u = torch.empty((B, k), dtype=torch.uint8, device=dev)
    c = torch.empty((B, code.n_mother), dtype=torch.uint8, device=dev)
    y = torch.empty((B, S, 2), dtype=torch.float32, device=dev)
    llr = torch.empty((B, code.e_tx), dtype=torch.float32, device=dev)
    bits = torch.empty((B, k), dtype=torch.uint8, device=dev)
    counts = torch.zeros((9, 3), dtype=torch.int64, device=dev)
    p_spa = lsim.params(lsim.SPA_F32, iters=20, llr_max=20.0)
    dec_timer = Timer(torch)

    def step(i, timed):
        seed = data_seed(2, i)
        lsim.source_bits(seed, 0, B, k, out=u)
        lsim.encode(code, u, out=c)
        lsim.map_awgn(code, m, c, no, seed, 0, out=y)
        lsim.demap(m, lsim.DEMAP_MAXLOG, y, no, out=llr)
        if timed:
            with dec_timer:
                lsim.decode(code, llr, p_spa, bits=bits)
        else:
            lsim.decode(code, llr, p_spa, bits=bits)
        lsim.count_errors(u, bits, tbins, 9, counts=counts)

    log(f"[bench] warmup {args.warmup} steps")
    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    counts.zero_()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(1000 + i, False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = B * k / (ms_step * 1e-3) / 1e9
    cnt = counts.cpu().numpy()

    # decoder kernel alone, HIP events on its stream
    for i in range(max(5, min(args.steps, 20))):
        step(2000 + i, True)
        dec_timer.collect()
    dec_ms = dec_timer.total / dec_timer.n
    E = code.E
    slots = B * 20 * E * SPA_SLOTS_PER_EDGE
    achieved = slots / (dec_ms * 1e-3) / 1e12
    hbm_bytes = B * (code.e_tx * 4 + k)            # LLRs in, bits out
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                "kernel": "flood_kernel<512,16,SPA>", "kernel_ms": round(dec_ms, 4),
                "algorithmic_slots_per_edge_round": SPA_SLOTS_PER_EDGE,
                "hbm_algorithmic_bytes": hbm_bytes,
                "hbm_frac": round(hbm_bytes / (dec_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    log(f"[bench] step {ms_step:.3f} ms, decoder {dec_ms:.3f} ms, {value:.3f} Gbit/s")

    extra = {"bler_by_ebn0": {f"{pts[j]:.1f}": [int(cnt[j, 1]), int(cnt[j, 2])] for j in range(9)},
             "ber_by_ebn0": {f"{pts[j]:.1f}": float(cnt[j, 0]) / max(1, cnt[j, 2] * k) for j in range(9)},
             "decoder_only_gbps": round(B * k / (dec_ms * 1e-3) / 1e9, 3)}

    legs = [x for x in args.legs.split(",") if x]
    if "oms" in legs:
        q8 = torch.empty((B, code.e_tx), dtype=torch.int8, device=dev)
        p = lsim.params(lsim.OMS_I8, iters=20, offset=1, sat=31)
        tm = Timer(torch)
        for i in range(10):
            lsim.demap_q8(m, lsim.DEMAP_MAXLOG, y, no, out=q8)
            with tm:
                lsim.decode(code, q8, p, bits=bits)
            tm.collect()
        ms = tm.total / tm.n
        a = B * 20 * E * OMS_SLOTS_PER_EDGE / (ms * 1e-3) / 1e12
        extra["oms_i8_bg2"] = {"decoder_ms": round(ms, 4), "gbps": round(B * k / (ms * 1e-3) / 1e9, 3),
                               "alu_frac": round(a / VALU_PEAK_TOPS, 4)}
        log(f"[bench] oms int8 decoder {ms:.3f} ms")
    if "nms" in legs:
        qb1 = BG1.load()
        code1 = lsim.Code.from_qcbase(qb1, 25344)
        B1 = 1024
        n0 = lsim.ebn0_to_n0(3.0, code1.k / code1.e_tx, 6)
        no1 = torch.full((B1,), float(n0), dtype=torch.float32, device=dev)
        u1 = lsim.source_bits(data_seed(3, 0), 0, B1, code1.k, dev)
        c1 = lsim.encode(code1, u1)
        y1 = lsim.map_awgn(code1, 6, c1, no1, data_seed(3, 0), 0)
        l1 = lsim.demap(6, lsim.DEMAP_MAXLOG, y1, no1)
        p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
        work = torch.empty(lsim.decode_workspace(code1, p, B1), dtype=torch.uint8, device=dev)
        b1 = torch.empty((B1, code1.k), dtype=torch.uint8, device=dev)
        tm = Timer(torch)
        for i in range(6):
            with tm:
                lsim.decode(code1, l1, p, bits=b1, work=work)
            tm.collect()
        ms = tm.total / tm.n
        state_bytes = B1 * 20 * code1.m_dec * 12 * 2
        extra["nms_layered_bg1"] = {
            "decoder_ms": round(ms, 4), "gbps": round(B1 * code1.k / (ms * 1e-3) / 1e9, 3),
            "alu_frac": round(B1 * 20 * code1.E * NMS_SLOTS_PER_EDGE / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
            "state_stream_gbs": round(state_bytes / (ms * 1e-3) / 1e9, 1)}
        log(f"[bench] nms layered bg1 decoder {ms:.3f} ms")

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(qb, args.cpu_sample)

    out = {
        "metric": "decoded info Gbit/s @20 BP iters (fwd; fwd+bwd) at matched BLER",
        "value": round(value, 4), "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bg2-shaped QC-LDPC 42x52 Z=128 (k=1280, 3840 tx bits), Gray 16-QAM, "
                               "max-log demapper, flooding FP32 sum-product 20 iters, Eb/N0 0:0.5:4 dB",
                   "global_batch": B, "seq_len": None, "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(qb, ncw):
    """The FP64 oracle's link (bits .. SPA decode .. count) on a bounded
    sample of the same workload, on the host cores."""
    from inputs.workloads import data_seed
    from oracle import pipeline, qc

    g = qc.graph_from_qcbase(qb, 3840)
    threads = int(os.environ.get("OMP_NUM_THREADS", "1") or 1)
    log(f"[bench] cpu baseline: oracle on {ncw} codewords")
    t0 = time.perf_counter()
    cnt, _ = pipeline.run_point(g, qb.family, data_seed(2, 0), ncw, 2.0, 4, "maxlog", "spa", 20,
                                chunk=128)
    dt = time.perf_counter() - t0
    return {"value": round(ncw * g.k / dt / 1e9, 6), "unit": "Gbit/s", "cores": 1,
            "kind": "oracle", "threads_env": threads,
            "sample": f"{ncw} codewords of the bg2 workload at Eb/N0 2 dB, full link with "
                      f"FP64 flooding sum-product (20 iters), {dt:.1f} s"}


if __name__ == "__main__":
    main()
