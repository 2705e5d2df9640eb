"""Throughput of the LDPC link hot path on one MI355X.

One step = one batch of the BG1-shaped workload through the whole link:
Philox information bits -> QC encoder -> Gray 64-QAM + AWGN -> max-log
demapper -> layered normalized min-sum decoder (FP32, alpha 0.75, 20
iterations) -> error count binned by Eb/N0.  The batch is 1024 codewords
(k = 8448, 26112 decoded variable nodes, 25344 transmitted bits); codeword b
sits at Eb/N0 point b mod 9 of 1:0.5:5 dB, so every step covers the whole
BLER curve.  Inputs are synthetic (counter-based Philox in-kernel), resident
in HBM before the timed region.

Printed: one JSON line with the decoded-information throughput (Gbit/s), the
decoder kernel's roofline position against the published peaks and against
peaks measured in the same job (device copy, LDS, VALU probes), the oracle's
CPU baseline on a bounded sample, BLER validity gates against the oracle for
every decoder and workload point, and secondary entries (the BG2-shaped
workload with FP32 sum-product and int8 offset min-sum, the mixed-shape
persistent batch, weighted BP fwd / fwd+bwd and a trained WBP + demapper
pair against plain decoding at equal conditions, the trainable
constellation, EXIT curves and iterative demapping and decoding, Polar SC /
SCL / SCL-CRC).
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
# LDS planning figure: 128 bytes per clock per CU (the measured rate is
# reported beside it)
LDS_PEAK_GBS = N_CU * 128 * CLOCK_GHZ

# HBM bytes per launch of a decoder kernel from rocprofv3 FETCH_SIZE /
# WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
# for the copy probe of known size (factors below).  Valid only for the
# kernel sources they were taken on (hash); any change there reports null
# until the counters are taken again.
LAYERED_TRAFFIC = {"bytes": (2722004 * 2 + 4066563) * 1024,
                   "sources": ("layered_tile.h", "k_layered.hip", "dispatch.h", "lds.h",
                               "devcode.h"),
                   "sha256_16": "d70f9144f73c24f6"}
FLOOD_SPA_TRAFFIC = {"bytes": (30955 * 2 + 5120) * 1024,
                     "sources": ("k_flood.hip", "spa_math.h", "dispatch.h", "lds.h", "devcode.h"),
                     "sha256_16": "b7c20661452a4d85"}

# Algorithmic VALU work per edge and round:
# sum-product in the sum / difference form: check side 13 simple ops
# (sign xor, prefix and suffix updates 2 + 2, combination 4, ratio product,
# clamp, sign insert 2) + 3 transcendentals (exp, rcp, log; quarter rate,
# 4 issue slots each), variable side 3 ops -> 28 issue slots.
SPA_SLOTS_PER_EDGE = 13 + 3 * 4 + 3
# offset min-sum: check side 9 ops, variable side 3 ops.
OMS_SLOTS_PER_EDGE = 9 + 3
# layered normalized min-sum: 12 ops per edge and layer visit.
NMS_SLOTS_PER_EDGE = 12
# layered decoder: bytes of the check record streamed per check and
# iteration (alpha*m1, alpha*m2, signs | argmin), and of a record kept in
# LDS (the same three words in a 16-byte slot)
NMS_RECORD_BYTES = 12
NMS_LDS_RECORD_BYTES = 16

# BLER validity gates: oracle sample sizes (codewords per Eb/N0 point)
GATE_ORACLE_CW = {"cfg1": 1000, "cfg2": 96, "cfg3": 48}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=96,
                    help="codewords of the oracle CPU baseline sample (0 = skip)")
    ap.add_argument("--cpu-pool", type=int, default=1,
                    help="also time the oracle in a process pool over the host's cores")
    ap.add_argument("--gates", type=int, default=1,
                    help="BLER validity gates against the oracle (0 = skip)")
    ap.add_argument("--legs", default="bg2,bler,mixed,wbp,wbpeval,const,exit,polar",
                    help="secondary legs: bg2,bler,mixed,wbp,wbpeval,const,exit,polar "
                         "(empty = none)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library "
              "decodes on one device per process", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]

    # The oracle runs first, before anything touches the GPU, so its worker
    # processes start from a process without a GPU context: the CPU baseline
    # on the headline workload, then the BLER gates' samples over a pool.
    cpu = cpu_pool = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(args.cpu_sample)
        if args.cpu_pool:
            cpu_pool = cpu_baseline_pool(args.cpu_sample)
    gate_jobs = gate_plan(args.steps) if args.gates else []
    gate_oracle = run_gate_oracle(gate_jobs) if gate_jobs else {}

    import torch

    import paper_2203_11854_amd as lsim
    from inputs.workloads import BG1, BG2, data_seed

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda:0"

    peaks = measure_peaks(torch, lsim, dev)
    log(f"[bench] measured peaks {peaks}")

    # ---------------- headline: BG1-shaped code, 64-QAM, batch 1024
    qb1 = BG1.load()
    code = lsim.Code.from_qcbase(qb1, 25344)
    B, k, m, T = 1024, code.k, 6, 20
    pts = 1.0 + np.arange(9) * 0.5
    rate = k / code.e_tx
    n0_pts = lsim.ebn0_to_n0(pts, rate, m)
    bins = np.arange(B) % 9
    no = torch.tensor(n0_pts[bins], dtype=torch.float32, device=dev)
    tbins = torch.tensor(bins, dtype=torch.int32, device=dev)
    p_nms = lsim.params(lsim.NMS_F32, iters=T, alpha=0.75)
    order_tuning = layer_order_tuning(torch, lsim, dev, code, p_nms)
    log(f"[bench] layer order: {order_tuning}")
    link = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p_nms, B, no, bins=tbins, nbins=9, device=dev)

    def step(i):
        link.run(data_seed(3, i), 0)

    log(f"[bench] warmup {args.warmup} steps")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    link.counts.zero_()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(1000 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = B * k / (ms_step * 1e-3) / 1e9
    cnt = link.counts.cpu().numpy()
    log(f"[bench] step {ms_step:.3f} ms, {value:.3f} Gbit/s")

    # decoder kernel alone: back-to-back launches between two HIP events on
    # the stream the kernels run on (the current stream)
    llr, bits = link.llr, link.bits
    work = link.work
    dec = lambda: lsim.decode(code, llr, p_nms, bits=bits, work=work)  # noqa: E731
    dec_ms = _elapsed(torch, dec, 10)
    dec_med = _median_ms(torch, dec, 20, 5)
    # decode time does not depend on the data: spot checks at 1 dB and 5 dB
    snr_ms = {}
    for pt in (1.0, 5.0):
        no_pt = torch.full((B,), float(lsim.ebn0_to_n0(pt, rate, m)), dtype=torch.float32,
                           device=dev)
        lk_pt = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p_nms, B, no_pt, device=dev)
        lk_pt.run(data_seed(3, 77), 0)
        snr_ms[f"{pt:.1f}"] = round(_median_ms(
            torch, lambda: lsim.decode(code, lk_pt.llr, p_nms, bits=bits, work=work), 20, 5), 4)
    roofline = layered_roofline(code, B, T, dec_ms, peaks, lsim.decode_launch(code, p_nms))
    roofline.update({"kernel_ms_median20": round(dec_med, 4),
                     "kernel_ms_median20_by_ebn0": snr_ms})
    curve = [cnt[j, 1] / max(1, cnt[j, 2]) for j in range(9)]
    e12 = ebn0_at_bler(pts, curve)
    extra = {"measured_peaks": peaks,
             "decoder_only_gbps": round(B * k / (dec_ms * 1e-3) / 1e9, 3),
             "decoder_ms": round(dec_ms, 4),
             "bler_by_ebn0": {f"{pts[j]:.1f}": [int(cnt[j, 1]), int(cnt[j, 2])] for j in range(9)},
             "ber_by_ebn0": {f"{pts[j]:.1f}": float(cnt[j, 0]) / max(1, cnt[j, 2] * k)
                             for j in range(9)},
             "ebn0_db_at_bler_1e-2": None if e12 is None else round(e12, 3),
             "layer_order": order_tuning}
    gpu_curves = {("cfg3", "nms" if order_tuning["chosen"] == "natural" else "nms_grouped"): cnt}

    if "bg2" in legs or "bler" in legs:
        extra["bg2"], bg2_counts = bg2_leg(torch, lsim, dev, args.steps, "bler" in legs)
        gpu_curves.update(bg2_counts)
        log(f"[bench] bg2: {extra['bg2']}")
    if "mixed" in legs:
        extra["mixed_persistent"] = mixed_leg(torch, lsim, dev)
        log(f"[bench] mixed: {extra['mixed_persistent']}")
    qb2 = BG2.load()
    code2 = lsim.Code.from_qcbase(qb2, 3840)
    if "wbp" in legs:
        extra["wbp_ndm_bg2"] = {f"T{t}": wbp_leg(torch, lsim, dev, code2, qb2, t) for t in (10, 20)}
        log(f"[bench] wbp: {extra['wbp_ndm_bg2']}")
    if "wbpeval" in legs:
        extra["wbp_ndm_trained_vs_spa"] = wbp_eval_leg(torch, lsim, dev, code2, qb2)
        log(f"[bench] wbp eval: {extra['wbp_ndm_trained_vs_spa']}")
    if "exit" in legs:
        extra["exit_bicm_id_bg2"] = exit_leg(torch, lsim, dev, code2, qb2)
        log(f"[bench] exit: {extra['exit_bicm_id_bg2']}")
    if "polar" in legs:
        extra["polar_n1024_k512"] = polar_leg(torch, lsim, dev)
        log(f"[bench] polar: {extra['polar_n1024_k512']}")
    if "const" in legs:
        extra["constellation_ndm_bg2"] = const_leg(torch, lsim, dev, code2, qb2)
        log(f"[bench] constellation: {extra['constellation_ndm_bg2']}")

    if gate_jobs:
        extra["matched_bler"] = gate_results(torch, lsim, dev, gate_jobs, gate_oracle, gpu_curves,
                                             args.steps)
        bad = [g for g in extra["matched_bler"]["points"] if not g["within"]]
        log(f"[bench] BLER gates: {len(extra['matched_bler']['points']) - len(bad)} of "
            f"{len(extra['matched_bler']['points'])} inside the oracle's 95% interval")
    if cpu_pool is not None:
        extra["cpu_baseline_pool"] = cpu_pool

    out = {
        "metric": "decoded info Gbit/s @20 BP iters (fwd; fwd+bwd) at matched BLER",
        "value": round(value, 4), "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bg1-shaped QC-LDPC 46x68 Z=384 (k=8448, n=26112, 25344 tx bits, "
                               "rate 1/3), Gray 64-QAM, max-log demapper, layered normalized "
                               "min-sum FP32 alpha 0.75, 20 iters, layer order chosen by the "
                               "schedule tuner (" + order_tuning["chosen"] + "), Eb/N0 1:0.5:5 dB, "
                               "whole link per step",
                   "global_batch": B, "seq_len": None, "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def measure_peaks(torch, lsim, dev):
    """Peak rates measured on this device with the library's probes: device
    copy and read (HBM), LDS reads and writes, FMA and exp2 issue."""
    nb = 1 << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    out = torch.empty(16384 * 256, dtype=torch.float32, device=dev)
    res = {}
    u = [0]

    def rate(kind, grid, rounds=1, s=None, d=out, nbytes=0):
        ms = _median_ms(torch, lambda: u.__setitem__(0, lsim.probe(kind, d, s, nbytes, rounds, grid)),
                        10, 2)
        return u[0] / (ms * 1e-3)

    res["hbm_copy_gbs"] = round(max(rate(lsim.PROBE_COPY, g, s=src, d=dst, nbytes=nb)
                                    for g in (1024, 2048)) / 1e9, 1)
    res["hbm_read_gbs"] = round(max(rate(lsim.PROBE_READ, g, s=src, nbytes=nb)
                                    for g in (1024, 2048)) / 1e9, 1)
    del src, dst
    res["lds_read_gbs"] = round(rate(lsim.PROBE_LDS_READ, 2048, 2048) / 1e9, 1)
    res["lds_write_gbs"] = round(rate(lsim.PROBE_LDS_WRITE, 2048, 2048) / 1e9, 1)
    res["valu_fma_tops"] = round(rate(lsim.PROBE_FMA, 2048, 4096) / 1e12, 3)
    res["valu_exp2_tops"] = round(rate(lsim.PROBE_EXP2, 2048, 4096) / 1e12, 3)
    return res


def layered_roofline(code, B, T, ms, peaks, launch):
    """Roofline position of one layered-decoder launch.  HBM algorithmic
    bytes: the 12-byte check records of the rows that stream through device
    memory (read in iterations 2..T, written in 1..T-1), the channel LLR of
    each private (degree-one) column read again in iterations 2..T, the LLRs
    in once and the bits out.  LDS: one 4-byte read and one write per edge
    and iteration whose posterior is in LDS, plus the records of the rows
    kept in LDS.  VALU: 12 lane operations per edge and iteration."""
    K = launch["lds_rows"]
    rec = B * (T - 1) * 2 * NMS_RECORD_BYTES * (code.rows - K) * code.Z
    priv = B * (T - 1) * 4 * code.n_private_rows * code.Z
    io = B * (4 * code.e_tx + code.k)
    hbm = rec + priv + io
    s = ms * 1e-3
    lds_edges = code.E - code.n_private_rows * code.Z
    lds = B * T * (8 * lds_edges + 2 * NMS_LDS_RECORD_BYTES * K * code.Z)
    valu = B * T * code.E * NMS_SLOTS_PER_EDGE
    achieved = hbm / s / 1e9
    D = 16 if code.max_row_deg <= 16 else 24 if code.max_row_deg <= 24 else 27
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _traffic(LAYERED_TRAFFIC),
            "kernel": f"layered_kernel<{launch['threads']},{D},{launch['waves_per_simd']}>",
            "launch": launch,
            "kernel_ms": round(ms, 4),
            "hbm_algorithmic_bytes": int(hbm),
            "measured_peak": peaks["hbm_copy_gbs"],
            "frac_of_measured": round(achieved / peaks["hbm_copy_gbs"], 4),
            "lds_algorithmic_bytes": int(lds),
            "lds_gbs": round(lds / s / 1e9, 1),
            "lds_frac_of_measured": round(lds / s / 1e9 / peaks["lds_read_gbs"], 4),
            "lds_frac_of_planning_peak": round(lds / s / 1e9 / LDS_PEAK_GBS, 4),
            "valu_algorithmic_lane_ops": int(valu),
            "valu_tops": round(valu / s / 1e12, 3),
            "valu_frac_of_measured": round(valu / s / 1e12 / peaks["valu_fma_tops"], 4),
            "valu_frac_of_published": round(valu / s / 1e12 / VALU_PEAK_TOPS, 4)}


def bg2_leg(torch, lsim, dev, steps, bler_legs):
    """The BG2-shaped workload (Z = 128, 16-QAM, batch 4096, Eb/N0 0:0.5:4
    dB): the whole link with the FP32 flooding sum-product decoder timed as
    a step, the decoders alone, and (with the bler leg) the same data
    through int8 offset min-sum and layered NMS for their BLER curves."""
    from inputs.workloads import BG2, data_seed

    qb = BG2.load()
    code = lsim.Code.from_qcbase(qb, 3840)
    B, k, m = 4096, code.k, 4
    pts = np.arange(9) * 0.5
    rate = k / code.e_tx
    bins = np.arange(B) % 9
    no = torch.tensor(lsim.ebn0_to_n0(pts, rate, m)[bins], dtype=torch.float32, device=dev)
    tbins = torch.tensor(bins, dtype=torch.int32, device=dev)
    p_spa = lsim.params(lsim.SPA_F32, iters=20, llr_max=20.0)
    link = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p_spa, B, no, bins=tbins, nbins=9, device=dev)
    for i in range(3):
        link.run(data_seed(2, i), 0)
    torch.cuda.synchronize()
    link.counts.zero_()
    t0 = time.perf_counter()
    for i in range(steps):
        link.run(data_seed(2, 1000 + i), 0)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    cnt = link.counts.cpu().numpy()
    llr, bits = link.llr, link.bits
    E = code.E
    spa_ms = _elapsed(torch, lambda: lsim.decode(code, llr, p_spa, bits=bits), 10)
    s = spa_ms * 1e-3
    lds = B * 20 * (16 * E + 8 * code.n_dec)
    out = {"workload": "bg2-shaped 42x52 Z=128 (k=1280, 3840 tx bits), Gray 16-QAM, max-log, "
                       "batch 4096, 20 iters, Eb/N0 0:0.5:4 dB",
           "spa_f32_step_ms": round(ms_step, 4),
           "spa_f32_step_gbps": round(B * k / (ms_step * 1e-3) / 1e9, 3),
           "spa_f32_decoder_ms": round(spa_ms, 4),
           "spa_f32_decoder_gbps": round(B * k / s / 1e9, 3),
           "spa_f32_kernel": "flood_kernel<512,16,SPA>",
           "spa_f32_valu_slots_frac": round(B * 20 * E * SPA_SLOTS_PER_EDGE / s / 1e12
                                            / VALU_PEAK_TOPS, 4),
           "spa_f32_lds_gbs": round(lds / s / 1e9, 1),
           "spa_f32_traffic": _traffic(FLOOD_SPA_TRAFFIC)}
    curves = {("cfg2", "spa"): cnt}
    p8 = lsim.params(lsim.OMS_I8, iters=20, offset=1, sat=31)
    lk8 = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p8, B, no, bins=tbins, nbins=9, device=dev)
    lk8.run(data_seed(2, 0), 0)
    q8 = lk8.llr
    oms_ms = _elapsed(torch, lambda: lsim.decode(code, q8, p8, bits=bits), 10)
    out["oms_i8_decoder_ms"] = round(oms_ms, 4)
    out["oms_i8_decoder_gbps"] = round(B * k / (oms_ms * 1e-3) / 1e9, 3)
    out["oms_i8_valu_slots_frac"] = round(B * 20 * E * OMS_SLOTS_PER_EDGE / (oms_ms * 1e-3)
                                          / 1e12 / VALU_PEAK_TOPS, 4)
    pn = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    lkn = lsim.Link(code, m, lsim.DEMAP_MAXLOG, pn, B, no, bins=tbins, nbins=9, device=dev)
    lkn.run(data_seed(2, 0), 0)
    nms_ms = _elapsed(torch, lambda: lsim.decode(code, lkn.llr, pn, bits=bits, work=lkn.work), 10)
    out["nms_f32_layered_decoder_ms"] = round(nms_ms, 4)
    out["nms_f32_layered_decoder_gbps"] = round(B * k / (nms_ms * 1e-3) / 1e9, 3)
    if bler_legs:
        for name, lk in (("oms", lk8), ("nms", lkn)):
            lk.counts.zero_()
            for i in range(steps):
                lk.run(data_seed(2, 1000 + i), 0)
            curves[("cfg2", name)] = lk.counts.cpu().numpy()
        out["ebn0_db_at_bler_1e-2"] = {}
        out["bler_curves"] = {}
        for (_, name), c in curves.items():
            cv = [c[j, 1] / max(1, c[j, 2]) for j in range(9)]
            e = ebn0_at_bler(pts, cv)
            out["ebn0_db_at_bler_1e-2"][name] = None if e is None else round(e, 3)
            out["bler_curves"][name] = [round(float(x), 5) for x in cv]
    return out, curves


# ------------------------------------------------------ BLER validity gates

def layer_order_tuning(torch, lsim, dev, code, p):
    """The schedule tuner's layer order for the headline code (natural or
    grouped, lsim.autotune.tune_layer_order) on its own batch: 2048
    codewords of the same link at 5.5 dB, where the BLER curve falls (at the
    workload's 1..5 dB every frame fails, so there the orders cannot be told
    apart)."""
    from inputs.workloads import data_seed
    from paper_2203_11854_amd import autotune
    nb, m = 2048, 6
    no = torch.full((nb,), float(lsim.ebn0_to_n0(5.5, code.k / code.e_tx, m)),
                    dtype=torch.float32, device=dev)
    lk = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p, nb, no, device=dev)
    lk.run(data_seed(3, 500), 0)
    return autotune.tune_layer_order(code, lk.llr, lk.u, p)


def _gate_configs():
    """(spec, e_tx, m, demap, Eb/N0 points, workload number, GPU batch).
    The BG1-shaped workload's grid runs on to 6 dB: at 1..5 dB its BLER is
    about 1, so the two points past the workload's range are where the
    curves can be told apart."""
    from inputs.workloads import BG1, BG2, SMALL
    return {"cfg1": (SMALL, 648, 1, "exact", np.array([1.0, 2.0, 3.0]), 1, 3000),
            "cfg2": (BG2, 3840, 4, "maxlog", np.arange(9) * 0.5, 2, 4096),
            "cfg3": (BG1, 25344, 6, "maxlog", 1.0 + np.arange(11) * 0.5, 3, 1024)}


def gate_plan(steps):
    """The gated (workload, decoder) pairs with the oracle's sample: the
    first codewords of the first timed step of the same workload (same
    Philox seed and codeword indices, so the GPU decodes the very same
    frames), codeword b at Eb/N0 point b mod (number of points)."""
    from inputs.workloads import data_seed
    cfgs = _gate_configs()
    plan = []
    for cfg, algos in (("cfg1", ("spa",)), ("cfg2", ("spa", "oms", "nms")),
                       ("cfg3", ("nms", "nms_grouped"))):
        npts = len(cfgs[cfg][4])
        n = GATE_ORACLE_CW[cfg] * npts
        seed = data_seed(cfgs[cfg][5], 1000)
        for a in algos:
            plan.append({"cfg": cfg, "algo": a, "seed": seed, "n": n})
    return plan


def _oracle_gate_chunk(job):
    """Oracle block-error flags of codewords cw0 .. cw0 + nb - 1 of a gate."""
    cfg, algo, seed, cw0, nb = job
    from oracle import pipeline, qc
    spec, e_tx, m, demap, pts, _, _ = _gate_configs()[cfg]
    qb = spec.load()
    g = qc.graph_from_qcbase(qb, e_tx)
    idx = np.arange(cw0, cw0 + nb)
    n0 = pipeline.n0_for(g, pts[idx % len(pts)], m)
    tx = pipeline.transmit(g, qb.family, seed, cw0, nb, n0, m, demap)
    bits, _ = pipeline.decode(g, tx["L"], algo, 20)
    return cw0, (bits != tx["u"]).any(axis=1)


def run_gate_oracle(plan):
    """Every gate's oracle sample over a process pool (the host's cores, at
    most 16); returns {(cfg, algo): block-error flags}."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    chunk = {"cfg1": 500, "cfg2": 48, "cfg3": 8}
    jobs = []
    for gp in plan:
        c = chunk[gp["cfg"]]
        jobs += [(gp["cfg"], gp["algo"], gp["seed"], lo, min(c, gp["n"] - lo))
                 for lo in range(0, gp["n"], c)]
    workers = max(1, min(16, _ncpu()))
    log(f"[bench] BLER gates: oracle on {sum(j[4] for j in jobs)} codewords, {workers} processes")
    t0 = time.perf_counter()
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_gate_chunk, jobs))
    finally:
        if old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = old
    flags = {}
    for (cfg, algo, _, _, _), (cw0, f) in zip(jobs, res):
        flags.setdefault((cfg, algo), {})[cw0] = f
    out = {key: np.concatenate([d[c] for c in sorted(d)]) for key, d in flags.items()}
    log(f"[bench] BLER gates: oracle done in {time.perf_counter() - t0:.1f} s")
    return out


def gate_results(torch, lsim, dev, plan, oracle, gpu_curves, steps):
    """Per gated point: the oracle's BLER and Wilson 95% interval on its
    sample, the GPU's BLER on the very same frames (and how many frames the
    two decide differently), the GPU's BLER on its full sample (the timed
    steps of the same workload, or as many steps of the gate's own grid) and
    whether it lies inside the interval; per curve, the Eb/N0 at BLER 1e-2 of
    both."""
    from inputs.workloads import data_seed
    from oracle import stats
    cfgs = _gate_configs()
    algos = {"spa": lsim.SPA_F32, "oms": lsim.OMS_I8, "nms": lsim.NMS_F32,
             "nms_grouped": lsim.NMS_F32}
    points, curves = [], {}
    for gp in plan:
        cfg, algo, seed, n = gp["cfg"], gp["algo"], gp["seed"], gp["n"]
        spec, e_tx, m, demap, pts, wl, batch = cfgs[cfg]
        code = lsim.Code.from_qcbase(spec.load(), e_tx)
        if algo == "nms_grouped":
            code.set_layer_order("grouped")
        npts = len(pts)
        n0_pts = lsim.ebn0_to_n0(pts, code.k / code.e_tx, m)
        p = lsim.params(algos[algo], iters=20, alpha=0.75, offset=1, sat=31)
        method = lsim.DEMAP_EXACT if demap == "exact" else lsim.DEMAP_MAXLOG
        idx = np.arange(n) % npts
        no = torch.tensor(n0_pts[idx], dtype=torch.float32, device=dev)
        per = lsim.Link(code, m, method, p, n, no, bins=torch.arange(n, dtype=torch.int32, device=dev),
                        nbins=n, device=dev)
        per.run(seed, 0)
        gflags = per.counts.cpu().numpy()[:, 1] > 0
        oflags = oracle[(cfg, algo)]
        full = gpu_curves.get((cfg, algo))
        if cfg == "cfg1":
            full = None                  # the workload is these 1000 codewords per point
        elif full is None or full.shape[0] != npts:
            bi = np.arange(batch) % npts
            lk = lsim.Link(code, m, method, p, batch,
                           torch.tensor(n0_pts[bi], dtype=torch.float32, device=dev),
                           bins=torch.tensor(bi, dtype=torch.int32, device=dev), nbins=npts,
                           device=dev)
            for i in range(steps):
                lk.run(data_seed(wl, 1000 + i), 0)
            full = lk.counts.cpu().numpy()
        oc, gc = [], []
        for j in range(npts):
            sel = idx == j
            ob, nn = int(oflags[sel].sum()), int(sel.sum())
            lo, hi = stats.wilson(ob, nn)
            pb = int(gflags[sel].sum())
            fb, fn = (pb, nn) if full is None else (int(full[j, 1]), int(full[j, 2]))
            gb = fb / max(1, fn)
            points.append({"workload": cfg, "decoder": algo, "ebn0_db": float(pts[j]),
                           "oracle_bler": round(ob / nn, 5), "oracle_codewords": nn,
                           "oracle_ci95": [round(float(lo), 5), round(float(hi), 5)],
                           "gpu_bler_same_frames": round(pb / nn, 5),
                           "frames_decided_differently": int((oflags[sel] != gflags[sel]).sum()),
                           "gpu_bler": round(gb, 5), "gpu_codewords": fn,
                           # the interval's ends at 0 and 1 come out of the
                           # formula within rounding of the exact value
                           "within": bool(lo - 1e-9 <= gb <= hi + 1e-9)})
            oc.append(ob / nn)
            gc.append(gb)
        eo, eg = ebn0_at_bler(pts, oc), ebn0_at_bler(pts, gc)
        curves[f"{cfg}/{algo}"] = {"oracle_ebn0_db_at_bler_1e-2": None if eo is None else round(eo, 3),
                                   "gpu_ebn0_db_at_bler_1e-2": None if eg is None else round(eg, 3)}
    return {"points": points, "curves": curves,
            "all_within": all(g["within"] for g in points),
            "frames_decided_differently": int(sum(g["frames_decided_differently"] for g in points)),
            "note": "oracle: FP64 (int8 OMS: exact integers) on the same Philox seeds and codeword "
                    "indices the GPU decodes in its first step; interval: Wilson 95%"}


def _ncpu():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _traffic(entry):
    import hashlib
    if entry["bytes"] is None:
        return None
    h = hashlib.sha256()
    for f in entry["sources"]:
        with open(os.path.join(ROOT, "paper_2203_11854_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return entry["bytes"] if h.hexdigest()[:16] == entry["sha256_16"] else None


def ebn0_at_bler(pts, blers, target=1e-2):
    """Eb/N0 where the BLER curve crosses ``target`` (linear in log10 BLER
    between the two bracketing points), or None if it does not cross."""
    for j in range(1, len(pts)):
        a, b = blers[j - 1], blers[j]
        if a >= target > b:
            if b <= 0:
                return float(pts[j])
            la, lb, lt = math.log10(a), math.log10(b), math.log10(target)
            return float(pts[j - 1] + (pts[j] - pts[j - 1]) * (la - lt) / (la - lb))
    return None


def _median_ms(torch, fn, reps, warm):
    """Median of `reps` launches, each between its own pair of HIP events on
    the current stream, after `warm` untimed ones."""
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def _elapsed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def mixed_leg(torch, lsim, dev):
    """Eight BG-shaped codes (Z 16..384, rates 1/3..8/9), counts drawn
    log-uniform in [16, 4096], QPSK/16-QAM per codeword, Eb/N0 ~ U[0, 6] dB:
    one persistent graph-replayed launch vs one launch per shape, with the
    layered NMS decoder (and the autotuner), and with int8 offset min-sum
    over the shapes whose state fits the LDS."""
    from inputs import rand
    from inputs.workloads import data_seed, mixed_counts, mixed_specs

    specs = mixed_specs()
    counts = mixed_counts()
    codes, parts, us = [], [], []
    p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    for s, ((spec, e_tx), cnt) in enumerate(zip(specs, counts)):
        qb = spec.load()
        code = lsim.Code.from_qcbase(qb, e_tx)
        codes.append(code)
        r = rand.rng(4000 + s)
        n_qpsk = int((r.random(cnt) < 0.5).sum())
        ebn0 = r.uniform(0.0, 6.0, cnt)
        seed = data_seed(4, s)
        u = lsim.source_bits(seed, 0, cnt, code.k, dev)
        us.append(u)
        c = lsim.encode(code, u)
        llr = torch.empty((cnt, code.e_tx), dtype=torch.float32, device=dev)
        for lo, hi, m in ((0, n_qpsk, 2), (n_qpsk, cnt, 4)):
            if hi <= lo:
                continue
            no = torch.tensor(lsim.ebn0_to_n0(ebn0[lo:hi], code.k / code.e_tx, m),
                              dtype=torch.float32, device=dev)
            y = lsim.map_awgn(code, m, c[lo:hi].contiguous(), no, seed, lo)
            llr[lo:hi] = lsim.demap(m, lsim.DEMAP_MAXLOG, y, no)
        parts.append(llr)
    cat = torch.cat([x.reshape(-1) for x in parts])
    plan = lsim.MixedPlan(codes, counts, p)
    work = plan.workspace(dev)
    bits = torch.empty(plan.n_bits, dtype=torch.uint8, device=dev)
    plan.decode(cat, bits=bits, work=work)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.decode(cat, bits=bits, work=work)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.decode(cat, bits=bits, work=work)
    ms_graph = _elapsed(torch, g.replay, 5)
    ms_pers = _elapsed(torch, lambda: plan.decode(cat, bits=bits, work=work), 5)
    sep_bits = [torch.empty((cnt, cd.k), dtype=torch.uint8, device=dev) for cd, cnt in zip(codes, counts)]
    sep_work = [torch.empty(max(1, lsim.decode_workspace(cd, p, cnt)), dtype=torch.uint8, device=dev)
                for cd, cnt in zip(codes, counts)]

    def per_shape():
        for cd, x, bb, ww in zip(codes, parts, sep_bits, sep_work):
            lsim.decode(cd, x, p, bits=bb, work=ww)

    ms_sep = _elapsed(torch, per_shape, 5)
    # autotuned launch knobs (result-invariant; the tuner checks the bits)
    from paper_2203_11854_amd import autotune
    best = autotune.tune_mixed(codes, counts, p, cat, cache_path=None)
    tplan = lsim.MixedPlan(codes, counts, p, codewords_per_tile=best["codewords_per_tile"],
                           threads=best["threads"])
    twork = tplan.workspace(dev)
    tbits = torch.empty_like(bits)
    ms_tuned = _elapsed(torch, lambda: tplan.decode(cat, bits=tbits, work=twork,
                                                    persistent=best["persistent"]), 5)
    same = all(torch.equal(bits[o:o + bb.numel()], bb.reshape(-1))
               for o, bb in zip(plan.bits_offsets, sep_bits))
    info = sum(cnt * cd.k for cd, cnt in zip(codes, counts))
    # the int8 offset min-sum decoder (flooding, codeword pairs in packed
    # 16-bit lanes, or one codeword per tile where a pair does not fit, whole
    # state in LDS) over every shape: persistent launch vs one per shape
    po = lsim.params(lsim.OMS_I8, iters=20)
    keep = [s for s, cd in enumerate(codes) if autotune.oms_fits(cd)]
    ocodes = [codes[s] for s in keep]
    ocounts = [counts[s] for s in keep]
    q8 = [lsim.quantize(parts[s]) for s in keep]
    qcat = torch.cat([x.reshape(-1) for x in q8])
    oplan = lsim.MixedPlan(ocodes, ocounts, po)
    owork = oplan.workspace(dev)
    obits = torch.empty(oplan.n_bits, dtype=torch.uint8, device=dev)
    ms_oms = _elapsed(torch, lambda: oplan.decode(qcat, bits=obits, work=owork), 5)
    osep = [torch.empty((cnt, cd.k), dtype=torch.uint8, device=dev)
            for cd, cnt in zip(ocodes, ocounts)]

    def per_shape_oms():
        for cd, x, bb in zip(ocodes, q8, osep):
            lsim.decode(cd, x, po, bits=bb)

    ms_oms_sep = _elapsed(torch, per_shape_oms, 5)
    osame = all(torch.equal(obits[o:o + bb.numel()], bb.reshape(-1))
                for o, bb in zip(oplan.bits_offsets, osep))
    oinfo = sum(cnt * cd.k for cd, cnt in zip(ocodes, ocounts))
    # schedule and placement tuning: per shape layered NMS or flooding int8
    # OMS (accepted only inside NMS's Wilson 95% BLER interval on this data),
    # check records in LDS or streamed; the chosen schedule's bits against
    # the per-shape decoders it names
    sched = autotune.tune_schedule(codes, counts, parts, us, p)
    lp = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75, lds_rows=sched["lds_rows"])
    sm = autotune.ScheduledMixed(codes, counts, sched["schedule"], lp, po)
    io = sm.inputs(parts)
    sm.decode(io)
    sbits = sm.bits(io)
    sched_same = True
    for s_, (cd, x) in enumerate(zip(codes, parts)):
        if sched["schedule"][s_] == "oms":
            rb, _ = lsim.decode(cd, lsim.quantize(x), po)
        elif sched["layer_order"][s_] == "natural":
            rb = sep_bits[s_]
        else:                      # the order the tuner left set on the code
            rb, _ = lsim.decode(cd, x, p)
        sched_same = sched_same and torch.equal(sbits[s_], rb)
    ms_sched = _elapsed(torch, lambda: sm.decode(io), 5)
    blk = {"default_nms": 0, "scheduled": 0}
    for s_, sh in enumerate(sched["shapes"]):
        blk["default_nms"] += sh["nms_block_errors"]
        blk["scheduled"] += (sh["oms_block_errors"] if sched["schedule"][s_] == "oms"
                             else sh["grouped_block_errors"]
                             if sched["layer_order"][s_] == "grouped" else sh["nms_block_errors"])
    for cd in codes:
        cd.set_layer_order("natural")
    return {"codewords": int(sum(counts)), "counts": counts, "info_bits": int(info),
            "graph_ms": round(ms_graph, 4), "persistent_ms": round(ms_pers, 4),
            "per_shape_ms": round(ms_sep, 4),
            "graph_gbps": round(info / (ms_graph * 1e-3) / 1e9, 3),
            "per_shape_gbps": round(info / (ms_sep * 1e-3) / 1e9, 3),
            "bit_identical_to_per_shape": bool(same),
            "autotuned": {"threads": best["threads"], "codewords_per_tile": best["codewords_per_tile"],
                          "persistent": best["persistent"], "ms": round(ms_tuned, 4),
                          "bit_identical": bool(torch.equal(tbits, bits))},
            "schedule_tuned": {"schedule": sched["schedule"], "layer_order": sched["layer_order"],
                               "lds_rows": sched["lds_rows"],
                               "ms": round(ms_sched, 4),
                               "gbps": round(info / (ms_sched * 1e-3) / 1e9, 3),
                               "default_persistent_ms": round(ms_pers, 4),
                               "block_errors": blk, "codewords": int(sum(counts)),
                               "per_shape": sched["shapes"], "candidates": sched["tried"],
                               "bit_identical_to_named_decoders": bool(sched_same)},
            "oms_i8": {"shapes": keep, "codewords": int(sum(ocounts)),
                       "persistent_ms": round(ms_oms, 4), "per_shape_ms": round(ms_oms_sep, 4),
                       "persistent_gbps": round(oinfo / (ms_oms * 1e-3) / 1e9, 3),
                       "per_shape_gbps": round(oinfo / (ms_oms_sep * 1e-3) / 1e9, 3),
                       "bit_identical_to_per_shape": bool(osame)}}


def wbp_leg(torch, lsim, dev, code, qb, T=10):
    """Weighted BP (T rounds, per-edge per-round weights) fed by the neural
    demapper on 16-QAM, batch 2048, Eb/N0 ~ U[1, 4] dB: one training step
    (forward; forward + backward + Adam) vs the plain sum-product decoder."""
    from inputs import rand
    from inputs.workloads import data_seed

    B, m = 2048, 4
    r = rand.rng(5005)
    ebn0 = r.uniform(1.0, 4.0, B)
    no = torch.tensor(lsim.ebn0_to_n0(ebn0, code.k / code.e_tx, m), dtype=torch.float32, device=dev)
    seed = data_seed(5, 0)
    u = lsim.source_bits(seed, 0, B, code.k, dev)
    c = lsim.encode(code, u)
    y = lsim.map_awgn(code, m, c, no, seed, 0)
    params = torch.tensor(glorot_params(5006), dtype=torch.float32, device=dev)
    w = torch.ones((T, code.E), dtype=torch.float32, device=dev)
    pm, pv = torch.zeros_like(params), torch.zeros_like(params)
    wm, wv = torch.zeros_like(w), torch.zeros_like(w)
    llr = torch.empty((B, code.e_tx), dtype=torch.float32, device=dev)
    lpost = torch.empty((B, code.n_dec), dtype=torch.float32, device=dev)
    ckpt = torch.empty((T, B, code.E), dtype=torch.float32, device=dev)
    gwork = torch.empty(lsim.wbp_workspace(code, T, B), dtype=torch.uint8, device=dev)
    scale = 1.0 / (B * code.n_dec)
    state = {"step": 0}

    def fwd():
        lsim.ndm_forward(params, y, no, out=llr)
        lsim.wbp_forward(code, w, llr, T, 20.0, ckpt=ckpt, lpost=lpost)
        return lsim.bce_grad(lpost, c, scale)

    def fwd_bwd():
        gpost, loss = fwd()
        gllr, gw = lsim.wbp_backward(code, w, llr, ckpt, gpost, T, 20.0, work=gwork)
        gp = lsim.ndm_backward(params, y, no, gllr)
        state["step"] += 1
        lsim.adam_step(w, gw, wm, wv, state["step"])
        lsim.adam_step(params, gp, pm, pv, state["step"])
        return loss

    ms_f = _elapsed(torch, fwd, 5)
    ms_fb = _elapsed(torch, fwd_bwd, 5)
    l0 = float(fwd()[1].item())
    spa = lsim.params(lsim.SPA_F32, iters=T)
    ms_plain = _elapsed(torch, lambda: lsim.decode(code, llr, spa), 5)
    info = B * code.k
    return {"batch": B, "iters": T, "fwd_ms": round(ms_f, 4), "fwd_bwd_ms": round(ms_fb, 4),
            "fwd_gbps": round(info / (ms_f * 1e-3) / 1e9, 3),
            "fwd_bwd_gbps": round(info / (ms_fb * 1e-3) / 1e9, 3),
            "plain_spa_ms": round(ms_plain, 4),
            "plain_spa_gbps": round(info / (ms_plain * 1e-3) / 1e9, 3),
            "loss_after_timing_steps": round(l0, 6)}


def polar_leg(torch, lsim, dev):
    """Polar code N = 1024, K = 512 (496 data bits + CRC-16 0x1021),
    Bhattacharyya construction at 2 dB, QPSK over AWGN, 4096 codewords at
    Eb/N0 1, 1.5, 2, 2.5 dB (codeword b at point b mod 4): SC, SCL-8,
    SCL-8-CRC and SCL-32-CRC decode time (one launch, event-timed) and BLER
    per point."""
    from inputs.workloads import data_seed

    n, K, r, poly = 10, 512, 16, 0x1021
    N, D, B, m = 1 << n, K - r, 4096, 2
    pc = lsim.PolarCode(n, lsim.polar_construct(n, K, 2.0), r, poly)
    pts = np.array([1.0, 1.5, 2.0, 2.5])
    bins = np.arange(B) % len(pts)
    no = torch.tensor(lsim.ebn0_to_n0(pts[bins], D / N, m), dtype=torch.float32, device=dev)
    tb = torch.tensor(bins, dtype=torch.int32, device=dev)
    seed = data_seed(8, 0)
    data = lsim.source_bits(seed, 0, B, D, dev)
    x = pc.encode(data)
    y = lsim.map_awgn_bits(m, x, no, seed, 0)
    llr = lsim.demap(m, lsim.DEMAP_EXACT, y, no)
    bits = torch.empty((B, D), dtype=torch.uint8, device=dev)
    out = {"batch": B, "ebn0_db": pts.tolist(), "encode_ms": round(_elapsed(
        torch, lambda: pc.encode(data, out=x), 5), 4)}
    for name, L, use in (("sc", 1, False), ("scl8", 8, False), ("scl8_crc", 8, True),
                         ("scl32_crc", 32, True)):
        pc.decode(llr, L, use, bits=bits)
        counts = lsim.count_errors(data, bits, bins=tb, nbins=len(pts)).cpu().numpy()
        ms = _elapsed(torch, lambda: pc.decode(llr, L, use, bits=bits), 3)
        out[name] = {"ms": round(ms, 4), "gbps": round(B * D / (ms * 1e-3) / 1e9, 3),
                     "bler": [round(float(c[1] / c[2]), 5) for c in counts]}
    return out


def exit_leg(torch, lsim, dev, code, qb):
    """EXIT chart simulation and iterative demapping and decoding on the
    bg2 code with Gray 16-QAM, batch 4096.

    * Demapper and decoder transfer curves in one batched pass each: the
      codewords are split over 11 a-priori strengths sigma_A = 0, 0.6, ..,
      6 (bin b mod 11); I_A and I_E are measured (per-bin mean of the
      mutual-information estimate) on the a-priori and extrinsic LLRs.  The
      demapper sees the channel at Eb/N0 3 dB; the decoder (sum-product,
      20 iterations) sees only the a-priori LLRs.
    * BICM-ID: 3 passes of demapper with prior + decoder (20 iterations) +
      extrinsic at Eb/N0 3 dB against one plain pass and against one
      60-iteration decoder run on the same data (BLER and time)."""
    from inputs.workloads import data_seed

    B, m, nb = 4096, 4, 11
    S = code.e_tx // m
    seed = data_seed(7, 0)
    bins = torch.tensor(np.arange(B) % nb, dtype=torch.int32, device=dev)
    sig_pts = np.linspace(0.0, 6.0, nb)
    sigma = torch.tensor(sig_pts[np.arange(B) % nb], dtype=torch.float32, device=dev)
    no = torch.full((B,), float(lsim.ebn0_to_n0(3.0, code.k / code.e_tx, m)), dtype=torch.float32,
                    device=dev)
    u = lsim.source_bits(seed, 0, B, code.k, dev)
    c = lsim.encode(code, u)
    ctx = c[:, code.tx_lo:]
    y = lsim.map_awgn(code, m, c, no, seed, 0)
    la = torch.empty((B, code.e_tx), dtype=torch.float32, device=dev)
    le = torch.empty_like(la)
    app = torch.empty((B, code.n_dec), dtype=torch.float32, device=dev)
    bits = torch.empty((B, code.k), dtype=torch.uint8, device=dev)
    mi_cw = torch.empty((B,), dtype=torch.float32, device=dev)
    ia = torch.empty((nb,), dtype=torch.float64, device=dev)
    ie = torch.empty_like(ia)
    p = lsim.params(lsim.SPA_F32, iters=20)
    work = torch.empty(max(1, lsim.decode_workspace(code, p, B)), dtype=torch.uint8, device=dev)

    def demapper_curve():
        lsim.apriori_llrs(code, c, sigma, seed, 0, out=la)
        lsim.mutual_info(la, ctx, bins, nb, mi_cw=mi_cw, mi_bins=ia)
        lsim.demap_prior(m, lsim.DEMAP_EXACT, y, no, la, out=le)
        lsim.mutual_info(le, ctx, bins, nb, mi_cw=mi_cw, mi_bins=ie)

    def decoder_curve():
        lsim.apriori_llrs(code, c, sigma, seed, 0, out=la)
        lsim.mutual_info(la, ctx, bins, nb, mi_cw=mi_cw, mi_bins=ia)
        lsim.decode(code, la, p, want_bits=False, want_app=True, app=app, work=work)
        lsim.extrinsic(code, app, la, out=le)
        lsim.mutual_info(le, ctx, bins, nb, mi_cw=mi_cw, mi_bins=ie)

    demapper_curve()
    dem = (ia.cpu().numpy(), ie.cpu().numpy())
    ms_dem = _elapsed(torch, demapper_curve, 5)
    decoder_curve()
    dec = (ia.cpu().numpy(), ie.cpu().numpy())
    ms_dec = _elapsed(torch, decoder_curve, 5)

    prior = torch.zeros((B, code.e_tx), dtype=torch.float32, device=dev)
    llr = torch.empty_like(prior)
    counts = torch.zeros((1, 3), dtype=torch.int64, device=dev)

    def bicm(passes):
        prior.zero_()
        for i in range(passes):
            lsim.demap_prior(m, lsim.DEMAP_EXACT, y, no, prior, out=llr)
            lsim.decode(code, llr, p, want_bits=(i == passes - 1), want_app=(i < passes - 1),
                        bits=bits, app=app, work=work)
            if i < passes - 1:
                lsim.extrinsic(code, app, llr, out=prior)

    def score():
        counts.zero_()
        lsim.count_errors(u, bits, counts=counts)
        cnt = counts.cpu().numpy()[0]
        return {"bler": round(float(cnt[1] / cnt[2]), 5),
                "ber": round(float(cnt[0] / (cnt[2] * code.k)), 7)}

    res = {}
    for passes in (1, 3):
        bicm(passes)
        res[f"passes_{passes}"] = {"ms": round(_elapsed(torch, lambda: bicm(passes), 3), 4),
                                   **score()}
    # the same 60 decoder iterations in one run, without demapper feedback
    p60 = lsim.params(lsim.SPA_F32, iters=60)
    lsim.demap_prior(m, lsim.DEMAP_EXACT, y, no, torch.zeros_like(prior), out=llr)
    lsim.decode(code, llr, p60, bits=bits, work=work)
    res["plain_60_iters"] = {"ms": round(_elapsed(torch, lambda: lsim.decode(code, llr, p60, bits=bits,
                                                                             work=work), 3), 4),
                             **score()}
    return {"batch": B, "sigma_a": [round(float(x), 2) for x in sig_pts],
            "demapper_ebn0_db": 3.0,
            "demapper_IA": [round(float(x), 5) for x in dem[0]],
            "demapper_IE": [round(float(x), 5) for x in dem[1]],
            "decoder_IA": [round(float(x), 5) for x in dec[0]],
            "decoder_IE": [round(float(x), 5) for x in dec[1]],
            "demapper_curve_ms": round(ms_dem, 4), "decoder_curve_ms": round(ms_dec, 4),
            "bicm_id_ebn0_db": 3.0, "bicm_id": res}


def const_leg(torch, lsim, dev, code, qb, steps=50):
    """End-to-end learning of the constellation with the neural demapper
    (16 trainable points, batch 2048 codewords of the bg2 code's coded bits,
    Eb/N0 ~ U[1, 4] dB): one training step (mapper with the point table,
    demapper, BCE, demapper backward with dL/dy, points adjoint, two Adam
    updates) against the same step with the fixed Gray mapper."""
    from inputs import rand
    from inputs.workloads import data_seed

    B, m = 2048, 4
    r = rand.rng(6006)
    no = torch.tensor(lsim.ebn0_to_n0(r.uniform(1.0, 4.0, B), code.k / code.e_tx, m),
                      dtype=torch.float32, device=dev)
    seed = data_seed(6, 0)
    c = lsim.encode(code, lsim.source_bits(seed, 0, B, code.k, dev))
    ctx = c[:, code.tx_lo:]
    S = code.e_tx // m
    gray = torch.tensor(_gray_points(m), dtype=torch.float32, device=dev)
    pts = gray.clone()
    params = torch.tensor(glorot_params(6007), dtype=torch.float32, device=dev)
    pm, pv = torch.zeros_like(pts), torch.zeros_like(pts)
    wm, wv = torch.zeros_like(params), torch.zeros_like(params)
    y = torch.empty((B, S, 2), dtype=torch.float32, device=dev)
    llr = torch.empty((B, code.e_tx), dtype=torch.float32, device=dev)
    gy = torch.empty_like(y)
    nwork = torch.empty(lsim.ndm_workspace(B, S), dtype=torch.uint8, device=dev)
    pwork = torch.empty(lsim.points_workspace(code, m, B), dtype=torch.uint8, device=dev)
    gpts = torch.empty_like(pts)
    scale = 1.0 / (B * code.e_tx)
    state = {"step": 0}

    def step(trainable=True):
        state["step"] += 1
        if trainable:
            lsim.map_points(code, m, pts, c, no, seed, state["step"] * B, out=y)
        else:
            lsim.map_awgn(code, m, c, no, seed, state["step"] * B, out=y)
        lsim.ndm_forward(params, y, no, out=llr)
        g, loss = lsim.bce_grad(llr, ctx, scale)
        if trainable:
            gp, _ = lsim.ndm_backward(params, y, no, g, work=nwork, gy=gy)
            lsim.points_grad(code, m, pts, c, gy, out=gpts, work=pwork)
            lsim.adam_step(pts, gpts, pm, pv, state["step"], lr=1e-2)
        else:
            gp = lsim.ndm_backward(params, y, no, g, work=nwork)
        lsim.adam_step(params, gp, wm, wv, state["step"], lr=1e-2)
        return loss

    l_first = float(step().item())
    for _ in range(steps - 1):
        loss = step()
    l_last = float(loss.item())
    ms_t = _elapsed(torch, step, 5)
    ms_map = _elapsed(torch, lambda: lsim.map_points(code, m, pts, c, no, seed, 0, out=y), 5)
    ms_pg = _elapsed(torch, lambda: lsim.points_grad(code, m, pts, c, gy, out=gpts, work=pwork), 5)
    ms_f = _elapsed(torch, lambda: step(False), 5)
    nsym = B * S
    return {"batch": B, "symbols": nsym, "step_ms": round(ms_t, 4),
            "fixed_gray_step_ms": round(ms_f, 4),
            "map_points_ms": round(ms_map, 4), "points_grad_ms": round(ms_pg, 4),
            "step_msym_per_s": round(nsym / (ms_t * 1e-3) / 1e6, 1),
            "loss_first_step": round(l_first, 5), f"loss_after_{steps}_steps": round(l_last, 5)}


def _gray_points(m):
    """Initial constellation: the mapper's square Gray QAM (3GPP TS 38.211
    Sec. 5.1) by label, first bit most significant; I takes bits 0, 2, ..,
    Q bits 1, 3, ..; per axis level (1-2a0)(2^(h-1) - (1-2a1)(2^(h-2) - ..))
    over 2^h levels, scaled to unit average energy."""
    h = m // 2

    def level(a):
        v = 1
        for q in range(h - 1, 0, -1):
            v = (1 << (h - q)) - (1 - 2 * a[q]) * v
        return (1 - 2 * a[0]) * v

    norm = math.sqrt(2.0 * (4 ** h - 1) / 3.0)
    out = np.zeros((1 << m, 2))
    for lab in range(1 << m):
        bits = [(lab >> (m - 1 - i)) & 1 for i in range(m)]
        out[lab] = (level(bits[0::2]) / norm, level(bits[1::2]) / norm)
    return out


def wbp_eval_leg(torch, lsim, dev, code, qb, T=10, pre_steps=300, joint_steps=300):
    """Weighted BP (T rounds) fed by the neural demapper, trained end to end,
    then compared with plain sum-product decoding at equal conditions.

    Training (16-QAM, batch 2048, Eb/N0 ~ U[1, 4] dB, fresh codewords every
    step): the demapper alone on the BCE of its LLRs (300 steps, Adam
    1e-2), then demapper and weights jointly on the BCE of the decoder's
    posteriors (300 steps, Adam 1e-3).  Evaluation on other data: 4096
    codewords at each Eb/N0 of 0:0.25:5 dB, BLER of the trained pair, of
    sum-product with the exact demapper at T and at 20 iterations, and the
    Eb/N0 each needs for BLER 1e-2."""
    from inputs import rand
    from inputs.workloads import data_seed

    B, m = 2048, 4
    rate = code.k / code.e_tx
    r = rand.rng(7007)
    params = torch.tensor(glorot_params(7008), dtype=torch.float32, device=dev)
    w = torch.ones((T, code.E), dtype=torch.float32, device=dev)
    pm, pv = torch.zeros_like(params), torch.zeros_like(params)
    wm, wv = torch.zeros_like(w), torch.zeros_like(w)
    y = torch.empty((B, code.e_tx // m, 2), dtype=torch.float32, device=dev)
    llr = torch.empty((B, code.e_tx), dtype=torch.float32, device=dev)
    lpost = torch.empty((B, code.n_dec), dtype=torch.float32, device=dev)
    ckpt = torch.empty((T, B, code.E), dtype=torch.float32, device=dev)
    gwork = torch.empty(lsim.wbp_workspace(code, T, B), dtype=torch.uint8, device=dev)
    nwork = torch.empty(lsim.ndm_workspace(B, code.e_tx // m), dtype=torch.uint8, device=dev)
    seed = data_seed(5, 1)
    losses = {}

    def batch(step):
        no = torch.tensor(lsim.ebn0_to_n0(r.uniform(1.0, 4.0, B), rate, m), dtype=torch.float32,
                          device=dev)
        c = lsim.encode(code, lsim.source_bits(seed, step * B, B, code.k, dev))
        lsim.map_awgn(code, m, c, no, seed, step * B, out=y)
        return c, no

    # one fixed evaluation batch (other seeds, Eb/N0 ~ U[1, 4] dB) on which the
    # posterior loss is taken before and after the joint stage
    fseed = data_seed(5, 3)
    fno = torch.tensor(lsim.ebn0_to_n0(rand.rng(7009).uniform(1.0, 4.0, B), rate, m),
                       dtype=torch.float32, device=dev)
    fc = lsim.encode(code, lsim.source_bits(fseed, 0, B, code.k, dev))
    fy = lsim.map_awgn(code, m, fc, fno, fseed, 0)

    def fixed_bce(wt):
        fl = lsim.ndm_forward(params, fy, fno)
        fp, _ = lsim.wbp_forward(code, wt, fl, T, 20.0, want_ckpt=False)
        _, fl_loss = lsim.bce_grad(fp, fc, 1.0 / (B * code.n_dec))
        return round(float(fl_loss.item()), 6)

    t0 = time.perf_counter()
    for step in range(1, pre_steps + 1):
        c, no = batch(step)
        lsim.ndm_forward(params, y, no, out=llr)
        g, loss = lsim.bce_grad(llr, c[:, code.tx_lo:], 1.0 / (B * code.e_tx))
        gp = lsim.ndm_backward(params, y, no, g, work=nwork)
        lsim.adam_step(params, gp, pm, pv, step, lr=1e-2)
        if step in (1, pre_steps):
            losses[f"demapper_bce_step{step}"] = round(float(loss.item()), 5)
    pm.zero_()
    pv.zero_()
    ones = torch.ones_like(w)
    fixed = {"posterior_bce_before_joint": fixed_bce(ones)}
    for step in range(1, joint_steps + 1):
        c, no = batch(pre_steps + step)
        lsim.ndm_forward(params, y, no, out=llr)
        lsim.wbp_forward(code, w, llr, T, 20.0, ckpt=ckpt, lpost=lpost)
        gpost, loss = lsim.bce_grad(lpost, c, 1.0 / (B * code.n_dec))
        gllr, gw = lsim.wbp_backward(code, w, llr, ckpt, gpost, T, 20.0, work=gwork)
        gp = lsim.ndm_backward(params, y, no, gllr, work=nwork)
        lsim.adam_step(w, gw, wm, wv, step, lr=1e-3)
        lsim.adam_step(params, gp, pm, pv, step, lr=1e-3)
        if step in (1, joint_steps):
            losses[f"posterior_bce_step{step}"] = round(float(loss.item()), 5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    fixed["posterior_bce_after_joint"] = fixed_bce(w)
    fixed["posterior_bce_after_joint_unit_weights"] = fixed_bce(ones)
    dw = (w - 1.0).double()
    fixed["weights"] = {"l2_norm_w_minus_1": round(float(dw.norm()), 5),
                        "max_abs_w_minus_1": round(float(dw.abs().max()), 5),
                        "mean_abs_w_minus_1": round(float(dw.abs().mean()), 6),
                        "count": int(w.numel())}

    Be = 4096
    pts = np.arange(21) * 0.25
    eseed = data_seed(5, 2)
    ye = torch.empty((Be, code.e_tx // m, 2), dtype=torch.float32, device=dev)
    le = torch.empty((Be, code.e_tx), dtype=torch.float32, device=dev)
    lpe = torch.empty((Be, code.n_dec), dtype=torch.float32, device=dev)
    bits = torch.empty((Be, code.k), dtype=torch.uint8, device=dev)
    counts = torch.zeros((1, 3), dtype=torch.int64, device=dev)
    curves = {"wbp_ndm_trained": [], f"spa_exact_{T}": [], "spa_exact_20": []}
    spaT = lsim.params(lsim.SPA_F32, iters=T)
    spa20 = lsim.params(lsim.SPA_F32, iters=20)
    for j, pt in enumerate(pts):
        no = torch.full((Be,), float(lsim.ebn0_to_n0(pt, rate, m)), dtype=torch.float32, device=dev)
        u = lsim.source_bits(eseed + j, 0, Be, code.k, dev)
        c = lsim.encode(code, u)
        lsim.map_awgn(code, m, c, no, eseed + j, 0, out=ye)

        def score(name):
            counts.zero_()
            lsim.count_errors(u, bits, counts=counts)
            cnt = counts.cpu().numpy()[0]
            curves[name].append(round(float(cnt[1] / cnt[2]), 5))

        lsim.ndm_forward(params, ye, no, out=le)
        lsim.wbp_forward(code, w, le, T, 20.0, lpost=lpe, want_ckpt=False)
        lsim.hard_bits(lpe, code.k, out=bits)
        score("wbp_ndm_trained")
        lsim.demap(m, lsim.DEMAP_EXACT, ye, no, out=le)
        lsim.decode(code, le, spaT, bits=bits)
        score(f"spa_exact_{T}")
        lsim.decode(code, le, spa20, bits=bits)
        score("spa_exact_20")
    return {"train_steps": {"demapper_only": pre_steps, "joint": joint_steps},
            "train_seconds": round(train_s, 2), "losses": losses, "fixed_batch": fixed,
            "eval_batch_per_point": Be,
            "ebn0_db": pts.tolist(), "bler": curves,
            "ebn0_db_at_bler_1e-2": {k: ebn0_at_bler(pts, v) for k, v in curves.items()}}


def glorot_params(seed):
    """Glorot-uniform weights, zero biases, flat in the library's order."""
    from inputs import rand
    r = rand.rng(seed)
    out = []
    for fan_out, fan_in in ((64, 3), (64, 64), (4, 64)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        out.append(r.uniform(-lim, lim, fan_out * fan_in))
        out.append(np.zeros(fan_out))
    return np.concatenate(out)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk(job):
    """The oracle's link on codewords cw0 .. cw0+nb-1 of the headline
    workload's first timed step (codeword b at Eb/N0 point b mod 9 of
    1:0.5:5 dB); returns (bit errors, block errors, codewords)."""
    from inputs.workloads import BG1, data_seed
    from oracle import pipeline, qc, stats
    cw0, nb = job
    qb = BG1.load()
    g = qc.graph_from_qcbase(qb, 25344)
    pts = 1.0 + np.arange(9) * 0.5
    n0 = pipeline.n0_for(g, pts[np.arange(cw0, cw0 + nb) % 9], 6)
    tx = pipeline.transmit(g, qb.family, data_seed(3, 1000), cw0, nb, n0, 6, "maxlog")
    bits, _ = pipeline.decode(g, tx["L"], "nms", 20)
    return stats.count_errors(tx["u"], bits)[0]


def cpu_baseline(ncw):
    """The FP64 oracle's link (bits .. layered NMS decode .. count) on a
    bounded sample of the headline workload, in this process."""
    log(f"[bench] cpu baseline: oracle on {ncw} codewords")
    c0 = os.times()
    t0 = time.perf_counter()
    tot = np.zeros(3, dtype=np.int64)
    for lo in range(0, ncw, 16):
        tot += _oracle_chunk((lo, min(16, ncw - lo)))
    dt = time.perf_counter() - t0
    c1 = os.times()
    cpu_s = (c1.user - c0.user) + (c1.system - c0.system)
    return {"value": round(ncw * 8448 / dt / 1e9, 7), "unit": "Gbit/s",
            "codewords_per_s": round(ncw / dt, 2),
            "cores": max(1, int(round(cpu_s / dt))), "kind": "oracle",
            "cpu_model": _cpu_model(), "cpu_seconds": round(cpu_s, 1),
            "sample": f"{ncw} codewords of the bg1 workload (Eb/N0 1:0.5:5 dB interleaved), full "
                      f"link (bits, encode, 64-QAM, AWGN, max-log, FP64 layered normalized "
                      f"min-sum 20 iters, count) in one process, {dt:.1f} s wall",
            "block_errors": int(tot[1])}


def cpu_baseline_pool(ncw):
    """The same oracle link over a process pool, one chunk per worker."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    workers = max(1, min(16, _ncpu()))
    per = max(1, ncw // 8)
    jobs = [(w * per, per) for w in range(workers)]
    log(f"[bench] cpu baseline: oracle pool of {workers} workers x {per} codewords")
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            list(ex.map(_oracle_chunk, [(0, 1)] * workers))      # start-up outside the clock
            t0 = time.perf_counter()
            tot = sum(ex.map(_oracle_chunk, jobs))
            dt = time.perf_counter() - t0
    finally:
        if old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = old
    n = workers * per
    return {"value": round(n * 8448 / dt / 1e9, 7), "unit": "Gbit/s", "cores": workers,
            "codewords_per_s": round(n / dt, 2),
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{n} codewords ({workers} processes x {per}), same link as cpu_baseline, "
                      f"{dt:.1f} s wall", "block_errors": int(tot[1])}


if __name__ == "__main__":
    main()
