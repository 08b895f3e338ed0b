#!/usr/bin/env python
"""Benchmark of the codec hot path on one MI355X.

A step is one encode + one decode of a synthetic frame (positions -> octree occupancy bytes,
attributes -> quantized RAHT coefficients, then octree expansion and inverse RAHT), with the
inputs resident in HBM. The default workload is the 1M-Gaussian frame at octree depth 12 with
56 attribute channels and grouped quantization steps.

Prints one JSON line: whole-job throughput in M Gaussians/s (encode + decode), the roofline
figure of the dominant kernel (timed live with HIP events on the library's stream), and the
FP64 CPU oracle timed on the host on the same workload.

Other workloads (--workload):
  frame100k_J10, frame4M_J14   single frames as above (every single-frame line also carries
                               the FP32-versus-FP64 coefficient error per channel group)
  seq30_J12                    the 30-frame sequence: per-frame launches, one batch, the batch
                               as a replayed HIP graph, and the graph with autotuned sort tiles
  diff500k_J11                 the straight-through differentiable coder: forward + rate-
                               distortion loss + backward, next to a plain encode + decode
  rlgr_frame1M_J12             the block entropy coder on the 1M frame's quantized
                               coefficients: time and size per block length
  color_frame1M                the colour decorrelation (YUV + per-channel KLT of the SH
                               coefficients) on a 1M frame with correlated SH: time, HBM
                               fraction and the coded size with and without it
  rans_frame1M_J12             the occupancy-byte rANS coder on the 1M frame's occupancy
                               bytes: time and size per chunk length
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "M Gaussians/s encode+decode (and frames/s at 1M), % HBM roofline vs CPU oracle"
# (stages 6 and 8, the upper RAHT levels, run inside the launches of stages 5 and 7)
STAGES = {"encode": 0, "decode": 1, "sort": 2, "occupancy": 3, "prelude": 4, "raht_fwd1": 5,
          "raht_inv1": 7, "octree_dec": 9}


# Algorithmic bytes (each input read once, each output written once; float32/int32 rows of C
# channels), per launch:
#   raht_fwd1 : the attribute rows of the n Gaussians (4C each); per voxel the input row of its
#               first member (4), its run start (4), one merge record (4) and the quantized
#               coefficient row written (4C)
#   raht_inv1 : per voxel the coefficient row (4C) + one merge record (4) read, the attribute
#               row written (4C)
def alg_bytes(stage, n, nv, C):
    if stage == "raht_fwd1":
        return n * 4 * C + nv * (4 + 4 + 4 + 4 * C)
    if stage == "raht_inv1":
        return nv * (4 * C + 4 + 4 * C)
    raise KeyError(stage)


# HBM bytes per launch of the first-level transforms on the 1M-Gaussian frame, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# same counter reads for a 512 MiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); see
# profiles/k_raht_transforms_frame1M_J12_pmc.md. They hold for the kernel sources they were
# taken on: with any other sources the figure is reported as null.
KERNEL_SOURCES = ("paper_2606_05650_amd/csrc/k_raht.hip", "paper_2606_05650_amd/csrc/gsc_device.h",
                  "paper_2606_05650_amd/csrc/gsc_internal.h")
PMC_TRAFFIC = {"workload": "frame1M_J12",
               "sources_sha256": "dad95ac0f3de1e7abc5656ae28dd6e92bdf63bc4274d9ef0f04169a914054597",
               "raht_fwd1": 597987115, "raht_inv1": 468067301}
KERNEL_NAMES = {"raht_fwd1": "k_raht_fwd", "raht_inv1": "k_raht_inv"}


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(stage, workload):
    if workload != PMC_TRAFFIC["workload"] or sources_sha256() != PMC_TRAFFIC["sources_sha256"]:
        return None
    return PMC_TRAFFIC[stage]


def alg_bytes_roundtrip(n, nv, C, occ_bytes):
    """Algorithmic bytes of one encode + decode: the encoder reads positions (12 B) and
    attribute rows (4C B) of the n Gaussians and writes the stream (header, occupancy bytes,
    padding, Nv int32 coefficient rows); the decoder reads the stream and writes Nv positions and
    attribute rows."""
    stream = 1024 + occ_bytes + (-(1024 + occ_bytes)) % 256 + nv * 4 * C
    return n * (12 + 4 * C) + 2 * stream + nv * (12 + 4 * C)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def phase_bytes(n, nv, J, occ_bytes):
    """Algorithmic bytes of the sort stage (voxelize, radix sort passes, unique; the bounding
    box runs in the setup launch, outside the stage) and of the occupancy stage."""
    bits = 9 if (3 * J + 8) // 9 < (3 * J + 7) // 8 else 8  # the radix digit width
    P = (3 * J + bits - 1) // bits
    sort = (12 * n + 8 * n) + (P * 24 * n - 4 * n) + (8 * n + 12 * nv)
    occ = 8 * nv + occ_bytes
    return sort, occ


class StageTimer:
    """HIP event pairs recorded by the library around each stage, one pair per step."""

    def __init__(self, gsc, torch, K, names=STAGES):
        self.gsc, self.K, self.events = gsc, K, {}
        for name in names:
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * K)]
            for e in evs:  # torch creates the HIP event on first record
                e.record()
            arr = (ctypes.c_void_p * (2 * K))(*[e.cuda_event for e in evs])
            gsc.lib().gsc_profile_events(STAGES[name], arr, K)
            self.events[name] = (evs, arr)

    def stop(self):
        import numpy as np
        for name in self.events:
            self.gsc.lib().gsc_profile_events(STAGES[name], None, 0)
        out = {}
        for name, (evs, _) in self.events.items():
            out[name] = float(np.mean([evs[2 * i].elapsed_time(evs[2 * i + 1])
                                       for i in range(self.K)]))
        return out


def timed(fn, K, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / K


def base_record(args, value, ms, config, dtype="f32"):
    return {"metric": METRIC, "value": round(value, 3), "unit": "M Gaussians/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


# ------------------------------------------------------------------------ single frame
def frame_bench(args):
    import numpy as np
    import torch
    from paper_2606_05650_amd import gsc, synth

    n, J, table = synth.WORKLOADS[args.workload]
    steps_q = synth.quant_steps(table)
    pos, attr = synth.make_frame(n, seed=2)
    C = attr.shape[1]
    dev = torch.device("cuda:0")
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    p = gsc.make_params(J, C, steps_q)
    ws = gsc.Workspace(n, J, C, dev)
    sbuf = torch.empty(gsc.stream_capacity(n, J, C), dtype=torch.uint8, device=dev)
    info_e = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
    info_d = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
    pos_out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    attr_out = torch.empty((n, C), dtype=torch.float32, device=dev)

    def step():
        gsc.encode_frame(tp, ta, p, ws=ws, stream_buf=sbuf, info=info_e)
        gsc.decode_frame(sbuf, J, C, n, ws=ws, pos_out=pos_out, attr_out=attr_out, info=info_d)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    enc = gsc.Encoded(sbuf, info_e, J, C).check()
    gsc.Decoded(pos_out, attr_out, None, None, info_d).check()
    nv = enc.n_vox()
    occ_bytes = int(gsc.parse_header(sbuf[:gsc.HEADER_BYTES].cpu().numpy())["occ_bytes"])

    K = args.steps
    # the timed steps run without instrumentation; the per-stage times come from K more steps
    # with the library's stage events recorded
    dt = timed(step, K, torch)
    timer = StageTimer(gsc, torch, K)
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    stage_ms = timer.stop()
    # the roofline kernel is timed again with a 512 MiB write before every step, so that the
    # 256 MB last-level cache holds none of its inputs when the step starts
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    cold_timer = StageTimer(gsc, torch, K, names=("raht_fwd1", "raht_inv1"))
    for _ in range(K):
        flush.fill_(1)
        step()
    torch.cuda.synchronize()
    cold_ms = cold_timer.stop()
    del flush

    ms = dt * 1e3
    value = n / dt / 1e6
    dom = max(("raht_fwd1", "raht_inv1"), key=lambda s: cold_ms[s])
    achieved = alg_bytes(dom, n, nv, C) / (cold_ms[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": KERNEL_NAMES[dom],
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(dom, args.workload),
            "alg_bytes_per_launch": alg_bytes(dom, n, nv, C),
            "avg_launch_ms": round(cold_ms[dom], 4),
            "avg_launch_ms_back_to_back": round(stage_ms[dom], 4),
            "timing": "HIP events recorded by the library on its stream around the launch, "
                      "mean over the steps, 512 MiB written before each step"}
    cfg = {"workload": args.workload, "gaussians": n, "voxels": nv, "depth": J, "channels": C,
           "parallelism": "single GPU"}
    out = base_record(args, value, ms, cfg)
    out["frames_per_s"] = round(1e3 / ms, 2)
    out["stage_ms"] = {k: round(v, 4) for k, v in stage_ms.items()}
    out["stage_ms_note"] = "HIP events recorded by the library around each stage, in a separate pass of the same steps (the timed steps run without them)"
    out["roofline"] = roof
    sort_b, occ_b = phase_bytes(n, nv, J, occ_bytes)
    raht_b = alg_bytes("raht_fwd1", n, nv, C) + alg_bytes("raht_inv1", n, nv, C)
    raht_ms = sum(stage_ms[s] for s in ("raht_fwd1", "raht_inv1"))
    out["phase_gbs"] = {"sort": round(sort_b / stage_ms["sort"] / 1e6, 1),
                        "occupancy": round(occ_b / stage_ms["occupancy"] / 1e6, 1),
                        "raht": round(raht_b / raht_ms / 1e6, 1)}
    # the whole step against the HBM peak: every input read once, every output written once
    rt = alg_bytes_roundtrip(n, nv, C, occ_bytes)
    roof["pipeline"] = {"alg_bytes_per_step": rt, "achieved": round(rt / dt / 1e9, 1),
                        "unit": "GB/s", "frac": round(rt / dt / 1e9 / HBM_PEAK_GBS, 4),
                        "ms_per_step": round(ms, 4)}
    roof["stage_frac"] = {
        "sort": round(sort_b / stage_ms["sort"] / 1e6 / HBM_PEAK_GBS, 4),
        "occupancy": round(occ_b / stage_ms["occupancy"] / 1e6 / HBM_PEAK_GBS, 4),
        "raht_fwd1": round(alg_bytes("raht_fwd1", n, nv, C) / stage_ms["raht_fwd1"] / 1e6 / HBM_PEAK_GBS, 4),
        "raht_inv1": round(alg_bytes("raht_inv1", n, nv, C) / stage_ms["raht_inv1"] / 1e6 / HBM_PEAK_GBS, 4)}
    ref = None
    if not args.no_cpu_baseline:
        # the oracle as it stands, single-threaded, on the same frame: encode + decode passes
        # until about cpu_seconds have elapsed (at least one)
        from oracle import oracle as orc
        reps, t0 = 0, time.perf_counter()
        while True:
            r = orc.encode_frame(pos, attr, J, steps_q, 0.5, want_y=(reps == 0))
            orc.decode_frame(r["occ"], r["level_sizes"], J, r["Q"], steps_q, r["bbox_min"],
                             r["cell"])
            if reps == 0:
                ref = r
            reps += 1
            t = time.perf_counter() - t0
            if t >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {"value": round(n * reps / t / 1e6, 4),
                               "unit": "M Gaussians/s", "cores": 1, "kind": "oracle",
                               "sample": f"{reps} encode+decode of the same {n}-Gaussian frame "
                                         f"({t:.1f} s, single-threaded FP64 C)", **cpu_info()}
    if not args.no_errors:
        out["coef_error"] = coefficient_errors(tp, ta, pos, attr, p, J, steps_q, nv, ref)
    print(json.dumps(out))


def coefficient_errors(tp, ta, pos, attr, p, J, steps_q, nv, ref=None):
    """Max over the channels of a group of max_i |y32 - y64| / max_i |y64| (and in steps): the
    FP32 coefficients of one more GPU encode of the frame against the oracle's FP64 ones (ref:
    an oracle encode of the same frame with want_y, else one is run here)."""
    import numpy as np
    import torch
    from oracle import oracle as orc
    from paper_2606_05650_amd import gsc, synth
    C = attr.shape[1]
    coef = torch.empty((tp.shape[0], C), dtype=torch.float32, device=tp.device)
    gsc.encode_frame(tp, ta, p, coef_f32=coef).check()
    y32 = coef[:nv].cpu().numpy().astype(np.float64)
    if ref is None:
        ref = orc.encode_frame(pos, attr, J, steps_q, 0.5, want_y=True)
    y64 = ref["Y"]
    err = np.abs(y32 - y64).max(axis=0)
    rel = err / np.maximum(np.abs(y64).max(axis=0), 1e-300)
    out = {"max_rel": float(rel.max()), "bar": 1e-5}
    for name, sl in synth.channel_group_slices().items():
        out[name] = {"max_rel": float(rel[sl].max()),
                     "max_abs_in_steps": float((err[sl] / steps_q[sl]).max())}
    return out


# ---------------------------------------------------------------------------- sequence
def seq_bench(args):
    import numpy as np
    import torch
    from paper_2606_05650_amd import gsc, synth

    _, J, table = synth.WORKLOADS["seq30_J12"]
    steps_q = synth.quant_steps(table)
    dev = torch.device("cuda:0")
    frames = []
    for t, (pos, attr) in enumerate(synth.make_sequence()):
        if t == 0:
            pos0, attr0 = pos, attr   # the CPU baseline's sample
        frames.append((torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)))
    F = len(frames)
    C = frames[0][1].shape[1]
    ns = [int(f[0].shape[0]) for f in frames]
    ntot = sum(ns)
    p = gsc.make_params(J, C, steps_q, bbox=(np.zeros(3), 1.0 / (1 << J)))
    wse = [gsc.Workspace(n, J, C, dev) for n in ns]
    wsd = [gsc.Workspace(n, J, C, dev) for n in ns]
    sb = [torch.empty(gsc.stream_capacity(n, J, C), dtype=torch.uint8, device=dev) for n in ns]
    ie = [torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev) for _ in ns]
    idd = [torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev) for _ in ns]
    po = [torch.empty((n, 3), dtype=torch.float32, device=dev) for n in ns]
    ao = [torch.empty((n, C), dtype=torch.float32, device=dev) for n in ns]

    def per_frame():
        for f in range(F):
            gsc.encode_frame(frames[f][0], frames[f][1], p, ws=wse[f], stream_buf=sb[f],
                             info=ie[f])
            gsc.decode_frame(sb[f], J, C, ns[f], ws=wsd[f], pos_out=po[f], attr_out=ao[f],
                             info=idd[f])

    def batch():
        outs = gsc.encode_batch(frames, p, workspaces=wse)
        gsc.decode_batch(outs, ns, workspaces=wsd)

    def capture():
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            outs = gsc.encode_batch(frames, p, workspaces=wse)
            decs = gsc.decode_batch(outs, ns, workspaces=wsd)
        return g, outs, decs

    K, W = args.steps, args.warmup
    res = {}
    for name, fn in (("per_frame", per_frame), ("batch", batch)):
        for _ in range(W):
            fn()
        res[name] = timed(fn, K, torch)
    for f in range(F):
        gsc.Encoded(sb[f], ie[f], J, C).check()
    g, outs, decs = capture()
    for _ in range(W):
        g.replay()
    res["graph"] = timed(g.replay, K, torch)
    ref_bytes = [o.check().to_bytes() for o in outs[:2]]
    chosen, vt, _ = gsc.autotune(frames, p, reps=2, workspaces=wse)
    g2, outs2, decs2 = capture()
    for _ in range(W):
        g2.replay()
    res["graph_autotuned"] = timed(g2.replay, K, torch)
    torch.cuda.synchronize()
    same = all(o.check().to_bytes() == b for o, b in zip(outs2[:2], ref_bytes))
    for d in decs2:
        d.check()
    dt = res["graph_autotuned"]
    cfg = {"workload": "seq30_J12", "frames": F, "gaussians": ntot, "depth": J, "channels": C,
           "parallelism": "single GPU"}
    out = base_record(args, ntot / dt / 1e6, dt * 1e3, cfg)
    out["frames_per_s"] = round(F / dt, 2)
    out["modes_ms_per_sequence"] = {k: round(v * 1e3, 3) for k, v in res.items()}
    out["modes_m_gaussians_per_s"] = {k: round(ntot / v / 1e6, 2) for k, v in res.items()}
    out["autotune"] = {"chosen_variant": chosen, "encode_ms_per_variant": [round(t, 3) for t in vt],
                       "streams_identical": same}
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        t0 = time.perf_counter()
        ref = orc.encode_frame(pos0, attr0, J, steps_q, 0.5, bbox=(np.zeros(3), 1.0 / (1 << J)))
        orc.decode_frame(ref["occ"], ref["level_sizes"], J, ref["Q"], steps_q, ref["bbox_min"],
                         ref["cell"])
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(pos0.shape[0] / t / 1e6, 4), "unit": "M Gaussians/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"encode+decode of frame 0 ({pos0.shape[0]} Gaussians, "
                                         f"{t:.1f} s, single-threaded FP64 C)"}
    print(json.dumps(out))


# ------------------------------------------------------------------- differentiable coder
def ste_bench(args):
    import torch
    from paper_2606_05650_amd import gsc, synth
    from paper_2606_05650_amd.ste import SteCoder, SteCoderPadded, rd_loss

    n, J, table = synth.WORKLOADS["diff500k_J11"]
    lam = 0.01
    steps_q = synth.quant_steps(table)
    pos, attr = synth.make_frame(n, seed=4)
    C = attr.shape[1]
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(pos).to(dev)
    ta = torch.from_numpy(attr).to(dev).requires_grad_(True)
    steps_t = torch.from_numpy(steps_q).to(dev)
    p = gsc.make_params(J, C, steps_q)

    def ste_step():
        # the layer that never waits for the device (rows past Nv zero, Nv on the device)
        ta.grad = None
        yhat, ahat, aref, nv = SteCoderPadded.apply(ta, tp, p)
        loss, _, _ = rd_loss(yhat, ahat, aref, steps_t, lam, nv=nv)
        loss.backward()

    def ste_step_sync():
        # the layer that cuts its outputs to Nv rows (one host synchronization per step)
        ta.grad = None
        yhat, ahat, aref = SteCoder.apply(ta, tp, p)
        loss, _, _ = rd_loss(yhat, ahat, aref, steps_t, lam)
        loss.backward()

    ws = gsc.Workspace(n, J, C, dev)
    sbuf = torch.empty(gsc.stream_capacity(n, J, C), dtype=torch.uint8, device=dev)
    pos_out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    attr_out = torch.empty((n, C), dtype=torch.float32, device=dev)
    tad = ta.detach()

    def plain():
        gsc.encode_frame(tp, tad, p, ws=ws, stream_buf=sbuf)
        gsc.decode_frame(sbuf, J, C, n, ws=ws, pos_out=pos_out, attr_out=attr_out)

    K, W = args.steps, args.warmup
    for _ in range(W):
        ste_step()
        ste_step_sync()
        plain()
    t_ste = timed(ste_step, K, torch)
    t_sync = timed(ste_step_sync, K, torch)
    t_plain = timed(plain, K, torch)
    cfg = {"workload": "diff500k_J11", "gaussians": n, "depth": J, "channels": C,
           "lambda": lam, "parallelism": "single GPU"}
    out = base_record(args, n / t_ste / 1e6, t_ste * 1e3, cfg)
    out["step"] = "straight-through forward + rate-distortion loss + backward to the attributes"
    out["synchronizing_layer_ms"] = round(t_sync * 1e3, 4)
    out["plain_encode_decode_ms"] = round(t_plain * 1e3, 4)
    out["plain_m_gaussians_per_s"] = round(n / t_plain / 1e6, 2)
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        t0 = time.perf_counter()
        orc.ste_grad(pos, attr, J, steps_q, 0.5, lam)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(n / t / 1e6, 4), "unit": "M Gaussians/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"one loss + gradient of the {n}-Gaussian frame "
                                         f"({t:.1f} s, single-threaded FP64 C)"}
    print(json.dumps(out))


# ------------------------------------------------------------------ block entropy coder
def rlgr_bench(args):
    """The block entropy coder (Sec. 3.4) on the quantized coefficients of the 1M-Gaussian frame:
    GPU encode and decode time and stream size per block length, next to one block per channel
    (the sequential coder, from the CPU oracle) and the oracle's time at the chosen block."""
    import numpy as np
    import torch
    from paper_2606_05650_amd import gsc, synth

    n, J, table = synth.WORKLOADS["frame1M_J12"]
    steps_q = synth.quant_steps(table)
    pos, attr = synth.make_frame(n, seed=2)
    C = attr.shape[1]
    dev = torch.device("cuda:0")
    enc = gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev),
                           gsc.make_params(J, C, steps_q))
    torch.cuda.synchronize()
    enc.check()
    blob = np.frombuffer(enc.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    nv = int(h["n_vox"])
    Q = blob[int(h["coef_offset"]):int(h["total_bytes"])].view(np.int32).reshape(nv, C)
    tq = torch.from_numpy(np.ascontiguousarray(Q)).to(dev)
    raw = Q.nbytes
    rows = []
    for B in (256, 512, 1024, 2048, 4096, 8192):
        cap = gsc.rlgr_capacity(nv, C, B)
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
        ws = torch.empty(gsc.rlgr_workspace_size(nv, B), dtype=torch.uint8, device=dev)
        info = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
        qd = torch.empty_like(tq)
        wsd = torch.empty(8, dtype=torch.uint8, device=dev)
        infod = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
        s = gsc.rlgr_encode(tq, B, out=out, ws=ws, info=info)
        torch.cuda.synchronize()
        s.check()
        nbytes = s.nbytes()
        for _ in range(args.warmup):
            gsc.rlgr_encode(tq, B, out=out, ws=ws, info=info)
            gsc.rlgr_decode(out, nv, C, B, nbytes=nbytes, q=qd, ws=wsd, info=infod)
        te = timed(lambda: gsc.rlgr_encode(tq, B, out=out, ws=ws, info=info), args.steps, torch)
        td = timed(lambda: gsc.rlgr_decode(out, nv, C, B, nbytes=nbytes, q=qd, ws=wsd, info=infod),
                   args.steps, torch)
        assert int(infod[0].item()) == 0 and torch.equal(qd, tq), "entropy coder round trip"
        rows.append({"block": B, "bytes": nbytes, "bits_per_coef": round(8 * nbytes / Q.size, 3),
                     "enc_ms": round(te * 1e3, 4), "dec_ms": round(td * 1e3, 4),
                     "enc_gbs_raw": round(raw / te / 1e9, 1), "dec_gbs_raw": round(raw / td / 1e9, 1)})
    out = {"workload": "rlgr_frame1M_J12", "coefficients": int(Q.size), "raw_bytes": raw,
           "blocks": rows}
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        # one block per channel: the sequential coder, the size every blocking is compared with
        off, w = orc.rlgr_encode(Q, nv)
        seq = 32 + 4 * len(off) + 4 * int(off[-1])
        for r in rows:
            r["delta_size_vs_one_block_per_channel"] = round(r["bytes"] / seq - 1.0, 5)
        t0 = time.perf_counter()
        orc.rlgr_encode(Q, 512)
        t = time.perf_counter() - t0
        out["one_block_per_channel_bytes"] = seq
        out["cpu_baseline"] = {"encode_ms_block512": round(t * 1e3, 1), "cores": 1, "kind": "oracle",
                               "sample": "one encode of the frame's coefficients (single-threaded C)"}
    print(json.dumps(out))


def color_bench(args):
    """The colour decorrelation (Sec. 4) on a 1M-Gaussian frame with correlated SH coefficients:
    GPU forward (Gram matrices, eigenvectors, per-row transform) and inverse time against the
    HBM peak, the round-trip error, and the effect on the coded size: the frame encoded with the
    grouped steps and its coefficients entropy-coded with blocks of 512, with and without the
    colour step, next to the SH reconstruction error of each (voxels holding one Gaussian)."""
    import numpy as np
    import torch
    from paper_2606_05650_amd import gsc, synth

    n, J, table = synth.WORKLOADS["frame1M_J12"]
    steps_q = synth.quant_steps(table)
    pos, attr = synth.make_color_frame(n, seed=2)
    C = attr.shape[1]
    dev = torch.device("cuda:0")
    tp, ta = torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev)
    out, back = torch.empty_like(ta), torch.empty_like(ta)
    klt = torch.empty((3, 15, 15), dtype=torch.float32, device=dev)
    eig = torch.empty((3, 15), dtype=torch.float64, device=dev)
    ws = torch.empty(gsc.color_workspace_size(n), dtype=torch.uint8, device=dev)
    info = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)

    def fwd():
        gsc.color_forward(ta, out=out, klt=klt, eig=eig, ws=ws, info=info)

    def inv():
        gsc.color_inverse(out, klt, out=back)

    for _ in range(args.warmup):
        fwd()
        inv()
    tf = timed(fwd, args.steps, torch)
    ti = timed(inv, args.steps, torch)
    # the Gram pass reads every row's 45 AC values; the transform reads and writes every row
    bytes_f, bytes_i = n * (45 * 4 + 2 * 4 * C), n * 2 * 4 * C
    rt_err = ((back - ta).abs().max() / ta.abs().max()).item()

    p = gsc.make_params(J, C, steps_q)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    vof = torch.empty(n, dtype=torch.int32, device=dev)

    def coded(rows):
        e = gsc.encode_frame(tp, rows, p, perm=perm, voxel_of=vof)
        torch.cuda.synchronize()
        e.check()
        blob = np.frombuffer(e.to_bytes(), dtype=np.uint8)
        h = gsc.parse_header(blob)
        nv = int(h["n_vox"])
        Q = blob[int(h["coef_offset"]):int(h["total_bytes"])].view(np.int32).reshape(nv, C)
        s_ = gsc.rlgr_encode(torch.from_numpy(np.ascontiguousarray(Q)).to(dev), 512)
        d = gsc.decode_frame(e.stream, J, C, n)
        torch.cuda.synchronize()
        s_.check()
        d.check()
        return int(h["occ_bytes"]), s_.nbytes(), d.attr[:nv], nv

    occ0, b0, dec0, nv = coded(ta)
    occ1, b1, dec1, _ = coded(out)
    rgb1 = gsc.color_inverse(dec1.contiguous(), klt)[:nv]
    v = vof.cpu().numpy().astype(np.int64)
    cnt = np.bincount(v, minlength=nv)
    single = np.nonzero(cnt[v] == 1)[0]          # Gaussians alone in their voxel
    vox = torch.from_numpy(v[single]).to(dev)
    src = ta[torch.from_numpy(single).to(dev)][:, 8:56]
    rmse = lambda dec: (dec[vox][:, 8:56] - src).pow(2).mean().sqrt().item()
    res = {"workload": "color_frame1M", "gaussians": n, "channels": C,
           "forward_ms": round(tf * 1e3, 4), "inverse_ms": round(ti * 1e3, 4),
           "forward_gbs": round(bytes_f / tf / 1e9, 1), "inverse_gbs": round(bytes_i / ti / 1e9, 1),
           "forward_frac_hbm": round(bytes_f / tf / 1e9 / HBM_PEAK_GBS, 4),
           "inverse_frac_hbm": round(bytes_i / ti / 1e9 / HBM_PEAK_GBS, 4),
           "round_trip_max_rel_error": rt_err,
           "eigenvalues_first3": [[round(float(x), 8) for x in row[:3]] for row in eig.cpu().numpy()],
           "coded_bytes": {"rgb": occ0 + b0, "yuv_klt": occ1 + b1, "occupancy": occ0,
                           "coefficients_rgb": b0, "coefficients_yuv_klt": b1},
           "sh_rmse": {"rgb": round(rmse(dec0), 6), "yuv_klt": round(rmse(rgb1), 6)},
           "steps": "grouped (scale 1/32, rotation 1/128, opacity 1/32, SH DC 1/64, SH rest 1/16) "
                    "on the stored channels, with and without the colour step",
           "data": "synthetic, correlated SH coefficients"}
    if not args.no_cpu_baseline:
        from oracle import color_oracle as co
        t0 = time.perf_counter()
        co.color_forward(attr, 8)
        t = time.perf_counter() - t0
        res["cpu_baseline"] = {"forward_ms": round(t * 1e3, 1), "kind": "oracle",
                               "sample": "one forward of the frame (numpy FP64)"}
    print(json.dumps(res))


def rans_bench(args):
    """The occupancy-byte rANS coder on the 1M-Gaussian frame's occupancy bytes: GPU encode and
    decode time and the coded size per chunk length, next to the order-0 entropy of the bytes
    and the oracle's encode time."""
    import numpy as np
    import torch
    from paper_2606_05650_amd import gsc, synth

    n, J, table = synth.WORKLOADS["frame1M_J12"]
    pos, attr = synth.make_frame(n, seed=2)
    dev = torch.device("cuda:0")
    enc = gsc.encode_frame(torch.from_numpy(pos).to(dev), torch.from_numpy(attr).to(dev),
                           gsc.make_params(J, attr.shape[1], synth.quant_steps(table)))
    torch.cuda.synchronize()
    enc.check()
    blob = np.frombuffer(enc.to_bytes(), dtype=np.uint8)
    h = gsc.parse_header(blob)
    occ = np.ascontiguousarray(blob[int(h["occ_offset"]):int(h["occ_offset"]) + int(h["occ_bytes"])])
    cnt = np.bincount(occ, minlength=256).astype(np.float64)
    p = cnt[cnt > 0] / occ.size
    entropy_bytes = float(-(p * np.log2(p)).sum() * occ.size / 8)
    t_occ = torch.from_numpy(occ).to(dev)
    rows = []
    for K in (256, 512, 1024, 4096, 16384):
        out = torch.empty(gsc.rans_capacity(occ.size, K), dtype=torch.uint8, device=dev)
        ws = torch.empty(gsc.rans_workspace_size(occ.size, K), dtype=torch.uint8, device=dev)
        info = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
        dec = torch.empty(occ.size, dtype=torch.uint8, device=dev)
        wsd = torch.empty(8, dtype=torch.uint8, device=dev)
        infod = torch.zeros(gsc.INFO_WORDS, dtype=torch.int32, device=dev)
        s_ = gsc.rans_encode(t_occ, K, out=out, ws=ws, info=info)
        torch.cuda.synchronize()
        s_.check()
        nbytes = s_.nbytes()
        for _ in range(args.warmup):
            gsc.rans_encode(t_occ, K, out=out, ws=ws, info=info)
            gsc.rans_decode(out, occ.size, K, nbytes=nbytes, out=dec, ws=wsd, info=infod)
        te = timed(lambda: gsc.rans_encode(t_occ, K, out=out, ws=ws, info=info), args.steps, torch)
        td = timed(lambda: gsc.rans_decode(out, occ.size, K, nbytes=nbytes, out=dec, ws=wsd, info=infod),
                   args.steps, torch)
        assert int(infod[0].item()) == 0 and torch.equal(dec, t_occ), "rANS round trip"
        rows.append({"chunk": K, "bytes": nbytes, "ratio": round(nbytes / occ.size, 4),
                     "enc_ms": round(te * 1e3, 4), "dec_ms": round(td * 1e3, 4),
                     "enc_gbs": round(occ.size / te / 1e9, 2), "dec_gbs": round(occ.size / td / 1e9, 2)})
    res = {"workload": "rans_frame1M_J12", "occupancy_bytes": int(occ.size),
           "order0_entropy_bytes": round(entropy_bytes), "chunks": rows}
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        t0 = time.perf_counter()
        orc.rans_encode(occ, 4096)
        t = time.perf_counter() - t0
        res["cpu_baseline"] = {"encode_ms_chunk4096": round(t * 1e3, 1), "cores": 1, "kind": "oracle",
                               "sample": "one encode of the frame's occupancy bytes (single-threaded C)"}
    print(json.dumps(res))


def copy_calibration(args):
    """Plain copies of a 512 MiB buffer: each launch reads and writes exactly 536,870,912 bytes."""
    import torch
    dev = torch.device("cuda:0")
    a = torch.ones(512 << 20, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    for _ in range(max(args.steps, 1)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": a.numel(), "launches": max(args.steps, 1)}))


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="frame1M_J12")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="single frames: oracle encode+decode passes until this many seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="single frames: skip the FP32-versus-FP64 coefficient error per channel "
                         "group (reported by default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 512 MiB device-to-device copies (the reference kernel "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this codec shards by frame (see the design notes), and "
              "this build runs on a single MI355X, so --gpus must be 1.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "seq30_J12":
        seq_bench(args)
    elif args.workload == "diff500k_J11":
        ste_bench(args)
    elif args.workload == "rlgr_frame1M_J12":
        rlgr_bench(args)
    elif args.workload == "color_frame1M":
        color_bench(args)
    elif args.workload == "rans_frame1M_J12":
        rans_bench(args)
    else:
        frame_bench(args)


if __name__ == "__main__":
    main()
