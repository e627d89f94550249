"""Throughput of the conjunctive ML-UDF query on one MI355X.

Workload (default): cnn4_u8_128, the largest single-GPU configuration: 1,048,576 synthetic frames
128x128x3 uint8 (51.5 GB, generated straight into HBM by the device frame generator, bit-identical
to the numpy recipe), four CNN predicates (conv 32-64-128-256, stride 2, global mean, FC 10) with
class-subset thresholds for selectivities 0.8 / 0.6 / 0.4 / 0.2.  Frames are resident in HBM before
timing starts; models are uploaded at session creation (setup, not timed).  --workload 1..4
selects the other synthetic workloads; a second, smaller line for the 65,536-frame 64x64 CNN
workload is added under "cnn3_drift64" (--no-secondary skips it).

A step is one whole query: reset, push every tuple (route, multi-split, evaluate, forward
survivors, materialise the sorted ids) and copy ids and statistics to the host.

Forms:
  full   learned content-based router (score routing as control arm, judge and fallback) +
         grouped persistent launches per round (MLP tile shapes from the autotuner, timed at
         setup), each whole push captured once in a HIP graph (at setup) and replayed + low
         precision first pass on MFMA (fp32 accumulate) with margins within tau re-scored in FP32
         and within tau32 in FP64.  `value`; timed over exactly --steps steps.
  eager  the full form launched kernel by kernel, with HIP events recorded around each round's
         phases: the roofline, phase times and statistics come from this run (`eager_value`).
  score  as eager, but score-driven routing only.
  plain  FP32 first pass (tau32 band -> FP64), score-driven routing, one launch per predicate,
         no graph.
  host   the full form pushed from pinned host memory in the workload's push batches, over a
         prefix of --host-blocks batches (PCIe-inclusive; never `value`).
  The eager / score / plain / host forms are ablations, timed over --ablation-steps steps.
  Every form's session calibrates its per-predicate bands at setup (untimed): tau_k and tau32_k
  are `--safety` (2) times the largest margin error of the first pass / FP32 pass against the
  FP64 pass on 8,192 separate frames of the same generator (--no-calibrate: fixed bands 0.015 /
  1e-5).

Prints one JSON line (the full form's throughput as `value`, the plain form beside it, the
dominant kernels' roofline from HIP events recorded by the library on its stream, and the FP64
oracle timed on the host cores on a bounded sample whose ids are also checked).  Two more
objects: `reuse` (the 65,536-frame workload's recurrent query after an exploratory one filled
the result cache, with and without reuse-aware routing; --no-reuse skips it) and `compaction`
(routing, multi-split, forwarding and result materialisation on 2^26 tuples with given outcomes,
against their algorithmic bytes; --no-compaction skips it, --compaction-only runs only it).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tuples/sec through ML-UDF conjunction at 1 GPU, learned+batched vs plain; MFMA util"
# HBM bytes of the first pass come from FETCH_SIZE / WRITE_SIZE runs of this script, scaled by the
# same counters on a 1 GiB device copy (the byte-counter summaries in profiles/), and are reported
# only while the kernel sources hash to the build those runs measured (None otherwise).
# The 4-layer CNN first pass (front + layer-3 + layer-4 launches, bf16): HBM bytes per evaluated
# frame from the same counters (profiles/cnn4_u8_128_first_pass.md), valid while the kernel
# sources hash to the recorded value; the figure per launch is this times the launch's frames.
FIRST_PASS_BYTES_PER_EVAL = {"cnn4_u8_128": ('abc034d3ba5f195a', 10.150e9 / 18280.8)}
FIRST_PASS_SOURCES = ("paper_2403_14902_amd/csrc/cnn4.hip", "paper_2403_14902_amd/csrc/common.h")


def sources_hash(paths) -> str:
    import hashlib
    h = hashlib.sha1()
    for f in paths:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK = {"bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}   # dense MFMA peaks, TFLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--n", type=int, default=0, help="tuples: a prefix of the workload (0: all)")
    ap.add_argument("--host", action="store_true",
                    help="also time the full form pushed from pinned host memory (workloads without "
                         "push batches; the streamed workload always adds it)")
    ap.add_argument("--host-blocks", type=int, default=16,
                    help="push batches of the pinned-host form (a prefix of the workload)")
    ap.add_argument("--ablation-steps", type=int, default=3)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--wave", type=int, default=16384)
    ap.add_argument("--tau", type=float, default=0.0)
    ap.add_argument("--no-calibrate", action="store_true",
                    help="fixed bands tau = 0.015, tau32 = 1e-5 instead of bands calibrated on separate frames")
    ap.add_argument("--safety", type=float, default=2.0)
    ap.add_argument("--route", default="learned")
    ap.add_argument("--precision", default="bf16", help="first pass of the full form: bf16 or fp8")
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 first-pass form")
    ap.add_argument("--no-rescore3", action="store_true",
                    help="no three-product re-score tier in the bf16 forms of the 4-layer CNN workload")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--check-sample", type=int, default=2048)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB: first copy a device buffer of this size three times (a plain copy kernel "
                         "of known traffic, to scale hardware byte counters)")
    ap.add_argument("--no-compaction", action="store_true", help="skip the standalone routing/compaction run")
    ap.add_argument("--no-reuse", action="store_true", help="skip the result-reuse (recurrent query) run")
    ap.add_argument("--no-concurrent", action="store_true", help="skip the concurrent host/GPU predicate run")
    ap.add_argument("--no-variable", action="store_true", help="skip the variable-size (crop) run")
    ap.add_argument("--variable-only", action="store_true", help="run only the variable-size (crop) run")
    ap.add_argument("--concurrent-only", action="store_true", help="run only the concurrent host/GPU predicate run")
    ap.add_argument("--concurrent-points", type=lambda v: [tuple(float(x) for x in p.split(":")) for p in v.split(",")],
                    default=[(0.0, 0.05), (0.1, 0.05), (0.2, 0.05), (0.1, 0.12)],
                    help="GPU-threshold shift : host threshold pairs of the concurrent run")
    ap.add_argument("--compaction-only", action="store_true",
                    help="run only the standalone routing/compaction measurement and print its JSON")
    ap.add_argument("--compaction-log2n", type=int, default=26)
    ap.add_argument("--errors", type=int, default=4096,
                    help="frames on which bf16 / fp32 logits and margins are compared with fp64 (0: skip)")
    return ap.parse_args()


def first_pass_traffic(cfg, n, ev, launches):
    """HBM bytes per first-pass launch from the byte-counter runs of this kernel build, else None."""
    if cfg.name in FIRST_PASS_BYTES_PER_EVAL:
        sha, per_eval = FIRST_PASS_BYTES_PER_EVAL[cfg.name]
        if sources_hash(FIRST_PASS_SOURCES) == sha:
            return per_eval * float(ev.sum()) / max(1, launches)
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_form(hydro, torch, specs, frames_dev, dtype, pt, seg_len, policy, steps, warmup, n, cal=None,
             safety=2.0, push_batch=0):
    """Session setup (weights, autotune and, with `cal`, band calibration) is untimed.  With
    push_batch > 0 the tuples are pushed in blocks of that size (from wherever frames_dev lives,
    e.g. pinned host memory)."""
    blk = push_batch if push_batch > 0 else n
    sess = hydro.Session(specs, policy, frames_dev.shape[1], blk)
    bands = sess.calibrate(cal, dtype, safety) if cal is not None else None
    run_form.tau16 = sess.bands()[1] if cal is not None else None
    res = None

    def one_query():
        sess.reset()
        for lo in range(0, n, blk):
            sess.push(frames_dev[lo:lo + blk], dtype, pt.thresholds, seg_len, id_base=lo)
        return sess.finish()

    for _ in range(warmup):
        res = one_query()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, stats_all = [], []
    for _ in range(steps):
        res = one_query()
        infos.append(sess.info())
        stats_all.append(res[1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sess.close()
    run_form.bands = bands
    return res[0], stats_all, infos, t1 - t0


def make_device_frames(hs, torch, cfg, n):
    """The workload's first n frames in HBM: structured frames come from the device generator
    (bit-identical to the numpy recipe, no 51.5 GB host copy); the small uniform fp32 workload is
    generated by numpy and copied."""
    if cfg.frame_kind == "uniform":
        return torch.from_numpy(hs.make_frames_parallel(cfg, 0, n)).cuda()
    from hydro_synth import device as hd
    t = time.perf_counter()
    out = hd.make_frames_device(cfg, 0, n, chunks_per_call=256)
    torch.cuda.synchronize()
    log(f"[bench] {n} frames generated on the device in {time.perf_counter() - t:.1f} s")
    return out


def host_frames(frames_dev, sel, torch):
    """Host (numpy) copy of the frames at indices `sel` of a device tensor."""
    idx = torch.from_numpy(np.ascontiguousarray(sel)).cuda()
    return frames_dev.index_select(0, idx).cpu().numpy()


def measure(args, wl, n_req, steps, warmup, abl_steps, hydro, torch, hs, primary):
    """Every form of one workload; returns the JSON object of its line."""
    cfg = hs.workload(wl)
    n = min(n_req if n_req > 0 else cfg.n, cfg.n)
    log(f"[bench] workload {cfg.name}: {n} tuples")
    frames_dev = make_device_frames(hs, torch, cfg, n)
    pt = hs.load_predicates(cfg)
    weights = [hs.make_model(d) for d in cfg.models]
    specs = [hydro.ModelSpec.from_weights(w, m) for w, m in zip(weights, pt.class_masks)]
    seg_len = cfg.n // cfg.n_seg
    flops = np.array([d.flops() for d in cfg.models])
    # band calibration sample: frames of the same generator, different seed (not the query's)
    cal = None if args.no_calibrate else torch.from_numpy(hs.calibration_frames(cfg)).cuda()

    extra = {}
    if args.no_calibrate:
        extra.update(tau=0.015, tau32=1e-5)      # the fixed bands
    if args.tau > 0:
        extra["tau"] = args.tau
    d0 = cfg.models[0]
    if d0.arch == "mlp":
        kernel_label = "mlp_gemm_kernel<bf16> + mlp_head_kernel (first pass, grouped over predicates)"
    elif cfg.hw == 64 and all(len(d.widths) == 3 for d in cfg.models):
        kernel_label = "cnn_fused_kernel<bf16, *> (first pass: one launch per width class)"
    elif cfg.hw == 128 and all(tuple(d.widths) == (32, 64, 128, 256) for d in cfg.models):
        kernel_label = ("c4_front_kernel<bf16> (layers 1-2) + c4_gemm_bf16_kernel<2> (layer 3) + "
                        "c4_gemm_bf16_kernel<3> (layer 4, pool, FC, decision): the first pass of a round")
    else:
        kernel_label = "gconv_* layer kernels + gcnn_head_kernel (first pass, grouped over predicates)"
    prec = args.precision
    c4 = cfg.hw == 128 and all(d.arch == "cnn" and tuple(d.widths) == (32, 64, 128, 256) for d in cfg.models)
    # the three-product re-score tier between the bf16 first pass and fp32 (4-layer CNN predicates)
    mid = {"rescore3": 1} if prec == "bf16" and c4 and not args.no_rescore3 else {}
    full_pol = hydro.make_policy(args.route, precision=prec, wave=args.wave, grouped=1, autotune=1, time_kernels=1,
                                 **extra, **mid)
    log(f"[bench] eager full form ({args.route} routing)")
    ids, stats_all, infos, dt = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, full_pol,
                                         abl_steps, 1, n, cal, args.safety)
    bands = run_form.bands
    tau16_full = run_form.tau16
    eager_value = n * abl_steps / dt

    # dominant kernels: the first-pass launches of every round
    ev = np.array([[s["evaluated"] for s in st] for st in stats_all], dtype=np.float64)
    first_flops = float((ev * flops).sum())
    first_ms = sum(i["first_pass_ms"] for i in infos)
    launches = sum(i["timed_rounds"] for i in infos)
    achieved = first_flops / (first_ms * 1e-3) / 1e12 if first_ms > 0 else 0.0
    resc = np.array([[s["rescored"] for s in st] for st in stats_all], dtype=np.float64)
    resc16 = np.array([[s["rescored16"] for s in st] for st in stats_all], dtype=np.float64)
    f32_in = resc16 if mid else resc                   # the frames the fp32 tier re-scored
    f32_flops = float((f32_in * flops).sum())
    f32_ms = sum(i["f32_pass_ms"] for i in infos)
    mid_ms = sum(i["mid_pass_ms"] for i in infos)
    last = stats_all[-1]

    # headline: the full form as deployed, each push replayed from its captured HIP graph
    log(f"[bench] full form, graph replay: {warmup} warmup + {steps} timed steps")
    gpol = hydro.make_policy(args.route, precision=prec, wave=args.wave, grouped=1, autotune=1, use_graph=1,
                             **extra, **mid)
    ids_g, _, _, dtg = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, gpol, steps, warmup, n,
                                cal, args.safety)
    assert np.array_equal(ids_g, ids), "graph replay and eager runs disagree"
    value = n * steps / dtg
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dtg * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {n} frames {cfg.hw}x{cfg.hw}x3 {cfg.dtype}, "
                               f"{cfg.k} predicates, {cfg.n_seg} threshold segments"
                               + (f" (first {n} of {cfg.n} tuples)" if n < cfg.n else ""),
                   "form": f"full: {prec} first pass + " + ("bf16/" if prec == "fp8" else "")
                           + ("three-product bf16/" if mid else "") + "fp32/fp64 re-score, "
                           + args.route + " routing, grouped, each push replayed from a captured HIP graph",
                   "frames_in": "HBM (generated on the device before timing)",
                   "wave": args.wave, "tuples_per_step": n, "ablation_steps": abl_steps},
        "roofline": {
            "bound": "mfma",
            "kernel": kernel_label,
            "achieved": achieved,
            "peak": PEAK[prec],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK[prec],
            "traffic": first_pass_traffic(cfg, n, ev, launches),
            "flops_per_launch": first_flops / max(1, launches),
            "avg_launch_ms": first_ms / max(1, launches),
        },
        "eager_value": eager_value,
        "eager_ms_per_step": dt * 1e3 / abl_steps,
        "phases_ms_per_step": {
            "route": sum(i["route_ms"] for i in infos) / abl_steps,
            "first_pass": first_ms / abl_steps,
            **({"three_product_rescore": mid_ms / abl_steps} if mid else {}),
            "fp32_rescore": f32_ms / abl_steps,
            "fp64_escalate": sum(i["f64_pass_ms"] for i in infos) / abl_steps,
        },
        "fp32_rescore_tflops": f32_flops / (f32_ms * 1e-3) / 1e12 if f32_ms > 0 else 0.0,
        **({"three_product_rescore_tflops": float((resc * flops).sum()) / (mid_ms * 1e-3) / 1e12 if mid_ms > 0
            else 0.0} if mid else {}),
        "per_predicate": [{"evaluated": s["evaluated"], "passed": s["passed"], "rescored": s["rescored"],
                           "rescored16": s["rescored16"], "escalated": s["escalated"],
                           "selectivity": round(s["selectivity"], 4)} for s in last],
        "band_fraction": {"first_pass": float(resc.sum() / max(1.0, ev.sum())),
                          **({"three_product": float(resc16.sum() / max(1.0, resc.sum()))} if mid else {}),
                          "fp32": float(sum(x["escalated"] for st in stats_all for x in st)
                                        / max(1.0, float(f32_in.sum())))},
        "n_result": int(ids.size),
        "bands": ({"calibrated_on": f"{cal.shape[0]} separate frames", "safety": args.safety,
                   "tau": [round(float(x), 6) for x in bands[0]],
                   **({"tau16": [float(x) for x in tau16_full]} if mid else {}),
                   "tau32": [float(x) for x in bands[1]]} if bands is not None else
                  {"tau": float(full_pol.tau), "tau32": float(full_pol.tau32)}),
        "rounds": infos[-1]["rounds"],
    }
    info_last = infos[-1]
    out["router"] = {k: info_last[k] for k in ("learned_routed", "stats_routed", "learned_active", "train_steps")}
    if info_last["arm_tuples"][0] > 0 and info_last["arm_tuples"][1] > 0:
        # the judge's figures: UDF work per finished tuple of each arm since the learned arm began
        out["router"]["mflop_per_finished_tuple"] = {
            "control": info_last["arm_flops"][0] / info_last["arm_tuples"][0] / 1e6,
            "learned": info_last["arm_flops"][1] / info_last["arm_tuples"][1] / 1e6,
            "tuples": [int(info_last["arm_tuples"][0]), int(info_last["arm_tuples"][1])]}
    out["udf_gflop_per_step"] = float((ev * flops).sum()) / abl_steps / 1e9

    if args.route != "score":
        log("[bench] score form")
        spol = hydro.make_policy("score", precision="bf16", wave=args.wave, grouped=1, autotune=1, time_kernels=1,
                                 **extra, **mid)
        ids_s, st_s, inf_s, dts = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, spol,
                                           abl_steps, 1, n, cal, args.safety)
        assert np.array_equal(ids_s, ids), "score and learned routing disagree"
        ev_s = np.array([[x["evaluated"] for x in st] for st in st_s], dtype=np.float64)
        out["score"] = {"value": n * abl_steps / dts, "unit": "tuples/s",
                        "udf_gflop_per_step": float((ev_s * flops).sum()) / abl_steps / 1e9,
                        "first_pass_ms_per_step": sum(i["first_pass_ms"] for i in inf_s) / abl_steps}

    if mid:
        # the same eager full form without the three-product tier (bf16 -> fp32 -> fp64)
        log("[bench] full form without the three-product tier")
        npol = hydro.make_policy(args.route, precision=prec, wave=args.wave, grouped=1, autotune=1, time_kernels=1,
                                 **extra)
        ids_n, st_n, inf_n, dtn = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, npol,
                                           abl_steps, 1, n, cal, args.safety)
        assert np.array_equal(ids_n, ids), "the forms with and without the three-product tier disagree"
        out["without_three_product_tier"] = {
            "value": n * abl_steps / dtn, "unit": "tuples/s", "form": "eager",
            "phases_ms_per_step": {"first_pass": sum(i["first_pass_ms"] for i in inf_n) / abl_steps,
                                   "fp32_rescore": sum(i["f32_pass_ms"] for i in inf_n) / abl_steps,
                                   "fp64_escalate": sum(i["f64_pass_ms"] for i in inf_n) / abl_steps}}

    if primary and not args.no_fp8 and prec != "fp8" and all(
            d.arch == "cnn" and d.in_hw == 128 and tuple(d.widths) == (32, 64, 128, 256) for d in cfg.models):
        # the FP8 first pass (e4m3, per-channel weight scales, calibrated activation scales) with its
        # BF16 -> FP32 -> FP64 re-score chain, eager with HIP events per tier
        log("[bench] fp8 form")
        fpol = hydro.make_policy(args.route, precision="fp8", wave=args.wave, grouped=1, time_kernels=1, **extra)
        ids_8, st_8, inf_8, dt8 = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, fpol,
                                           abl_steps, 1, n, cal, args.safety)
        assert np.array_equal(ids_8, ids), "fp8 and bf16 first passes disagree"
        ev8 = np.array([[x["evaluated"] for x in st] for st in st_8], dtype=np.float64)
        r8 = np.array([[x["rescored"] for x in st] for st in st_8], dtype=np.float64)
        r16 = np.array([[x["rescored16"] for x in st] for st in st_8], dtype=np.float64)
        fp8_ms = sum(i["first_pass_ms"] for i in inf_8)
        out["fp8"] = {"value": n * abl_steps / dt8, "unit": "tuples/s",
                      "band_fraction": {"fp8_to_bf16": float(r8.sum() / ev8.sum()),
                                        "bf16_to_fp32": float(r16.sum() / max(1.0, r8.sum()))},
                      "bands": ({"tau": [round(float(x), 5) for x in run_form.bands[0]]} if run_form.bands else None),
                      "phases_ms_per_step": {"first_pass_fp8": fp8_ms / abl_steps,
                                             "bf16_rescore": sum(i["mid_pass_ms"] for i in inf_8) / abl_steps,
                                             "fp32_rescore": sum(i["f32_pass_ms"] for i in inf_8) / abl_steps,
                                             "fp64_escalate": sum(i["f64_pass_ms"] for i in inf_8) / abl_steps},
                      "first_pass_tflops": float((ev8 * flops).sum()) / (fp8_ms * 1e-3) / 1e12 if fp8_ms > 0 else 0.0,
                      "first_pass_frac_of_fp8_peak": float((ev8 * flops).sum()) / (fp8_ms * 1e-3) / 1e12 / PEAK["fp8"]
                      if fp8_ms > 0 else 0.0}

    if primary and (args.host or cfg.push_batch > 0):
        blk = cfg.push_batch if cfg.push_batch > 0 else 16384
        nh = min(n, blk * args.host_blocks)
        log(f"[bench] full form pushed from pinned host memory: {nh} tuples in blocks of {blk}")
        frames_host = torch.empty(tuple(frames_dev[:nh].shape), dtype=frames_dev.dtype, pin_memory=True)
        frames_host.copy_(frames_dev[:nh])
        hpol = hydro.make_policy(args.route, precision="bf16", wave=args.wave, grouped=1, autotune=1, **extra, **mid)
        ids_h, _, _, dth = run_form(hydro, torch, specs, frames_host, cfg.dtype, pt, seg_len, hpol,
                                    abl_steps, 1, nh, cal, args.safety, push_batch=blk)
        assert np.array_equal(ids_h, ids[ids < nh]), "host-pushed and device-resident runs disagree"
        out["host_pinned"] = {"value": nh * abl_steps / dth, "unit": "tuples/s", "tuples": nh,
                              "push_batch": blk, "note": "PCIe-inclusive: frames start in pinned host memory",
                              "h2d_gb_per_s_equiv": frames_host.numel() * frames_host.element_size() * abl_steps
                              / dth / 1e9}
        # pinned-copy peak of the same bytes, for the H2D fraction
        dst = torch.empty_like(frames_dev[:blk])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lo in range(0, nh, blk):
            dst.copy_(frames_host[lo:lo + blk], non_blocking=True)
        torch.cuda.synchronize()
        out["host_pinned"]["pinned_copy_gb_per_s"] = frames_host.numel() * frames_host.element_size() / \
            (time.perf_counter() - t0) / 1e9
        del frames_host, dst

    if not args.no_plain:
        log("[bench] plain form")
        plain_pol = hydro.make_policy("score", precision="fp32", wave=args.wave, grouped=0, time_kernels=0, **extra)
        ids_p, _, _, dtp = run_form(hydro, torch, specs, frames_dev, cfg.dtype, pt, seg_len, plain_pol,
                                    abl_steps, 1, n, cal, args.safety)
        assert np.array_equal(ids_p, ids), "plain and full forms disagree"
        vp = n * abl_steps / dtp
        out["plain"] = {"value": vp, "unit": "tuples/s",
                        "form": "fp32 first pass, score routing, per-predicate launches, no graph"}
        out["speedup_vs_plain"] = value / vp

    if args.errors > 0 and primary:
        # error of the bf16 and fp32 passes against the library's FP64 pass (which the parity
        # tests pin to the oracle to ~1e-15)
        m = min(args.errors, n)
        log(f"[bench] logit / margin error on {m} frames")
        es = hydro.Session(specs, hydro.make_policy(args.route, precision="bf16"), cfg.hw, m)

        def margin(z, mask):
            inside = np.array([(mask >> c) & 1 for c in range(10)], dtype=bool)
            zin = np.where(inside, z, -np.inf).max(axis=1)
            zout = np.where(~inside, z, -np.inf).max(axis=1)
            return zin - zout

        rep = {"frames": m, "reference": "library fp64 pass"}
        z64 = [es.logits(j, 2, frames_dev[:m], cfg.dtype) for j in range(cfg.k)]
        sessions = [(es, 0, "bf16"), (es, 1, "fp32")]
        f8s = None
        if "fp8" in out:
            f8s = hydro.Session(specs, hydro.make_policy(args.route, precision="fp8"), cfg.hw, m)
            if cal is not None:
                f8s.calibrate(cal, cfg.dtype, args.safety)   # sets the activation scales
            sessions.append((f8s, 0, "fp8"))
        for sess_e, tier, name in sessions:
            ml, mm, pm = [], [], []
            for j in range(cfg.k):
                z = sess_e.logits(j, tier, frames_dev[:m], cfg.dtype)
                dd = np.abs(margin(z, pt.class_masks[j]) - margin(z64[j], pt.class_masks[j]))
                ml.append(float(np.abs(z - z64[j]).max()))
                mm.append(float(dd.max()))
                pm.append(float(np.quantile(dd, 0.999)))
            rep[name] = {"max_logit_err": ml, "max_margin_err": mm, "p999_margin_err": pm}
        es.close()
        if f8s is not None:
            f8s.close()
        out["logit_error"] = rep

    if not args.no_cpu and primary:
        # FP64 oracle on a bounded, evenly spread sample of the same workload
        from threadpoolctl import threadpool_info
        from oracle import hydro_oracle as ho
        # bounded sample: about 1e13 FP64 FLOPs of oracle work (every predicate on every tuple)
        m = int(min(args.cpu_sample, n, max(1024, 1e13 // float(flops.sum()))))
        sel = np.linspace(0, n - 1, m).astype(np.int64)
        fr_s = host_frames(frames_dev, sel, torch)
        cores = min(16, os.cpu_count() or 1)
        log(f"[bench] cpu oracle on {m} sampled tuples, {cores} threads")
        t0 = time.perf_counter()
        P = np.zeros((m, cfg.k), dtype=bool)
        D = np.zeros((m, cfg.k), dtype=np.float64)
        th = ho.tuple_thresholds(pt.thresholds, seg_len, sel)
        for j, w in enumerate(weights):
            z = ho.model_logits(w, fr_s, cfg.dtype, workers=cores)
            D[:, j] = ho.predicate_margin(z, pt.class_masks[j])
            P[:, j] = ho.decide(D[:, j], th[:, j])
        tc = time.perf_counter() - t0
        exp_in = P.all(axis=1)
        got_in = np.isin(sel, ids)
        out["cpu_baseline"] = {"value": m / tc, "unit": "tuples/s", "cores": cores, "kind": "oracle",
                               "sample": f"{m} tuples evenly spaced over the {n} tuples, every predicate "
                                         f"evaluated in fp64 (numpy, BLAS 1 thread per worker)",
                               "os_cpu_count": os.cpu_count(),
                               "blas": [d.get("internal_api") for d in threadpool_info()]}
        # near-tie audit of the sample: exactness against FP64 is well defined where no margin lies
        # within FP64 rounding noise of its threshold
        gap = float(np.abs(D - th)[np.isfinite(D)].min()) if np.isfinite(D).any() else float("inf")
        out["sample_check"] = {"tuples": m, "mismatches": int((exp_in != got_in).sum()), "min_margin_gap": gap}
        if (exp_in != got_in).any():
            log("[bench] WARNING: GPU ids differ from the oracle on the sample")
    del frames_dev, cal
    torch.cuda.empty_cache()
    return out


def compaction(args, hydro, torch):
    """Routing, multi-split, forwarding and result materialisation on 2^26 tuples whose outcomes
    for four predicates (pass rates 0.5 / 0.7 / 0.8 / 0.9, independent) are drawn on the device:
    the query path with the inference tiers replaced by a bitmap lookup, timed with HIP events per
    phase, against the algorithmic bytes of each phase."""
    n, k = 1 << args.compaction_log2n, 4
    rates = [0.5, 0.7, 0.8, 0.9]
    g = torch.Generator(device="cuda").manual_seed(26)
    weights = (torch.ones(32, dtype=torch.int64, device="cuda") << torch.arange(32, device="cuda"))
    rows = []
    for p in rates:
        b = torch.rand(n, generator=g, device="cuda") < p
        rows.append((b.view(-1, 32).to(torch.int64) * weights).sum(dim=1).to(torch.int32))   # bit t % 32 of word t / 32
    bits = torch.stack(rows).contiguous()
    del rows
    out_ids = torch.empty(n, dtype=torch.int64, device="cuda")
    runs = []
    for _ in range(3):
        cnt, stats, ms = hydro.compaction_debug(k, n, bits, out_ids, route="fixed", wave=1 << 22)
        runs.append(ms)
    ms = min(runs, key=lambda m: m[3])
    ev = sum(x["evaluated"] for x in stats)
    surv = ev - n                      # entries re-routed from a live list (admitted ones are generated)
    words = (n + 31) // 32
    route_b = 4 * ev + 4 * surv        # queue entry writes + live-list reads
    decide_b = 4 * ev + 4 * surv + 4 * words * k + 4 * words   # queue reads, survivor writes, outcome bitmaps, result bits
    result_b = 3 * 4 * words + 8 * cnt                          # bitmap clear, count and write passes; ids
    tot_b = route_b + decide_b + result_b
    del bits, out_ids
    torch.cuda.empty_cache()
    return {"n": n, "k": k, "pass_rates": rates, "route": "fixed", "wave": 1 << 22, "result": int(cnt),
            "evaluated": [int(x["evaluated"]) for x in stats],
            "ms": {"fold_route": ms[0], "decide_forward": ms[1], "results": ms[2], "total": ms[3]},
            "bytes": {"fold_route": route_b, "decide_forward": decide_b, "results": result_b},
            "GB_per_s": {"fold_route": route_b / ms[0] / 1e6, "decide_forward": decide_b / ms[1] / 1e6,
                         "results": result_b / ms[2] / 1e6, "total": tot_b / ms[3] / 1e6},
            "frac_of_hbm_peak": tot_b / ms[3] / 1e6 / 8000.0,
            "note": "HIP-event phase sums over all rounds (fold + route, bitmap decisions + forwarding, "
                    "result materialisation), best of 3 runs; algorithmic bytes, 8 TB/s peak"}


def reuse_leg(args, hydro, torch, hs):
    """Result reuse on the 65,536-frame CNN workload (UC2's recurrent query, section 4.3): an
    exploratory query (written order, most expensive predicate first) fills the session's result
    cache on the middle half of the ids; the recurrent query then runs over all of them with cost
    routing (static costs), once reuse-unaware (cached decisions used, ranking unchanged) and once
    reuse-aware ((1 - hit rate) x cost per batch of 64).  The cache is cleared and refilled before
    each timed recurrent query (untimed), which alone is timed."""
    cfg = hs.workload(2)
    n = cfg.n
    frames_dev = make_device_frames(hs, torch, cfg, n)
    pt = hs.load_predicates(cfg)
    weights = [hs.make_model(d) for d in cfg.models]
    specs = [hydro.ModelSpec.from_weights(w, m) for w, m in zip(weights, pt.class_masks)]
    seg_len = cfg.n // cfg.n_seg
    flops = np.array([d.flops() for d in cfg.models])
    order = sorted(range(cfg.k), key=lambda j: -flops[j])
    lo, hi = n // 4, 3 * n // 4
    cal = torch.from_numpy(hs.calibration_frames(cfg)).cuda()
    out, ids_ref = {}, None
    for reuse in (1, 2):
        pol = hydro.make_policy("cost", wave=args.wave, reuse=reuse, cost_source="static")
        s = hydro.Session(specs, pol, cfg.hw, n)
        s.calibrate(cal, cfg.dtype, args.safety)
        s.set_order(order)
        times, gf = [], []
        for step in range(4):
            s.cache_clear()
            s.set_route("fixed")
            s.reset()
            s.push(frames_dev[lo:hi], cfg.dtype, pt.thresholds, seg_len, id_base=lo)
            s.finish()
            s.set_route("cost")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.reset()
            s.push(frames_dev, cfg.dtype, pt.thresholds, seg_len)
            ids, st = s.finish()
            t1 = time.perf_counter()
            if step > 0:                     # the first recurrent query is warm-up
                times.append(t1 - t0)
                gf.append(float(np.dot([x["evaluated"] for x in st], flops)) / 1e9)
        s.close()
        if ids_ref is None:
            ids_ref = ids
        assert np.array_equal(ids, ids_ref), "reuse-aware and reuse-unaware results differ"
        out["reuse_aware" if reuse == 2 else "reuse_unaware"] = {
            "value": n / float(np.median(times)), "unit": "tuples/s", "udf_gflop": float(np.mean(gf)),
            "cache_hits": [int(x["cache_hits"]) for x in st], "evaluated": [int(x["evaluated"]) for x in st]}
    out["speedup"] = out["reuse_aware"]["value"] / out["reuse_unaware"]["value"]
    out["workload"] = {"name": cfg.name, "tuples": n, "cached_range": [lo, hi], "route": "cost (static)",
                       "steps": 3, "note": "exploratory query (untimed) fills the cache before each recurrent query"}
    del frames_dev, cal
    torch.cuda.empty_cache()
    return out


def concurrent_leg(args, hydro, torch, hs):
    """Section 4.1's concurrent setting on one MI355X and its host: the 65,536-frame CNN workload's
    widest predicate on the GPU and a colour-box predicate decided by the host's CPU threads (every
    8th pixel row and column), frames resident in HBM for the GPU and in host memory for the CPU.
    Each round the CPU decides its queue while the GPU evaluates the other, so a query takes about
    the longer of the two per round.
    The three routing policies are timed (median of 3 queries each) at three host thresholds;
    the selectivities are the ones each query measured."""
    cfg = hs.workload(2)
    n = cfg.n
    frames_host = hs.make_frames_parallel(cfg, 0, n)
    frames = torch.from_numpy(frames_host).cuda()
    pt = hs.load_predicates(cfg)
    weights = [hs.make_model(d) for d in cfg.models]
    gpu = hydro.ModelSpec.from_weights(weights[2], pt.class_masks[2])
    lo, hi, stride = [0.5, 0.5, 0.5], [1.0, 1.0, 1.0], 8
    host = hydro.ModelSpec.host_color(cfg.hw, lo, hi, stride)
    seg_len = cfg.n // cfg.n_seg
    points = []
    for gpu_shift, theta in args.concurrent_points:
        th = np.stack([pt.thresholds[:, 2] + np.float32(gpu_shift), np.full(cfg.n_seg, theta, dtype=np.float32)],
                      axis=1).astype(np.float32)
        pt_out = {"gpu_threshold_shift": gpu_shift, "host_threshold": theta, "ms": {}, "evaluated": {}}
        for route in ("cost", "score", "selectivity"):
            s = hydro.Session([gpu, host], hydro.make_policy(route, wave=args.wave), cfg.hw, n)
            times, ids_ref = [], None
            for rep in range(4):
                s.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.push(frames, cfg.dtype, th, seg_len, host_copy=frames_host)
                ids, st = s.finish()
                t1 = time.perf_counter()
                if rep > 0:
                    times.append(t1 - t0)
                if ids_ref is None:
                    ids_ref = ids
            s.close()
            if "ids" in pt_out:
                assert np.array_equal(pt_out["ids"], ids_ref), "routing policies disagree"
            pt_out["ids"] = ids_ref
            pt_out["ms"][route] = float(np.median(times)) * 1e3
            pt_out["evaluated"][route] = [int(x["evaluated"]) for x in st]
            if route == "cost":
                pt_out["selectivity"] = {"gpu_cnn": round(st[0]["selectivity"], 3), "host_color": round(st[1]["selectivity"], 3)}
                pt_out["cost_us_per_tuple"] = {"gpu_cnn": st[0]["cost_us_per_tuple"], "host_color": st[1]["cost_us_per_tuple"]}
        pt_out["n_result"] = int(pt_out.pop("ids").size)
        points.append(pt_out)
    del frames, frames_host
    torch.cuda.empty_cache()
    return {"workload": f"{cfg.name}: {n} frames in HBM, with a host copy for the CPU predicate",
            "predicates": {"gpu": "CNN (64, 128, 256), 79 MFLOP per tuple",
                           "host": {"box": [lo, hi], "stride": stride, "threads": os.cpu_count()}},
            "points": points,
            "note": "median of 3 queries per policy; cost units: device time per tuple summed over compute "
                    "units (host: thread time x compute units / threads)"}


def variable_leg(args, hydro, torch, hs):
    """Variable-size inputs (section 5.3): a CNN (16, 32, 64) on each tuple's crop of the
    65,536-frame workload's frames, crop sides log-uniform from 2 to 64 (many small crops, a few
    large: the work per tuple spans three orders of magnitude).  Query time with the round's
    tuples dealt to the workgroups in queue order against largest-estimated-work-first from a
    shared counter (the input-size heuristic), at two admission wave sizes (fewer tuples per
    workgroup and round make the imbalance of a fixed assignment larger).  Median of 3 queries."""
    cfg = hs.workload(2)
    n = cfg.n
    frames = make_device_frames(hs, torch, cfg, n)
    pt = hs.load_predicates(cfg)
    w0 = hs.make_model(cfg.models[0])
    rng = np.random.default_rng(23)
    side = cfg.hw
    hh = np.minimum(side, np.round(np.exp(rng.uniform(np.log(2), np.log(side), n)))).astype(np.int32)
    ww = np.minimum(side, np.round(np.exp(rng.uniform(np.log(2), np.log(side), n)))).astype(np.int32)
    crops = np.stack([(rng.random(n) * (side - hh + 1)).astype(np.int32),
                      (rng.random(n) * (side - ww + 1)).astype(np.int32), hh, ww], axis=1).astype(np.int32)
    spec = hydro.ModelSpec.from_weights(w0, pt.class_masks[0], on_crop=True, in_hw=side)
    th = np.zeros((1, 1), dtype=np.float32)
    out = {"workload": f"{cfg.name}: {n} frames, one crop per tuple (sides log-uniform 2..{side})",
           "predicate": "CNN (16, 32, 64) on the crop, FP64", "points": []}
    ids_ref = None
    for wave in (2048, 16384):
        pt_out = {"wave": wave, "ms": {}}
        for balance in (0, 1):
            s = hydro.Session([spec], hydro.make_policy("score", wave=wave, balance=balance), side, n)
            times = []
            for rep in range(4):
                s.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.push(frames, cfg.dtype, th, n, crops=crops)
                ids, st = s.finish()
                if rep > 0:
                    times.append(time.perf_counter() - t0)
            s.close()
            if ids_ref is None:
                ids_ref = ids
            assert np.array_equal(ids, ids_ref), "the two schedules disagree"
            pt_out["ms"]["data_aware" if balance else "queue_order"] = float(np.median(times)) * 1e3
        pt_out["speedup"] = pt_out["ms"]["queue_order"] / pt_out["ms"]["data_aware"]
        out["points"].append(pt_out)
    out["n_result"] = int(ids_ref.size)
    del frames
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus above 1 is not supported "
                                   "(sharding across GPUs is a design note only, nothing runs on several)"}))
        sys.exit(2)
    import torch
    import hydro_synth as hs
    from paper_2403_14902_amd import hydro

    torch.cuda.set_device(0)
    hydro.lib()
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.compaction_only:
        print(json.dumps({"compaction": compaction(args, hydro, torch)}), flush=True)
        return
    if args.variable_only:
        print(json.dumps({"variable": variable_leg(args, hydro, torch, hs)}), flush=True)
        return
    if args.concurrent_only:
        print(json.dumps({"concurrent": concurrent_leg(args, hydro, torch, hs)}), flush=True)
        return
    abl = max(1, min(args.ablation_steps, args.steps))
    out = measure(args, args.workload, args.n, args.steps, args.warmup, abl, hydro, torch, hs, True)
    if not args.no_secondary and args.workload != 2:
        # the 65,536-frame 64x64 CNN workload (fused per-frame kernel), as a second line
        sec = measure(args, 2, 0, max(1, min(args.steps, 10)), 2, abl, hydro, torch, hs, False)
        out["cnn3_drift64"] = {k: sec[k] for k in ("value", "ms_per_step", "steps", "eager_value", "roofline",
                                                    "plain", "speedup_vs_plain", "score", "n_result", "config")
                               if k in sec}
    if not args.no_reuse:
        log("[bench] result reuse (recurrent query)")
        out["reuse"] = reuse_leg(args, hydro, torch, hs)
    if not args.no_concurrent:
        log("[bench] concurrent host and GPU predicates")
        out["concurrent"] = concurrent_leg(args, hydro, torch, hs)
    if not args.no_variable:
        log("[bench] variable-size inputs")
        out["variable"] = variable_leg(args, hydro, torch, hs)
    if not args.no_compaction:
        log("[bench] standalone routing / compaction")
        out["compaction"] = compaction(args, hydro, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
