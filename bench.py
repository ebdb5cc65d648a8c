#!/usr/bin/env python3
"""Benchmark of the hierarchy-cut-code path on one MI355X.

Workload (paper-shaped frame): a 1,012,012-triangle room holding 100 icospheres and 100
tori, a 1920x1080 camera at 8 samples per pixel; the bounce-1 cosine-weighted diffuse
secondary rays (one per primary hit, 16.6M) are the measured batch, and the two shadow
rays per primary hit (33.2M) give the any-hit numbers.  Rays are generated once (primary
hits come from the library's own trace) and stay resident in HBM.

A step = HCC encode + stable radix sort + closest-hit trace through the sorted permutation
over the whole batch.  The same batch is also timed for NoSort (trace in generation order)
and TwoPoint (6-D Morton key).  Each method runs in its own fastest configuration, chosen
before the timed region by the autotuner (trace launch options; key length; for HCC the cut
size C from 32 to 4,096 with C >= K -- the frame configuration's cut sizes -- or only the paper's
C = K pairs with --paper-exact; key lengths 16 / 32 / 64; low key bits left out of the sort).  Prints one JSON line on stdout; progress goes to stderr.

Beside the headline the line carries: the roofline of the trace kernel, the CPU oracle's rate,
a grid of reordering methods on the same batch, wavefront packets against per-lane launches by ray
order (primary and shadow rays), bounces 2 and 3 of the frame, the 10M-triangle boundary-drift
workload, the uneven-batch engine workload and the request-server workload (each can be skipped
with its --no-... flag).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "secondary Mrays/s incl. encode+sort vs NoSort; serve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
NODE_BYTES, WIDE_NODE_BYTES, TRI_BYTES = 64, 128, 48
QUANT_NODE_BYTES = 64      # quantised 4-wide node
RAY_BYTES, PERM_BYTES, HIT_BYTES = 32, 4, 16


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spp", type=int, default=8)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--tune", type=int, default=1, help="autotune each method (0: use the flags below)")
    ap.add_argument("--cut", type=int, default=32)
    ap.add_argument("--hcc-cuts", default="16,32,64", help="cut sizes the HCC tuning tries")
    ap.add_argument("--truncate", action="store_true",
                    help="HCC tuning also over C > K (the key holds the K cut nodes of highest HAD); "
                         "by default C = K, the paper's hierarchy cut code")
    ap.add_argument("--skips", default="0,2,4,8,16,32",
                    help="low key bits the tuned sort may leave out (the paper's shortened sort)")
    ap.add_argument("--min-sorted-frac", type=float, default=0.5,
                    help="tuned sorts keep at least this fraction of the key's bits")
    ap.add_argument("--skip", type=int, default=0, help="skipped low key bits without tuning")
    ap.add_argument("--tune-key-bits", default="16,32,64", help="key lengths the reordering tuning tries")
    ap.add_argument("--key-bits", type=int, default=32)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--stack", type=int, default=2, help="0 scratch, 1 LDS, 2 LDS+scratch")
    ap.add_argument("--persistent", type=int, default=1)
    ap.add_argument("--refill", type=int, default=32)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--waves", type=int, default=8192)
    ap.add_argument("--flags", type=int, default=2)
    ap.add_argument("--remap", type=int, default=0, help="1 = XCD-contiguous block order")
    ap.add_argument("--methods", default="nosort,twopoint,hcc,hcc_paper_exact")
    ap.add_argument("--no-stats", action="store_true", help="skip the fetch-counting trace (kernel-counted bytes)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg (CPU baseline and the wave model behind the roofline)")
    ap.add_argument("--cpu-stride", type=int, default=8, help="oracle sample: every k-th secondary ray")
    ap.add_argument("--model-wave-stride", type=int, default=8,
                    help="the oracle's wave model runs on every k-th wavefront of each trace order")
    ap.add_argument("--no-shadow", action="store_true")
    ap.add_argument("--no-packets", action="store_true",
                    help="skip the table of wavefront-packet against per-lane trace launches by ray order")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-batch engine workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server workload")
    ap.add_argument("--no-grid", action="store_true", help="skip the frame workload's method grid")
    ap.add_argument("--grid-reps", type=int, default=5)
    ap.add_argument("--no-drift", action="store_true", help="skip the 10M-triangle boundary-drift workload")
    ap.add_argument("--no-bounces", action="store_true", help="skip the frame workload's bounces 2 and 3")
    ap.add_argument("--drift-tris", type=int, default=10_000_000)
    ap.add_argument("--drift-spp", type=int, default=4)
    ap.add_argument("--drift-keys", default="16,24,32,48,64")
    ap.add_argument("--drift-reps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-direct-min", type=int, default=0,
                    help="continuous server: requests of at least this many rays take the full-device kernels "
                         "(0 = the library default; 4294967295 = every request through the engine)")
    ap.add_argument("--full-out", default="bench_full.json",
                    help="file that receives the full record (every table); the last stdout line is a summary")
    return ap.parse_args(argv)


def cut_composition(H, cut, n_tris: int, sorted_bits: int) -> dict:
    """What the sorted key bits encode: of the cut nodes owning them, how many are leaves
    (single triangles) and how many distinct boxes they have."""
    ids, _, boxes = cut.export()
    m = min(sorted_bits, ids.shape[0])
    ids, boxes = ids[:m], boxes[:m]
    leaves = int((ids >= max(n_tris - 1, 0)).sum()) if n_tris > 1 else m
    distinct = len({b.tobytes() for b in boxes})
    return dict(sorted_nodes=int(m), leaves=leaves, distinct_boxes=distinct)


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rays would be sharded by contiguous ranges with a BVH replica per GPU); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_16652_amd as H
    from paper_2305_16652_amd import autotune as AT
    import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    methods = [m for m in args.methods.split(",") if m]
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst

    # ------------------------------------------------------------------ workload
    t0 = time.time()
    spec = W.frame_scene()
    tris_h = spec.tris
    tris = torch.from_numpy(tris_h).to(dev)
    log(f"scene {tris_h.shape[0]} triangles ({time.time() - t0:.1f}s)")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    e0, e1 = ev(), ev()
    e0.record()
    bvh = H.build_bvh(tris)
    e1.record()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)

    flag_opts = H.TraceOpts(args.block, args.stack, args.remap, args.persistent, args.refill, args.chunk,
                            args.waves, args.flags)
    t0 = time.time()
    prim = W.pinhole_rays(spec, args.width, args.height, args.spp, seed=2)
    prim_d = torch.from_numpy(prim).to(dev)
    ph = H.trace(bvh, prim_d, opts=flag_opts).cpu().numpy()
    del prim_d
    p_t = ph[:, 0].copy()
    p_prim = ph[:, 1].copy().view(np.uint32)
    sec, _ = W.spawn_diffuse(prim, p_t, p_prim, tris_h, seed=7, bounce=0)
    rays = torch.from_numpy(sec).to(dev)
    R = rays.shape[0]
    log(f"{prim.shape[0]} primary rays, {R} secondary rays ({time.time() - t0:.1f}s)")
    shadow = None
    if not args.no_shadow:
        shd, _ = W.spawn_shadow(prim, p_t, p_prim, tris_h, spec.lights)
        shadow = torch.from_numpy(shd).to(dev)
        log(f"{shadow.shape[0]} shadow rays")
    packets = None
    if not args.no_packets and shadow is not None:
        packets = run_packets(H, bvh, torch.from_numpy(prim).to(dev), shadow)
    del prim, ph

    # ------------------------------------------------------------------ configuration per method
    # nosort: trace options only.  twopoint / hcc: key length, skipped low bits (keeping at least
    # --min-sorted-frac of the key in the sort) and trace options; hcc over C = K (a real cut whose
    # every node owns a key bit).  hcc_paper_exact: C = K = 32, full 32-bit sort (the paper's
    # configuration), trace options tuned.
    t0 = time.time()
    conf = {}
    sk = tuple(int(x) for x in args.skips.split(","))
    kb = tuple(int(x) for x in args.tune_key_bits.split(","))
    for m in methods:
        if m == "nosort":
            o = AT.tune_trace(bvh, rays, None)[0] if args.tune else flag_opts
            conf[m] = dict(cut=0, key_bits=0, skip=0, opts=o)
        elif m == "hcc_paper_exact":
            ch, _ = AT.tune_reorder(bvh, rays, "hcc", cuts=(32,), key_bits=(32,), skips=(0,)) if args.tune else \
                (None, None)
            conf[m] = dict(cut=32, key_bits=32, skip=0, opts=ch.opts if ch else flag_opts)
        elif m in ("twopoint", "hcc"):
            if args.tune:
                cs = tuple(int(c) for c in args.hcc_cuts.split(",")) if m == "hcc" else (0,)
                ch, _ = AT.tune_reorder(bvh, rays, m, cuts=cs, key_bits=kb, paper_exact=not args.truncate,
                                        skips=sk, min_sorted_frac=args.min_sorted_frac)
                conf[m] = dict(cut=ch.cut, key_bits=ch.key_bits, skip=ch.skip, opts=ch.opts)
            else:
                conf[m] = dict(cut=args.cut if m == "hcc" else 0, key_bits=args.key_bits, skip=args.skip,
                               opts=flag_opts)
    if args.tune:
        log(f"autotuned in {time.time() - t0:.1f}s: " +
            "; ".join(f"{m} C={c['cut']} K={c['key_bits']} skip={c.get('skip', 0)} {AT.opts_dict(c['opts'])}"
                      for m, c in conf.items()))
    e0.record()
    cuts = {m: H.select_cut(bvh, c["cut"]) for m, c in conf.items() if m.startswith("hcc")}
    e1.record()
    torch.cuda.synchronize()
    cut_ms = e0.elapsed_time(e1)

    hits = torch.empty((R, 4), dtype=torch.float32, device=dev)
    bufs = {}
    for m, c in conf.items():
        if m == "nosort":
            continue
        k = c["key_bits"]
        bufs[m] = dict(keys=torch.empty(R, dtype=torch.int32 if k <= 32 else torch.int64, device=dev),
                       perm=torch.empty(R, dtype=torch.int32, device=dev),
                       ws=torch.empty(H.sort_workspace_bytes(R, k), dtype=torch.uint8, device=dev))

    def run(method: str, evs=None, rr=None, closest=True, out=None, b=None, opts=None):
        rr = rays if rr is None else rr
        out = hits if out is None else out
        b = bufs.get(method) if b is None else b
        c = conf[method]
        if evs:
            evs[0].record()
        perm = None
        if method != "nosort":
            k = c["key_bits"]
            if method.startswith("hcc"):
                H.encode(bvh, cuts[method], H.KEY_HCC, k, rr, out=b["keys"])
            else:
                H.encode(bvh, None, H.KEY_TWOPOINT, k, rr, out=b["keys"])
            if evs:
                evs[1].record()
            H.sort_ex(b["keys"], k, c["skip"], 0, perm=b["perm"], ws=b["ws"])
            perm = b["perm"]
        elif evs:
            evs[1].record()
        if evs:
            evs[2].record()
        H.trace(bvh, rr, perm, closest=closest, out=out, opts=c["opts"] if opts is None else opts)
        if evs:
            evs[3].record()

    def timed(method: str):
        for _ in range(args.warmup):
            run(method)
        torch.cuda.synchronize()
        evs = [[ev() for _ in range(4)] for _ in range(args.steps)]
        start, stop = ev(), ev()
        torch.cuda.synchronize()
        t_wall = time.time()
        start.record()
        for s in range(args.steps):
            run(method, evs[s])
        stop.record()
        torch.cuda.synchronize()
        wall = time.time() - t_wall
        ms = start.elapsed_time(stop) / args.steps
        enc = [e[0].elapsed_time(e[1]) for e in evs]
        srt = [e[1].elapsed_time(e[2]) for e in evs]
        trc = [e[2].elapsed_time(e[3]) for e in evs]
        res = dict(ms_per_step=ms, mrays_s=R / (ms * 1e-3) / 1e6, encode_ms=float(np.median(enc)),
                   sort_ms=float(np.median(srt)), trace_ms=float(np.median(trc)), trace_ms_mean=float(np.mean(trc)),
                   trace_only_mrays_s=R / (np.median(trc) * 1e-3) / 1e6, wall_s=wall)
        log(f"{method}: {ms:.3f} ms/step ({res['mrays_s']:.1f} Mrays/s), encode {res['encode_ms']:.3f} "
            f"sort {res['sort_ms']:.3f} trace {res['trace_ms']:.3f} ms")
        return res

    results = {m: timed(m) for m in conf}
    hcc_hits = hits.clone()
    head = "hcc" if "hcc" in results else next(iter(results))
    composition = (cut_composition(H, cuts[head], tris_h.shape[0], conf[head]["key_bits"] - conf[head]["skip"])
                   if head in cuts else None)

    # any-hit (shadow) rays, each method with its secondary-ray key (cut, key length, skipped bits)
    # and its trace options tuned on the shadow rays in its own order (per-lane 4-wide launches and
    # wavefront packets, which pay on these more coherent rays)
    shadow_res = None
    if shadow is not None:
        S = shadow.shape[0]
        occ = torch.empty(S, dtype=torch.uint8, device=dev)
        shadow_res = {"rays": S}
        for m in conf:
            sb = None
            if m != "nosort":
                k = conf[m]["key_bits"]
                sb = dict(keys=torch.empty(S, dtype=torch.int32 if k <= 32 else torch.int64, device=dev),
                          perm=torch.empty(S, dtype=torch.int32, device=dev),
                          ws=torch.empty(H.sort_workspace_bytes(S, k), dtype=torch.uint8, device=dev))
            s_opts = conf[m]["opts"]
            if args.tune:
                run(m, rr=shadow, closest=False, out=occ, b=sb)     # leaves the order in sb["perm"]
                s_opts = AT.tune_trace(bvh, shadow, sb["perm"] if sb else None, closest=False,
                                       candidates=AT.WIDE + AT.PACKET)[0]
            times = []
            for s in range(args.warmup + args.steps):
                a, b = ev(), ev()
                a.record()
                run(m, rr=shadow, closest=False, out=occ, b=sb, opts=s_opts)
                b.record()
                torch.cuda.synchronize()
                if s >= args.warmup:
                    times.append(a.elapsed_time(b))
            ms = float(np.median(times))
            shadow_res[m] = dict(ms=round(ms, 4), mrays_s=round(S / (ms * 1e-3) / 1e6, 2),
                                 trace_opts=AT.opts_dict(s_opts))
            del sb
        log("shadow Mrays/s: " + ", ".join(f"{m} {shadow_res[m]['mrays_s']:.0f}" for m in conf))

    counted = None
    if not args.no_stats:
        counted = {m: kernel_counted_fetches(H, bvh, rays, bufs[m]["perm"] if m in bufs else None, conf[m]["opts"])
                   for m in conf}
    oracle_leg = None
    if not args.no_cpu and "hcc" in conf:
        oracle_leg = run_oracle_leg(tris_h, sec, args, hcc_hits.cpu().numpy(), conf, head)
    roofline = roofline_of(H, R, results[head]["trace_ms_mean"], conf[head]["opts"],
                           oracle_leg["model"].get(head) if oracle_leg else None,
                           counted.get(head) if counted else None)
    cpu = oracle_leg["cpu_baseline"] if oracle_leg else None

    grid = None
    if not args.no_grid and "hcc" in conf:
        grid = run_method_grid(H, bvh, rays, conf["hcc"]["opts"], args.grid_reps)
    del bufs
    bounces = None if args.no_bounces else run_bounces(H, args, bvh, tris_h, sec, rays)
    drift = None if args.no_drift else run_drift(H, args)
    batched = None if args.no_batched else run_batched(H, args)
    serve = None if args.no_serve else run_serving(H, args)

    hc = conf[head]
    workload = (f"frame: {tris_h.shape[0]:,}-triangle room with 100 icospheres + 100 tori, "
                f"{args.width}x{args.height}x{args.spp} spp, bounce-1 diffuse secondary rays")
    full = {
        "metric": METRIC, "workload": workload, "steps": args.steps, "warmup": args.warmup,
        "triangles": int(tris_h.shape[0]), "rays": int(R), "headline": head,
        "methods": {m: dict({k: round(v, 4) for k, v in r.items()}, cut=conf[m]["cut"],
                            key_bits=conf[m]["key_bits"], skip_bits=conf[m].get("skip", 0),
                            trace_opts=AT.opts_dict(conf[m]["opts"]))
                    for m, r in results.items()},
        "cut_composition": composition,
        "shadow": shadow_res,
        "packets": packets,
        "build_ms": round(build_ms, 2),
        "select_cut_ms": round(cut_ms, 2),
        "fetches": dict(model=oracle_leg["model"] if oracle_leg else None, kernel_counted=counted),
        "method_grid": grid,
        "frame_bounces": bounces,
        "drift": drift,
        "batched": batched,
        "serve": serve,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.full_out:
        with open(args.full_out, "w") as f:
            json.dump(full, f, indent=1)
    line = compact_line(full, args, workload)
    print(json.dumps(line, separators=(",", ":")), flush=True)


def compact_line(full: dict, args, workload: str) -> dict:
    """The one JSON line the benchmark prints last: the headline, every method's rate and stage
    times, speedups, roofline, CPU baseline and one-number summaries of the other workloads.
    The tables behind them are in the full record (args.full_out)."""
    head = full["headline"]
    res = full["methods"]
    hc = res[head]

    def mrow(m):
        r = res[m]
        out = dict(mrays_s=round(r["mrays_s"], 1), ms=round(r["ms_per_step"], 3), enc=round(r["encode_ms"], 3),
                   sort=round(r["sort_ms"], 3), trace=round(r["trace_ms"], 3))
        if m != "nosort":
            out.update(C=r["cut"], K=r["key_bits"], skip=r["skip_bits"])
        return out

    def speed(a, b):
        return round(res[a]["mrays_s"] / res[b]["mrays_s"], 3) if a in res and b in res else None

    line = {
        "metric": METRIC,
        "value": round(hc["mrays_s"], 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hc["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload + f"; {head} C={hc['cut']} K={hc['key_bits']}"
                   + (f" sorted on the top {hc['key_bits'] - hc['skip_bits']} bits" if hc["skip_bits"] else ""),
                   "triangles": full["triangles"], "rays": full["rays"], "cut": hc["cut"], "key_bits": hc["key_bits"],
                   "skip_bits": hc["skip_bits"], "trace_opts": hc["trace_opts"]},
        "methods": {m: mrow(m) for m in res},
        "speedup_vs_nosort": speed(head, "nosort"),
        "speedup_vs_twopoint": speed(head, "twopoint"),
        "paper_exact_vs_nosort": speed("hcc_paper_exact", "nosort"),
        "cut_composition": full.get("cut_composition"),
    }
    pk = full.get("packets")
    if pk:
        line["packet_vs_lane_ms"] = {k: [v["lane_ms"], v["packet_ms"]] for k, v in pk.items()}
    sh = full.get("shadow")
    if sh:
        line["shadow_mrays_s"] = {m: sh[m]["mrays_s"] for m in res if m in sh}
        for base in ("nosort", "twopoint"):
            if head in sh and base in sh and head != base:
                line[f"shadow_speedup_vs_{base}"] = round(sh[head]["mrays_s"] / sh[base]["mrays_s"], 3)
    pe = res.get("hcc_paper_exact")
    if pe and pe.get("key_bits") == 32 and pe.get("skip_bits") == 0 and pe["sort_ms"] > 0:
        # the full 32-bit sort of the frame's keys against its algorithmic bytes (68 B per key)
        achieved = 68.0 * full["rays"] / (pe["sort_ms"] * 1e-3) / 1e9
        line["sort32"] = dict(ms=round(pe["sort_ms"], 4), bytes_per_key=68, achieved_gbs=round(achieved, 1),
                              frac=round(achieved / HBM_PEAK_GBS, 4))
    fm = (full.get("fetches") or {}).get("model")
    if fm:
        line["model_fetches_per_ray"] = {m: [v["node_fetches_per_ray"], v["tri_fetches_per_ray"]] for m, v in fm.items()}
    b = full.get("frame_bounces")
    if b:
        line["bounces_mrays_s"] = {k: {r["method"]: r["mrays_s"] for r in v["rows"]} for k, v in b.items()}
        # the frame's three diffuse bounces together (the paper-shaped frame traces three), each
        # method in its tuned configuration of each bounce: all secondary rays / all step time
        agg = {}
        for m in ("nosort", "twopoint", "hcc"):
            if m not in res:
                continue
            rays, ms = float(full["rays"]), res[m]["ms_per_step"]
            for v in b.values():
                tuned = [r for r in v["rows"] if r.get("tuned") and r["method"].split(" ")[0] == m]
                if not tuned:
                    break
                rays += v["rays"]
                ms += tuned[0]["ms"]
            else:
                agg[m] = round(rays / (ms * 1e-3) / 1e6, 1)
        if agg:
            line["frame_3_bounces_mrays_s"] = agg
    bt = full.get("batched")
    if bt:
        line["batched_mrays_s"] = {k.replace("_mrays_s", ""): bt[k] for k in (
            "engine_hcc_mrays_s", "plain_hcc_mrays_s", "engine_hcc_real_cut_mrays_s", "plain_hcc_real_cut_mrays_s",
            "engine_nosort_mrays_s", "plain_nosort_mrays_s") if k in bt}
        line["batched_mrays_s"]["pick"] = f"C={bt.get('cut')} K={bt.get('key_bits')}"
    sv = full.get("serve")
    if sv:
        line["serve_p50_p99_ms"] = {rho: {k: [v["p50_ms"], v["p99_ms"]] for k, v in row.items()}
                                    for rho, row in sv["loads"].items()}
    d = full.get("drift")
    if d:
        line["drift_best_mrays_s"] = {bn: list(max((r["mrays_s"], r["method"]) for r in v["rows"]))
                                      for bn, v in d["bounces"].items()}
        # the best HCC row (C = K, encode + sort included) against NoSort on the scene that does
        # not fit the caches
        ratio = {}
        for bn, v in d["bounces"].items():
            hcc = [r["mrays_s"] for r in v["rows"] if r["method"].startswith("hcc")]
            base = [r["mrays_s"] for r in v["rows"] if r["method"] == "nosort"]
            if hcc and base:
                ratio[bn] = round(max(hcc) / base[0], 3)
        if ratio:
            line["drift_hcc_vs_nosort"] = ratio
        sh = d.get("shadow")
        if sh:
            base = [r["mrays_s"] for r in sh["rows"] if r["method"] == "nosort"]
            line["drift_shadow_best_mrays_s"] = list(max((r["mrays_s"], r["method"]) for r in sh["rows"]))
            hcc = [r["mrays_s"] for r in sh["rows"] if r["method"].startswith("hcc")]
            if hcc and base:
                line["drift_shadow_hcc_vs_nosort"] = round(max(hcc) / base[0], 3)
    line["roofline"] = full.get("roofline")
    line["cpu_baseline"] = full.get("cpu_baseline")
    line["full_record"] = args.full_out
    return line


_SCENES = None


def cluster_scenes(H):
    """The four resident cluster scenes (10K, 100K, 1M, 2M triangles) with device ray pools:
    bounce-1 diffuse rays and shadow rays from a 1024x512 camera (primary hits from the
    library's trace)."""
    global _SCENES
    if _SCENES is not None:
        return _SCENES
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    scenes = []
    for i, n in enumerate((10_000, 100_000, 1_000_000, 2_000_000)):
        spec = W.cluster_scene(n, seed=40 + i)
        bvh = H.build_bvh(torch.from_numpy(spec.tris).to(dev))
        prim = W.pinhole_rays(spec, 1024, 512, 1, seed=50 + i)
        ph = H.trace(bvh, torch.from_numpy(prim).to(dev)).cpu().numpy()
        pt, pp = ph[:, 0].copy(), ph[:, 1].copy().view(np.uint32)
        dif, _ = W.spawn_diffuse(prim, pt, pp, spec.tris, seed=60 + i, bounce=0)
        shd, _ = W.spawn_shadow(prim, pt, pp, spec.tris, spec.lights)
        scenes.append(dict(n=n, bvh=bvh, diffuse=torch.from_numpy(dif).to(dev), shadow=torch.from_numpy(shd).to(dev)))
    _SCENES = scenes
    return scenes


def run_serving(H, args):
    """Poisson stream of trace requests (ray count log-uniform in [4K, 4M], scene uniform over
    the 4 resident scenes, 70% closest / 30% any hit) at 3 offered loads relative to the plain
    one-request-at-a-time capacity, admitted under a 64 GiB budget.  Reports p50/p99 latency
    and Mrays/s for the continuous-batching server and for the plain FIFO path."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    scenes = cluster_scenes(H)
    cuts = [H.select_cut(s["bvh"], 32) for s in scenes]
    n_req = args.serve_requests + args.serve_warmup
    plan = W.batch_plan(n_req, seed=77, lo=4096, hi=4_194_304)
    pools = {}
    for si, s in enumerate(scenes):
        for kind in ("diffuse", "shadow"):
            p = s[kind]
            reps = (4_194_304 + p.shape[0] - 1) // p.shape[0] + 1
            pools[(si, kind)] = p.repeat(reps, 1)[: 4_194_304 + p.shape[0]].contiguous()
    reqs = []
    for b in plan:
        pool = pools[(b["scene"], "diffuse" if b["closest"] else "shadow")]
        off = b["offset"] % (pool.shape[0] - b["n"] + 1)
        reqs.append(H.Batch(scenes[b["scene"]]["bvh"], pool[off:off + b["n"]], b["closest"], cut=cuts[b["scene"]]))
    total_rays = sum(b["n"] for b in plan[args.serve_warmup:])

    def serve(server, rate=None):
        """Submit every request (at Poisson times if rate is given, else all at once)."""
        rng = np.random.default_rng(5)
        gaps = rng.exponential(1.0 / rate, n_req) if rate else np.zeros(n_req)
        ids = []
        t_start = time.perf_counter()
        t_next = t_start
        for i, b in enumerate(reqs):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                pass
            ids.append(server.submit(b))
        server.drain()
        t_end = time.perf_counter()
        lat = np.array([server.poll(i)[1] for i in ids[args.serve_warmup:]])
        return lat, t_end - t_start

    # plain capacity: the FIFO path with every request queued at once
    plain = H.Server(key_mode=H.KEY_HCC, key_bits=32, plain=True)
    _, wall = serve(plain)
    capacity = n_req / wall
    out = dict(requests=args.serve_requests, warmup=args.serve_warmup, rays=int(total_rays),
               plain_capacity_req_s=round(capacity, 1), budget_gib=64, loads={})
    for rho in (0.5, 0.8, 0.95):
        rate = rho * capacity
        row = {}
        for name, server in (("plain", plain), ("continuous", None)):
            if server is None:
                server = H.Server(key_mode=H.KEY_HCC, key_bits=32, max_group=16, streams=4,
                                  batch=H.BatchOpts(0, 0, 0, H.TRACE_WIDE | H.TRACE_QUANT, 0),
                                  direct_min=args.serve_direct_min)
            lat, wall = serve(server, rate)
            row[name] = dict(p50_ms=round(float(np.percentile(lat, 50)) / 1e3, 3),
                             p99_ms=round(float(np.percentile(lat, 99)) / 1e3, 3),
                             mrays_s=round(total_rays / wall / 1e6, 1))
            if name == "continuous":
                server.close()
        out["loads"][str(rho)] = row
        log(f"serve rho={rho}: plain p50 {row['plain']['p50_ms']} p99 {row['plain']['p99_ms']} ms; "
            f"continuous p50 {row['continuous']['p50_ms']} p99 {row['continuous']['p99_ms']} ms")
    plain.close()
    return out


def run_batched(H, args):
    """Uneven-batch workload: 4 resident cluster scenes (10K, 100K, 1M, 2M triangles), 64 batches
    of log-uniform size in [1K, 2M] rays, 70% closest-hit diffuse / 30% any-hit shadow.  Times
    the plain path (per batch: encode, sort, trace launches) against the engine's single
    persistent launch, each for NoSort and for HCC, with the engine's options autotuned."""
    import torch
    import workloads as W
    from paper_2305_16652_amd import autotune as AT

    dev = torch.device("cuda:0")
    t0 = time.time()
    scenes = cluster_scenes(H)
    plan = W.batch_plan(64, seed=21)
    batches = []
    for b in plan:
        s = scenes[b["scene"]]
        pool = s["diffuse"] if b["closest"] else s["shadow"]
        idx = (torch.arange(b["n"], device=dev, dtype=torch.int64) + b["offset"] % pool.shape[0]) % pool.shape[0]
        batches.append(H.Batch(s["bvh"], pool[idx].contiguous(), b["closest"]))
    total = sum(b["n"] for b in plan)
    log(f"batched workload: {len(plan)} batches, {total} rays over 4 scenes ({time.time() - t0:.1f}s)")

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            e.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(e))
        return float(np.median(ts))

    topts = H.TraceOpts(64, 2, 0, 1, 32, 64, 8192, H.TRACE_WIDE | H.TRACE_QUANT)
    bufs = {}

    def plain(mode, K):
        for b in batches:
            n = b.rays.shape[0]
            perm = None
            if mode == H.KEY_HCC:
                key = (id(b), K)
                if key not in bufs:
                    bufs[key] = (torch.empty(n, dtype=torch.int32 if K <= 32 else torch.int64, device=dev),
                                 torch.empty(n, dtype=torch.int32, device=dev),
                                 torch.empty(H.sort_workspace_bytes(n, K), dtype=torch.uint8, device=dev))
                keys, perm, ws = bufs[key]
                H.encode(b.bvh, b.cut, H.KEY_HCC, K, b.rays, out=keys)
                H.sort(keys, K, perm=perm, ws=ws)
            H.trace(b.bvh, b.rays, perm, closest=b.closest, out=b.out, opts=topts)

    res = {}
    cuts = {}
    # engine tuning in two stages: key length K and cut size C (C = K, or a 256-node cut whose K
    # nodes of highest HAD form the key) under default options; then, for the best pair and for
    # the best real cut (C = K >= 16), rays per trace item (chunk), refill, trace flags and the
    # 4-wide trace phase's stack placement
    pairs = [(K, C) for K in (2, 4, 8, 16, 24, 32) for C in sorted({K, 256})]
    for K, C in pairs:
        cuts[C] = cuts.get(C) or [H.select_cut(s["bvh"], C) for s in scenes]

    def set_cut(C):
        for b, p in zip(batches, plan):
            b.cut = cuts[C][p["scene"]]

    stage1 = []
    for K, C in pairs:
        set_cut(C)
        ws = H.batch_run(batches, H.KEY_HCC, K)
        o = H.BatchOpts(256, 32, 8192, H.TRACE_WIDE)
        stage1.append((timeit(lambda: H.batch_run(batches, H.KEY_HCC, K, opts=o, ws=ws), reps=2), K, C))
    table = []

    def tune_opts(K, C):
        set_cut(C)
        ws = H.batch_run(batches, H.KEY_HCC, K)
        best = None
        for chunk in (128, 256, 512):
            for refill in (24, 32):
                wq = H.TRACE_WIDE | H.TRACE_QUANT
                for flags, stacks in ((0, (0,)), (H.TRACE_WIDE, (0, H.STACK_LDS, H.BATCH_STACK_SCRATCH)),
                                      (H.TRACE_WIDE | H.TRACE_SLAB, (0,)),
                                      (wq, (0, H.STACK_LDS, H.BATCH_STACK_SCRATCH)), (wq | H.TRACE_SLAB, (0,))):
                    for st in stacks:
                        o = H.BatchOpts(chunk, refill, 8192, flags, 0, st)
                        ms = timeit(lambda: H.batch_run(batches, H.KEY_HCC, K, opts=o, ws=ws), reps=2)
                        table.append((ms, K, C, chunk, refill, flags, st))
                        if best is None or ms < best[0]:
                            best = (ms, K, C, chunk, refill, flags, st)
        return best

    _, K1, C1 = min(stage1)
    best = tune_opts(K1, C1)
    real = [t for t in stage1 if t[1] >= 16 and t[1] == t[2]]
    _, Kr, Cr = min(real)
    best_real = tune_opts(Kr, Cr) if (Kr, Cr) != (K1, C1) else best
    _, K, C, chunk, refill, flags, st = best
    set_cut(C)
    o = H.BatchOpts(chunk, refill, 8192, flags, 0, st)
    ws = H.batch_run(batches, H.KEY_HCC, K, opts=o)
    res["engine_hcc_ms"] = timeit(lambda: H.batch_run(batches, H.KEY_HCC, K, opts=o, ws=ws))
    wsn = H.batch_run(batches, 0, K, opts=o)
    res["engine_nosort_ms"] = timeit(lambda: H.batch_run(batches, 0, K, opts=o, ws=wsn))
    # the same call with large batches sent through the full-device kernels (direct_min tuned)
    hyb = []
    for dmin in (65536, 262144, 1048576):
        od = H.BatchOpts(chunk, refill, 8192, flags, dmin, st)
        hyb.append((timeit(lambda: H.batch_run(batches, H.KEY_HCC, K, opts=od, ws=ws), reps=3), dmin))
    res["hybrid_hcc_ms"], direct_min = min(hyb)
    od = H.BatchOpts(chunk, refill, 8192, flags, direct_min, st)
    res["hybrid_nosort_ms"] = timeit(lambda: H.batch_run(batches, 0, K, opts=od, ws=wsn))
    res["plain_hcc_ms"] = timeit(lambda: plain(H.KEY_HCC, K))
    res["plain_nosort_ms"] = timeit(lambda: plain(0, K))
    # the best real cut (C = K >= 16) in its own tuned options, and the plain path with its keys
    _, Kr, Cr, chr_, rfr, flr, str_ = best_real
    set_cut(Cr)
    o_r = H.BatchOpts(chr_, rfr, 8192, flr, 0, str_)
    ws_r = H.batch_run(batches, H.KEY_HCC, Kr, opts=o_r)
    res["engine_hcc_real_cut_ms"] = timeit(lambda: H.batch_run(batches, H.KEY_HCC, Kr, opts=o_r, ws=ws_r))
    res["plain_hcc_real_cut_ms"] = timeit(lambda: plain(H.KEY_HCC, Kr))
    set_cut(C)
    out = {k.replace("_ms", "_mrays_s"): round(total / (v * 1e-3) / 1e6, 1) for k, v in res.items()}
    out.update({k: round(v, 3) for k, v in res.items()})
    out.update(dict(batches=len(plan), rays=total, key_bits=K, cut=C,
                    engine_opts=dict(chunk=chunk, refill=refill, flags=flags, stack=st), hybrid_direct_min=direct_min,
                    real_cut=dict(key_bits=Kr, cut=Cr, chunk=chr_, refill=rfr, flags=flr, stack=str_),
                    plain_trace_opts=AT.opts_dict(topts),
                    speedup_engine_vs_plain_hcc=round(res["plain_hcc_ms"] / res["engine_hcc_ms"], 3),
                    scenes="cluster 10K/100K/1M/2M triangles",
                    key_tuning=[dict(ms=round(t[0], 3), key_bits=t[1], cut=t[2]) for t in sorted(stage1)],
                    tuning=[dict(ms=round(t[0], 3), key_bits=t[1], cut=t[2], chunk=t[3], refill=t[4], flags=t[5],
                                 stack=t[6]) for t in sorted(table)[:8]]))
    log(f"batched: engine HCC {out['engine_hcc_mrays_s']} Mrays/s (with direct launches >= {direct_min} rays: "
        f"{out['hybrid_hcc_mrays_s']}) vs plain {out['plain_hcc_mrays_s']}; NoSort engine "
        f"{out['engine_nosort_mrays_s']} ({out['hybrid_nosort_mrays_s']}) vs plain {out['plain_nosort_mrays_s']}")
    return out


def variant_name(v) -> str:
    m = v["mode"]
    if m == "hcc":
        name = f"hcc C={v['C']} K={v['K']}"
    elif m == "mlhcc":
        name = f"mlhcc{v['top'] + v['low']} ({v['top']}+{v['low']})"
    elif m == "nosort":
        return "nosort"
    else:
        name = f"{m} K={v['K']}"
    if v.get("skip"):
        name += f" skip {v['skip']}"
    if v.get("tile"):
        name += f" tile {v['tile']}"
    return name


def measure_variant(H, bvh, rays, v, opts, reps=5, closest=True, stats=True):
    """encode + sort + trace of one reordering variant: median stage times over `reps` steps
    (after one warm-up), wavefront node/triangle fetches per ray and ANC (distinct keys per
    group of 32 and of 64 consecutive rays in trace order)."""
    import torch
    R = rays.shape[0]
    dev = rays.device
    mode, K = v["mode"], v.get("K", 0)
    cut = None
    if mode == "hcc":
        cut = H.select_cut(bvh, v["C"])
    elif mode == "mlhcc":
        cut = H.select_mlhcc_cut(bvh, v["top"], v["low"])
    elif mode == "grid":
        cut = H.grid_cut(bvh, *H.grid_dims(K))
    kmode = {"twopoint": H.KEY_TWOPOINT, "hcc": H.KEY_HCC, "grid": H.KEY_HCC, "mlhcc": H.KEY_MLHCC,
             "ppc": H.KEY_PPC}.get(mode, 0)
    skip, tile = v.get("skip", 0), v.get("tile", 0)
    out = (torch.empty((R, 4), dtype=torch.float32, device=dev) if closest
           else torch.empty(R, dtype=torch.uint8, device=dev))
    keys = perm = ws = None
    if mode != "nosort":
        keys = torch.empty(R, dtype=torch.int32 if K <= 32 else torch.int64, device=dev)
        perm = torch.empty(R, dtype=torch.int32, device=dev)
        ws = torch.empty(H.sort_workspace_bytes(R, K), dtype=torch.uint8, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(e=None):
        if e:
            e[0].record()
        if mode != "nosort":
            H.encode(bvh, cut, kmode, K, rays, out=keys)
        if e:
            e[1].record()
        if mode != "nosort":
            if skip or tile:
                H.sort_ex(keys, K, skip_bits=skip, tile=tile, perm=perm, ws=ws)
            else:
                H.sort(keys, K, perm=perm, ws=ws)
        if e:
            e[2].record()
        H.trace(bvh, rays, perm, closest=closest, out=out, opts=opts)
        if e:
            e[3].record()

    step()
    torch.cuda.synchronize()
    evs = [[ev() for _ in range(4)] for _ in range(reps)]
    for e in evs:
        step(e)
    torch.cuda.synchronize()
    enc = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    srt = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    trc = float(np.median([e[2].elapsed_time(e[3]) for e in evs]))
    tot = float(np.median([e[0].elapsed_time(e[3]) for e in evs]))
    res = dict(method=variant_name(v), ms=round(tot, 4), encode_ms=round(enc, 4), sort_ms=round(srt, 4),
               trace_ms=round(trc, 4), mrays_s=round(R / (tot * 1e-3) / 1e6, 1),
               trace_only_mrays_s=round(R / (trc * 1e-3) / 1e6, 1))
    if cut is not None:
        res["cut_eff"] = H.cut_shape(cut)[1]
    if stats:
        _, _, _, wn, wt = H.trace_stats(bvh, rays, perm, closest=closest)
        res["node_fetches_per_ray"] = round(int(wn.to(torch.int64).sum().item()) / R, 3)
        res["tri_fetches_per_ray"] = round(int(wt.to(torch.int64).sum().item()) / R, 3)
        if keys is not None:
            sk = keys[perm.long()]
            for w in (32, 64):
                d = torch.ones(R, dtype=torch.int64, device=dev)
                d[1:] = (sk[1:] != sk[:-1]).to(torch.int64)
                d[::w] = 1
                res[f"anc{w}"] = round(int(d.sum().item()) / ((R + w - 1) // w), 3)
    return res


def run_method_grid(H, bvh, rays, opts, reps):
    """The frame workload's method grid: TwoPoint K in {32, 64}; HCC with the paper-exact cut
    (C = K) and with larger cuts C in {256 ... 4096} truncated to K bits; MLHCC16 (8+8) and
    MLHCC32 (16+16); the regular-grid control and the prefix path code at K in {32, 64}; and
    HCC / TwoPoint with the shorter sorts (low bits skipped, or tile-local sorts)."""
    vs = [dict(mode="twopoint", K=k) for k in (32, 64)]
    vs += [dict(mode="hcc", C=c, K=k) for k in (32, 64) for c in (k, 256, 512, 1024, 2048, 4096)]
    vs += [dict(mode="mlhcc", top=8, low=8, K=16), dict(mode="mlhcc", top=16, low=16, K=32)]
    vs += [dict(mode="grid", K=k) for k in (32, 64)]
    vs += [dict(mode="ppc", K=k) for k in (32, 64)]
    vs += [dict(mode="hcc", C=32, K=32, skip=8), dict(mode="hcc", C=32, K=32, skip=16),
           dict(mode="hcc", C=32, K=32, tile=1024), dict(mode="hcc", C=32, K=32, tile=4096),
           dict(mode="twopoint", K=32, tile=4096), dict(mode="twopoint", K=32, skip=16)]
    rows = []
    for v in vs:
        rows.append(measure_variant(H, bvh, rays, v, opts, reps))
    best = max(rows, key=lambda r: r["mrays_s"])
    log("method grid: " + "; ".join(f"{r['method']} {r['mrays_s']:.0f} ({r['node_fetches_per_ray']:.1f} nf/ray)"
                                    for r in rows))
    log(f"method grid best: {best['method']} {best['mrays_s']} Mrays/s")
    return rows


def run_bounces(H, args, bvh, tris_h, sec, rays):
    """Bounces 2 and 3 of the frame workload: diffuse rays spawned at the previous bounce's
    closest hits (origins now scattered over the scene, directions random).  Per bounce: NoSort
    with trace options tuned on its own order; TwoPoint and HCC (C = K) with key length, skipped
    bits and trace options tuned on the bounce's own rays in their own orders (at least half of
    the key sorted); and the untuned rows HCC C = K = 32 and 64, MLHCC16 (8+8) and MLHCC32
    (16+16), TwoPoint K = 32, each with a full sort and the trace options of its method's tuned
    row.  Node / triangle fetches per ray are the one-ray-per-lane kernel's
    wavefront counts (equal to the oracle's wave model, see the tests)."""
    import torch
    import workloads as W
    from paper_2305_16652_amd import autotune as AT
    out = {}
    prev, prev_d = sec, rays
    sk = tuple(int(x) for x in args.skips.split(","))
    for bounce in (2, 3):
        t0 = time.time()
        h = H.trace(bvh, prev_d, opts=H.TraceOpts(64, 2, 0, 1, 32, 128, 8192, H.TRACE_WIDE)).cpu().numpy()
        nxt, _ = W.spawn_diffuse(prev, h[:, 0].copy(), h[:, 1].copy().view(np.uint32), tris_h, seed=7,
                                 bounce=bounce - 1)
        rd = torch.from_numpy(nxt).to(rays.device)
        opts = AT.tune_trace(bvh, rd, None, candidates=AT.WIDE)[0]
        tw, _ = AT.tune_reorder(bvh, rd, "twopoint", key_bits=(16, 32), skips=sk, candidates=AT.WIDE,
                                min_sorted_frac=args.min_sorted_frac)
        hc, _ = AT.tune_reorder(bvh, rd, "hcc", cuts=(16, 32), key_bits=(16, 32), skips=sk, paper_exact=True,
                                candidates=AT.WIDE, min_sorted_frac=args.min_sorted_frac)
        method_opts = {"nosort": opts, "twopoint": tw.opts, "hcc": hc.opts, "mlhcc": hc.opts}
        variants = [dict(mode="nosort"), dict(mode="twopoint", K=tw.key_bits, skip=tw.skip),
                    dict(mode="hcc", C=hc.cut, K=hc.key_bits, skip=hc.skip),
                    dict(mode="hcc", C=32, K=32), dict(mode="hcc", C=64, K=64),
                    dict(mode="mlhcc", top=8, low=8, K=16), dict(mode="mlhcc", top=16, low=16, K=32),
                    dict(mode="twopoint", K=32)]
        seen, rows = set(), []
        for v in variants:
            name = variant_name(v)
            if name in seen:
                continue
            seen.add(name)
            row = measure_variant(H, bvh, rd, v, method_opts[v["mode"]], args.grid_reps)
            # the tuned configuration of each method (NoSort, and the first TwoPoint and HCC rows)
            row["tuned"] = v is variants[0] or v is variants[1] or v is variants[2]
            rows.append(row)
        out[str(bounce)] = dict(rays=int(rd.shape[0]), trace_opts={m: AT.opts_dict(o) for m, o in method_opts.items()},
                                rows=rows)
        log(f"frame bounce {bounce} ({rd.shape[0]} rays, {time.time() - t0:.1f}s): " +
            "; ".join(f"{r['method']} {r['mrays_s']:.0f} Mrays/s (trace {r['trace_ms']:.2f} ms, "
                      f"{r['node_fetches_per_ray']:.1f} nf/ray)" for r in rows))
        if prev_d is not rays:
            del prev_d
        prev, prev_d = nxt, rd
    del prev_d
    return out


def run_packets(H, bvh, prim, shadow) -> dict:
    """Wavefront packets against per-lane launches, by ray order: the frame's primary rays in
    pixel order (closest hit) and its shadow rays (any hit) in pixel order, HCC order (C = K = 32,
    full sort; C = K = 16 sorted on the top 8 bits) and TwoPoint order (K = 32, full sort).  Each
    entry: the fastest per-lane 4-wide launch and the fastest packet launch for that order, each
    tuned over its candidates (trace time only; the order's encode and sort are not included).
    A packet walks the union of its 64 rays' traversals, so its time follows the coherence the
    order gives each wavefront (Section 3.1), while the per-lane launch barely depends on it."""
    from paper_2305_16652_amd import autotune as AT
    out = {}

    def row(name, rays, perm, closest):
        lane = AT.tune_trace(bvh, rays, perm, closest=closest, candidates=AT.WIDE)
        pack = AT.tune_trace(bvh, rays, perm, closest=closest, candidates=AT.PACKET)
        out[name] = dict(lane_ms=round(lane[1], 4), packet_ms=round(pack[1], 4),
                         lane_opts=AT.opts_dict(lane[0]), packet_opts=AT.opts_dict(pack[0]))
        log(f"packets {name}: per-lane {lane[1]:.3f} ms, packets {pack[1]:.3f} ms")

    row("primary nosort", prim, None, True)
    row("shadow nosort", shadow, None, False)
    for name, mode, cut, k, skip in (("shadow hcc C=32 K=32", H.KEY_HCC, 32, 32, 0),
                                     ("shadow hcc C=16 K=16 skip 8", H.KEY_HCC, 16, 16, 8),
                                     ("shadow twopoint K=32", H.KEY_TWOPOINT, 0, 32, 0)):
        cut_h = H.select_cut(bvh, cut) if mode == H.KEY_HCC else None
        perm = H.sort_ex(H.encode(bvh, cut_h, mode, k, shadow), k, skip)
        row(name, shadow, perm, False)
        del perm
    return out


def drift_shadow_rows(H, bvh, rd, args) -> dict:
    """Any-hit rows of the drift scene's shadow rays: per-lane 4-wide trace options tuned on the
    rays in pixel order (NoSort) and in TwoPoint order (every reordered row), as for the diffuse
    rows; encode + sort included in each row's rate."""
    from paper_2305_16652_amd import autotune as AT
    opts = AT.tune_trace(bvh, rd, None, closest=False, candidates=AT.WIDE)[0]
    tperm = H.sort(H.encode(bvh, None, H.KEY_TWOPOINT, 32, rd), 32)
    sorted_opts = AT.tune_trace(bvh, rd, tperm, closest=False, candidates=AT.WIDE)[0]
    del tperm
    rows = [measure_variant(H, bvh, rd, dict(mode="nosort"), opts, args.drift_reps, closest=False)]
    for v in (dict(mode="twopoint", K=32), dict(mode="hcc", C=16, K=16), dict(mode="hcc", C=32, K=32),
              dict(mode="mlhcc", top=16, low=16, K=32)):
        rows.append(measure_variant(H, bvh, rd, v, sorted_opts, args.drift_reps, closest=False))
    log(f"drift shadow ({rd.shape[0]} rays): " +
        "; ".join(f"{r['method']} {r['mrays_s']:.0f} Mrays/s (trace {r['trace_ms']:.2f} ms)" for r in rows))
    return dict(rays=int(rd.shape[0]), rows=rows, trace_opts=AT.opts_dict(opts),
                sorted_trace_opts=AT.opts_dict(sorted_opts))


def run_drift(H, args):
    """Boundary-drift workload: 10M thin triangles in 64 Gaussian clusters inside the unit room,
    1920x1080x4 camera, two diffuse bounces.  For each bounce: NoSort, and TwoPoint, HCC (C = K)
    and the regular grid at K in {16, 24, 32, 48, 64}, with node fetches/ray and ANC.  Also the
    any-hit shadow rays of the camera rays' hits (two lights): NoSort, TwoPoint K = 32, HCC C = K
    = 16 and 32, MLHCC32, each with encode + sort included."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    t0 = time.time()
    spec = W.cluster_scene(args.drift_tris, seed=90)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).to(dev))
    opts = H.TraceOpts(64, 2, 0, 1, 32, 64, 8192, H.TRACE_WIDE)
    rays = W.pinhole_rays(spec, args.width, args.height, args.drift_spp, seed=91)
    from paper_2305_16652_amd import autotune as AT
    log(f"drift scene: {spec.tris.shape[0]} triangles, {rays.shape[0]} primary rays ({time.time() - t0:.1f}s)")
    out = dict(triangles=int(spec.tris.shape[0]), camera=f"{args.width}x{args.height}x{args.drift_spp}",
               bounces={})
    ks = [int(k) for k in args.drift_keys.split(",")]
    for bounce in (1, 2):
        rd = torch.from_numpy(rays).to(dev)
        h = H.trace(bvh, rd, opts=opts).cpu().numpy()
        del rd
        t, prim = h[:, 0].copy(), h[:, 1].copy().view(np.uint32)
        if bounce == 1 and not args.no_shadow:
            shd, _ = W.spawn_shadow(rays, t, prim, spec.tris, spec.lights)
            out["shadow"] = drift_shadow_rows(H, bvh, torch.from_numpy(shd).to(dev), args)
            del shd
        rays, _ = W.spawn_diffuse(rays, t, prim, spec.tris, seed=92, bounce=bounce - 1)
        rd = torch.from_numpy(rays).to(dev)
        # 4-wide trace options per bounce: tuned on the unsorted rays for NoSort, and on one
        # sorted order (TwoPoint, K = 32, full sort) for every reordered row
        opts = AT.tune_trace(bvh, rd, None, candidates=AT.WIDE)[0]
        tkeys = H.encode(bvh, None, H.KEY_TWOPOINT, 32, rd)
        sorted_opts = AT.tune_trace(bvh, rd, H.sort(tkeys, 32), candidates=AT.WIDE)[0]
        del tkeys
        rows = [measure_variant(H, bvh, rd, dict(mode="nosort"), opts, args.drift_reps)]
        for k in ks:
            for v in (dict(mode="twopoint", K=k), dict(mode="hcc", C=k, K=k), dict(mode="grid", K=k)):
                rows.append(measure_variant(H, bvh, rd, v, sorted_opts, args.drift_reps))
        # the paper's two-level code (a 16- and a 32-bit key from 8 + 8 and 16 + 16 cut nodes)
        for v in (dict(mode="mlhcc", top=8, low=8, K=16), dict(mode="mlhcc", top=16, low=16, K=32)):
            rows.append(measure_variant(H, bvh, rd, v, sorted_opts, args.drift_reps))
        out["bounces"][str(bounce)] = dict(rays=int(rd.shape[0]), rows=rows, trace_opts=AT.opts_dict(opts),
                                           sorted_trace_opts=AT.opts_dict(sorted_opts))
        log(f"drift bounce {bounce} ({rd.shape[0]} rays): " +
            "; ".join(f"{r['method']} {r['mrays_s']:.0f} Mrays/s {r['node_fetches_per_ray']:.1f} nf/ray "
                      f"anc32 {r.get('anc32', 0):.2f}" for r in rows))
        del rd
    return out


def measured_traffic(kernel: str, opts):
    """HBM bytes per trace launch from the committed PMC summary: the entry taken for this
    kernel with these launch options (flags, refill, chunk, wavefronts, stack), while the trace
    kernel sources still hash to what they were then (else None)."""
    path = os.path.join(ROOT, "profiles", "trace_traffic.txt")
    if not os.path.exists(path):
        return None
    lines = [l.strip() for l in open(path) if "=" in l and not l.startswith("#")]
    kv = dict(l.split("=", 1) for l in lines if not l.startswith("launch="))
    if kv.get("kernel") != kernel:
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_2305_16652_amd", "csrc", f), "rb").read()
                   for f in ("trace.hip", "hcc_internal.h"))
    if hashlib.sha256(src).hexdigest()[:16] != kv.get("kernel_sha256_16"):
        return None
    want = [int(opts.flags), int(opts.refill), int(opts.chunk), int(opts.waves), int(opts.stack)]
    for l in lines:
        if l.startswith("launch="):
            f = [int(x) for x in l.split("=", 1)[1].split()]
            if f[:5] == want:
                return f[5] + f[6]
    return None


def kernel_name(H, opts) -> str:
    if opts.flags & H.TRACE_WIDE:
        return "k_trace_wide"
    return "k_trace_persistent" if opts.persistent else "k_trace"


def kernel_counted_fetches(H, bvh, rays, perm, opts) -> dict:
    """Wavefront-distinct node and triangle fetches per ray as the launch itself counts them
    (hcc_trace_count for persistent and 4-wide launches, hcc_trace_stats otherwise)."""
    import torch
    R = rays.shape[0]
    wide = bool(opts.flags & H.TRACE_WIDE)
    if wide or opts.persistent:
        _, nodes, tris = H.trace_count(bvh, rays, perm, opts=opts)
    else:
        _, _, _, wn, wt = H.trace_stats(bvh, rays, perm)
        nodes, tris = int(wn.to(torch.int64).sum().item()), int(wt.to(torch.int64).sum().item())
    node_bytes = (QUANT_NODE_BYTES if opts.flags & H.TRACE_QUANT else WIDE_NODE_BYTES) if wide else NODE_BYTES
    return dict(node_fetches_per_ray=round(nodes / R, 3), tri_fetches_per_ray=round(tris / R, 3),
                node_bytes=node_bytes, bytes_per_ray=round((node_bytes * nodes + TRI_BYTES * tris) / R, 1))


def roofline_of(H, R, trace_ms_mean, opts, model, counted):
    """Roofline of the headline's trace kernel.  Algorithmic bytes per launch: the oracle's
    lockstep wave model of the rays in the launch's order (distinct 64-byte BVH2 nodes and
    48-byte triangles per 64-lane wavefront and step, child-test traversal), plus each ray's
    record, permutation entry and hit record; divided by the kernel's mean launch time over the
    timed steps (HIP events on the launch stream).  The kernel's own fetch count is reported
    beside it; without the oracle leg (--no-cpu) it takes the model's place."""
    io = RAY_BYTES + PERM_BYTES + HIT_BYTES
    if model is not None:
        per_ray, numerator = model["bytes_per_ray"], "oracle wave model (BVH2 nodes, 64-lane waves)"
    elif counted is not None:
        per_ray, numerator = counted["bytes_per_ray"], "kernel-counted fetches"
    else:
        return None
    bytes_per_launch = R * (per_ray + io)
    achieved = bytes_per_launch / (trace_ms_mean * 1e-3) / 1e9
    kernel = kernel_name(H, opts)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(kernel, opts),
                    kernel=kernel + "<closest>", launch_ms=round(trace_ms_mean, 4), bytes_per_ray=round(per_ray + io, 1),
                    numerator=numerator)
    if counted is not None:
        roofline["kernel_counted_bytes_per_ray"] = round(counted["bytes_per_ray"] + io, 1)
    if roofline["traffic"]:
        # where the launch sits against HBM by the bytes it actually moves (PMC): far below, because
        # the modelled fetch stream is served by L2 and the Infinity Cache; the kernel is bound by
        # vector-memory instruction issue instead
        roofline["traffic_frac"] = round(roofline["traffic"] / (trace_ms_mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    log(f"roofline: {achieved:.0f} GB/s of algorithmic traffic ({roofline['frac']:.3f} of HBM peak) from the "
        f"{numerator}; {per_ray + io:.0f} B/ray" +
        (f" (kernel-counted {counted['bytes_per_ray'] + io:.0f} B/ray)" if counted else ""))
    return roofline


def run_oracle_leg(tris_h, sec, args, gpu_hits, conf, head):
    """The part of the benchmark that runs the CPU oracle: (1) its encode + sort + trace timed on
    a strided sample of the secondary rays in the headline configuration (the CPU baseline), and
    (2) its lockstep wave model over every k-th 64-ray wavefront of each method's trace order
    (keys and sort computed by the oracle over all rays), which gives the roofline's numerator."""
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    R = sec.shape[0]
    ob = O.build_bvh(tris_h)
    had = O.had(ob)

    def order(m):
        c = conf[m]
        if m == "nosort":
            return None, None
        k, skip = c["key_bits"], c["skip"]
        if m.startswith("hcc"):
            keys = O.encode_hcc(sec, O.cut_boxes(ob, O.select_cut(ob, had, c["cut"])), k, threads=cores)
        else:
            keys = O.encode_twopoint(sec, O.scene_box(tris_h), k, threads=cores)
        return keys, (O.sort(keys) if skip == 0 else O.sort_prefix(keys, k, skip))

    # (1) CPU baseline on the headline configuration
    c = conf[head]
    sample = np.ascontiguousarray(sec[:: args.cpu_stride])
    n = sample.shape[0]
    log(f"CPU oracle on {n} rays with {cores} threads")
    cb = O.cut_boxes(ob, O.select_cut(ob, had, c["cut"])) if head.startswith("hcc") else None
    t0 = time.time()
    if cb is not None:
        keys = O.encode_hcc(sample, cb, c["key_bits"], threads=cores)
        perm = O.sort_prefix(keys, c["key_bits"], c["skip"])
    else:
        perm = None
    h = O.trace(ob, sample, perm=perm, threads=cores)
    dt = time.time() - t0
    g = gpu_hits[:: args.cpu_stride]
    agree = float(np.mean(g[:, 1].copy().view(np.uint32) == h.prim))
    log(f"CPU oracle: {dt:.1f}s, {n / dt / 1e6:.3f} Mrays/s; prim agreement with GPU {agree:.6f}")
    one = np.ascontiguousarray(sec[:: args.cpu_stride * 8])
    t0 = time.time()
    p1 = O.sort_prefix(O.encode_hcc(one, cb, c["key_bits"]), c["key_bits"], c["skip"]) if cb is not None else None
    O.trace(ob, one, perm=p1, threads=1)
    dt1 = time.time() - t0
    log(f"CPU oracle, 1 thread: {one.shape[0]} rays in {dt1:.1f}s, {one.shape[0] / dt1 / 1e6:.4f} Mrays/s")
    cpu = dict(value=round(n / dt / 1e6, 4), unit="Mrays/s", cores=cores, kind="oracle",
               sample=f"every {args.cpu_stride}th bounce-1 secondary ray ({n} rays): {head} encode (C={c['cut']}, "
                      f"K={c['key_bits']}) + stable sort (top {c['key_bits'] - c['skip']} bits) + closest-hit trace, "
                      f"{dt:.1f} s wall",
               prim_agreement_with_gpu=agree,
               single_thread=dict(value=round(one.shape[0] / dt1 / 1e6, 4), cores=1,
                                  sample=f"every {args.cpu_stride * 8}th ray ({one.shape[0]} rays), {dt1:.1f} s"))

    # (2) wave model of each method's trace order
    model = {}
    n_waves = (R + 63) // 64
    waves = np.arange(0, n_waves, args.model_wave_stride, dtype=np.uint32)
    for m in conf:
        t0 = time.time()
        keys, perm = order(m)
        nodes, tris, _ = O.wave_fetches(ob, sec, perm, 64, True, 1, waves, threads=cores)
        # wavefronts modelled: every stride-th, the ragged last one counted at its own size
        rays_modelled = sum(min(64, R - 64 * int(w)) for w in waves)
        nf = float(nodes.sum()) / rays_modelled
        tf = float(tris.sum()) / rays_modelled
        model[m] = dict(node_fetches_per_ray=round(nf, 3), tri_fetches_per_ray=round(tf, 3),
                        bytes_per_ray=round(NODE_BYTES * nf + TRI_BYTES * tf, 1),
                        waves_modelled=int(waves.shape[0]), wave_stride=args.model_wave_stride)
        if keys is not None:
            model[m]["anc64"] = round(O.anc(keys, perm, 64), 3)
            model[m]["anc32"] = round(O.anc(keys, perm, 32), 3)
        log(f"wave model {m}: {nf:.2f} node + {tf:.2f} triangle fetches per ray "
            f"({waves.shape[0]} wavefronts, {time.time() - t0:.1f}s)")
    return dict(cpu_baseline=cpu, model=model)


if __name__ == "__main__":
    main()
