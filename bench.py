"""Throughput of the photon-path verification hot path on one MI355X.

One step = one frame of the paper-scale workload: new object / light
transforms, transform + hierarchy refit, origin update + dynamic-occlusion
verification, work-queue compaction, error-based re-trace (T = 1%) and photon
compaction.  Inputs are resident in HBM before the timed region.  Prints one
JSON line (metric: verified path segments per second).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def light_moved(sc, f):
    import numpy as np
    a, b = sc.light_xforms[f], sc.light_xforms[f - 1]
    return [not np.array_equal(a[l].view(np.uint32), b[l].view(np.uint32)) for l in range(a.shape[0])]


def cpu_baseline(sc, engine, torch, T, target_s):
    """The oracle (untuned) timed on a bounded sample of the same workload:
    sampled paths of the full-size store, frame 1, verification and re-trace
    timed apart (median of 3 runs each).  The same sampled paths, loaded from
    the oracle's frame-0 store into a full-size device store, are verified and
    re-traced on the GPU too, and compared with the oracle outside its
    decision bands (excluded paths counted)."""
    import numpy as np
    import oracle as O
    N, B = sc.n_paths, sc.max_bounces
    rng = np.random.default_rng(17)
    fs0 = O.frame_scene(sc, 0)
    fs1 = O.frame_scene(sc, 1, 0)
    n = 2048
    while True:
        cols = np.unique(rng.choice(N, n, replace=False))
        ora, amb0, _ = O.initial_trace(fs0, N, B, sc.seed, paths=cols)
        snap = ora.select(cols)
        tv, tr = [], []
        for rep in range(3):
            for k in ("pos", "hit", "energy", "radius"):
                getattr(ora, k)[:, cols] = getattr(snap, k)
            ora.origin[cols] = snap.origin
            ora.info[cols] = snap.info
            t0 = time.perf_counter()
            ambv, ex = O.verify(fs1, ora, paths=cols)
            t1 = time.perf_counter()
            replaced = int(((ora.info[cols] >> 30) & 1).sum())
            ambr, rays = O.retrace(fs1, ora, T, sc.seed, 1, paths=cols)
            t2 = time.perf_counter()
            tv.append(t1 - t0)
            tr.append(t2 - t1)
        total = sum(tv) + sum(tr)
        log("cpu baseline: %d sampled paths, %.2f s (3 runs)" % (cols.size, total))
        if total >= target_s * 0.4 or n >= 1 << 18:
            break
        n = int(min(1 << 18, n * max(2.0, min(8.0, target_s / max(total, 1e-3)))))
    mv, mr = sorted(tv)[1], sorted(tr)[1]
    seg = float(ex.sum())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {"value": seg / (mv + mr), "unit": "segments/s", "cores": cores, "kind": "oracle",
           "sample": "%d sampled paths of the full-size store, frame 1 (verify + error-based re-trace), "
                     "median of 3 runs, %.1f s in all" % (cols.size, total),
           "verify_s": mv, "retrace_s": mr, "verify_segments_per_s": seg / mv,
           "retrace_rays_per_s": float(rays.sum()) / mr, "replaced_paths": replaced}
    # parity of the GPU on the same sampled paths, frame 1
    ctx = engine.Context(sc)
    st = ctx.new_store()
    ctx.frame_begin(0)
    ctx.initial_trace(st, sc.seed, 0)
    st.load_numpy(dict(pos=snap.pos, hit=snap.hit, energy=snap.energy, radius=snap.radius, origin=snap.origin,
                       info=snap.info), cols=cols)
    ctx.frame_begin(1)
    ctx.verify(st)
    ctx.retrace(st, T, sc.seed, 1)
    torch.cuda.synchronize()
    g = st.to_numpy(cols)
    ctx.close()
    o = ora.select(cols)
    ok = (amb0 == 0) & (ambv == 0) & (ambr == 0)
    nrow = (o.info >> 22) & 15
    rows = np.arange(B)[:, None] < nrow[None, :]
    info_bad = int((g["info"][ok] != o.info[ok]).sum())
    hit_bad = int(((g["hit"] != o.hit) & rows)[:, ok].sum())
    dp = np.abs(g["pos"] - o.pos).max(-1)[rows & ok[None, :]]
    res["parity_sample"] = {"paths": int(cols.size), "excluded": int((~ok).sum()), "compared": int(ok.sum()),
                            "info_mismatches": info_bad, "hit_mismatches": hit_bad,
                            "max_position_diff": float(dp.max()) if dp.size else 0.0}
    return res


def set_tuning(ctx, tuning):
    if tuning:
        ctx.set_tuning(tuning["retrace_variant"], tuning["retrace_blocks_per_cu"], tuning["walk_min_active"],
                       tuning["verify_blocks_per_cu"], tuning["verify_min_active"])


def headline_graph(args, engine, sc, torch, np, T, tuning):
    """The measured workload itself in the batched form: the whole frame of
    the one scene captured in a HIP graph and replayed, and all the timed
    frames captured in one graph and launched once, against the plain
    per-frame calls, from identical frame-0 stores (stores compared bit for
    bit after the timed frames)."""
    K = args.headline_graph_frames
    seed = sc.seed
    if K + 2 > sc.n_frames:
        # more frames than the scene holds: the same scene, its motion played
        # back and forth (0 .. n-1, n-2 .. 0, 1 ..), so that frames 2 .. K + 1
        # exist and consecutive frames still differ
        import dataclasses
        per = 2 * max(1, sc.n_frames - 1)
        idx = [f % per if f % per < sc.n_frames else per - f % per for f in range(K + 2)]
        sc = dataclasses.replace(sc, obj_xforms=sc.obj_xforms[idx], light_xforms=sc.light_xforms[idx])
    consecutive = 1 + K <= sc.n_frames - 1  # frames 2 .. K + 1 exist (one launch runs consecutive frames)
    runs = []
    for mode in ("plain", "graph", "frames"):
        if mode == "frames" and not consecutive:
            runs.append(None)
            continue
        ctx = engine.Context(sc)
        set_tuning(ctx, tuning)
        st = ctx.new_store()
        ctx.frame_begin(0)
        ctx.initial_trace(st, seed, 0)
        b = engine.Batch([ctx], [st], T, seed) if mode != "plain" else None
        cap = sc.n_paths * sc.max_bounces
        o = (torch.empty((cap, 3), dtype=torch.float32, device="cuda"),
             torch.empty((cap, 3), dtype=torch.float32, device="cuda"),
             torch.zeros(1, dtype=torch.int32, device="cuda"))
        stats = ctx.new_stats()

        def frame(f, s=None):
            if b is not None:
                b.frame(f, s)
            else:
                ctx.frame_begin(f)
                ctx.verify(st, s)
                ctx.retrace(st, T, seed, f)
                ctx.compact_photons_into(st, *o)

        frame(1, stats)  # warm-up (graph capture)
        torch.cuda.synchronize()
        if mode == "frames":
            # capture the K-frame graph outside the timed region, then return
            # to the state after frame 1: transforms of frame 1 (one more
            # frame 1), the store as it was
            snap = st.to_numpy()
            b.frames(2, K, stats)
            frame(1, stats)
            torch.cuda.synchronize()
            st.load_numpy(snap)
        stats.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        if mode == "frames":
            b.frames(2, K, stats)
        else:
            for i in range(K):
                frame(1 + (1 + i) % max(1, sc.n_frames - 1), stats)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        seg = ctx.stats_dict(stats)["segments_examined"]
        runs.append((dt / K * 1e3, seg / dt, st.to_numpy()))
        if b is not None:
            b.close()
        ctx.close()
    (pm, ps, sp), (bm, bs, sb) = runs[0], runs[1]
    same = all(np.array_equal(sp[k].view(np.uint32), sb[k].view(np.uint32)) for k in sp)
    res = {"frames_timed": K, "plain_ms_per_frame": pm, "graph_ms_per_frame": bm, "plain_segments_per_s": ps,
           "graph_segments_per_s": bs, "speedup": pm / bm, "stores_bit_identical": bool(same)}
    if runs[2] is not None:
        fm, fs, sf = runs[2]
        res.update({"frames_per_launch": K, "one_launch_ms_per_frame": fm, "one_launch_segments_per_s": fs,
                    "one_launch_speedup": pm / fm,
                    "one_launch_stores_bit_identical": bool(all(np.array_equal(sp[k].view(np.uint32),
                                                                               sf[k].view(np.uint32)) for k in sp))})
    return res


def method_modes(engine, scenes, torch, sc_paper, T, tuning, frames=6):
    """The method's other forms on the paper-scale workload, each on its own
    context from its own frame-0 trace: distribution maps (4x4 positions x
    8 rings x 16 sectors per light, updated after every verification), the
    cosine-ratio reading of Equation 2, and the same rooms lit by two moving
    spotlights or two cameras.  Per-phase times are HIP events on the
    context's stream, averaged over the timed frames."""
    out = {}
    for mode in ("distribution_maps", "cosine_ratio", "spot_lights", "cameras"):
        if mode in ("spot_lights", "cameras"):
            kind, param = (1, (0.8, 0.0)) if mode == "spot_lights" else (2, (0.6, 0.4))
            sc = scenes.make_rooms("paper", 6, 6, 300_000, 8, (100, 50), 3_000_000, 7, frames + 3, T, 3,
                                   n_lights=2, lights_move=True, torus_size=(0.2, 0.07), light_kind=kind,
                                   light_param=param)
        else:
            sc = sc_paper if sc_paper.n_frames >= frames + 3 else scenes.make_paper(frames=frames + 3)
        ctx = engine.Context(sc)
        set_tuning(ctx, tuning)
        if mode == "distribution_maps":
            ctx.set_distribution_map((4, 4, 8, 16))
        if mode == "cosine_ratio":
            ctx.set_energy_test(True)
        st = ctx.new_store()
        ctx.frame_begin(0)
        ctx.initial_trace(st, sc.seed, 0)
        cap = sc.n_paths * sc.max_bounces
        o = (torch.empty((cap, 3), dtype=torch.float32, device="cuda"),
             torch.empty((cap, 3), dtype=torch.float32, device="cuda"),
             torch.zeros(1, dtype=torch.int32, device="cuda"))
        names = ["frame_begin", "verify", "distribution", "queue", "retrace", "compact_photons"]
        acc = {k: 0.0 for k in names}
        seg = rays = inv = 0
        for i in range(2 + frames):
            f = 1 + i
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            s = ctx.new_stats()
            ev[0].record()
            ctx.frame_begin(f)
            ev[1].record()
            ctx.verify(st, s, build_queue=False)
            ev[2].record()
            if mode == "distribution_maps":
                ctx.update_distribution(st, sc.seed, f)
            ev[3].record()
            ctx.build_queue(st)
            ev[4].record()
            ctx.retrace(st, T, sc.seed, f, s)
            ev[5].record()
            ctx.compact_photons_into(st, *o)
            ev[6].record()
            torch.cuda.synchronize()
            if i < 2:
                continue  # warm-up frames
            for j, k in enumerate(names):
                acc[k] += ev[j].elapsed_time(ev[j + 1]) / frames
            d = ctx.stats_dict(s)
            seg += d["segments_examined"]
            rays += d["rays_traced"]
            inv += d["paths_invalid"]
        ctx.close()
        del st, o
        torch.cuda.empty_cache()
        ms = sum(acc.values())
        out[mode] = {"ms_per_frame": ms, "segments_per_s": seg / frames / (ms / 1e3),
                     "phases_ms": {k: v for k, v in acc.items() if k != "distribution" or mode == "distribution_maps"},
                     "paths_invalid_per_frame": inv / frames, "rays_per_frame": rays / frames}
        log("mode %s: %.3f ms per frame" % (mode, ms))
    return out


def cache_resident_mid(engine, scenes, torch, tuning):
    """The mid workload (1M paths x 7 bounces, 3 moving objects): its
    verification reads (about 130 MB) fit in the 256 MB Infinity Cache, so
    its rate is the cache-resident one, not an HBM figure."""
    sc = scenes.make_mid(frames=8, threshold=0.01)
    ctx = engine.Context(sc)
    set_tuning(ctx, tuning)
    st = ctx.new_store()
    ctx.frame_begin(0)
    ctx.initial_trace(st, sc.seed, 0)
    ms, byts = [], []
    for f in range(1, 8):
        s = ctx.new_stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.frame_begin(f)
        e0.record()
        ctx.verify(st, s, build_queue=False)
        e1.record()
        ctx.retrace(st, 0.01, sc.seed, f)
        torch.cuda.synchronize()
        if f > 2:
            ms.append(e0.elapsed_time(e1))
            byts.append(20 * sc.n_paths + 16 * ctx.stats_dict(s)["segments_examined"])
    ctx.close()
    v = sum(ms) / len(ms)
    gbs = sum(byts) / len(byts) / (v / 1e3) / 1e9
    return {"workload": "mid: %d paths x %d bounces, %d static + %d dynamic triangles" % (
        sc.n_paths, sc.max_bounces, sc.n_static, sc.n_dynamic_tris()), "verify_ms": v,
        "algorithmic_bytes_per_launch": sum(byts) / len(byts), "achieved_gbs": gbs,
        "frac_of_hbm_peak": gbs / PEAK_HBM_GBS, "note": "cache-resident (verification set below the 256 MB MALL)"}


def batched(args, engine, scenes, torch, np, tuning=None):
    """64 uneven scenes: per-scene launches (plain) against one graph-captured
    launch per phase (batched), from identical frame-0 stores; the stores must
    stay bit-identical."""
    K = args.batch_steps
    t0 = time.perf_counter()
    scs = scenes.make_batch(n_scenes=args.batch_scenes, frames=K + 2)
    T, seed = 0.01, 4
    sets = []
    for _ in range(2):
        ctxs = [engine.Context(s) for s in scs]
        sts = [c.new_store() for c in ctxs]
        for c, st in zip(ctxs, sts):
            c.frame_begin(0)
            c.initial_trace(st, seed, 0)
        sets.append((ctxs, sts))
    torch.cuda.synchronize()
    log("batch: %d scenes, %d paths, set up in %.1f s" % (len(scs), sum(s.n_paths for s in scs),
                                                          time.perf_counter() - t0))
    (pc, ps), (bc, bs) = sets
    for c in pc + bc:
        set_tuning(c, tuning)
    caps = [st.n_paths * st.B for st in ps]
    outs = [(torch.empty((c, 3), dtype=torch.float32, device="cuda"),
             torch.empty((c, 3), dtype=torch.float32, device="cuda"),
             torch.zeros(1, dtype=torch.int32, device="cuda")) for c in caps]
    b = engine.Batch(bc, bs, T, seed)
    stats_p = pc[0].new_stats()
    stats_b = bc[0].new_stats()
    # frame 1: warmup (graph capture for the batch)
    for c, st, o in zip(pc, ps, outs):
        c.frame_begin(1)
        c.verify(st)
        c.retrace(st, T, seed, 1)
        c.compact_photons_into(st, *o)
    b.frame(1, stats_b)
    torch.cuda.synchronize()
    stats_b.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for f in range(2, 2 + K):
        for c, st, o in zip(pc, ps, outs):
            c.frame_begin(f)
            c.verify(st, stats_p)
            c.retrace(st, T, seed, f)
            c.compact_photons_into(st, *o)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    t = time.perf_counter()
    for f in range(2, 2 + K):
        b.frame(f, stats_b)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t
    same = all(np.array_equal(x.to_numpy()[k].view(np.uint32), y.to_numpy()[k].view(np.uint32))
               for x, y in zip(ps, bs) for k in ("pos", "hit", "energy", "info", "origin"))
    sp, sb = pc[0].stats_dict(stats_p), bc[0].stats_dict(stats_b)
    b.close()
    for c in pc + bc:
        c.close()
    return {"scenes": len(scs), "paths": int(sum(s.n_paths for s in scs)), "frames_timed": K,
            "plain_ms_per_frame": plain_s / K * 1e3, "batched_ms_per_frame": batch_s / K * 1e3,
            "plain_segments_per_s": sp["segments_examined"] / plain_s,
            "batched_segments_per_s": sb["segments_examined"] / batch_s,
            "speedup": plain_s / batch_s, "stores_bit_identical": bool(same),
            "segments_examined_equal": sp["segments_examined"] == sb["segments_examined"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="paper", choices=["tiny", "mid", "paper"])
    ap.add_argument("--paths", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-box-test", action="store_true",
                    help="skip the frames with the paper's box test (counter runs of the triangle test)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--no-headline-graph", action="store_true")
    ap.add_argument("--no-cache-resident", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the distribution-map, cosine-ratio, spotlight and camera frames")
    ap.add_argument("--headline-graph-frames", type=int, default=30)
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=5)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs a path store on one device "
              "(stores would shard by path range across GPUs, each with its own replica of the scene)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2111_06906_amd import engine, scenes

    cfg = {"tiny": scenes.make_tiny, "mid": scenes.make_mid, "paper": scenes.make_paper}[args.config]
    frames = 1 + args.warmup + args.steps
    kw = {"frames": max(frames, 2)}
    if args.paths:
        kw["n_paths"] = args.paths
    t0 = time.perf_counter()
    sc = cfg(**kw)
    T = sc.threshold if sc.threshold >= 0 else 0.01
    log("scene %s: %d static + %d dynamic tris, %d paths, B=%d, %d frames (%.1f s)" % (
        sc.name, sc.n_static, sc.n_dynamic_tris(), sc.n_paths, sc.max_bounces, frames, time.perf_counter() - t0))

    torch.cuda.set_device(0)
    # achievable HBM bandwidth of a plain 1 GiB device copy (read + write),
    # the practical ceiling beside the 8 TB/s peak
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    copy_ms = []
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        if i:
            copy_ms.append(e0.elapsed_time(e1))
    copy_gbs = 2.0 * a.numel() * 4 / (sum(copy_ms) / len(copy_ms) / 1e3) / 1e9
    del a, b
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ctx = engine.Context(sc)
    st = ctx.new_store()
    N, B = sc.n_paths, sc.max_bounces
    cap = N * B
    out_pos = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    out_en = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    out_cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.frame_begin(0)
    ctx.initial_trace(st, sc.seed, 0)
    torch.cuda.synchronize()
    log("frame 0 traced")

    # the photon compaction runs on the context's stream in the timed frames
    # (clean per-phase events); a later section overlaps it with the next frame
    cstream = None

    def step(f, ev, stats):
        ev[0].record()
        ctx.frame_begin(f)
        ev[1].record()
        ctx.verify(st, stats, build_queue=False)
        ev[2].record()
        ctx.build_queue(st)
        ev[3].record()
        ctx.retrace(st, T, sc.seed, f, stats)
        ev[4].record()
        if cstream is None:
            ctx.compact_photons_into(st, out_pos, out_en, out_cnt)
            ev[5].record()
        else:
            # overlapped with the next frame's begin, verification and queue
            # (the next re-trace waits for it)
            ctx.compact_photons_into(st, out_pos, out_en, out_cnt, stream=cstream)
            ev[5].record(cstream)

    tuning = None
    for f in range(1, 1 + args.warmup):
        if f == 1 and not args.no_autotune:
            # autotuner: re-trace variant and grid on this workload (frame 1 on
            # a snapshot of the store, which it restores)
            ctx.frame_begin(f)
            tuning = ctx.autotune(st, T, sc.seed, f)
            log("autotune: %s" % tuning)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            ev[0].record()
            ev[1].record()
            ctx.verify(st, None, build_queue=False)
            ctx.build_queue(st)
            ctx.retrace(st, T, sc.seed, f)
            ctx.compact_photons_into(st, out_pos, out_en, out_cnt)
            continue
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        step(f, ev, None)
    torch.cuda.synchronize()
    log("warmup done")

    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
    stats = [ctx.new_stats() for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        step(1 + args.warmup + i, evs[i], stats[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    names = ["frame_begin", "verify", "queue", "retrace", "compact_photons"]
    phase = {n: 0.0 for n in names}
    verify_ms = []
    seg = 0
    bytes_verify = 0
    sd = [ctx.stats_dict(s) for s in stats]
    for i in range(K):
        f = 1 + args.warmup + i
        for j, n in enumerate(names):
            phase[n] += evs[i][j].elapsed_time(evs[i][j + 1])
        verify_ms.append(evs[i][1].elapsed_time(evs[i][2]))
        seg += sd[i]["segments_examined"]
        moved_paths = sum(int(sc.light_paths[l]) for l, m in enumerate(light_moved(sc, f)) if m)
        origin_writes = max(0, moved_paths - sd[i]["paths_light_lost"])
        bytes_verify += 20 * N + 16 * sd[i]["segments_examined"] + 12 * origin_writes
    tot = {k: sum(s[k] for s in sd) for k in sd[0]}
    avg_verify_s = sum(verify_ms) / K / 1e3
    achieved = bytes_verify / K / avg_verify_s / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "verify_traffic.json")
    if os.path.exists(tf):
        # counters only count for the kernel source they were taken with
        try:
            from paper_2111_06906_amd.traffic import sources_sha1
            rec = json.load(open(tf))
            if rec.get("sources_sha1") == sources_sha1():
                traffic = rec.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    res = {
        "metric": "verified path segments/s",
        "value": seg / wall,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d paths x %d bounces, %d static + %d dynamic triangles in %d objects, "
                               "%d lights (%s), energy threshold %g" % (
                                   sc.name, N, B, sc.n_static, sc.n_dynamic_tris(), sc.n_dynamic,
                                   sc.light_half.shape[0], "moving" if sc.meta.get("lights_move") else "static", T),
                   "paths": N, "max_bounces": B, "frames_timed": K},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "verification call (k_verify_scan, task scan + k_verify_gather, k_verify_trace, "
                               "k_verify_finish, k_verify_stats)",
                     "algorithmic_bytes_per_launch": bytes_verify / K, "avg_launch_ms": avg_verify_s * 1e3},
        "phases_ms_per_frame": {k: v / K for k, v in phase.items()},
        "hbm_reference": {"copy_1gib_gbs": copy_gbs,
                          "compact_photons_gbs": 56.0 * int(out_cnt.item()) / (phase["compact_photons"] / K / 1e3) / 1e9,
                          "note": "device copy: bytes read + written per second; compaction: 32 B read + 24 B "
                                  "written per existing photon"},
        "tuning": tuning,
        "per_frame": {"segments_examined": tot["segments_examined"] / K, "paths_invalid": tot["paths_invalid"] / K,
                      "paths_light_lost": tot["paths_light_lost"] / K, "rays_traced": tot["rays_traced"] / K,
                      "photons_written": tot["photons_written"] / K, "reuse_accepted": tot["reuse_accepted"] / K,
                      "verify_box_hits": tot["verify_box_hits"] / K, "photons_compacted": int(out_cnt.item())},
    }
    rt_s = phase["retrace"] / K / 1e3
    rays = tot["rays_traced"] / K
    res["retrace"] = {"rays_per_s": rays / rt_s, "ms": rt_s * 1e3,
                      "algorithmic_gbs": (48.0 * rays + 4.0 * tot["paths_invalid"] / K) / rt_s / 1e9,
                      "note": "latency-bound traversal; algorithmic bytes: 16 B origin vertex read + 32 B photon "
                              "written per ray, 4 B information word per queued path"}
    log(json.dumps(res["phases_ms_per_frame"]))
    # the paper's comparator on the same GPU: re-trace every path every frame
    base_ms = []
    for i in range(3):
        f = 1 + args.warmup + (i % K)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.frame_begin(f)
        e0.record()
        ctx.queue_all(st)
        ctx.retrace(st, -1.0, sc.seed, 1000 + i)
        e1.record()
        torch.cuda.synchronize()
        base_ms.append(e0.elapsed_time(e1))
    res["baseline_retrace_all_ms"] = sum(base_ms) / len(base_ms)
    # the paper's own dynamic-occlusion test (moved objects' bounding boxes,
    # PV_VERIFY_BOXES) on the frames that follow: cheaper verification, more
    # paths to re-trace
    ctx.set_verify_mode(True)
    bx = {"verify": [], "retrace": [], "frame": [], "paths_invalid": [], "rays_traced": []}
    bx_bytes = []
    for i in range(0 if args.no_box_test else 5):
        f = 1 + (3 + args.warmup + i) % max(1, sc.n_frames - 1)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        s = ctx.new_stats()
        step(f, ev, s)
        torch.cuda.synchronize()
        d = ctx.stats_dict(s)
        if i == 0:
            continue  # first frame after the full re-trace baseline
        bx["verify"].append(ev[1].elapsed_time(ev[2]))
        bx["retrace"].append(ev[3].elapsed_time(ev[4]))
        bx["frame"].append(ev[0].elapsed_time(ev[5]))
        bx["paths_invalid"].append(d["paths_invalid"])
        bx["rays_traced"].append(d["rays_traced"])
        moved_paths = sum(int(sc.light_paths[l]) for l, m in enumerate(light_moved(sc, f)) if m)
        bx_bytes.append(20 * N + 16 * d["segments_examined"] + 12 * max(0, moved_paths - d["paths_light_lost"]))
    ctx.set_verify_mode(False)
    # the overlap form of the compaction (side stream, beside the next frame's
    # begin, verification and queue): whole frames, wall clock
    cstream = torch.cuda.Stream()
    ov_frames = [1 + (8 + args.warmup + i) % max(1, sc.n_frames - 1) for i in range(11)]
    ov_seg = 0
    ov_stats = [ctx.new_stats() for _ in ov_frames]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    step(ov_frames[0], ev, None)  # warm-up
    torch.cuda.synchronize()
    t_ov = time.perf_counter()
    for f, s in zip(ov_frames[1:], ov_stats[1:]):
        step(f, ev, s)
    torch.cuda.synchronize()
    t_ov = time.perf_counter() - t_ov
    ov_seg = sum(ctx.stats_dict(s)["segments_examined"] for s in ov_stats[1:])
    res["overlapped_compaction"] = {"frames": len(ov_frames) - 1,
                                    "ms_per_step": t_ov / (len(ov_frames) - 1) * 1e3,
                                    "segments_per_s": ov_seg / t_ov}
    cstream = None
    if not args.no_box_test:
        res["box_test_mode"] = {k + ("" if k in ("paths_invalid", "rays_traced") else "_ms"): sum(v) / len(v)
                                for k, v in bx.items()}
        # the same algorithmic bytes per call as the headline's roofline, for
        # the paper's own (box) test: context, not the headline figure
        vb = sum(bx_bytes) / len(bx_bytes)
        vgbs = vb / (sum(bx["verify"]) / len(bx["verify"]) / 1e3) / 1e9
        res["box_test_mode"].update({"verify_algorithmic_bytes": vb, "verify_achieved_gbs": vgbs,
                                     "verify_frac_of_hbm_peak": vgbs / PEAK_HBM_GBS})
    # frame begin (object transforms, hierarchies, top-level trees) with the
    # objects' hierarchies refit, then with every object's hierarchy rebuilt on
    # the device as a linear BVH (last: the mode keeps larger traversal stacks)
    fb = {}
    for mode in (0, 1):
        ctx.set_tuning(object_rebuild=mode)
        ms = []
        for i in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.frame_begin(1 + (i % max(1, sc.n_frames - 1)))
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        fb["rebuild_ms" if mode else "refit_ms"] = sum(ms[1:]) / len(ms[1:])
    res["frame_begin_objects"] = fb
    ctx.close()
    del st, out_pos, out_en
    torch.cuda.empty_cache()
    if not args.no_batch:
        res["batched"] = batched(args, engine, scenes, torch, np, tuning)
    if not args.no_headline_graph:
        res["batched_headline"] = headline_graph(args, engine, sc, torch, np, T, tuning)
    if not args.no_cache_resident and args.config == "paper":
        res["cache_resident_mid"] = cache_resident_mid(engine, scenes, torch, tuning)
    if not args.no_modes and args.config == "paper":
        res["method_modes"] = method_modes(engine, scenes, torch, sc, T, tuning)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc, engine, torch, T, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
