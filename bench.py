#!/usr/bin/env python3
"""Throughput of the streaming Count-Sketch halo-finder hot path on one MI355X.

One step = one pass of the whole hot path over the resident synthetic stream:
zero the sketch, Add every particle (update), collect the distinct cells whose
estimate passes theta (second pass), select the top-k.  `value` is particles/s of
whole steps.  The roofline object covers csk_sketch_update (bin + accumulate
kernels), timed with HIP events on the stream the library launches on.

Workload (default): 2^30 float32 particles, L = 1000 Mpc/h, 2^20 Plummer halos
(power-law masses, slope -1.9, 50..1e6 particles), 30 % uniform background;
cells of 0.25 Mpc/h (4000^3), d = 5 rows, w = 2^24 counters, k = 1e4.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
BYTES_PER_PARTICLE = 12         # algorithmic: each float32 position read once

# HBM bytes moved by one update (bin + accumulate) of the 2^30-particle workload, from
# rocprofv3 FETCH_SIZE (x2.000) and WRITE_SIZE (x1.000) scaled by a 1 GiB device copy
# (profiles/update_kernels_plummer_2e30.md).  Reported only while the kernel sources hash
# to what was profiled; any change to them makes `traffic` null until measured again.
TRAFFIC = {"bytes": 45_239_779_984, "particles": 1 << 30,
           "sources_sha256": "e0e1f7bd342daf50b0b5635228e7ed48f7592ae02dc0c50787f91da9329cb834"}
TRAFFIC_SOURCES = ["csk_update.hip", "csk_sortbin.hip", "csk_sortbin_body.h", "csk_kernel_util.h", "csk_device.h",
                   "csk_internal.h"]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_00975_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n):
    if TRAFFIC["bytes"] is None or n != TRAFFIC["particles"]:
        return None
    return TRAFFIC["bytes"] if sources_sha256() == TRAFFIC["sources_sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["scale", "small"], default="scale")
    ap.add_argument("--n", type=int, default=0, help="override the particle count (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured ceilings (stream read, LDS and global atomic rates)")
    ap.add_argument("--no-small", action="store_true", help="skip the 2^20-particle warm/cold update")
    ap.add_argument("--no-packed", action="store_true",
                    help="skip the packed 8-byte particle stream")
    ap.add_argument("--no-router", action="store_true",
                    help="skip the learned router vs plain sketch comparison at equal memory")
    ap.add_argument("--router-n", type=int, default=1 << 28, help="particles per router snapshot")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched update of 64 uneven sub-volumes")
    ap.add_argument("--no-hierarchy", action="store_true",
                    help="skip the two-layer (super-cell) search")
    ap.add_argument("--no-dictionary", action="store_true",
                    help="skip the full-dictionary search (every cell of the mesh estimated once)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--no-protocols", action="store_true",
                    help="skip the per-2^26-chunk update timing and the 2^28-particle w = 2^22 update")
    ap.add_argument("--oracle-full", action="store_true",
                    help="time the oracle on the whole stream on every host core (minutes; own JSON line)")
    ap.add_argument("--large", action="store_true",
                    help="run the large combined workload (2^34 particles, three grids, router) instead")
    ap.add_argument("--large-n", type=int, default=0, help="particles of the large run (default 2^34)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates the HBM byte counters)")
    return ap.parse_args()


def make_positions(wl, n, torch):
    """Generate the stream on the host in chunks and copy it into one device tensor."""
    import numpy as np
    chunk = wl.chunk or n
    dev = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    host = torch.empty((min(chunk, n), 3), dtype=torch.float32).pin_memory()
    hv = host.numpy()
    t0 = time.time()
    if wl.f_bg < 0:
        dev.copy_(torch.from_numpy(wl.generate()))
    else:
        for a in range(0, n, chunk):
            m = min(chunk, n - a)
            wl.generate(a, m, out=hv[:m])
            dev[a:a + m].copy_(host[:m], non_blocking=False)
            log(f"  generated {a + m}/{n} particles ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return dev


def calibrate_theta(s, pos, wl, csk):
    """Geometric search for a threshold that leaves at least k candidates (the paper
    moves its threshold geometrically, Sec. 3.1 item 4).  With >= k candidates the
    top-k does not depend on theta."""
    theta = 1 << 22
    while True:
        s.clear_candidates()
        s.collect(pos, wl.delta, wl.L, theta)
        keys, est, rc = s.topk(wl.k)
        if rc == csk.CSK_OK:
            return theta, int(est[-1].item())
        if theta <= 1:
            return csk.INT32_MIN, None
        theta //= 2


def host_info():
    """The host the oracle runs on: logical CPUs, the ones this process may use, the model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    info = {"nproc": os.cpu_count(), "usable": aff, "cpu_model": model}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info["lscpu_" + key.strip().lower().replace("(s)", "s").replace(" ", "_")] = val.strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(pos_dev, wl, sample, threads):
    """The oracle as it stands on the first `sample` particles.  With threads > 1 the Add
    phase runs on that many threads (one sketch per thread, summed); the estimates of
    every distinct cell and the top-k run on one thread either way."""
    import oracle
    pos = pos_dev[:sample].cpu().numpy()
    t0 = time.perf_counter()
    M, _ = oracle.sketch(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, threads=threads)
    t1 = time.perf_counter()
    oracle.topk_sketch(M, oracle.hash_tables(wl.seed, wl.d), pos, wl.delta, wl.L, oracle.INT32_MIN, wl.k)
    t2 = time.perf_counter()
    return {"value": sample / (t2 - t0), "unit": "particles/s", "cores": threads, "kind": "oracle",
            "host": host_info(),
            "sample": f"first {sample} particles of the same stream; keys + Add ({t1 - t0:.1f} s on {threads} "
                      f"thread{'s' if threads > 1 else ''}), estimates of every distinct cell + top-{wl.k} "
                      f"({t2 - t1:.1f} s, one thread)"}


def oracle_full(pos_dev, wl, threads, chunk=1 << 26, key_block=1 << 24, s=None, theta=None):
    """The oracle on the whole stream, in pieces that each report when done:
    - Add (oracle.sketch) on `threads` host threads per chunk of `chunk` particles; the
      counters of the chunks are summed, which is the sketch of the stream (Add is additive);
    - the distinct cell keys (oracle.keys per chunk, then one np.unique over the chunks');
    - the top-k of Sec. 2.2 over every distinct cell with theta = INT32_MIN: oracle.topk_keys
      on disjoint blocks of `key_block` distinct keys, then the same order (estimate desc,
      key asc) over the blocks' winners.
    With a sketch handle s (and its calibrated theta), the GPU's counters and top-k of the
    same stream are compared with the oracle's."""
    import numpy as np
    import oracle
    n = pos_dev.shape[0]
    T = oracle.hash_tables(wl.seed, wl.d)
    t0 = time.perf_counter()
    M = np.zeros((wl.d, wl.w), dtype=np.int64)
    skipped = 0
    uniq_parts = []
    t_add = t_keys = 0.0
    for a in range(0, n, chunk):
        pos = pos_dev[a:a + chunk].cpu().numpy()
        ta = time.perf_counter()
        Mc, sk = oracle.sketch(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, threads=threads)
        tb = time.perf_counter()
        M += Mc
        skipped += int(sk)
        uniq_parts.append(np.unique(oracle.keys(pos, wl.delta, wl.L)))
        tc = time.perf_counter()
        t_add += tb - ta
        t_keys += tc - tb
        log(f"  oracle: particles {a + pos.shape[0]}/{n}: Add {tb - ta:.1f} s, keys {tc - tb:.1f} s")
    M = M.astype(np.int32)     # exact: every counter of the whole stream fits int32 (n < 2^31)
    t1 = time.perf_counter()
    uniq = np.unique(np.concatenate(uniq_parts))
    del uniq_parts
    t2 = time.perf_counter()
    log(f"  oracle: {uniq.size} distinct cells ({t2 - t1:.1f} s)")
    wk, we = [], []
    for b in range(0, uniq.size, key_block):
        kk, ee = oracle.topk_keys(M, T, uniq[b:b + key_block], oracle.INT32_MIN, wl.k)
        wk.append(kk)
        we.append(ee)
        log(f"  oracle: estimates and top-k of distinct cells {min(b + key_block, uniq.size)}/{uniq.size}")
    kk, ee = np.concatenate(wk), np.concatenate(we)
    order = np.lexsort((kk, -ee.astype(np.int64)))[:wl.k]
    ko, eo = kk[order], ee[order]
    t3 = time.perf_counter()
    out = {"particles": n, "threads_add": threads, "host": host_info(), "chunk": chunk,
           "keys_add_s": t_add, "distinct_keys_s": t_keys + (t2 - t1), "estimates_topk_s": t3 - t2,
           "whole_s": t3 - t0, "add_particles_per_s": n / t_add, "whole_particles_per_s": n / (t3 - t0),
           "distinct_cells": int(uniq.size), "skipped": skipped, "kth_estimate": int(eo[-1]) if len(eo) else None}
    if s is not None:
        s.reset()
        s.update(pos_dev, wl.delta, wl.L)
        s.collect(pos_dev, wl.delta, wl.L, theta)
        gk, ge, _ = s.topk(wl.k)
        gk = gk.cpu().numpy().view(np.uint64)
        ge = ge.cpu().numpy()
        out["gpu_counters_equal"] = bool(np.array_equal(s.counters().cpu().numpy(), M))
        # the GPU's candidate pass keeps every cell whose estimate is >= theta: its top-k is
        # the oracle's whenever the oracle's k-th estimate is >= theta
        out["gpu_theta"] = theta
        out["gpu_topk_equal"] = bool(np.array_equal(gk, ko) and np.array_equal(ge, eo))
    return {"oracle_full": out}


def update_protocols(pos, wl, csk, torch, reps=10):
    """The update under the stream's own chunking (2^26 particles per csk_sketch_update call,
    each call complete: bin + accumulate), and the 2^28-particle stream into w = 2^22
    counters (80 MiB, MALL-resident): per call, median of `reps`."""
    import numpy as np
    stream = torch.cuda.current_stream()
    out = {}
    n = pos.shape[0]
    chunk = wl.chunk or n
    s = csk.Sketch(wl.d, wl.w, wl.seed)
    s.update(pos[:chunk], wl.delta, wl.L)
    per_call, whole = [], []
    for _ in range(3):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(n // chunk + 1)]
        torch.cuda.synchronize()
        evs[0].record(stream)
        for i, a in enumerate(range(0, n, chunk)):
            s.update(pos[a:a + chunk], wl.delta, wl.L)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        per_call += [evs[i].elapsed_time(evs[i + 1]) for i in range(len(evs) - 1)]
        whole.append(evs[0].elapsed_time(evs[-1]))
    s.close()
    ms = float(np.median(whole))
    out["chunked"] = {"chunk": chunk, "calls": n // chunk, "stream_ms": ms,
                      "call_ms_median": float(np.median(per_call)),
                      "particles_per_s": n / (ms / 1e3),
                      "roofline_frac": BYTES_PER_PARTICLE * n / (ms / 1e3) / (HBM_PEAK_GBS * 1e9),
                      "note": "median of 3 passes over the stream, one csk_sketch_update per chunk; each call "
                              "adds its tokens to the counters (a read-modify-write of all d w counters)"}
    m = min(n, 1 << 28)
    w4 = 1 << 22
    s = csk.Sketch(wl.d, w4, wl.seed)
    s.update(pos[:m], wl.delta, wl.L)
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.update(pos[:m], wl.delta, wl.L)
        e1.record(stream)
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1))
    s.close()
    ms4 = float(np.median(t))
    out["w2e22_2e28"] = {"particles": m, "w": w4, "update_ms": ms4, "particles_per_s": m / (ms4 / 1e3),
                         "roofline_frac": BYTES_PER_PARTICLE * m / (ms4 / 1e3) / (HBM_PEAK_GBS * 1e9),
                         "note": "the first 2^28 particles of the stream into d = 5, w = 2^22 (80 MiB of "
                                 "counters, MALL-resident): the learned-router configuration's plain sketch"}
    return out


def dictionary_search(s, wl, theta, keys_top, torch):
    """Count Sketch with Full Search on the step's final counters: every key of the G^3
    mesh is estimated once (csk_collect_dictionary), then the same top-k.  Timed with HIP
    events on the launch stream; compared with the stream top-k of the step."""
    G = round(wl.L / wl.delta)
    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    s.clear_candidates()
    e0.record(stream)
    s.collect_dictionary(wl.delta, wl.L, theta)
    e1.record(stream)
    keys, est, rc = s.topk(wl.k)
    e2.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    same = torch.isin(keys, keys_top).sum().item()
    return {"keys": G ** 3, "theta": theta, "collect_ms": ms, "keys_per_s": G ** 3 / (ms / 1e3),
            "topk_ms": e1.elapsed_time(e2), "status": rc,
            "shared_with_stream_topk": same / max(1, keys_top.numel()),
            "note": "every cell of the mesh, occupied or not (Sec. 2.2 item 1, Alg. 1)"}


def hierarchical_search(s, pos, wl, theta, keys_top, csk, torch, group=1000, c=3):
    """Count Sketch Hierarchical (Alg. 3) on the step's counters: a second sketch of the
    same shape counts super-cells key // group over the same stream; its c*k heaviest
    super-cells (threshold found by halving, as for theta) are searched cell by cell in
    the step's sketch.  Times each stage with HIP events; compares the top-k with the
    stream top-k of the step."""
    stream = torch.cuda.current_stream()
    coarse = csk.Sketch(wl.d, wl.w, wl.seed + 1, max_candidates=1 << 22, group=group)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev[0].record(stream)
    coarse.update(pos, wl.delta, wl.L)
    ev[1].record(stream)
    theta1 = 1 << 22
    while True:   # threshold that leaves at least c*k heavy super-cells
        coarse.clear_candidates()
        coarse.collect_dictionary(wl.delta, wl.L, theta1)
        _, est1, rc1 = coarse.topk(c * wl.k)
        if rc1 == csk.CSK_OK or theta1 <= 1:
            break
        theta1 //= 2
    coarse.clear_candidates()
    ev[2].record(stream)
    coarse.collect_dictionary(wl.delta, wl.L, theta1)
    ev[3].record(stream)
    s.clear_candidates()
    s.collect_children(coarse, theta)
    ev[4].record(stream)
    keys, est, rc = s.topk(wl.k)
    torch.cuda.synchronize()
    G = round(wl.L / wl.delta)
    out = {"group": group, "super_cells": -(-G ** 3 // group), "theta1": theta1, "theta2": theta,
           "coarse_update_ms": ev[0].elapsed_time(ev[1]), "super_dictionary_ms": ev[2].elapsed_time(ev[3]),
           "children_ms": ev[3].elapsed_time(ev[4]), "status": rc,
           "shared_with_stream_topk": torch.isin(keys, keys_top).sum().item() / max(1, keys_top.numel()),
           "note": "heavy super-cells key // group first, then their cells (Sec. 2.2 item 3, Alg. 3)"}
    coarse.close()
    return out


def batched_subvolumes(csk, torch, reps=5):
    """64 independent sub-volumes of uneven size (2^16..2^24 particles, w = 2^14..2^20,
    Plummer halos in L = 100 at delta = 0.1): the batched update (one bin and one
    accumulate launch, workgroup budget from the autotuner) against the same sketches
    updated one after another, and the whole update -> collect -> top-k pipeline of all
    64 (batched reset, update, candidate pass and top-k) eager against one HIP graph replay."""
    from concurrent.futures import ThreadPoolExecutor
    import workloads
    from paper_1711_00975_amd import autotune
    subs = workloads.batch_subvolumes()
    t0 = time.time()
    with ThreadPoolExecutor(host_threads()) as ex:   # one generator thread each: no nested OpenMP teams
        host = list(ex.map(lambda wl: wl.generate(threads=1), subs))
    pos = [torch.from_numpy(h).cuda() for h in host]
    del host
    log(f"  generated {len(subs)} sub-volumes ({time.time() - t0:.1f} s)")
    # candidate sets sized to each sub-volume (8 k keys, or all n when n <= 2^18, so that a
    # small stream cannot overflow): clearing and compacting a set costs time in proportion
    # to its slots
    sk = [csk.Sketch(wl.d, wl.w, wl.seed, max_candidates=max(1 << 14, 8 * wl.k, min(wl.n, 1 << 18)))
          for wl in subs]
    counts = [wl.n for wl in subs]
    total = sum(counts)
    tuner = autotune.Tuner()
    tuned = tuner.tune_batch(sk, pos, 0.1, 100.0)
    log(f"  tuned the batch: {tuned['wg_budget']} workgroups")
    for s, n in zip(sk, counts):
        if not tuner.apply(s, n):
            tuner.tune_update(s.d, s.w, n)
            tuner.apply(s, n)
            log(f"  tuned w={s.w} n={n}: {tuner.lookup(autotune.size_class(s.w, n))['all_ms']}")
    try:
        tuner.save()
    except OSError:
        pass
    b = csk.Batch(sk, counts, 0.1, 100.0, wg_budget=tuned["wg_budget"])
    stream = torch.cuda.current_stream()

    def timed(fn):
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def sequential():
        for s, p in zip(sk, pos):
            s.update(p, 0.1, 100.0)

    b.update(pos)
    sequential()
    t_batch = timed(lambda: b.update(pos))
    t_seq = timed(sequential)
    log(f"  batched update {t_batch:.3f} ms, one by one {t_seq:.3f} ms")
    # a threshold per sub-volume, as for the main stream: halved from 2^16 until k cells pass
    # (the paper's geometric threshold, Sec. 3.1 item 4), on fresh counters
    ks = [wl.k for wl in subs]
    for s_ in sk:
        s_.reset()
    b.update(pos)
    thetas = []
    for s_, p, k_ in zip(sk, pos, ks):
        th = 1 << 16
        while th > 1:
            s_.clear_candidates()
            s_.collect(p, 0.1, 100.0, th)
            try:
                kk, ee, rc = s_.topk(k_)
            except csk.CskError:      # the set overflowed: the previous threshold is the lowest that fits
                th *= 2
                s_.reset()
                s_.update(p, 0.1, 100.0)
                break
            if kk.numel() == k_ and int(ee[k_ - 1].item()) >= th:
                break
            th //= 2
        thetas.append(th)
    log(f"  thresholds per sub-volume: {min(thetas)} .. {max(thetas)}")
    # the whole pipeline: batched update, then per sketch a filtered collect and top-k
    keys = [torch.empty(k, dtype=torch.int64, device="cuda") for k in ks]
    est = [torch.empty(k, dtype=torch.int32, device="cuda") for k in ks]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in ks]

    def pipeline():   # one step of the batch: fresh counters, update, candidate passes, top-k
        b.reset()                     # the 64 resets in one launch
        b.update(pos)                 # one bin and one accumulate launch
        b.collect(pos, thetas)        # the 64 candidate passes in one set of launches
        b.topk(ks, keys, est, outs)   # the 64 selections in one set of launches

    pipeline()
    torch.cuda.synchronize()
    t_eager = timed(pipeline)
    log(f"  eager pipeline {t_eager:.3f} ms; capturing the graph")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipeline()
    g.replay()
    torch.cuda.synchronize()
    t_graph = timed(g.replay)
    del g
    for s in sk:   # surfaces a latched device error (capacity, domain) of the last replay
        s.check()
    complete = sum(int(o[0].item()) == k_ for o, k_ in zip(outs, ks))   # k returned by the last replay
    b.close()
    for s in sk:
        s.close()
    return {"sub_volumes": len(subs), "particles": total, "widths": sorted(set(wl.w for wl in subs)),
            "wg_budget": tuned["wg_budget"], "budget_ms": tuned["all_ms"],
            "batch_update_ms": t_batch, "sequential_update_ms": t_seq,
            "particles_per_s": total / (t_batch / 1e3),
            "roofline_frac": BYTES_PER_PARTICLE * total / (t_batch / 1e3) / 1e9 / HBM_PEAK_GBS,
            "pipeline_eager_ms": t_eager, "pipeline_graph_ms": t_graph,
            "thresholds": [min(thetas), max(thetas)], "complete_topk": complete,
            "note": "sum over sub-volumes; update counters identical to one-by-one updates"}


def learned_router(csk, torch, workloads, n=1 << 28, k=10_000, w_plain=1 << 22, train_seeds=range(2, 10),
                   eval_seed=1, exact_slots=1 << 29, epochs=4, sweep_widths=(1 << 20, 1 << 18)):
    """Learned router vs the plain sketch at equal memory on the plain-at-scale recipe cut to
    n particles.  The model trains on the exact top-k labels of other-seed snapshots; the
    evaluation snapshot is routed (sample pre-pass -> features -> MLP -> admission ->
    split -> rest sketch -> merged top-k) and compared with a plain d x w_plain sketch
    on recall of the exact top-k."""
    from paper_1711_00975_amd.router import Router, RoutedStep, rest_width, TABLE_BYTES_PER_SLOT
    base = workloads.SCALE.with_(n=n, w=w_plain, k=k, name=f"plummer-2^{n.bit_length() - 1}-L1000-d0.25")
    r = Router(base.delta, base.L)
    snaps = []
    for sd in train_seeds:
        pos = make_positions(base.with_(seed=sd), n, torch)
        info = r.add_snapshot(pos, k, exact_slots)
        del pos
        snaps.append(info)
        log(f"  training snapshot seed {sd}: {info}")
    t0 = time.perf_counter()
    tr = r.train(epochs=epochs)
    torch.cuda.synchronize()
    tr["seconds"] = time.perf_counter() - t0
    log(f"  trained: {tr}")

    wl = base.with_(seed=eval_seed)
    pos = make_positions(wl, n, torch)
    tk, tc = csk.new_table(exact_slots)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    csk.exact_counts(pos, wl.delta, wl.L, tk, tc, err)
    ex_keys, ex_counts = csk.table_topk(tk, tc, 2 * k)
    assert err.item() == 0
    del tk, tc
    kth = int(ex_counts[k - 1].item())
    exact_top = ex_keys[:k]
    at_least_kth = ex_keys[ex_counts >= kth]

    def score(keys):
        keys = keys[:k]
        return {"strict": torch.isin(keys, exact_top).sum().item() / k,
                "tie_tolerant": torch.isin(keys, at_least_kth).sum().item() / k, "returned": int(keys.numel())}

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best, res = None, None
        for _ in range(reps):
            t = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) * 1e3
            best = dt if best is None else min(best, dt)
        return best, res

    def search_theta(run):
        # the top-k is final once k candidates were found and the k-th value is at least
        # theta (no key left out of the candidate set can beat it); the exact table's keys
        # are candidates whatever their counts, so the second condition matters there
        theta = 1 << 22
        while True:
            keys, est, rc = run(theta)
            if rc == csk.CSK_OK and keys.numel() == k and int(est[k - 1].item()) >= theta:
                return theta
            if theta <= 1:
                return csk.INT32_MIN
            theta //= 2

    # plain sketch: update + collect + top-k
    plain = csk.Sketch(wl.d, w_plain, wl.seed, max_candidates=1 << 22)

    def plain_run(theta):
        plain.reset()
        plain.update(pos, wl.delta, wl.L)
        plain.collect(pos, wl.delta, wl.L, theta)
        return plain.topk(k)
    theta_p = search_theta(plain_run)
    plain_ms, (plain_keys, _, _) = timed(lambda: plain_run(theta_p))
    log(f"  plain: theta {theta_p}, {plain_ms:.2f} ms")

    # routed: the sync-free step (admission, the rest update with the split fused in, the
    # candidate pass over the whole stream, the merged top-k), eager and as a HIP graph
    w_rest = rest_width(w_plain, wl.d, r.table_slots)
    rs = csk.Sketch(wl.d, w_rest, wl.seed, max_candidates=1 << 22)
    step = RoutedStep(r, rs, k)
    stage = {}

    def routed_run(theta, times=None):
        marks = [time.perf_counter()]

        def mark():
            if times is not None:
                torch.cuda.synchronize()
                marks.append(time.perf_counter())
        step.admit(pos)
        mark()
        step.update(pos)
        mark()
        step.select(pos, theta)
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        if times is not None:
            for nm, a, b in zip(["admit_ms", "update_routed_ms", "collect_topk_ms"], marks[:-1], marks[1:]):
                times[nm] = min(times.get(nm, 1e30), (b - a) * 1e3)
        keys, est, partial = step.result()
        return keys, est, (csk.CSK_W_INCOMPLETE if partial else csk.CSK_OK)
    theta_r = search_theta(routed_run)
    routed_ms, (routed_keys, _, _) = timed(lambda: routed_run(theta_r))
    for _ in range(2):
        routed_run(theta_r, stage)
    na = int(step.na.item())
    stage["admitted_cells"] = na
    stage["scored_cells"] = int(step.m.item())
    stage["table_particles"] = int(step.table_counts.sum().item())
    assert step.err.item() == 0 and stage["scored_cells"] <= step.cells.numel()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step.run(pos, theta_r)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(step.result()[0], routed_keys)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    graph_ms = None
    for _ in range(3):
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        graph_ms = t if graph_ms is None else min(graph_ms, t)
    del g
    log(f"  routed: theta {theta_r}, {routed_ms:.2f} ms eager, {graph_ms:.2f} ms as a graph, {stage}")
    # the same trained router at smaller memory (recall only, untimed)
    sweep = []
    for wp in sweep_widths:
        ps = csk.Sketch(wl.d, wp, wl.seed, max_candidates=1 << 22)

        def small_plain(theta):
            ps.reset()
            ps.update(pos, wl.delta, wl.L)
            ps.collect(pos, wl.delta, wl.L, theta)
            return ps.topk(k)
        tp = search_theta(small_plain)
        pk = small_plain(tp)[0]
        wr = rest_width(wp, wl.d, r.table_slots)
        rs2 = csk.Sketch(wl.d, wr, wl.seed, max_candidates=1 << 22)
        step2 = RoutedStep(r, rs2, k)

        def small_routed(theta):
            step2.run(pos, theta)
            torch.cuda.synchronize()
            keys, est, partial = step2.result()
            return keys, est, (csk.CSK_W_INCOMPLETE if partial else csk.CSK_OK)
        tr2 = search_theta(small_routed)
        rk = small_routed(tr2)[0]
        sweep.append({"w_plain": wp, "w_rest": wr, "plain_theta": tp, "routed_theta": tr2,
                      "plain_recall": score(pk), "routed_recall": score(rk)})
        log(f"  width {wp}: plain {sweep[-1]['plain_recall']}, routed {sweep[-1]['routed_recall']}")
        ps.close()
        rs2.close()
    out = {"workload": wl.name, "particles": n, "k": k, "exact_kth_count": kth,
           "train": {"seeds": list(train_seeds), "snapshots": snaps, **tr},
           "plain": {"d": wl.d, "w": w_plain, "bytes": wl.d * w_plain * 4, "theta": theta_p, "ms": plain_ms,
                     "particles_per_s": n / (plain_ms / 1e3), "recall": score(plain_keys)},
           "routed": {"d": wl.d, "w_rest": w_rest, "table_slots": r.table_slots,
                      "bytes": wl.d * w_rest * 4 + r.table_slots * TABLE_BYTES_PER_SLOT, "max_admitted": r.max_admit,
                      "theta": theta_r, "ms": routed_ms, "graph_ms": graph_ms,
                      "particles_per_s": n / (routed_ms / 1e3), "vs_plain": routed_ms / plain_ms,
                      "stages": stage, "recall": score(routed_keys)},
           "smaller_memory": sweep,
           "note": "eager times: one host synchronization at the end of each step (plain: the top-k's "
                   "readback); graph_ms: the routed step captured once and replayed; recall against the exact "
                   "top-k from csk_exact_counts + csk_table_topk"}
    plain.close()
    rs.close()
    r.close()
    return out


def packed_input(pos, wl, theta, keys_top, csk, torch, steps):
    """The same stream packed to 8 bytes per particle (three 21-bit coordinates, Sec. 4.1):
    update + collect + top-k timed as in the main step.  The packed stream defines its own
    cells (the mesh of 4000 cells does not divide 2^21), so the top-k is compared with the
    float stream's as overlap, not parity."""
    n = pos.shape[0]
    words = csk.pack_positions(pos, wl.L)
    s = csk.Sketch(wl.d, wl.w, wl.seed, max_candidates=1 << 22)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        s.reset()
        if ev is not None:
            ev[0].record(stream)
        s.update_packed(words, wl.delta, wl.L)
        if ev is not None:
            ev[1].record(stream)
        s.collect_packed(words, wl.delta, wl.L, theta)
        if ev is not None:
            ev[2].record(stream)
        return s.topk(wl.k)

    step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        keys, est, rc = step(evs[i])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    upd = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
    col = sum(e[1].elapsed_time(e[2]) for e in evs) / steps
    overlap = torch.isin(keys, keys_top).sum().item() / max(1, keys_top.numel())
    s.close()
    del words
    achieved = 8 * n / (upd / 1e3) / 1e9
    return {"bytes_per_particle": 8, "ms_per_step": ms, "particles_per_s": n / (ms / 1e3), "update_ms": upd,
            "update_particles_per_s": n / (upd / 1e3), "collect_ms": col, "status": rc,
            "update_roofline": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": achieved / HBM_PEAK_GBS},
            "topk_overlap_with_float_stream": overlap}


def large_run(args, csk, torch, workloads):
    """The large combined run: 2^34 particles generated on the device in 2^27-particle
    chunks (L = 3000, 2^24 halos), streamed into three grids (0.25, 0.5, 1.0) as one batch
    of w = 2^24 sketches, with the learned router on the 0.25 grid (its table and rest
    sketch take the memory of one plain sketch), top-10^5 per sketch.

    Passes over the stream (each regenerates its chunks): a 1 % sample pass for the router,
    the update pass, and the candidate pass (repeated with half the threshold if fewer than
    k candidates pass).  The router's model is trained first on eight boxes of the same
    density and recipe at 1/64 of the volume (L = 750, 2^28 particles, 2^18 halos, exact
    top-1563 labels)."""
    from paper_1711_00975_amd.router import Router, rest_width
    wl = workloads.LARGE
    n = args.large_n or wl.n
    chunk = min(wl.chunk, n)
    k = wl.k
    L = wl.L
    deltas = [0.25, 0.5, 1.0]
    out = {"metric": "particles/s sketched into three grids (update pass) + top-10^5 per grid; learned router "
                     "vs plain at equal memory on the 0.25 grid",
           "unit": "particles/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int32",
           "data": "synthetic (seeded Plummer halos + uniform background, generated on the device)",
           "config": {"workload": wl.name, "particles": n, "chunk": chunk, "L": L, "deltas": deltas, "d": wl.d,
                      "w": wl.w, "k": k, "halos": wl.n_halo}}
    # ---- the router's model, trained on small boxes of the same density
    t0 = time.perf_counter()
    scale = 4
    tw = wl.with_(L=L / scale, n=1 << 28, n_halo=wl.n_halo // scale ** 3, chunk=0)
    k_train = round(k / scale ** 3)
    rt = Router(wl.delta, tw.L)
    for sd in range(2, 10):
        pos = workloads.DeviceGenerator(tw.with_(seed=sd)).generate(0, tw.n)
        info = rt.add_snapshot(pos, k_train, 1 << 29)
        del pos
        log(f"  training box seed {sd}: {info}")
    tr = rt.train()
    params = rt.mlp.params()
    rt.close()
    del rt
    torch.cuda.empty_cache()
    out["router_training"] = {"box_L": tw.L, "particles": tw.n, "halos": tw.n_halo, "k": k_train, **tr,
                              "seconds": time.perf_counter() - t0}
    log(f"  router trained: {tr}")

    gen = workloads.DeviceGenerator(wl)
    buf = torch.empty((chunk, 3), dtype=torch.float32, device="cuda")
    nchunks = (n + chunk - 1) // chunk

    def chunks():
        for c in range(nchunks):
            a = c * chunk
            m = min(chunk, n - a)
            yield a, gen.generate(a, m, buf)

    # ---- pass 0: the 1 % sample of the whole stream, admission
    r = Router(wl.delta, L)
    r.mlp.set_params(params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, pos in chunks():
        csk.sample_counts(pos, r.delta_c, L, r.sample_seed, r.counts, index0=a, bitmap=r.bitmap)
    cells = csk.cell_list(r.counts, r.min_count, bitmap=r.bitmap)
    x = csk.cell_features(r.counts, r.delta_c, L, cells)
    admitted = csk.route_admit(cells, r.mlp.forward(x), r.max_admit)
    torch.cuda.synchronize()
    t_sample = time.perf_counter() - t0
    scored = int(cells.numel())
    del cells, x
    r.counts = r.bitmap = None            # the 108 GB of coarse counts are not needed again
    torch.cuda.empty_cache()
    log(f"  sample pass: {t_sample:.1f} s, {scored} cells scored, {admitted.numel()} admitted")

    # ---- pass 1: updates (three grids batched; the routed rest separately)
    mc = 1 << 23
    plain = [csk.Sketch(wl.d, wl.w, wl.seed, max_candidates=mc) for _ in deltas]
    w_rest = rest_width(wl.w, wl.d, r.table_slots)
    rest_sk = csk.Sketch(wl.d, w_rest, wl.seed, max_candidates=mc)
    batch = csk.Batch(plain, [chunk] * 3, deltas, [L] * 3)
    ttk, ttc = csk.new_table(r.table_slots)
    rest = torch.empty((chunk, 3), dtype=torch.float32, device="cuda")
    rcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    rerr = torch.zeros(1, dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t_gen = t_batch = t_route = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, (a, pos) in enumerate(chunks()):
        ev[0].record()
        batch.update([pos, pos, pos])
        ev[1].record()
        rcount.zero_()
        r.split(pos, admitted, ttk, ttc, rest, rcount, rerr)
        nr = int(rcount.item())
        rest_sk.update(rest[:nr], wl.delta, L)
        torch.cuda.synchronize()
        t_batch += ev[0].elapsed_time(ev[1])
        if c % 16 == 15:
            log(f"  update pass: {a + pos.shape[0]}/{n} particles ({time.perf_counter() - t0:.1f} s)")
    t_update = time.perf_counter() - t0
    batch.close()
    for sk in plain + [rest_sk]:
        sk.check()
    assert rerr.item() == 0
    # generation alone, for the split of the update pass's time
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(4):
        gen.generate(0, chunk, buf)
    torch.cuda.synchronize()
    t_gen = (time.perf_counter() - g0) / 4 * nchunks
    log(f"  update pass: {t_update:.1f} s (batched three-grid update {t_batch / 1e3:.2f} s, generation about "
        f"{t_gen:.2f} s)")

    # ---- pass 2: candidates, threshold from chunk 0, halved until k pass everywhere
    names = ["plain_0.25", "plain_0.5", "plain_1.0", "routed_0.25"]
    sketches = plain + [rest_sk]
    dl = deltas + [wl.delta]

    def collect_pass(thetas):
        for sk in sketches:
            sk.clear_candidates()
        for a, pos in chunks():
            for sk, dd, th in zip(sketches[:3], dl[:3], thetas[:3]):
                sk.collect(pos, dd, L, th)
            rcount.zero_()
            ttk2, ttc2 = scratch_table
            ttk2.fill_(-1)
            ttc2.zero_()
            r.split(pos, admitted, ttk2, ttc2, rest, rcount, rerr)
            nr = int(rcount.item())
            rest_sk.collect(rest[:nr], wl.delta, L, thetas[3])

    scratch_table = csk.new_table(r.table_slots)   # the split's table of pass 2 is discarded
    g0 = time.perf_counter()
    pos0 = gen.generate(0, chunk, buf)
    thetas = []
    for i, sk in enumerate(sketches[:3]):
        th = 1 << 22
        while th > 1:
            sk.clear_candidates()
            sk.collect(pos0, dl[i], L, th)
            kk, ee, rc = sk.topk(k)
            if kk.numel() == k:
                break
            th //= 2
        thetas.append(th)
    th = 1 << 22
    while th > 1:
        rcount.zero_()
        ttk2, ttc2 = scratch_table
        ttk2.fill_(-1)
        ttc2.zero_()
        r.split(pos0, admitted, ttk2, ttc2, rest, rcount, rerr)
        rest_sk.clear_candidates()
        rest_sk.collect(rest[:int(rcount.item())], wl.delta, L, th)
        kk, ee, rc = csk.topk_with_table(rest_sk, ttk, ttc, k)
        if kk.numel() == k and int(ee[k - 1].item()) >= th:
            break
        th //= 2
    thetas.append(th)
    results = {}
    for attempt in range(6):
        collect_pass(thetas)
        done = True
        for i, (nm, sk) in enumerate(zip(names, sketches)):
            if nm.startswith("routed"):
                kk, ee, rc = csk.topk_with_table(sk, ttk, ttc, k)
            else:
                kk, ee, rc = sk.topk(k)
            ok = kk.numel() == k and int(ee[k - 1].item()) >= thetas[i]
            results[nm] = (kk, ee, rc)
            if not ok:
                thetas[i] //= 2
                done = False
        log(f"  candidate pass {attempt + 1}: thetas {thetas}, complete {done}")
        if done:
            break
    t_collect = time.perf_counter() - g0
    grids = {}
    for i, nm in enumerate(names):
        kk, ee, rc = results[nm]
        grids[nm] = {"theta": thetas[i], "returned": int(kk.numel()), "kth_estimate": int(ee[-1].item()),
                     "max_estimate": int(ee[0].item()), "status": rc}
    pk, rk = results["plain_0.25"][0], results["routed_0.25"][0]
    # coarse consistency: the 0.5 cell of each 0.25 top cell (floor nesting) among the 0.5 top cells
    G1, G2 = round(L / 0.25), round(L / 0.5)
    ix, iy, iz = pk // (G1 * G1), (pk // G1) % G1, pk % G1
    parent = ((ix // 2) * G2 + iy // 2) * G2 + iz // 2
    out.update({
        "value": n / t_update, "ms_per_step": t_update * 1e3, "steps": 1, "warmup": 0, "scaling": "weak",
        "vs_baseline": None,
        "passes_s": {"sample": t_sample, "update": t_update, "candidates": t_collect},
        "update_pass": {"batched_three_grid_update_s": t_batch / 1e3,
                        "three_grid_particles_per_s": 3 * n / (t_batch / 1e3),
                        "generation_s_estimate": t_gen},
        "router": {"scored_cells": scored, "admitted": int(admitted.numel()), "w_rest": w_rest,
                   "table_slots": r.table_slots,
                   "table_particles": int(ttc.to(torch.int64).sum().item())},
        "grids": grids,
        "routed_vs_plain_top_overlap": torch.isin(rk, pk).sum().item() / k,
        "fine_top_parents_in_0.5_top": torch.isin(parent, results["plain_0.5"][0]).sum().item() / k,
    })
    for sk in sketches:
        sk.close()
    r.close()
    return out


def ceilings(pos, torch, reps=5):
    """Measured ceilings (libcsk_probe.so): the read bandwidth of the 12-byte particle
    records with the update's own load pattern, the LDS atomic rate (128 KiB array, random
    addresses), and the device-scope global atomic rate into tables of 64 KiB, 64 MiB and
    1 GiB.  Each is the best of `reps` timed launches after one warm-up."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_1711_00975_amd", "libcsk_probe.so"))
    P, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
    lib.probe_stream_read.argtypes = [P, u64, P, u32, P]
    lib.probe_lds_atomics.argtypes = [u64, u32, P, P]
    lib.probe_global_atomics.argtypes = [P, u32, u64, u32, P]
    lib.probe_xcd_atomics.argtypes = [P, u32, u64, u32, P]
    for f in (lib.probe_stream_read, lib.probe_lds_atomics, lib.probe_global_atomics, lib.probe_xcd_atomics):
        f.restype = C.c_int
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def timed(launch):
        assert launch() == 0
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            assert launch() == 0
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    n = pos.shape[0]
    blocks = 1024
    sink = torch.empty(blocks * 1024, dtype=torch.int32, device="cuda")
    read_ms = timed(lambda: lib.probe_stream_read(pos.data_ptr(), n, sink.data_ptr(), blocks, st))
    lds_iters, lds_blocks = 2048, 512
    lds_ms = timed(lambda: lib.probe_lds_atomics(lds_iters, lds_blocks, sink.data_ptr(), st))
    glob = {}
    g_iters, g_blocks = 64, 4096
    for lw, label in ((14, "64KiB"), (24, "64MiB"), (28, "1GiB")):
        table = torch.zeros(1 << lw, dtype=torch.int32, device="cuda")
        ms = timed(lambda: lib.probe_global_atomics(table.data_ptr(), lw, g_iters, g_blocks, st))
        glob[label] = g_iters * g_blocks * 256 / (ms / 1e3)
        del table
    xcd = {}
    for lw, label in ((14, "64KiB"), (18, "1MiB"), (22, "16MiB")):
        table = torch.zeros(8 << lw, dtype=torch.int32, device="cuda")
        ms = timed(lambda: lib.probe_xcd_atomics(table.data_ptr(), lw, g_iters, g_blocks, st))
        xcd[label] = g_iters * g_blocks * 256 / (ms / 1e3)
        del table
    return {"stream_read_GBs": 12 * n / (read_ms / 1e3) / 1e9,
            "xcd_private_atomics_per_s": xcd,
            "lds_atomics_per_s": lds_iters * lds_blocks * 1024 / (lds_ms / 1e3),
            "global_atomics_per_s": glob,
            "note": "libcsk_probe.so: 12-byte records read with eight dwordx3 loads in flight per thread; random "
                    "ds_add on 2^15 LDS words; random device-scope atomicAdd into 2^14, 2^24 and 2^28 words; random workgroup-scope atomicAdd, each "
                    "into the issuing XCD's own copy of a 2^14, 2^18 or 2^22-word table (performed in that XCD's L2)"}


def small_workload(csk, torch, workloads, reps=1000, cold_reps=20):
    """The 2^20-particle configuration: the update warm (1000 updates replayed from one HIP
    graph; positions and counters stay on chip) and cold (a 512 MiB write before each
    update flushes the MALL), and recall@100 against the exact histogram."""
    import numpy as np
    wl = workloads.SMALL
    pos = torch.from_numpy(wl.generate()).cuda()
    n = pos.shape[0]
    s = csk.Sketch(wl.d, wl.w, wl.seed)
    s.update(pos, wl.delta, wl.L)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            s.update(pos, wl.delta, wl.L)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    warm_us = e0.elapsed_time(e1) * 1e3 / reps
    del g
    flush = torch.empty(1 << 27, dtype=torch.int32, device="cuda")
    cold = []
    for r in range(cold_reps):
        flush.fill_(r)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        s.update(pos, wl.delta, wl.L)
        b.record()
        torch.cuda.synchronize()
        cold.append(a.elapsed_time(b) * 1e3)
    del flush
    cold_us = float(np.median(cold))
    s.reset()
    s.update(pos, wl.delta, wl.L)
    s.collect(pos, wl.delta, wl.L, csk.INT32_MIN)
    keys, est, rc = s.topk(wl.k)
    s.close()
    ck = csk.cell_keys(pos, wl.delta, wl.L)
    uniq, counts = torch.unique(ck, sorted=True, return_counts=True)
    order = np.lexsort((uniq.cpu().numpy(), -counts.cpu().numpy()))
    u, c = uniq.cpu().numpy()[order], counts.cpu().numpy()[order]
    kth = c[wl.k - 1]
    got = keys.cpu().numpy()
    return {"workload": wl.name, "particles": n,
            "warm_update_us": warm_us, "warm_particles_per_s": n / (warm_us / 1e6),
            "warm_roofline_frac": 12 * n / (warm_us / 1e6) / (HBM_PEAK_GBS * 1e9),
            "cold_update_us_median": cold_us, "cold_particles_per_s": n / (cold_us / 1e6),
            "recall": {"k": wl.k, "strict": float(np.isin(got, u[:wl.k]).mean()),
                       "tie_tolerant": float(np.isin(got, u[c >= kth]).mean())},
            "note": "warm: one HIP graph of 1000 updates, per update; cold: median of 20 updates, each after "
                    "writing 512 MiB"}


def host_threads():
    """Host threads this process may use, capped at the 16 that one GPU's share allows."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def recall(pos, wl, keys_top, est_top, csk, torch):
    """Top-k recall of the sketch against the exact histogram of the whole stream.  The
    exact counts come from torch.unique over the cell keys (csk_cell_keys, whose keys are
    checked bit-exactly against the oracle in the tests).  strict: shared keys with the
    exact top-k (ties at the k-th count broken by smaller key); tie_tolerant: returned keys
    whose exact count is at least the exact k-th count.  Also the median and largest
    relative error of the returned estimates against the exact counts."""
    k = wl.k
    keys = csk.cell_keys(pos, wl.delta, wl.L)
    uniq, counts = torch.unique(keys, sorted=True, return_counts=True)
    del keys
    ck = torch.topk(counts, k).values[-1]
    above = uniq[counts > ck]
    ties = uniq[counts == ck]
    exact = torch.cat([above, ties[: k - above.numel()]])
    f = counts[torch.searchsorted(uniq, keys_top)]
    rel = (est_top.to(torch.float64) - f.to(torch.float64)).abs() / f.to(torch.float64)
    out = {"k": k, "strict": torch.isin(keys_top, exact).sum().item() / k,
           "tie_tolerant": (f >= ck).sum().item() / k,
           "rel_err_median": rel.median().item(), "rel_err_max": rel.max().item(),
           "exact_kth_count": int(ck.item()), "distinct_cells": int(uniq.numel()),
           "exact": "torch.unique over csk_cell_keys of the whole stream"}
    del uniq, counts
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        log("bench.py measures one GPU only: multi-GPU runs are not part of this build")
        sys.exit(2)
    import torch
    import workloads
    import paper_1711_00975_amd as csk

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_copy": src.numel() * 4}), flush=True)
        return

    if args.large:
        torch.cuda.set_device(0)
        print(json.dumps(large_run(args, csk, torch, workloads)), flush=True)
        return

    wl = workloads.SCALE if args.workload == "scale" else workloads.SMALL
    n = args.n or wl.n
    torch.cuda.set_device(0)
    log(f"workload {wl.name}: n={n} d={wl.d} w={wl.w} k={wl.k}")
    pos = make_positions(wl, n, torch)
    s = csk.Sketch(wl.d, wl.w, wl.seed, max_candidates=1 << 22)
    stream = torch.cuda.current_stream()

    def step(theta, ev=None):
        s.reset()
        if ev is not None:
            ev[0].record(stream)
        s.update(pos, wl.delta, wl.L)
        if ev is not None:
            ev[1].record(stream)
        s.collect(pos, wl.delta, wl.L, theta)
        if ev is not None:
            ev[2].record(stream)
        keys, est, rc = s.topk(wl.k)
        return rc, keys, est

    # warm-up: first update allocates scratch; then find theta
    s.update(pos, wl.delta, wl.L)
    torch.cuda.synchronize()
    t_theta = time.perf_counter()
    theta, kth = calibrate_theta(s, pos, wl, csk)
    theta_ms = (time.perf_counter() - t_theta) * 1e3

    if args.oracle_full:
        log(f"oracle on all {n} particles, {host_threads()} threads for Add ...")
        print(json.dumps(oracle_full(pos, wl, host_threads(), s=s, theta=theta)), flush=True)
        return
    log(f"theta = {theta} (k-th estimate {kth}; search {theta_ms:.1f} ms)")
    for _ in range(args.warmup):
        step(theta)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    rcs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rc, keys_top, est_top = step(theta, evs[i])
        rcs.append(rc)
        log(f"  step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert all(rc == csk.CSK_OK for rc in rcs), "a timed step returned an incomplete top-k"
    ms = (t1 - t0) * 1e3 / args.steps
    upd_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    col_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    value = n / (ms / 1e3)
    achieved = BYTES_PER_PARTICLE * n / (upd_ms / 1e3) / 1e9
    out = {
        "metric": "particles/s sketched + top-10^4 recall; learned router vs plain at equal memory",
        "value_is": "particles per second of whole steps (update + candidate pass + top-10^4) on the scale "
                    "workload; recall is in `recall`, the router comparison in `learned_router`",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded Plummer halos + uniform background, generated on the host)",
        "config": {"workload": wl.name, "particles": n, "L": wl.L, "delta": wl.delta, "d": wl.d, "w": wl.w,
                   "k": wl.k, "seed": wl.seed, "theta": theta, "parallelism": "single GPU"},
        "theta_search": {"ms": theta_ms, "theta": theta,
                         "note": "untimed: halving from 2^22, one collect + top-k per try, on the counters of "
                                 "the warm-up update of the same stream, before the timed steps"},
        "update_ms": upd_ms,
        "update_particles_per_s": n / (upd_ms / 1e3),
        "collect_ms": col_ms,
        "roofline": {"kernel": "csk_sketch_update (sortbin_kernel + accumulate_kernel)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(n)},
    }
    if not args.no_ceilings:
        log("measured ceilings ...")
        out["ceilings"] = c = ceilings(pos, torch)
        out["roofline"]["frac_of_measured_stream_read"] = achieved / c["stream_read_GBs"]
    if not args.no_protocols:
        log("chunked update and the 2^28-particle w = 2^22 update ...")
        out["update_protocols"] = update_protocols(pos, wl, csk, torch)
    if not args.no_small:
        log("2^20-particle workload, warm and cold ...")
        out["small_workload"] = small_workload(csk, torch, workloads)
    if not args.no_packed:
        log("packed 8-byte stream ...")
        out["packed_input"] = packed_input(pos, wl, theta, keys_top, csk, torch, args.steps)
    if not args.no_dictionary:
        log("full-dictionary search ...")
        out["dictionary_search"] = dictionary_search(s, wl, theta, keys_top, torch)
    if not args.no_batch:
        log("batched sub-volumes ...")
        out["batched"] = batched_subvolumes(csk, torch)
    if not args.no_hierarchy:
        log("hierarchical search ...")
        out["hierarchical_search"] = hierarchical_search(s, pos, wl, theta, keys_top, csk, torch)
    if not args.no_recall:
        log("recall against the exact histogram ...")
        try:
            out["recall"] = recall(pos, wl, keys_top, est_top, csk, torch)
        except RuntimeError as e:   # e.g. not enough device memory for the exact histogram
            out["recall"] = {"error": str(e)[:200]}
    if not args.no_router:
        log("learned router vs plain sketch at equal memory ...")
        out["learned_router"] = learned_router(csk, torch, workloads, n=args.router_n)
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        log("cpu baseline (oracle, one thread) ...")
        out["cpu_baseline"] = cpu_baseline(pos, wl, sample, 1)
        nt = host_threads()
        if nt > 1:
            log(f"cpu baseline (oracle, {nt} threads for Add) ...")
            out["cpu_baseline_all_cores"] = cpu_baseline(pos, wl, sample, nt)
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
