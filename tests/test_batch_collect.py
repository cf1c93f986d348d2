"""The batched candidate pass and reset (csk_batch_collect, csk_batch_reset) against the
oracle, sketch by sketch: a batch must give every sketch exactly what csk_collect and
csk_reset give it alone (Sec. 3.1 item 4 per sketch; Sec. 2.2 UpdateHeap for the top-k),
in eager calls, in a HIP graph replayed several times, and on a 64-sub-volume batch of
the batched configuration's shape with every stream cut down."""
import numpy as np
import pytest

import oracle
import workloads
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu

INT32_MIN = csk.INT32_MIN


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _clustered(n, L, seed, frac=0.6, sigma=0.15, nclump=12):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (nclump, 3))
    clump = centres[rng.integers(0, nclump, n)] + rng.normal(0, sigma, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < frac)[:, None], clump, bg)
    return np.mod(pos, L).astype(np.float32)


# (n, w, seed, theta): an empty stream, one particle, ragged tails, every width class of
# the batched configuration, no threshold, thresholds that leave few or no candidates
SHAPES = [(0, 1 << 14, 71, 4), (1, 1 << 14, 72, INT32_MIN), (8193, 1 << 16, 73, 2),
          (70_000, 1 << 15, 74, 6), (300_000, 1 << 18, 75, 12), (250_000, 1 << 20, 76, 1 << 20),
          (9_000, 1 << 16, 77, INT32_MIN), (120_000, 1 << 17, 78, 25)]


def _oracle_topk(pos, w, seed, theta, k):
    Mo, _ = oracle.sketch(pos, 5, w, seed, 0.1, 100.0, threads=8)
    return oracle.topk_sketch(Mo, oracle.hash_tables(seed, 5), pos, 0.1, 100.0, theta, k)


def _check(keys, est, out, ko, eo, st, tag):
    got = int(out[0])
    assert got == len(ko), (tag, got, len(ko))
    assert int(out[1]) == (1 if st == oracle.W_INCOMPLETE else 0), tag
    assert np.array_equal(keys[:got].view(np.uint64), ko), tag
    assert np.array_equal(est[:got], eo), tag


def test_batch_collect_and_reset_match_oracle():
    import torch
    print("batch collect", len(SHAPES), flush=True)
    sk = [csk.Sketch(5, w, seed) for _, w, seed, _ in SHAPES]
    host = [_clustered(n, 100.0, 400 + j) for j, (n, _, _, _) in enumerate(SHAPES)]
    pos = [_dev(p) for p in host]
    b = csk.Batch(sk, [max(1, p.shape[0]) for p in host], 0.1, 100.0)
    ks = [50] * len(sk)
    keys = [torch.empty(k, dtype=torch.int64, device="cuda") for k in ks]
    est = [torch.empty(k, dtype=torch.int32, device="cuda") for k in ks]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in ks]
    thetas = [t for _, _, _, t in SHAPES]
    try:
        # dirty every handle first: the batched reset must clear counters and candidate sets
        junk = _dev(_clustered(5000, 100.0, 9))
        for s in sk:
            s.update(junk, 0.1, 100.0)
            s.collect(junk, 0.1, 100.0, INT32_MIN)
        b.reset()
        b.update(pos)
        b.collect(pos, thetas)
        b.topk(ks, keys, est, outs)
        torch.cuda.synchronize()
        for j, (n, w, seed, theta) in enumerate(SHAPES):
            ko, eo, st = _oracle_topk(host[j], w, seed, theta, ks[j])
            _check(keys[j].cpu().numpy(), est[j].cpu().numpy(), outs[j].cpu().numpy(), ko, eo, st, (j, n, w, theta))
            Mo, _ = oracle.sketch(host[j], 5, w, seed, 0.1, 100.0, threads=8)
            assert np.array_equal(sk[j].counters().cpu().numpy(), Mo), j
    finally:
        b.close()
        for s in sk:
            s.close()


def test_batch_pipeline_with_batched_collect_in_a_hip_graph():
    # reset -> update -> collect -> top-k of the whole batch captured once and replayed
    # three times, with eager work and synchronizations between the replays
    import torch
    print("batch graph", flush=True)
    shapes = SHAPES[2:]
    sk = [csk.Sketch(5, w, seed) for _, w, seed, _ in shapes]
    host = [_clustered(n, 100.0, 500 + j) for j, (n, _, _, _) in enumerate(shapes)]
    pos = [_dev(p) for p in host]
    b = csk.Batch(sk, [p.shape[0] for p in host], 0.1, 100.0)
    ks = [40] * len(sk)
    thetas = [t for _, _, _, t in shapes]
    keys = [torch.empty(k, dtype=torch.int64, device="cuda") for k in ks]
    est = [torch.empty(k, dtype=torch.int32, device="cuda") for k in ks]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in ks]

    def pipeline():
        b.reset()
        b.update(pos)
        b.collect(pos, thetas)
        b.topk(ks, keys, est, outs)

    try:
        pipeline()        # eager (also sizes the selection scratch)
        torch.cuda.synchronize()
        want = []
        for j, (n, w, seed, theta) in enumerate(shapes):
            ko, eo, st = _oracle_topk(host[j], w, seed, theta, ks[j])
            _check(keys[j].cpu().numpy(), est[j].cpu().numpy(), outs[j].cpu().numpy(), ko, eo, st, ("eager", j))
            want.append((ko, eo, st))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pipeline()
        for rep in range(3):
            for s in sk:          # eager work between replays
                s.update(pos[0], 0.1, 100.0)
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for j in range(len(shapes)):
                ko, eo, st = want[j]
                _check(keys[j].cpu().numpy(), est[j].cpu().numpy(), outs[j].cpu().numpy(), ko, eo, st, (rep, j))
        del g
    finally:
        b.close()
        for s in sk:
            s.close()


def test_batch_of_64_subvolumes_scaled_down():
    # the batched configuration's 64 sub-volumes (widths 2^14..2^20, k = 1 % of w, Plummer
    # halos in L = 100 at delta = 0.1) with every stream cut to 1/64 of its size
    import torch
    subs = workloads.batch_subvolumes()
    print("64 sub-volumes", flush=True)
    host = []
    for wl in subs:
        n = max(1000, wl.n // 64)
        host.append(np.ascontiguousarray(wl.with_(n=n, n_halo=max(1, wl.n_halo // 64)).generate(threads=8)[:n]))
    sk = [csk.Sketch(wl.d, wl.w, wl.seed) for wl in subs]
    pos = [_dev(p) for p in host]
    ks = [wl.k for wl in subs]
    thetas = [2 if j % 2 else INT32_MIN for j in range(len(subs))]
    keys = [torch.empty(k, dtype=torch.int64, device="cuda") for k in ks]
    est = [torch.empty(k, dtype=torch.int32, device="cuda") for k in ks]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in ks]
    b = csk.Batch(sk, [p.shape[0] for p in host], 0.1, 100.0)
    try:
        b.reset()
        b.update(pos)
        b.collect(pos, thetas)
        b.topk(ks, keys, est, outs)
        torch.cuda.synchronize()
        for j, wl in enumerate(subs):
            Mo, _ = oracle.sketch(host[j], wl.d, wl.w, wl.seed, wl.delta, wl.L, threads=8)
            assert np.array_equal(sk[j].counters().cpu().numpy(), Mo), j
            ko, eo, st = oracle.topk_sketch(Mo, oracle.hash_tables(wl.seed, wl.d), host[j], wl.delta, wl.L,
                                            thetas[j], ks[j])
            _check(keys[j].cpu().numpy(), est[j].cpu().numpy(), outs[j].cpu().numpy(), ko, eo, st, j)
    finally:
        b.close()
        for s in sk:
            s.close()
