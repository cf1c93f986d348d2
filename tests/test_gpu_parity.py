"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Counters, estimates, cell keys and the top-k are integer results of a fully
specified computation, so every comparison here is exact equality.
"""
import struct

import numpy as np
import pytest

import oracle
import workloads
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu

# (L, delta): exact G/L = 10 (binary64 path), G/L = 4, 2, 1 (binary32 path), and two
# meshes whose G/L is not exact (floor estimate + fma residual path)
MESHES = [(100.0, 0.1), (1000.0, 0.25), (3000.0, 0.25), (3000.0, 0.5), (3000.0, 1.0), (7.0, 0.7),
          (123.456, 0.123456)]


def torch():
    import torch as t
    return t


def dev(a):
    return torch().from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


def clustered(n, L, seed, frac=0.6, sigma=0.15, nclump=12):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (nclump, 3))
    clump = centres[rng.integers(0, nclump, n)] + rng.normal(0, sigma, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < frac)[:, None], clump, bg)
    return np.mod(pos, L).astype(np.float32)


def gpu_counters(pos, d, w, seed, delta, L, variant=0, chunks=1):
    s = csk.Sketch(d, w, seed, variant)
    t = dev(pos)
    bounds = np.linspace(0, len(pos), chunks + 1).astype(int)
    for a, b in zip(bounds[:-1], bounds[1:]):
        s.update(t[a:b], delta, L)
    return s, s.counters().cpu().numpy()


def f32_neighbours(x):
    b = struct.unpack("I", struct.pack("f", x))[0]
    out = [x]
    for db in (-1, 1):
        out.append(struct.unpack("f", struct.pack("I", (b + db) & 0xFFFFFFFF))[0])
    return out


# ------------------------------------------------------------------ cell keys

@pytest.mark.parametrize("L,delta", MESHES)
def test_cell_keys_match_oracle(L, delta):
    say("cell keys", L, delta)
    G = oracle.grid(delta, L)
    rng = np.random.default_rng(7)
    vals = list(rng.uniform(-2 * L, 2 * L, 30000))
    for j in rng.integers(-2 * G, 2 * G, 3000):
        vals += f32_neighbours(float(np.float32(j * L / G)))
    vals += [0.0, -0.0, L, -L, 2 * L, -2 * L, float("nan"), float("inf"), -float("inf"), 1e-45, -1e-45]
    v = np.array(vals, dtype=np.float32)
    n = len(v) - len(v) % 3
    pos = v[:n].reshape(-1, 3)
    pos = np.concatenate([pos, np.roll(pos, 1, axis=1), np.roll(pos, 2, axis=1)])
    keys = csk.cell_keys(dev(pos), delta, L).cpu().numpy().view(np.uint64)
    ok = np.all(np.isfinite(pos) & (np.abs(pos.astype(np.float64)) < 2 * L), axis=1)
    want = oracle.keys(pos[ok], delta, L)
    assert np.array_equal(keys[ok], want)
    assert np.all(keys[~ok] == np.uint64(0xFFFFFFFFFFFFFFFF))


@pytest.mark.parametrize("L,delta", [(100.0, 0.1), (1000.0, 0.25), (7.0, 0.7)])
def test_cell_keys_exhaustive_float_sweep(L, delta):
    # every float32 in [0, L], as all three coordinates at once, against the oracle's
    # exact-rational floor (one mesh per way the kernels compute the floor)
    from concurrent.futures import ThreadPoolExecutor
    G = oracle.grid(delta, L)
    top = struct.unpack("I", struct.pack("f", L))[0]
    batch = 1 << 25
    mism = 0
    with ThreadPoolExecutor(16) as ex:
        for lo in range(0, top + 1, batch):
            bits = np.arange(lo, min(top + 1, lo + batch), dtype=np.uint32)
            p = bits.view(np.float32)
            parts = np.array_split(p, 16)
            want = np.concatenate(list(ex.map(lambda a: oracle.cell_index_many(a, G, L), parts)))
            pos = np.repeat(p[:, None], 3, axis=1)
            keys = csk.cell_keys(dev(pos), delta, L).cpu().numpy().astype(np.int64)
            ix, rest = np.divmod(keys, G * G)
            iy, iz = np.divmod(rest, G)
            mism += int((ix != want).sum() + (iy != want).sum() + (iz != want).sum())
    say("swept", top + 1, "floats")
    assert mism == 0


# ------------------------------------------------------------------ counters

def test_counters_small_workload_full():
    wl = workloads.SMALL
    pos = wl.generate()
    say("small workload", wl.name)
    s, M = gpu_counters(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L)
    Mo, skipped = oracle.sketch(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, threads=8)
    assert skipped == 0
    assert np.array_equal(M, Mo)
    s.close()


CASES = [
    # n, d, w, L, delta, seed, variant
    (0, 5, 1 << 16, 100.0, 0.1, 1, 0),
    (1, 5, 1 << 16, 100.0, 0.1, 1, 0),
    (8191, 5, 1 << 16, 100.0, 0.1, 2, 0),
    (8193, 5, 1 << 16, 100.0, 0.1, 3, 0),
    (100_000, 1, 1, 100.0, 0.1, 4, 0),
    (100_000, 2, 3, 100.0, 0.1, 5, 0),
    (100_000, 4, 1000, 100.0, 0.1, 6, 0),
    (100_000, 5, 32768, 1000.0, 0.25, 7, 0),
    (100_000, 5, 32769, 1000.0, 0.25, 8, 0),
    (200_000, 5, 4154983, 1000.0, 0.25, 9, 0),
    (150_000, 8, 1 << 20, 3000.0, 0.25, 10, 0),
    (100_000, 9, 12345, 3000.0, 1.0, 11, 0),
    (60_000, 16, 1 << 14, 100.0, 0.1, 12, 0),
    (40_000, 32, 777, 100.0, 0.1, 13, 0),
    (70_000, 6, 50_000, 1000.0, 0.25, 16, 0),
    (70_000, 3, 1 << 18, 1000.0, 0.25, 17, 0),
    (90_000, 5, 1 << 16, 7.0, 0.7, 18, 0),
    (90_000, 5, 3333, 123.456, 0.123456, 19, 0),
    (100_000, 5, 1 << 16, 100.0, 0.1, 14, 1),
    (100_000, 7, 999, 3000.0, 0.5, 15, 1),
    # packed hash fields (w = 2^lw, lw + 1 <= floor(128 / d)) at each d's largest lw, and the
    # shift path one step beyond it
    (120_000, 5, 1 << 24, 1000.0, 0.25, 25, 0),
    (80_000, 6, 1 << 20, 1000.0, 0.25, 20, 0),
    (80_000, 6, 1 << 21, 1000.0, 0.25, 21, 0),
    (80_000, 7, 1 << 17, 100.0, 0.1, 22, 0),
    (80_000, 8, 1 << 15, 100.0, 0.1, 23, 1),
    (80_000, 8, 1 << 16, 100.0, 0.1, 24, 0),
]


@pytest.mark.parametrize("n,d,w,L,delta,seed,variant", CASES)
def test_counters_match_oracle(n, d, w, L, delta, seed, variant):
    say("counters", n, d, w, L, delta, seed, variant)
    pos = clustered(n, L, seed)
    s, M = gpu_counters(pos, d, w, seed, delta, L, variant)
    Mo, _ = oracle.sketch(pos, d, w, seed, delta, L, variant=variant, threads=8)
    assert np.array_equal(M, Mo)
    if variant == 1:
        assert np.all(M.astype(np.int64).sum(axis=1) == n)
    s.close()


def test_one_cell_stream_overflows_regions_and_stays_exact():
    # every particle in one cell: all tokens of a row land in one slice, far above
    # the region capacity, so the overflow path carries most of them
    n = 300_000
    pos = np.full((n, 3), 12.34, dtype=np.float32)
    s, M = gpu_counters(pos, 5, 1 << 16, 3, 0.1, 100.0)
    Mo, _ = oracle.sketch(pos, 5, 1 << 16, 3, 0.1, 100.0)
    assert np.array_equal(M, Mo)
    assert sorted(np.abs(M).max(axis=1).tolist()) == [n] * 5
    s.close()


def test_halo_ordered_stream():
    # stream sorted by cell (the opposite of the paper's unsorted assumption)
    pos = clustered(200_000, 100.0, 21, frac=0.9, sigma=0.05)
    keys = oracle.keys(pos, 0.1, 100.0)
    pos = pos[np.argsort(keys, kind="stable")]
    s, M = gpu_counters(pos, 5, 1 << 16, 5, 0.1, 100.0)
    Mo, _ = oracle.sketch(pos, 5, 1 << 16, 5, 0.1, 100.0, threads=8)
    assert np.array_equal(M, Mo)
    s.close()


def test_direct_path_for_very_wide_rows():
    # 2^28 counters in one row: more slices than the binned plan holds in LDS
    pos = clustered(50_000, 100.0, 31)
    s, M = gpu_counters(pos, 1, 1 << 28, 6, 0.1, 100.0)
    Mo, _ = oracle.sketch(pos, 1, 1 << 28, 6, 0.1, 100.0)
    assert np.array_equal(M, Mo)
    s.close()


def test_chunking_order_determinism_and_merge():
    pos = clustered(300_000, 1000.0, 41)
    d, w, seed, L, delta = 5, 1 << 20, 9, 1000.0, 0.25
    s1, M1 = gpu_counters(pos, d, w, seed, delta, L)
    s2, M2 = gpu_counters(pos, d, w, seed, delta, L, chunks=7)
    perm = np.random.default_rng(1).permutation(len(pos))
    s3, M3 = gpu_counters(pos[perm], d, w, seed, delta, L)
    s4, M4 = gpu_counters(pos, d, w, seed, delta, L)
    assert np.array_equal(M1, M2) and np.array_equal(M1, M3) and np.array_equal(M1, M4)
    # merge: sketch(A) + sketch(B) loaded with set_counters == sketch(A u B)
    sa, Ma = gpu_counters(pos[:100_000], d, w, seed, delta, L)
    sb, Mb = gpu_counters(pos[100_000:], d, w, seed, delta, L)
    merged = (Ma.view(np.uint32) + Mb.view(np.uint32)).view(np.int32)
    sm = csk.Sketch(d, w, seed)
    sm.set_counters(dev(merged))
    assert np.array_equal(sm.counters().cpu().numpy(), M1)
    # resume: checkpoint after part A, continue with part B on a fresh handle
    sr = csk.Sketch(d, w, seed)
    sr.set_counters(dev(Ma))
    sr.update(dev(pos[100_000:]), delta, L)
    assert np.array_equal(sr.counters().cpu().numpy(), M1)
    for s in (s1, s2, s3, s4, sa, sb, sm, sr):
        s.close()


def test_domain_errors_latch_and_skip():
    pos = clustered(50_000, 100.0, 51)
    pos[::101, 0] = np.nan
    pos[5::103, 1] = np.inf
    pos[7::107, 2] = 250.0
    s = csk.Sketch(5, 4096, 2)
    s.update(dev(pos), 0.1, 100.0)
    with pytest.raises(csk.CskError) as e:
        s.check()
    assert e.value.code == csk.CSK_E_DOMAIN
    s.check()   # latch cleared
    Mo, skipped = oracle.sketch(pos, 5, 4096, 2, 0.1, 100.0)
    assert skipped > 0
    assert np.array_equal(s.counters().cpu().numpy(), Mo)
    with pytest.raises(csk.CskError) as e:
        s.update(dev(pos), 0.2, 100.0)   # a different mesh on a latched handle
    assert e.value.code == csk.CSK_E_STATE
    s.reset()
    s.update(dev(pos[:10]), 0.2, 100.0)   # reset releases the mesh
    s.close()


def test_reset_gives_a_fresh_handle():
    # reset clears counters, latch, candidate set and its count in one launch: after it the
    # handle must behave exactly like a new one, for the update and for a filtered collect
    a = clustered(120_000, 100.0, 71)
    a[::997, 0] = np.nan                      # latches a domain error before the reset
    b = clustered(90_000, 100.0, 72)
    s = csk.Sketch(5, 1 << 14, 4, max_candidates=1 << 15)
    s.update(dev(a), 0.1, 100.0)
    s.collect(dev(a), 0.1, 100.0, 5)
    s.reset()
    assert not s.counters().cpu().numpy().any()
    s.check()                                 # the latch is clear
    kk, ee, rc = s.topk(10)                   # the set is empty and not partial
    assert kk.numel() == 0 and rc == csk.CSK_OK
    s.update(dev(b), 0.1, 100.0)
    M = oracle.sketch(b, 5, 1 << 14, 4, 0.1, 100.0)[0]
    assert np.array_equal(s.counters().cpu().numpy(), M)
    T = oracle.hash_tables(4, 5)
    keys = oracle.keys(b, 0.1, 100.0)
    for theta in (6, 40):                     # the filter and hot set are rebuilt per collect
        s.clear_candidates()
        s.collect(dev(b), 0.1, 100.0, theta)
        got_k, got_e, rc = s.topk(200)
        want_k, want_e = oracle.topk_keys(M, T, keys, theta, 200)
        assert got_k.cpu().numpy().view(np.uint64).tolist() == want_k.tolist()
        assert got_e.cpu().numpy().tolist() == want_e.tolist()
    s.close()


# ------------------------------------------------------------------ estimates, top-k

def test_query_matches_oracle():
    wl = workloads.SMALL
    pos = wl.generate()
    s, M = gpu_counters(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L)
    T = oracle.hash_tables(wl.seed, wl.d)
    uniq, f = oracle.histogram(oracle.keys(pos, wl.delta, wl.L))
    rnd = np.random.default_rng(3).integers(0, 2 ** 48, 100_000, dtype=np.uint64)
    keys = np.concatenate([uniq, rnd])
    est = s.query(dev(keys.view(np.int64))).cpu().numpy()
    assert np.array_equal(est, oracle.estimate(M, T, keys))
    s.close()


@pytest.mark.parametrize("d", [2, 5, 9])
def test_query_even_and_global_table_rows(d):
    pos = clustered(80_000, 100.0, 61 + d)
    s, M = gpu_counters(pos, d, 3000, 17, 0.1, 100.0)
    uniq, _ = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    est = s.query(dev(uniq.view(np.int64))).cpu().numpy()
    assert np.array_equal(est, oracle.estimate(M, oracle.hash_tables(17, d), uniq))
    s.close()


def topk_case(pos, d, w, seed, delta, L, k, theta, variant=0):
    s, M = gpu_counters(pos, d, w, seed, delta, L, variant)
    s.collect(dev(pos), delta, L, theta)
    keys, est, rc = s.topk(k)
    T = oracle.hash_tables(seed, d)
    Mo, _ = oracle.sketch(pos, d, w, seed, delta, L, variant=variant, threads=8)   # the oracle's own counters
    assert np.array_equal(M, Mo)
    ko, eo, st = oracle.topk_sketch(Mo, T, pos, delta, L, theta, k, variant)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
    assert np.array_equal(est.cpu().numpy(), eo)
    assert rc == (csk.CSK_W_INCOMPLETE if st == oracle.W_INCOMPLETE else csk.CSK_OK)
    s.close()
    return ko, eo


def test_topk_small_workload_all_cells():
    wl = workloads.SMALL
    pos = wl.generate()
    say("topk small, theta = INT32_MIN")
    ko, eo = topk_case(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, wl.k, oracle.INT32_MIN)
    assert len(ko) == wl.k


def test_topk_theta_invariance_and_incomplete():
    wl = workloads.SMALL
    pos = wl.generate()
    ko, eo = topk_case(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, wl.k, oracle.INT32_MIN)
    kth = int(eo[-1])
    for theta in (kth, kth - 3):
        k2, e2 = topk_case(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, wl.k, theta)
        assert np.array_equal(k2, ko) and np.array_equal(e2, eo)
    topk_case(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, wl.k, int(eo[0]))   # incomplete


@pytest.mark.parametrize("k", [1, 37, 1000, 5000])
def test_topk_ties_and_sizes(k):
    rng = np.random.default_rng(k)
    cells = rng.uniform(0, 100, (3000, 3))
    counts = rng.integers(1, 5, 3000)
    pos = np.repeat(cells, counts, axis=0).astype(np.float32)
    pos = pos[rng.permutation(len(pos))]
    topk_case(pos, 5, 1 << 16, 8, 0.1, 100.0, k, oracle.INT32_MIN)
    topk_case(pos, 4, 1 << 12, 8, 0.1, 100.0, k, 2)
    topk_case(pos, 3, 97, 8, 0.1, 100.0, k, oracle.INT32_MIN, variant=1)


@pytest.mark.parametrize("d,w,theta,variant", [(8, 4096, 3, 0), (9, 4096, 3, 0), (6, 2000, 4, 0),
                                               (3, 1000, 20, 1), (5, 1 << 12, 1, 0), (5, 1 << 16, 3, 0),
                                               (6, 1 << 14, 3, 0), (7, 1 << 10, 3, 1)])
def test_topk_filtered_collect(d, w, theta, variant):
    # theta > 0 puts a Bloom filter of hot (row, bucket, sign) items in front of the
    # exact test (d <= 8); theta = 1 makes the filter too dense, so it is skipped
    pos = clustered(120_000, 100.0, 80 + d, frac=0.7, sigma=0.05)
    topk_case(pos, d, w, 23, 0.1, 100.0, 500, theta, variant)


def test_topk_empty_and_k_above_candidates():
    s = csk.Sketch(5, 1024, 1)
    s.collect(dev(np.zeros((0, 3), np.float32)), 0.1, 100.0, oracle.INT32_MIN)
    keys, est, rc = s.topk(10)
    assert len(keys) == 0 and rc == csk.CSK_OK
    pos = clustered(500, 100.0, 3)
    topk_case(pos, 5, 1024, 1, 0.1, 100.0, 100_000, oracle.INT32_MIN)
    s.close()


def test_candidate_capacity_error():
    pos = clustered(50_000, 100.0, 71, frac=0.0)
    s = csk.Sketch(5, 1 << 16, 1, max_candidates=1000)
    s.update(dev(pos), 0.1, 100.0)
    s.collect(dev(pos), 0.1, 100.0, oracle.INT32_MIN)
    with pytest.raises(csk.CskError) as e:
        s.topk(10)
    assert e.value.code == csk.CSK_E_CAPACITY
    s.clear_candidates()
    s.collect(dev(pos[:500]), 0.1, 100.0, oracle.INT32_MIN)
    keys, est, rc = s.topk(10)
    assert len(keys) == 10
    s.close()


def test_candidate_set_far_over_capacity_stays_fast():
    # Regression: a set asked to take ~2000x its capacity (4 million distinct cells into
    # 2048 slots) stops inserting at max_candidates and bounds every probe run, so the pass
    # ends in well under a second and reports CSK_E_CAPACITY; the full dictionary of 10^9
    # cells into a small set does the same.
    import time
    pos = clustered(1 << 22, 100.0, 72, frac=0.0)
    s = csk.Sketch(5, 1 << 12, 2, max_candidates=1000)
    s.update(dev(pos), 0.1, 100.0)
    t0 = time.time()
    s.collect(dev(pos), 0.1, 100.0, oracle.INT32_MIN)
    with pytest.raises(csk.CskError) as e:
        s.topk(10)
    assert e.value.code == csk.CSK_E_CAPACITY
    s.clear_candidates()
    s.collect_dictionary(0.1, 100.0, oracle.INT32_MIN)
    with pytest.raises(csk.CskError) as e:
        s.topk(10)
    assert e.value.code == csk.CSK_E_CAPACITY
    assert time.time() - t0 < 30.0
    s.close()


@pytest.mark.parametrize("d,w,G,theta,variant", [
    (5, 1 << 12, 20, oracle.INT32_MIN, 0),   # every key of the dictionary is a candidate
    (5, 1 << 16, 40, 3, 0),                  # Bloom filter + exact hot set, packed hash fields
    (3, 1000, 30, 2, 1),                     # Count-Min, multiply-high buckets
    (8, 1 << 12, 25, 2, 0),                  # packed fields at d = 8
    (6, 50000, 30, 4, 0),                    # multiply-high buckets with the filter
    (9, 4096, 16, 1, 0),                     # d > 8: tables read from global memory
    (5, 1 << 12, 24, 1 << 20, 0),            # nothing passes: empty result, incomplete
])
def test_dictionary_topk_matches_oracle(d, w, G, theta, variant):
    # Count Sketch with Full Search (Sec. 2.2 item 1; Alg. 1): every key of the G^3 mesh
    delta = 0.5
    L = G * delta
    say("dictionary", d, w, G, theta, variant)
    pos = clustered(60_000, L, 100 + d, frac=0.7, sigma=0.3)
    seed = 31 + d
    s, M = gpu_counters(pos, d, w, seed, delta, L, variant)
    Mo, _ = oracle.sketch(pos, d, w, seed, delta, L, variant=variant, threads=8)
    assert np.array_equal(M, Mo)
    k = 300
    s.clear_candidates()
    s.collect_dictionary(delta, L, theta)
    keys, est, rc = s.topk(k)
    ko, eo, st = oracle.topk_dictionary(Mo, oracle.hash_tables(seed, d), G, theta, k, variant)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
    assert np.array_equal(est.cpu().numpy(), eo)
    assert rc == (csk.CSK_W_INCOMPLETE if st == oracle.W_INCOMPLETE else csk.CSK_OK)
    s.close()


def test_dictionary_capacity_and_mesh_latch():
    # More dictionary keys than max_candidates with theta = INT32_MIN latches the capacity
    # error; a mesh other than the latched one is refused.
    s = csk.Sketch(5, 1 << 12, 3, max_candidates=1000)
    s.collect_dictionary(0.5, 10.0, oracle.INT32_MIN)    # 20^3 = 8000 keys
    with pytest.raises(csk.CskError) as e:
        s.topk(10)
    assert e.value.code == csk.CSK_E_CAPACITY
    with pytest.raises(csk.CskError) as e:
        s.collect_dictionary(0.25, 10.0, 0)
    assert e.value.code == csk.CSK_E_STATE
    s.close()


@pytest.mark.parametrize("d,w,R,L,delta", [
    (5, 1 << 12, 7, 100.0, 0.1),          # exact-ratio mesh, packed hash fields
    (5, 1 << 12, 1000, 1000.0, 0.25),     # power-of-two ratio mesh; the paper's group of 1000
    (3, 999, 1 << 20, 123.456, 0.123456), # general mesh, multiply-high buckets
    (9, 4096, 64, 100.0, 0.1),            # d > 8: global-table bin kernel
    (5, 1 << 12, 1, 100.0, 0.1),          # group 1 is the plain sketch
])
def test_grouped_counters_match_oracle(d, w, R, L, delta):
    # The coarse layer of the hierarchy adds key // R (Sec. 2.2 item 3; Alg. 3 Add(M1, s / 1000))
    say("grouped counters", d, w, R, L, delta)
    pos = clustered(150_000, L, 60 + d)
    s = csk.Sketch(d, w, 5, group=R)
    s.update(dev(pos), delta, L)
    Mo = oracle.super_sketch(pos, d, w, 5, delta, L, R)
    assert np.array_equal(s.counters().cpu().numpy(), Mo)
    # the stream candidate pass on super-items: distinct key // R with estimate >= theta
    theta = 40
    s.collect(dev(pos), delta, L, theta)
    keys, est, rc = s.topk(200)
    T = oracle.hash_tables(5, d)
    sup = np.unique(oracle.keys(pos, delta, L) // np.uint64(R))
    e = oracle.estimate(Mo, T, sup)
    want = sorted((-int(x), int(k)) for k, x in zip(sup, e) if x >= theta)[:200]
    assert keys.cpu().numpy().view(np.uint64).tolist() == [k for _, k in want]
    assert est.cpu().numpy().tolist() == [-x for x, _ in want]
    s.close()


@pytest.mark.parametrize("R,theta1,theta2,k", [
    (1000, 30, 5, 300),                   # the paper's group size
    (64, 10, oracle.INT32_MIN, 200),      # every child of the heavy super-items
    (7, oracle.INT32_MIN, 3, 150),        # every super-item: the full dictionary search
    (500, 1 << 20, 0, 50),                # no heavy super-item: empty, incomplete
])
def test_hierarchical_topk_matches_oracle(R, theta1, theta2, k):
    # Count Sketch Hierarchical (Sec. 2.2 item 3; Alg. 3): heavy super-items from the coarse
    # sketch, then their children from the fine sketch
    delta, L, G = 0.5, 15.0, 30
    say("hierarchical", R, theta1, theta2, k)
    pos = clustered(80_000, L, 77, frac=0.7, sigma=0.3)
    coarse = csk.Sketch(5, 1 << 12, 21, group=R)
    fine = csk.Sketch(5, 1 << 14, 22)
    for s in (coarse, fine):
        s.update(dev(pos), delta, L)
    coarse.collect_dictionary(delta, L, theta1)
    fine.collect_children(coarse, theta2)
    keys, est, rc = fine.topk(k)
    M1 = oracle.super_sketch(pos, 5, 1 << 12, 21, delta, L, R)
    M2, _ = oracle.sketch(pos, 5, 1 << 14, 22, delta, L, threads=8)
    assert np.array_equal(coarse.counters().cpu().numpy(), M1)
    assert np.array_equal(fine.counters().cpu().numpy(), M2)
    ko, eo, st = oracle.topk_hierarchical(M1, oracle.hash_tables(21, 5), M2, oracle.hash_tables(22, 5), G, R,
                                          theta1, theta2, k)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
    assert np.array_equal(est.cpu().numpy(), eo)
    assert rc == (csk.CSK_W_INCOMPLETE if st == oracle.W_INCOMPLETE else csk.CSK_OK)
    coarse.close()
    fine.close()


def test_hierarchical_argument_and_state_errors():
    coarse = csk.Sketch(5, 1 << 10, 1, group=10)
    fine = csk.Sketch(5, 1 << 10, 2)
    with pytest.raises(csk.CskError) as e:      # no mesh latched yet
        fine.collect_children(coarse, 0)
    assert e.value.code == csk.CSK_E_STATE
    pos = dev(clustered(1000, 10.0, 3))
    coarse.update(pos, 0.5, 10.0)
    fine.update(pos, 0.25, 10.0)
    with pytest.raises(csk.CskError) as e:      # different meshes
        fine.collect_children(coarse, 0)
    assert e.value.code == csk.CSK_E_STATE
    with pytest.raises(csk.CskError) as e:      # the fine layer must count cells (group 1)
        coarse.collect_children(fine, 0)
    assert e.value.code == csk.CSK_E_INVALID
    coarse.close()
    fine.close()


BATCH_SHAPES = [   # (n first call, n second call, w, seed): empty, tiny, ragged, uneven widths
    (0, 10, 1 << 14, 41), (1, 0, 1 << 14, 42), (8193, 100, 1 << 16, 43), (70_000, 5000, 1 << 15, 44),
    (300_000, 20_000, 1 << 18, 45), (120_000, 120_000, 1 << 20, 46), (9_000, 1, 1 << 16, 47),
]


def batch_case(shapes, L=100.0, delta=0.1):
    sk, pos1, pos2 = [], [], []
    for j, (n1, n2, w, seed) in enumerate(shapes):
        sk.append(csk.Sketch(5, w, seed))
        pos1.append(clustered(n1, L, 200 + j))
        pos2.append(clustered(n2, L, 300 + j))
    return sk, pos1, pos2


def test_batch_update_matches_oracle_per_sketch():
    # one bin and one accumulate launch for uneven sketches give each sketch exactly the
    # counters of its own stream (Sec. 2.2 Add); a second, smaller call adds on top
    say("batch update", len(BATCH_SHAPES))
    sk, pos1, pos2 = batch_case(BATCH_SHAPES)
    max_n = [max(a, b) for a, b, _, _ in BATCH_SHAPES]
    b = csk.Batch(sk, max_n, 0.1, 100.0, wg_budget=64)
    b.update([dev(p) for p in pos1])
    b.update([dev(p) for p in pos2])
    for j, (n1, n2, w, seed) in enumerate(BATCH_SHAPES):
        Mo, _ = oracle.sketch(np.concatenate([pos1[j], pos2[j]]), 5, w, seed, 0.1, 100.0, threads=8)
        assert np.array_equal(sk[j].counters().cpu().numpy(), Mo), j
    with pytest.raises(csk.CskError):                      # above max_n
        b.update([dev(clustered(n + 1, 100.0, 9)) for n in max_n])
    b.close()
    for s in sk:
        s.close()


def test_batch_topk_matches_oracle_and_replays_in_a_graph():
    # the top-k of all sketches of a batch in one set of launches equals the oracle's top-k
    # of each (counts, incomplete flags, keys, estimates), for uneven k (0 included) and
    # thresholds, eagerly and from three replays of a captured graph
    import torch
    say("batch top-k", len(BATCH_SHAPES))
    sk, pos1, _ = batch_case(BATCH_SHAPES)
    pos = [dev(p) for p in pos1]
    b = csk.Batch(sk, [max(1, p.shape[0]) for p in pos1], 0.1, 100.0)
    ks = [7, 0, 64, 300, 1000, 2500, 1]
    thetas = [3, 2, oracle.INT32_MIN, 4, 3, oracle.INT32_MIN, 2]
    keys = [torch.empty(max(k, 1), dtype=torch.int64, device="cuda") for k in ks]
    est = [torch.empty(max(k, 1), dtype=torch.int32, device="cuda") for k in ks]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in ks]

    def pipeline():
        b.update(pos)
        for j, s in enumerate(sk):
            s.clear_candidates()
            s.collect(pos[j], 0.1, 100.0, thetas[j])
        b.topk(ks, keys, est, outs)

    for s in sk:
        s.reset()
    pipeline()
    torch.cuda.synchronize()
    want = []
    for j, (n1, _, w, seed) in enumerate(BATCH_SHAPES):
        Mo, _ = oracle.sketch(pos1[j], 5, w, seed, 0.1, 100.0, threads=8)
        ko, eo, st = oracle.topk_sketch(Mo, oracle.hash_tables(seed, 5), pos1[j], 0.1, 100.0, thetas[j], ks[j])
        o = outs[j].cpu().numpy()
        got = int(o[0])
        assert got == len(ko), (j, got, len(ko))
        assert o[1] == (1 if (st == oracle.W_INCOMPLETE and ks[j] > 0) else 0), (j, o, st)
        assert np.array_equal(keys[j].cpu().numpy()[:got].view(np.uint64), ko), j
        assert np.array_equal(est[j].cpu().numpy()[:got], eo), j
        want.append((o.copy(), keys[j].cpu().numpy()[:got].copy(), est[j].cpu().numpy()[:got].copy()))
    for s in sk:
        s.reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipeline()
    for rep in range(3):
        for s in sk:
            s.reset()
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (o, kk, e) in enumerate(want):
            got = int(o[0])
            assert np.array_equal(outs[j].cpu().numpy(), o), (rep, j)
            assert np.array_equal(keys[j].cpu().numpy()[:got], kk), (rep, j)
            assert np.array_equal(est[j].cpu().numpy()[:got], e), (rep, j)
    del g
    b.close()
    for s in sk:
        s.close()


def test_batch_create_rejects_mixed_sketches():
    a, c = csk.Sketch(5, 1 << 14, 1), csk.Sketch(4, 1 << 14, 2)
    with pytest.raises(csk.CskError) as e:
        csk.Batch([a, c], [10, 10], 0.1, 100.0)
    assert e.value.code == csk.CSK_E_INVALID
    with pytest.raises(csk.CskError) as e:
        csk.Batch([a, a], [10, 10], 0.1, 100.0)
    assert e.value.code == csk.CSK_E_INVALID
    a.close()
    c.close()


def test_batch_pipeline_in_a_hip_graph():
    # batched update -> per-sketch collect -> asynchronous top-k, captured once and
    # replayed: every replay equals the eager pipeline and the oracle (zero-filled work
    # between replays, eager launches and synchronizations in between)
    import torch
    shapes = BATCH_SHAPES[2:6]
    sk, pos1, _ = batch_case(shapes)
    pos = [dev(p) for p in pos1]
    b = csk.Batch(sk, [p.shape[0] for p in pos1], 0.1, 100.0)
    k, theta = 64, 3
    keys = [torch.empty(k, dtype=torch.int64, device="cuda") for _ in sk]
    est = [torch.empty(k, dtype=torch.int32, device="cuda") for _ in sk]
    outs = [torch.zeros(2, dtype=torch.int32, device="cuda") for _ in sk]

    def pipeline():
        b.update(pos)
        for j, s in enumerate(sk):
            s.clear_candidates()
            s.collect(pos[j], 0.1, 100.0, theta)
            s.topk_async(k, keys[j], est[j], outs[j])

    def reset_all():
        for s in sk:
            s.reset()

    reset_all()
    pipeline()                                    # eager run (also sizes the top-k scratch)
    torch.cuda.synchronize()
    want = [(o.cpu().numpy().copy(), kk.cpu().numpy().copy(), e.cpu().numpy().copy())
            for o, kk, e in zip(outs, keys, est)]
    for j, (n1, _, w, seed) in enumerate(shapes):
        Mo, _ = oracle.sketch(pos1[j], 5, w, seed, 0.1, 100.0, threads=8)
        ko, eo, st = oracle.topk_sketch(Mo, oracle.hash_tables(seed, 5), pos1[j], 0.1, 100.0, theta, k)
        got = int(want[j][0][0])
        assert got == len(ko) and want[j][0][1] == (1 if st == oracle.W_INCOMPLETE else 0)
        assert np.array_equal(want[j][1][:got].view(np.uint64), ko) and np.array_equal(want[j][2][:got], eo)
    reset_all()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipeline()
    for rep in range(3):
        reset_all()                               # eager work between replays
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (o, kk, e) in enumerate(zip(outs, keys, est)):
            got = int(want[j][0][0])
            assert np.array_equal(o.cpu().numpy(), want[j][0]), (rep, j)
            assert np.array_equal(kk.cpu().numpy()[:got], want[j][1][:got]), (rep, j)
            assert np.array_equal(e.cpu().numpy()[:got], want[j][2][:got]), (rep, j)
    del g
    b.close()
    for s in sk:
        s.close()


# ------------------------------------------------------------------ headline configuration

def test_headline_config_prefix_update_collect_topk():
    # The 2^30-particle configuration (L = 1000, delta = 0.25, 4000^3 cells, d = 5, w = 2^24,
    # k = 10^4) on the first 2^24 particles of its own stream: one update call of 2048 tiles of
    # 8192 particles over 256 bin workgroups (8 tiles each), then the candidate pass through
    # the Bloom filter and the exact hot-item set (w = 2^24: 24-bit buckets in the packed
    # fields) and the top-10^4, each against the oracle (Sec. 2.2 Add, Estimate, UpdateHeap;
    # Sec. 3.1 item 4).  theta is the oracle's own 10^4-th estimate, so the result is complete;
    # theta = 1024 leaves about a thousand candidates: an incomplete result.
    wl = workloads.SCALE
    n = 1 << 24
    say("headline prefix", wl.name, n)
    pos = wl.generate(0, n)
    s, M = gpu_counters(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L)
    Mo, skipped = oracle.sketch(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L, threads=16)
    assert skipped == 0
    assert np.array_equal(M, Mo)
    T = oracle.hash_tables(wl.seed, wl.d)
    uniq, _ = oracle.histogram(oracle.keys(pos, wl.delta, wl.L))
    est_all = oracle.estimate(Mo, T, uniq)
    kth = int(np.sort(est_all)[::-1][wl.k - 1])
    hot = int((np.abs(Mo.astype(np.int64)) >= kth).sum())
    say("10^4-th estimate", kth, "rows x buckets at or above it", hot)
    assert 1 <= kth and hot <= 131072          # the filter and the hot-item set are both in use
    t = dev(pos)
    for theta, complete in ((kth, True), (1024, False)):
        s.clear_candidates()
        s.collect(t, wl.delta, wl.L, theta)
        keys, est, rc = s.topk(wl.k)
        ko, eo, st = oracle.topk_sketch(Mo, T, pos, wl.delta, wl.L, theta, wl.k)
        say("theta", theta, "returned", len(ko))
        assert (st == oracle.OK) == complete and (len(ko) == wl.k) == complete
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
        assert np.array_equal(est.cpu().numpy(), eo)
        assert rc == (csk.CSK_OK if complete else csk.CSK_W_INCOMPLETE)
    s.close()
