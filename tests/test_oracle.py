"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer values, exact rational arithmetic, hand-derived fixtures, brute
force on tiny inputs, closed forms and invariants of the Count Sketch (Sec. 2.2),
chosen so that a dropped term, a wrong sign or index, or a transposed operand in
the oracle fails at least one of them.
"""
import json
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CONFIG_MESHES = [(100.0, 0.1), (1000.0, 0.25), (3000.0, 0.25), (3000.0, 0.5), (3000.0, 1.0)]


def f32_below(x):
    b = struct.unpack("I", struct.pack("f", x))[0]
    return struct.unpack("f", struct.pack("I", b - 1))[0]


def exact_index(p: float, G: int, L: float) -> int:
    """floor(p*G/L) on exact rationals, wrapped — with Python's Fraction."""
    q = Fraction(p) * G / Fraction(L)
    return math.floor(q) % G


# ------------------------------------------------------------------ SplitMix64

def test_splitmix64_known_answers():
    # Published reference outputs of SplitMix64 (Steele, Lea & Flood 2014).
    assert [int(x) for x in oracle.splitmix64(0, 3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(x) for x in oracle.splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_hash_tables_layout_follows_generator_stream():
    seed, d = 12345, 5
    T = oracle.hash_tables(seed, d).ravel()
    z = oracle.splitmix64(seed, T.size // 2)
    assert np.array_equal(T[0::2], (z & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    assert np.array_equal(T[1::2], (z >> np.uint64(32)).astype(np.uint32))


def test_hash_tables_prefix_rows_do_not_depend_on_d():
    assert np.array_equal(oracle.hash_tables(7, 3), oracle.hash_tables(7, 5)[:3])


# ------------------------------------------------------------------ mesh (O1)

def test_grid_valid_and_invalid():
    assert oracle.grid(0.1, 100.0) == 1000
    assert oracle.grid(0.25, 1000.0) == 4000
    assert oracle.grid(0.25, 3000.0) == 12000
    assert oracle.grid(0.1, 500.0) == 5000          # the paper's Millennium mesh, Sec. 4.1
    for bad in [(0.0, 100.0), (-0.1, 100.0), (0.3, 100.0), (0.001, 100.0), (float("nan"), 1.0),
                (1.0, float("inf")), (1e-3, 1000.0)]:
        with pytest.raises(ValueError):
            oracle.grid(*bad)


# ------------------------------------------------------------ cell index (O2)

def test_cell_index_golden_fixture():
    doc = json.load(open(os.path.join(GOLDEN, "cell_keys.json")))
    for c in doc["cell_index"]:
        p = float.fromhex(c["p_hex"]) if "0x" in c["p_hex"] else float(c["p_hex"])
        G = oracle.grid(c["delta"], c["L"])
        got = oracle.cell_index(p, G, c["L"])
        want = -1 if c["expected"] is None else c["expected"]
        assert got == want, c


def test_cell_key_golden_fixture():
    doc = json.load(open(os.path.join(GOLDEN, "cell_keys.json")))
    for c in doc["cell_key"]:
        xyz = np.array([[float.fromhex(h) for h in c["xyz_hex"]]], dtype=np.float32)
        assert int(oracle.keys(xyz, c["delta"], c["L"])[0]) == c["expected_key"], c


@pytest.mark.parametrize("L,delta", CONFIG_MESHES)
def test_cell_index_matches_exact_rationals(L, delta):
    G = oracle.grid(delta, L)
    rng = np.random.default_rng(1)
    ps = list(rng.uniform(-L, 2 * L, 3000).astype(np.float32))
    # floats adjacent to cell boundaries j * L / G
    for j in rng.integers(0, 2 * G, 600):
        b = np.float32(j * L / G)
        ps += [b, np.nextafter(b, np.float32(np.inf)), np.nextafter(b, np.float32(-np.inf))]
    ps += [np.float32(0.0), np.float32(-0.0), np.float32(L), np.float32(1e-38), np.float32(-1e-45)]
    got = oracle.cell_index_many(np.array(ps, dtype=np.float32), G, L)
    for p, g in zip(ps, got):
        want = exact_index(float(p), G, L) if abs(float(p)) < 2 * L else -1
        assert g == want, (float(p), g, want)


def test_cell_index_nests_across_resolutions():
    # floor(floor(p G / L) / m) = floor(p (G/m) / L) for an integer m dividing G:
    # the 0.25 -> 0.5 -> 1.0 Mpc/h meshes of one box nest exactly.
    L = 3000.0
    rng = np.random.default_rng(2)
    p = rng.uniform(0, L, 20000).astype(np.float32)
    fine = oracle.cell_index_many(p, 12000, L)
    for m, G in [(2, 6000), (4, 3000)]:
        assert np.array_equal(fine // m, oracle.cell_index_many(p, G, L))


def test_keys_round_trip_and_order():
    L, delta = 1000.0, 0.25
    G = oracle.grid(delta, L)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, L, (5000, 3)).astype(np.float32)
    k = oracle.keys(pos, delta, L).astype(np.int64)
    ix, rest = np.divmod(k, G * G)
    iy, iz = np.divmod(rest, G)
    for axis, idx in enumerate([ix, iy, iz]):
        assert np.array_equal(idx, oracle.cell_index_many(pos[:, axis], G, L))
    assert k.max() < G ** 3


def test_keys_skip_out_of_domain_particles():
    pos = np.array([[1, 2, 3], [np.nan, 1, 1], [1, np.inf, 1], [1, 1, 250.0], [4, 5, 6]], dtype=np.float32)
    k = oracle.keys(pos, 1.0, 100.0)
    assert list(k) == [(1 * 100 + 2) * 100 + 3, (4 * 100 + 5) * 100 + 6]


def test_periodic_wrap_gives_same_key():
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 100, (2000, 3)).astype(np.float32)
    shifted = (pos.astype(np.float64) - 100.0).astype(np.float32)
    exact_shift = (shifted.astype(np.float64) + 100.0) == pos.astype(np.float64)
    rows = exact_shift.all(axis=1)
    assert rows.sum() > 100
    assert np.array_equal(oracle.keys(pos[rows], 0.1, 100.0), oracle.keys(shifted[rows], 0.1, 100.0))


# ------------------------------------------------------------ row hash (O5)

def test_tabulation_structure():
    # Simple tabulation: two keys that differ only in byte c have hashes that differ
    # by T[r][c][a] ^ T[r][c][b], whatever the other bytes are.
    T = oracle.hash_tables(99, 4)
    rng = np.random.default_rng(5)
    base = rng.integers(0, 2 ** 48, 200, dtype=np.uint64)
    for c in range(6):
        a, b = 17, 201
        mask = ~np.uint64(0xFF << (8 * c))
        k1 = (base & mask) | np.uint64(a << (8 * c))
        k2 = (base & mask) | np.uint64(b << (8 * c))
        for r in range(4):
            x = oracle.row_hash(T, r, k1) ^ oracle.row_hash(T, r, k2)
            assert np.all(x == (T[r, c, a] ^ T[r, c, b]))
    assert oracle.row_hash(T, 2, np.array([0], dtype=np.uint64))[0] == np.bitwise_xor.reduce(T[2, :, 0])


def test_bucket_range_reduction():
    rng = np.random.default_rng(6)
    hs = [int(x) for x in rng.integers(0, 2 ** 32, 2000, dtype=np.uint64)] + [0, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]
    for w in [1, 2, 3, 1000, 4154983, 1 << 16, 1 << 24, 1 << 30]:
        for h in hs:
            b = oracle.bucket(h, w)
            assert 0 <= b < w
            # floor(h31 * w / 2^31) with h31 the low 31 bits
            assert b == ((h & 0x7FFFFFFF) * w) >> 31
            if w & (w - 1) == 0:
                lg = w.bit_length() - 1
                assert b == (h & 0x7FFFFFFF) >> (31 - lg)


def test_sign_from_top_bit():
    assert oracle.sign(0) == 1 and oracle.sign(0x7FFFFFFF) == 1
    assert oracle.sign(0x80000000) == -1 and oracle.sign(0xFFFFFFFF) == -1


def test_hash_statistics():
    # Buckets uniform (chi-square), signs balanced, rows independent (collision
    # rate of two rows ~ 1/w^2 per pair of keys rather than 1/w).
    T = oracle.hash_tables(2024, 3)
    keys = np.arange(200_000, dtype=np.uint64) * np.uint64(7919)
    w = 1024
    H = [oracle.row_hash(T, r, keys) for r in range(3)]
    B = [((h.astype(np.uint64) & np.uint64(0x7FFFFFFF)) * np.uint64(w)) >> np.uint64(31) for h in H]
    for r in range(3):
        counts = np.bincount(B[r].astype(np.int64), minlength=w)
        e = keys.size / w
        chi2 = ((counts - e) ** 2 / e).sum()
        assert abs(chi2 - (w - 1)) < 6 * math.sqrt(2 * (w - 1))
        s = (H[r] >> np.uint32(31)).astype(np.int64)
        assert abs(s.mean() - 0.5) < 5 * 0.5 / math.sqrt(keys.size)
    joint = B[0] * np.uint64(w) + B[1]
    cj = np.bincount(joint.astype(np.int64), minlength=w * w)
    e = keys.size / (w * w)
    assert abs(cj.mean() - e) < 1e-9
    assert cj.max() < 20


# ------------------------------------------------------------ Add (O6)

def small_stream(n=20000, L=100.0, seed=0):
    """Clustered stream: a few dense clumps plus uniform background."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (12, 3))
    which = rng.integers(0, 12, n)
    clump = centres[which] + rng.normal(0, 0.15, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < 0.6)[:, None], clump, bg)
    return np.mod(pos, L).astype(np.float32)


def brute_counters(T, d, w, keys_, variant=oracle.VARIANT_CS):
    """Histogram-driven brute force: M[r][b] = sum over distinct keys j with
    bucket_r(j) = b of f_j * sign_r(j)."""
    uniq, f = oracle.histogram(keys_)
    M = np.zeros((d, w), dtype=np.int64)
    for r in range(d):
        h = oracle.row_hash(T, r, uniq).astype(np.uint64)
        b = ((h & np.uint64(0x7FFFFFFF)) * np.uint64(w)) >> np.uint64(31)
        s = np.where(h >> np.uint64(31), -1, 1) if variant == oracle.VARIANT_CS else np.ones_like(f)
        np.add.at(M[r], b.astype(np.int64), f * s)
    return ((M + 2 ** 31) % 2 ** 32 - 2 ** 31).astype(np.int32)


@pytest.mark.parametrize("d,w", [(5, 1 << 10), (3, 1000), (1, 1), (8, 4154983 // 4096)])
def test_stream_counters_equal_histogram_brute_force(d, w):
    pos = small_stream()
    M, skipped = oracle.sketch(pos, d, w, 11, 0.1, 100.0)
    assert skipped == 0
    assert np.array_equal(M, brute_counters(oracle.hash_tables(11, d), d, w, oracle.keys(pos, 0.1, 100.0)))


def test_count_min_rows_sum_to_n():
    pos = small_stream(15000)
    pos[::97] = np.nan
    n_valid = len(oracle.keys(pos, 0.1, 100.0))
    M, skipped = oracle.sketch(pos, 5, 777, 3, 0.1, 100.0, variant=oracle.VARIANT_CM)
    assert skipped == len(pos) - n_valid > 0
    assert np.all(M.astype(np.int64).sum(axis=1) == n_valid)


def test_count_sketch_row_sums_are_signed_totals():
    pos = small_stream(15000)
    d, w, seed = 5, 512, 8
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    T = oracle.hash_tables(seed, d)
    k = oracle.keys(pos, 0.1, 100.0)
    for r in range(d):
        s = np.where(oracle.row_hash(T, r, k) >> np.uint32(31), -1, 1)
        assert M[r].astype(np.int64).sum() == s.sum()


def test_single_counter_is_signed_sum():
    # d = w = 1: one counter = sum_j f_j s(j) (the single +-1 counter of Fig. 2).
    pos = small_stream(5000)
    M, _ = oracle.sketch(pos, 1, 1, 5, 0.1, 100.0)
    T = oracle.hash_tables(5, 1)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    s = np.where(oracle.row_hash(T, 0, uniq) >> np.uint32(31), -1, 1)
    assert int(M[0, 0]) == int((f * s).sum())


def test_permutation_chunking_and_merge_invariance():
    pos = small_stream(12000)
    d, w, seed = 5, 333, 21
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    perm = np.random.default_rng(9).permutation(len(pos))
    Mp, _ = oracle.sketch(pos[perm], d, w, seed, 0.1, 100.0)
    assert np.array_equal(M, Mp)
    # sketches of disjoint parts sum to the sketch of the whole (mergeability, Sec. 5)
    A, _ = oracle.sketch(pos[:5000], d, w, seed, 0.1, 100.0)
    B, _ = oracle.sketch(pos[5000:], d, w, seed, 0.1, 100.0)
    assert np.array_equal(M, (A.view(np.uint32) + B.view(np.uint32)).view(np.int32))
    # incremental update equals one update over the concatenation
    T = oracle.hash_tables(seed, d)
    Mi = np.zeros((d, w), np.int32)
    oracle.sketch_update(Mi, T, pos[:7000], 0.1, 100.0)
    oracle.sketch_update(Mi, T, pos[7000:], 0.1, 100.0)
    assert np.array_equal(M, Mi)
    Mt, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0, threads=4)
    assert np.array_equal(M, Mt)


def test_counters_wrap_modulo_2_32():
    d, w = 1, 1
    T = oracle.hash_tables(0, 1)
    M = np.full((d, w), 2 ** 31 - 1, dtype=np.int32)
    pos = np.zeros((1, 3), np.float32)
    key0 = oracle.keys(pos, 1.0, 10.0)
    s = 1 if oracle.row_hash(T, 0, key0)[0] < 2 ** 31 else -1
    if s < 0:
        M[:] = -(2 ** 31)
    oracle.sketch_update(M, T, pos, 1.0, 10.0)
    assert int(M[0, 0]) == (-(2 ** 31) if s > 0 else 2 ** 31 - 1)


# ------------------------------------------------------------ Estimate (O7)

def per_row_estimates(M, T, keys_):
    d, w = M.shape
    out = []
    for r in range(d):
        h = oracle.row_hash(T, r, keys_).astype(np.uint64)
        b = (((h & np.uint64(0x7FFFFFFF)) * np.uint64(w)) >> np.uint64(31)).astype(np.int64)
        s = np.where(h >> np.uint64(31), -1, 1)
        out.append(M[r, b].astype(np.int64) * s)
    return np.array(out)


@pytest.mark.parametrize("d", [1, 2, 4, 5, 7])
def test_estimate_is_lower_median_of_row_estimates(d):
    pos = small_stream(8000)
    w, seed = 64, 13
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    T = oracle.hash_tables(seed, d)
    uniq, _ = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    E = per_row_estimates(M, T, uniq)
    want = np.sort(E, axis=0)[(d - 1) // 2]
    assert np.array_equal(oracle.estimate(M, T, uniq), want)


def test_estimate_exact_without_collisions():
    # If key j shares its bucket with no other present key in at least floor(d/2)+1
    # rows, every such row returns f_j exactly and the median of d (odd) is f_j.
    rng = np.random.default_rng(10)
    cells = rng.uniform(0, 100, (50, 3))
    counts = rng.integers(1, 300, 50)
    pos = np.repeat(cells, counts, axis=0).astype(np.float32)
    pos = pos[rng.permutation(len(pos))]
    d, w, seed = 5, 1 << 20, 17
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    T = oracle.hash_tables(seed, d)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    est = oracle.estimate(M, T, uniq)
    clean = 0
    for j in range(len(uniq)):
        free_rows = 0
        for r in range(d):
            h = oracle.row_hash(T, r, uniq).astype(np.uint64)
            b = ((h & np.uint64(0x7FFFFFFF)) * np.uint64(w)) >> np.uint64(31)
            free_rows += int((b == b[j]).sum() == 1)
        if free_rows >= d // 2 + 1:
            assert est[j] == f[j]
            clean += 1
    assert clean >= 45
    # with exact estimates the sketch top-k is the exact top-k
    ks, es, st = oracle.topk_sketch(M, T, pos, 0.1, 100.0, oracle.INT32_MIN, 10)
    kx, fx = oracle.topk_exact(uniq, f, 10)
    assert np.array_equal(ks, kx) and np.array_equal(es, fx)


def test_count_min_never_underestimates():
    pos = small_stream(10000)
    M, _ = oracle.sketch(pos, 4, 97, 1, 0.1, 100.0, variant=oracle.VARIANT_CM)
    T = oracle.hash_tables(1, 4)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    est = oracle.estimate(M, T, uniq, variant=oracle.VARIANT_CM)
    assert np.all(est >= f)
    assert np.array_equal(est, per_row_estimates(M.astype(np.int64), T, uniq).__abs__().min(axis=0))


def test_row_estimate_is_unbiased_over_seeds():
    # E[M[r][h(j)] * s(j)] = f_j under pairwise-independent hashing (Sec. 2.2).
    pos = small_stream(3000, seed=3)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    j = int(np.argmax(f))
    d, w = 1, 16
    vals = []
    for seed in range(400):
        M, _ = oracle.sketch(pos, d, w, 1000 + seed, 0.1, 100.0)
        vals.append(int(oracle.estimate(M, oracle.hash_tables(1000 + seed, d), uniq[j:j + 1])[0]))
    vals = np.array(vals, dtype=np.float64)
    f2_rest = float((f.astype(np.float64) ** 2).sum() - f[j] ** 2)
    sd = math.sqrt(f2_rest / w)
    assert abs(vals.mean() - f[j]) < 5 * sd / math.sqrt(len(vals))


def test_additive_error_scale():
    # |est - f| ~ sqrt(F2_res / w) (Sec. 4.3: additive error set by the l2 norm).
    pos = small_stream(60000, seed=5)
    d, w, seed = 5, 2048, 2
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    est = oracle.estimate(M, oracle.hash_tables(seed, d), uniq)
    top = np.argsort(-f)[:200]
    f2_res = float((np.sort(f.astype(np.float64))[:-200] ** 2).sum())
    err = np.abs(est[top].astype(np.int64) - f[top])
    assert np.median(err) < 3 * math.sqrt(f2_res / w)


# ------------------------------------------------------------ histogram (O8)

def test_histogram_matches_dense_counting():
    rng = np.random.default_rng(12)
    L, delta = 10.0, 0.5          # G = 20: a dense array of 8000 cells
    pos = rng.uniform(-L, 2 * L, (30000, 3)).astype(np.float32)
    k = oracle.keys(pos, delta, L)
    uniq, f = oracle.histogram(k)
    dense = np.bincount(k.astype(np.int64), minlength=20 ** 3)
    nz = np.nonzero(dense)[0]
    assert np.array_equal(uniq.astype(np.int64), nz)
    assert np.array_equal(f, dense[nz])
    assert f.sum() == len(pos)


# ------------------------------------------------------------ top-k (O9, O10)

def python_topk(keys_, vals, k, theta=None):
    items = [(-int(v), int(kk)) for kk, v in zip(keys_, vals) if theta is None or v >= theta]
    items.sort()
    return [kk for _, kk in items[:k]], [-v for v, _ in items[:k]]


def test_topk_tie_order_and_theta_invariance():
    # Many equal counts: the order is (estimate desc, key asc).
    rng = np.random.default_rng(13)
    cells = rng.uniform(0, 100, (300, 3))
    counts = rng.integers(1, 6, 300)
    pos = np.repeat(cells, counts, axis=0).astype(np.float32)
    d, w, seed = 5, 1 << 18, 4
    M, _ = oracle.sketch(pos, d, w, seed, 0.1, 100.0)
    T = oracle.hash_tables(seed, d)
    uniq, f = oracle.histogram(oracle.keys(pos, 0.1, 100.0))
    est = oracle.estimate(M, T, uniq)
    for k in [1, 7, 50, 299, 1000]:
        ks, es, st = oracle.topk_sketch(M, T, pos, 0.1, 100.0, oracle.INT32_MIN, k)
        wk, we = python_topk(uniq, est, k)
        assert list(ks) == wk and list(es) == we and st == oracle.OK
        kth = we[-1]
        for theta in [kth, kth - 1, -5]:
            ks2, es2, st2 = oracle.topk_sketch(M, T, pos, 0.1, 100.0, theta, k)
            assert np.array_equal(ks, ks2) and np.array_equal(es, es2)
            assert st2 == (oracle.W_INCOMPLETE if len(wk) < k else oracle.OK)
    # a theta above the k-th estimate returns fewer items and says so
    n_max = int((est == est.max()).sum())
    ks3, es3, st3 = oracle.topk_sketch(M, T, pos, 0.1, 100.0, int(est.max()), n_max + 1)
    assert st3 == oracle.W_INCOMPLETE and len(ks3) == n_max and np.all(es3 == est.max())
    kx, fx = oracle.topk_exact(uniq, f, 40)
    wk, wf = python_topk(uniq, f, 40)
    assert list(kx) == wk and list(fx) == wf


def test_empty_stream():
    pos = np.zeros((0, 3), np.float32)
    M, sk = oracle.sketch(pos, 5, 64, 1, 0.1, 100.0)
    assert sk == 0 and not M.any()
    ks, es, st = oracle.topk_sketch(M, oracle.hash_tables(1, 5), pos, 0.1, 100.0, oracle.INT32_MIN, 10)
    assert len(ks) == 0 and st == oracle.OK
    uniq, f = oracle.histogram(np.zeros(0, np.uint64))
    assert len(uniq) == 0


def test_small_workload_recall():
    # Heavy-hitter recovery (Sec. 2.2: the median of t unbiased row estimates tracks the
    # frequencies of the heavy items) and the relative error |c - c_hat| / c of Sec. 4.3: on
    # the 2^20-particle Plummer workload (d = 5, w = 2^16, k = 100) the sketch's top-k is
    # checked against the exact top-k of the oracle's histogram.  The single-row noise
    # sqrt(F2 / w) is about 6.5 while the 100th count is about 60, so nearly all of the top
    # 100 must come back with small relative error; a wrong sign, bucket or median would
    # destroy this.
    import workloads
    wl = workloads.SMALL
    pos = wl.generate()
    M, _ = oracle.sketch(pos, wl.d, wl.w, wl.seed, wl.delta, wl.L)
    T = oracle.hash_tables(wl.seed, wl.d)
    ks, es, st = oracle.topk_sketch(M, T, pos, wl.delta, wl.L, oracle.INT32_MIN, wl.k)
    assert st == oracle.OK and len(ks) == wl.k
    uniq, f = oracle.histogram(oracle.keys(pos, wl.delta, wl.L))
    kx, fx = oracle.topk_exact(uniq, f, wl.k)
    fmap = dict(zip(uniq.tolist(), f.tolist()))
    strict = len(set(ks.tolist()) & set(kx.tolist())) / wl.k
    tie_tolerant = sum(fmap[k] >= fx[-1] for k in ks.tolist()) / wl.k
    rel = np.array([abs(int(e) - fmap[k]) / fmap[k] for k, e in zip(ks.tolist(), es.tolist())])
    assert strict >= 0.95 and tie_tolerant >= 0.95
    assert np.median(rel) < 0.05 and rel.max() < 0.25


def test_dictionary_topk_brute_force_and_semantics():
    # Count Sketch with Full Search (Sec. 2.2 item 1; Alg. 1): every key of the G^3 mesh is
    # estimated, occupied or not.  Checked against a Python selection over all keys, with the
    # estimates recomputed row by row from the counters (Sec. 2.2 Estimate).
    G, d, w, seed, L = 12, 5, 256, 4, 12.0
    rng = np.random.default_rng(7)
    pos = (rng.random((3000, 3)) ** 2 * L).astype(np.float32)   # skewed occupancy
    M, _ = oracle.sketch(pos, d, w, seed, 1.0, L)
    T = oracle.hash_tables(seed, d)
    keys = np.arange(G ** 3, dtype=np.uint64)
    rows = per_row_estimates(M.astype(np.int64), T, keys)         # [d][G^3] signed row estimates
    est = np.sort(rows, axis=0)[(d - 1) // 2].astype(np.int64)   # lower median
    for theta, k in [(oracle.INT32_MIN, 40), (3, 40), (3, 10 ** 5), (int(est.max()) + 1, 5)]:
        order = sorted((int(-e), int(kk)) for kk, e in zip(keys, est) if e >= theta)[:k]
        ks, es, st = oracle.topk_dictionary(M, T, G, theta, k)
        assert [int(x) for x in ks] == [kk for _, kk in order]
        assert [int(x) for x in es] == [-e for e, _ in order]
        short = len(order) < k and theta != oracle.INT32_MIN
        assert st == (oracle.W_INCOMPLETE if short else oracle.OK)
    # an invalid mesh is refused
    _, _, st = oracle.topk_dictionary(M, T, 0, 0, 5)
    assert st == oracle.E_INVALID


def test_dictionary_topk_without_collisions_is_exact():
    # With w far above the number of occupied cells every estimate is exact (no collision in
    # a majority of rows), so the dictionary top-k is the exact top-k of the stream followed,
    # for theta = INT32_MIN, by empty cells (estimate 0) in key order (Sec. 2.2).
    G, d, w, seed, L = 10, 5, 1 << 16, 9, 10.0
    rng = np.random.default_rng(3)
    centres = rng.random((6, 3)) * L
    pos = np.concatenate([c + rng.normal(0, 0.3, (400, 3)) for c in centres]) % L
    pos = pos.astype(np.float32)
    M, _ = oracle.sketch(pos, d, w, seed, 1.0, L)
    T = oracle.hash_tables(seed, d)
    uniq, f = oracle.histogram(oracle.keys(pos, 1.0, L))
    est = oracle.estimate(M, T, uniq)
    assert np.array_equal(est, f)   # no collisions at this width
    k = len(uniq) + 20
    ks, es, st = oracle.topk_dictionary(M, T, G, oracle.INT32_MIN, k)
    kx, fx = oracle.topk_exact(uniq, f, len(uniq))
    assert st == oracle.OK
    assert np.array_equal(ks[:len(uniq)], kx) and np.array_equal(es[:len(uniq)], fx)
    empty = [x for x in range(G ** 3) if x not in set(uniq.tolist())][:20]
    assert ks[len(uniq):].tolist() == empty and not es[len(uniq):].any()


def hier_case():
    G, L, seed1, seed2, R = 12, 12.0, 41, 42, 7
    rng = np.random.default_rng(11)
    pos = (rng.random((4000, 3)) ** 2 * L).astype(np.float32)
    M1 = oracle.super_sketch(pos, 5, 64, seed1, 1.0, L, R)
    M2, _ = oracle.sketch(pos, 5, 512, seed2, 1.0, L)
    return G, L, R, pos, M1, oracle.hash_tables(seed1, 5), M2, oracle.hash_tables(seed2, 5)


def test_super_sketch_counts_key_div_group():
    # The coarse layer adds key // R (Sec. 2.2 item 3: super-items s_j / 1000); with R = 1
    # it is the plain sketch, and its counters equal a sketch of the divided keys.
    G, L, R, pos, M1, T1, M2, T2 = hier_case()
    assert np.array_equal(oracle.super_sketch(pos, 5, 512, 42, 1.0, L, 1), M2)
    k = oracle.keys(pos, 1.0, L)
    manual = np.zeros((5, 64), np.int64)
    for r in range(5):
        h = oracle.row_hash(T1, r, k // np.uint64(R)).astype(np.uint64)
        b = (((h & np.uint64(0x7FFFFFFF)) * np.uint64(64)) >> np.uint64(31)).astype(np.int64)
        np.add.at(manual[r], b, np.where(h >> np.uint64(31), -1, 1))
    assert np.array_equal(M1, manual.astype(np.int32))


def test_hierarchical_topk_brute_force():
    # Alg. 3 query: heavy super-items by M1, then their children by M2; checked against a
    # Python walk over all super-items with row-by-row estimates, and against the full
    # dictionary search when every super-item passes (theta1 = INT32_MIN).
    G, L, R, pos, M1, T1, M2, T2 = hier_case()
    nkeys = G ** 3
    sup = np.arange((nkeys + R - 1) // R, dtype=np.uint64)
    e1 = np.sort(per_row_estimates(M1.astype(np.int64), T1, sup), axis=0)[2]
    allk = np.arange(nkeys, dtype=np.uint64)
    e2 = np.sort(per_row_estimates(M2.astype(np.int64), T2, allk), axis=0)[2]
    for theta1, theta2, k in [(5, 2, 50), (20, oracle.INT32_MIN, 30), (10 ** 6, 0, 10), (3, 4, 10 ** 5)]:
        cand = [(int(-e2[c]), c) for j in range(len(sup)) if e1[j] >= theta1
                for c in range(j * R, min((j + 1) * R, nkeys)) if e2[c] >= theta2]
        want = sorted(cand)[:k]
        ks, es, st = oracle.topk_hierarchical(M1, T1, M2, T2, G, R, theta1, theta2, k)
        assert [int(x) for x in ks] == [c for _, c in want]
        assert [int(x) for x in es] == [-e for e, _ in want]
        short = len(want) < k and (theta1 != oracle.INT32_MIN or theta2 != oracle.INT32_MIN)
        assert st == (oracle.W_INCOMPLETE if short else oracle.OK)
    for theta2 in [oracle.INT32_MIN, 3]:
        a = oracle.topk_hierarchical(M1, T1, M2, T2, G, R, oracle.INT32_MIN, theta2, 200)
        b = oracle.topk_dictionary(M2, T2, G, theta2, 200)
        assert all(np.array_equal(x, y) for x, y in zip(a[:2], b[:2])) and a[2] == b[2]
    assert oracle.topk_hierarchical(M1, T1, M2, T2, G, 0, 0, 0, 5)[2] == oracle.E_INVALID


# ------------------------------------------------------------------ learned router reference

def test_router_features_and_sample_by_brute_force():
    from oracle import router
    import workloads
    # features: neighbour counts enumerated one by one on a tiny periodic mesh
    Gc = 5
    counts = np.arange(Gc ** 3, dtype=np.uint32) * 7 % 11
    cells = np.array([0, 62, 124, 31], dtype=np.int64)
    f = router.features(counts, Gc, cells)
    for r, c in enumerate(cells):
        x, y, z = c // 25, (c // 5) % 5, c % 5
        q = 0
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    nb = (((x + dx) % 5) * 5 + (y + dy) % 5) * 5 + (z + dz) % 5
                    assert f[r, q] == np.float32(np.log1p(np.float32(counts[nb])))
                    q += 1
        assert not f[r, 27:].any()
    # the sample: about 1 % of the stream, and particle g's coin is word g mod 4 of the
    # published Philox block at counter g / 4
    m = router.sample_mask(200_000, 9)
    assert 0.009 < m.mean() < 0.011
    for g in (12344, 12345, 12346, 12347):
        w = workloads.philox4x32_10([g // 4, 0, 4, 0], [9, 0])[g % 4]
        assert m[g] == (w < router.SAMPLE_THRESHOLD)


def test_router_forward_and_gradients_by_loops_and_differences():
    from oracle import router
    rng = np.random.default_rng(4)
    p = rng.normal(0, 0.3, router.N_PARAMS).astype(np.float32)
    w = router.unpack(p)
    w["W1"][:, 27:] = 0
    p = router.pack(w)
    x = np.zeros((6, 32), np.float32)
    x[:, :27] = rng.random((6, 27)) * 3
    z, _, _ = router.forward(p, x)
    assert np.allclose(z, router.forward_loops(p, x), atol=1e-4)
    # bf16 rounding: ties to even, and 1 + 2^-8 (a tie) rounds down to 1
    assert router.bf16(np.float32(1 + 2 ** -8)) == 1.0 and router.bf16(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)
    # gradients of the loss at float64 without rounding, by central differences, agree with
    # the rounded analytic gradients to bf16 accuracy
    y = (rng.random(6) < 0.5).astype(np.float32)
    g = router.gradients(p, x, y)

    def loss(q):
        wq = router.unpack(q.astype(np.float32))
        h1 = np.maximum(x @ wq["W1"].T.astype(np.float64) + wq["b1"], 0)
        h2 = np.maximum(h1 @ wq["W2"].T.astype(np.float64) + wq["b2"], 0)
        zz = h2 @ wq["w3"].astype(np.float64) + wq["b3"][0]
        return np.mean(np.maximum(zz, 0) - zz * y + np.log1p(np.exp(-np.abs(zz))))
    for idx in [router.OFF["W1"][0] + 3, router.OFF["b1"][0] + 5, router.OFF["W2"][0] + 100,
                router.OFF["b2"][0] + 7, router.OFF["w3"][0] + 9, router.OFF["b3"][0]]:
        e = np.zeros(router.N_PARAMS)
        e[idx] = 1e-3
        num = (loss(p + e) - loss(p - e)) / 2e-3
        assert abs(num - g[idx]) < 0.03 * max(1e-3, abs(num)) + 2e-3, (idx, num, g[idx])


def test_router_split_invariants():
    from oracle import router
    rng = np.random.default_rng(2)
    pos = (rng.random((20_000, 3)) ** 3 * 10.0).astype(np.float32)     # crowded near the origin
    admitted = np.array([0, 1, 101, 4444], dtype=np.uint64)            # coarse keys of the 25^3 mesh
    tk, tc, rest = router.route(pos, 0.1, 10.0, 4, admitted)
    assert tc.sum() + len(rest) == len(pos)
    G, Gc = 100, 25
    for kk in tk:
        ix, iy, iz = kk // (G * G), (kk // G) % G, kk % G
        assert ((ix // 4) * Gc + iy // 4) * Gc + iz // 4 in set(admitted.tolist())
    rk = oracle.keys(rest, 0.1, 10.0)
    ck = ((rk // np.uint64(G * G) // np.uint64(4)) * np.uint64(Gc) + (rk // np.uint64(G)) % np.uint64(G) // np.uint64(4)) \
        * np.uint64(Gc) + rk % np.uint64(G) // np.uint64(4)
    assert not np.isin(ck, admitted).any()


def test_router_lists_labels_and_admission_by_brute_force():
    from oracle import router
    rng = np.random.default_rng(6)
    counts = rng.integers(0, 4, 300).astype(np.uint32)
    for mc in (0, 1, 3, 5):
        assert router.cell_list(counts, mc).tolist() == [j for j in range(300) if counts[j] >= mc]
    # labels: a coarse cell is positive iff one of its factor^3 children, enumerated one by
    # one, is among the fine keys
    G, f = 12, 3
    Gc = G // f
    fine = rng.choice(G ** 3, 40, replace=False).astype(np.uint64)
    fs = set(fine.tolist())
    cells = np.arange(Gc ** 3, dtype=np.int64)
    lab = router.labels(cells, fine, G, f)
    for c in cells:
        cx, cy, cz = c // (Gc * Gc), (c // Gc) % Gc, c % Gc
        kids = {((cx * f + a) * G + cy * f + b) * G + cz * f + e for a in range(f) for b in range(f) for e in range(f)}
        assert lab[c] == (1.0 if kids & fs else 0.0)
    # admission: A cells, ascending, and no cell left out outranks one taken by (logit, -key)
    m = 60
    cells = rng.choice(10 ** 6, m, replace=False).astype(np.int64)
    z = rng.integers(-3, 4, m).astype(np.float32) / 2      # many ties
    z[:4] = [0.0, -0.0, 0.0, -0.0]
    for A in (1, 7, 25, 60, 80):
        adm = router.admit(cells, z, A)
        assert len(adm) == min(A, m) and np.all(np.diff(adm) > 0)
        taken = set(adm.tolist())
        for j in range(m):
            for i in range(m):
                if cells[i] in taken and cells[j] not in taken:
                    assert (z[i] > z[j]) or (z[i] == z[j] and cells[i] < cells[j])


def test_exact_topk_by_counting():
    from oracle import router
    rng = np.random.default_rng(3)
    pos = (rng.random((5000, 3)) ** 2 * 10).astype(np.float32)
    keys, cnt = router.exact_topk(pos, 1.0, 10.0, 15)
    tally = {}
    for p in pos:
        k = (int(p[0]) * 10 + int(p[1])) * 10 + int(p[2])
        tally[k] = tally.get(k, 0) + 1
    want = sorted(tally.items(), key=lambda kv: (-kv[1], kv[0]))[:15]
    assert keys.tolist() == [k for k, _ in want] and cnt.tolist() == [c for _, c in want]


# ------------------------------------------------------------------ packed particle input

def test_pack_by_exact_rationals():
    from fractions import Fraction
    rng = np.random.default_rng(12)
    for L in (100.0, 1000.0, 64.0, 3.7):
        p = np.concatenate([rng.uniform(-1.9 * L, 1.9 * L, 300),
                            [0.0, -0.0, L, -L, np.nextafter(np.float32(L), np.float32(0)), 2 * L, -2 * L, np.inf,
                             np.nan, 1e-30]]).astype(np.float32)
        pos = np.stack([p, p[::-1], np.roll(p, 7)], axis=1)
        words = oracle.pack(pos, L)
        for row, wd in zip(pos, words):
            qs = []
            for c in row:
                c = float(c)
                if not np.isfinite(c) or abs(c) >= 2 * L:
                    qs = None
                    break
                q = (Fraction(c) * 2 ** 21 // Fraction(L)) % (2 ** 21)
                qs.append(int(q))
            if qs is None:
                assert wd == oracle.PACK_OUTSIDE
            else:
                assert int(wd) == qs[0] | qs[1] << 21 | qs[2] << 42


def test_packed_keys_by_integer_formula_and_nesting():
    rng = np.random.default_rng(13)
    pos = rng.uniform(0, 64.0, (3000, 3)).astype(np.float32)
    words = oracle.pack(pos, 64.0)
    for delta in (0.25, 0.256, 1.0):            # G = 256, 250, 64
        G = oracle.grid(delta, 64.0)
        keys = oracle.keys_packed(words, delta, 64.0)
        want = []
        for wd in words.tolist():
            i = [((wd >> sh) & (2 ** 21 - 1)) * G >> 21 for sh in (0, 21, 42)]
            want.append((i[0] * G + i[1]) * G + i[2])
        assert keys.tolist() == want
    # G dividing 2^21 (here 256 = 64 / 0.25): floor(floor(p 2^21 / L) G / 2^21) = floor(p G / L),
    # so the packed stream has the float stream's cells
    assert np.array_equal(oracle.keys_packed(words, 0.25, 64.0), oracle.keys(pos, 0.25, 64.0))
    # outside-domain words are dropped like out-of-domain particles
    pos[5] = (200.0, 1.0, 1.0)
    assert len(oracle.keys_packed(oracle.pack(pos, 64.0), 0.25, 64.0)) == len(pos) - 1


def test_topk_keys_matches_exact_top_without_collisions():
    rng = np.random.default_rng(14)
    keys = rng.zipf(1.6, 20000).astype(np.uint64) % np.uint64(5000)
    M = oracle.sketch_keys(keys, 5, 1 << 22, 3)
    T = oracle.hash_tables(3, 5)
    uniq, cnt = oracle.histogram(keys)
    # a wide sketch estimates every key exactly here, so the top-k is the exact one
    assert np.array_equal(oracle.estimate(M, T, uniq), cnt.astype(np.int32))
    k_keys, k_est = oracle.topk_keys(M, T, keys, oracle.INT32_MIN, 50)
    e_keys, e_cnt = oracle.topk_exact(uniq, cnt, 50)
    assert np.array_equal(k_keys, e_keys) and np.array_equal(k_est, e_cnt.astype(np.int32))
    k2, e2 = oracle.topk_keys(M, T, keys, int(e_cnt[9]), 50)         # theta cuts at the 10th count
    assert np.array_equal(k2, k_keys[k_est >= e_cnt[9]])


# ------------------------------------------------------------ router reference pins

@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    """PyTorch's own Philox4x32-10 engine (Salmon et al., SC'11), built from its header:
    an implementation that shares nothing with the workload generator's."""
    import ctypes
    import subprocess
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    src = os.path.join(os.path.dirname(__file__), "torch_philox_ref.cpp")
    so = str(tmp_path_factory.mktemp("philox") / "torch_philox_ref.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I", inc, "-o", so, src], check=True)
    lib = ctypes.CDLL(so)

    def words(ctr, key):
        c = np.ascontiguousarray(ctr, dtype=np.uint32)
        k = np.ascontiguousarray(key, dtype=np.uint32)
        out = np.zeros(4, dtype=np.uint32)
        lib.torch_philox4x32_10(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                                out.ctypes.data_as(ctypes.c_void_p))
        return out
    return words


def test_philox_matches_an_independent_engine(torch_philox):
    import workloads
    rng = np.random.default_rng(77)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2), ([1, 0, 0, 0], [0, 0]),
             ([0, 0, 0, 1], [1, 0]), ([12345, 0, 4, 0], [9, 0])]
    cases += [(rng.integers(0, 2 ** 32, 4, dtype=np.uint64), rng.integers(0, 2 ** 32, 2, dtype=np.uint64))
              for _ in range(500)]
    for ctr, key in cases:
        assert np.array_equal(workloads.philox4x32_10(ctr, key), torch_philox(ctr, key)), (ctr, key)
    # the stream form: word g is word g mod 4 at counter (g / 4 mod 2^32, g / 4 / 2^32,
    # stream, 0), key = seed; ranges that start and end inside a block and cross 2^34
    for index0, stream, seed in [(0, 1, 1), (2 ** 34 - 3, 4, 2 ** 40 + 5), (10 ** 12 + 1, 2, 9)]:
        got = workloads.philox_words(index0, 7, stream, seed)
        for i in range(7):
            g = index0 + i
            c = g // 4
            want = torch_philox([c & 0xFFFFFFFF, c >> 32, stream, 0], [seed & 0xFFFFFFFF, seed >> 32])[g % 4]
            assert got[i] == want, (index0, stream, seed, i)


def test_router_sample_counts_by_particle_loop(torch_philox):
    # One particle at a time: the coin of particle g is word g mod 4 of the independent
    # engine at counter (g / 4, stream 4), the cell is the exact floor by rationals, and a
    # particle outside the domain is never counted.
    from oracle import router
    rng = np.random.default_rng(31)
    L, dc, seed = 10.0, 2.5, 2 ** 33 + 17
    Gc = 4
    pos = (rng.random((3000, 3)) ** 2 * L).astype(np.float32)
    pos[5] = [np.nan, 1.0, 1.0]
    pos[6] = [1.0, 2 * L, 1.0]
    pos[7] = [-1.0, 0.0, np.float32(L)]        # wraps into the box
    for index0, threshold in [(0, 2 ** 31), (2 ** 34 - 1001, 2 ** 30), (123, router.SAMPLE_THRESHOLD)]:
        want = np.zeros(Gc ** 3, dtype=np.int64)
        for i, p in enumerate(pos):
            g = index0 + i
            c = g // 4
            coin = torch_philox([c & 0xFFFFFFFF, c >> 32, router.SAMPLE_STREAM, 0],
                                [seed & 0xFFFFFFFF, seed >> 32])[g % 4]
            if coin >= threshold:
                continue
            if not all(math.isfinite(float(c)) and abs(float(c)) < 2 * L for c in p):
                continue
            ix, iy, iz = (exact_index(float(c), Gc, L) for c in p)
            want[(ix * Gc + iy) * Gc + iz] += 1
        got = router.sample_counts(pos, dc, L, seed, index0, threshold)
        assert got.dtype == np.uint32 and np.array_equal(got.astype(np.int64), want), (index0, threshold)


def test_router_topk_routed_by_dict_merge():
    # The merged top-k of the routed pair, rebuilt with a dictionary: table keys enter with
    # their exact counts whatever theta is; a rest cell enters with the lower median of its
    # per-row estimates (computed row by row here) when that is >= theta; the order is
    # (value desc, key asc) and at most k come out.
    from oracle import router
    rng = np.random.default_rng(12)
    L, delta, d, w, seed = 10.0, 0.5, 5, 64, 3           # w = 64: many collisions
    G = 20
    rest = small_stream(4000, L, seed=4)
    rk_all = oracle.keys(rest, delta, L)
    present = set(int(x) for x in np.unique(rk_all))
    absent = [c for c in range(G ** 3) if c not in present]
    tkeys = np.sort(rng.choice(absent, 30, replace=False)).astype(np.uint64)
    tcounts = rng.integers(1, 40, 30).astype(np.int64)
    tcounts[:6] = [7, 7, 7, 1, 1, 300]                     # ties, and counts below theta
    M, _ = oracle.sketch(rest, d, w, seed, delta, L)
    T = oracle.hash_tables(seed, d)
    uniq = np.unique(rk_all)
    E = np.sort(per_row_estimates(M, T, uniq), axis=0)[(d - 1) // 2]
    for theta, k in [(oracle.INT32_MIN, 50), (5, 40), (20, 10 ** 4), (10 ** 6, 12), (8, 1)]:
        cand = {int(kk): int(c) for kk, c in zip(tkeys, tcounts)}
        for kk, e in zip(uniq, E):
            if e >= theta:
                cand[int(kk)] = int(e)
        want = sorted(cand.items(), key=lambda kv: (-kv[1], kv[0]))[:k]
        gk, gv = router.topk_routed(tkeys, tcounts, M, T, rest, delta, L, theta, k)
        assert list(gk) == [kk for kk, _ in want] and list(gv) == [v for _, v in want], (theta, k)
        assert len(gk) == min(k, len(cand))


def test_router_fp32_forward_matches_exact_loops():
    # the unrounded float32 reference against float64 loops over neurons: only float32
    # summation and storage rounding separate them (a pin of forward_fp32, which the GPU
    # logits are held to within 2e-2)
    from oracle import router as ref
    rng = np.random.default_rng(17)
    w = ref.unpack(rng.normal(0, 0.3, ref.N_PARAMS).astype(np.float32))
    w["W1"][:, 27:] = 0
    p = ref.pack(w)
    x = np.zeros((24, 32), np.float32)
    x[:, :27] = np.log1p(rng.poisson(4.0, (24, 27))).astype(np.float32)
    z = ref.forward_fp32(p, x).astype(np.float64)
    ze = ref.forward_loops_exact(p, x)
    assert np.max(np.abs(z - ze)) < 1e-4 * max(1.0, np.max(np.abs(ze)))
    # a wrong layer (the bf16 one) is visibly different from the exact reference
    zb = ref.forward(p, x)[0].astype(np.float64)
    assert np.max(np.abs(zb - ze)) > 10 * np.max(np.abs(z - ze))
