"""GPU parity of the packed particle input (three 21-bit coordinates in 64 bits): packing,
keys, counters and the top-k bit for bit against the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk
import workloads

pytestmark = pytest.mark.gpu

OUT = np.uint64(2 ** 64 - 1)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def as_u64(t):
    return t.cpu().numpy().view(np.uint64)


def stream(n, L, seed):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (16, 3))
    pos = np.where((rng.random(n) < 0.6)[:, None], centres[rng.integers(0, 16, n)] + rng.normal(0, 0.02 * L, (n, 3)),
                   rng.uniform(-L, 2 * L, (n, 3)))      # wrapped coordinates too
    return pos.astype(np.float32)


@pytest.mark.parametrize("L", [100.0, 1000.0, 64.0, 3.7])
def test_pack_matches_oracle(L):
    import torch
    pos = stream(50_000, L, 1)
    edge = np.array([0.0, -0.0, L, -L, np.nextafter(np.float32(L), np.float32(0)), 2 * L, -2 * L, np.inf, np.nan,
                     1e-30, -1e-30, 1.5 * L], np.float32)
    pos[:len(edge), 0] = edge
    pos[len(edge):2 * len(edge), 2] = edge
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = as_u64(csk.pack_positions(dev(pos), L, err))
    want = oracle.pack(pos, L)
    assert np.array_equal(got, want)
    assert err.item() == 1 and (want == OUT).any()


def test_packed_keys_match_oracle():
    pos = stream(100_000, 100.0, 2)
    pos[:3] = (300.0, 1.0, 1.0)
    words = oracle.pack(pos, 100.0)
    for delta in (0.1, 0.25, 0.390625):           # G = 1000, 400, 256
        got = as_u64(csk.cell_keys_packed(dev(words.view(np.int64)), delta, 100.0))
        inside = words != OUT
        assert (got[~inside] == OUT).all()
        assert np.array_equal(got[inside], oracle.keys_packed(words, delta, 100.0))


CASES = [  # (L, delta, d, w, n, seed)
    (100.0, 0.1, 5, 1 << 16, 0, 1),
    (100.0, 0.1, 5, 1 << 16, 1, 1),
    (100.0, 0.1, 5, 1 << 16, 8193, 2),
    (1000.0, 0.25, 5, 4154983, 300_000, 3),
    (1000.0, 0.25, 5, 1 << 24, 200_000, 4),
    (64.0, 0.25, 3, 1000, 100_000, 5),
    (100.0, 0.1, 8, 1 << 15, 100_000, 6),
    (100.0, 0.1, 9, 1 << 15, 50_000, 7),
]


@pytest.mark.parametrize("L,delta,d,w,n,seed", CASES)
def test_packed_update_matches_oracle(L, delta, d, w, n, seed):
    import torch
    pos = stream(n, L, seed)
    words = oracle.pack(pos, L)
    s = csk.Sketch(d, w, seed)
    s.update_packed(dev(words.view(np.int64)), delta, L)
    keys = oracle.keys_packed(words, delta, L)
    want = oracle.sketch_keys(keys, d, w, seed)
    if (words == OUT).any():
        with pytest.raises(csk.CskError):
            s.check()
    assert np.array_equal(s.counters().cpu().numpy(), want)
    s.close()


def test_packed_workload_update_collect_topk_match_oracle():
    wl = workloads.SMALL
    pos = wl.generate()
    words = oracle.pack(pos, wl.L)
    wd = dev(words.view(np.int64))
    s = csk.Sketch(wl.d, wl.w, wl.seed)
    s.update_packed(wd, wl.delta, wl.L)
    keys = oracle.keys_packed(words, wl.delta, wl.L)
    M = oracle.sketch_keys(keys, wl.d, wl.w, wl.seed)
    assert np.array_equal(s.counters().cpu().numpy(), M)
    T = oracle.hash_tables(wl.seed, wl.d)
    for theta in (oracle.INT32_MIN, 5, 40):          # no filter, then the Bloom-filtered pass
        s.clear_candidates()
        s.collect_packed(wd, wl.delta, wl.L, theta)
        got_k, got_e, rc = s.topk(wl.k)
        want_k, want_e = oracle.topk_keys(M, T, keys, theta, wl.k)
        assert got_k.cpu().numpy().view(np.uint64).tolist() == want_k.tolist()
        assert got_e.cpu().numpy().tolist() == want_e.tolist()
    s.close()


def test_packed_direct_plan_matches_oracle():
    pos = stream(60_000, 100.0, 9)
    words = oracle.pack(pos, 100.0)
    s = csk.Sketch(5, 1 << 14, 2)
    s.set_update_plan(csk.CSK_UPDATE_DIRECT)
    s.update_packed(dev(words.view(np.int64)), 0.1, 100.0)
    want = oracle.sketch_keys(oracle.keys_packed(words, 0.1, 100.0), 5, 1 << 14, 2)
    assert np.array_equal(s.counters().cpu().numpy(), want)
    s.close()


def test_packed_equals_float_when_the_mesh_divides_2_21():
    # G = 256 divides 2^21: packing keeps every particle in its cell, so packed and float
    # updates (also mixed on one handle) give the float stream's counters
    import torch
    pos = stream(200_000, 64.0, 11)
    pos = np.mod(pos, 64.0).astype(np.float32)
    words = csk.pack_positions(dev(pos), 64.0)
    a = csk.Sketch(5, 1 << 16, 3)
    a.update(dev(pos), 0.25, 64.0)
    b = csk.Sketch(5, 1 << 16, 3)
    b.update_packed(words, 0.25, 64.0)
    c = csk.Sketch(5, 1 << 16, 3)
    c.update(dev(pos[:77_777]), 0.25, 64.0)
    c.update_packed(words[77_777:], 0.25, 64.0)
    want = oracle.sketch(pos, 5, 1 << 16, 3, 0.25, 64.0, threads=8)[0]
    for s in (a, b, c):
        assert np.array_equal(s.counters().cpu().numpy(), want)
        s.close()
