"""GPU parity of the learned router: sample counts and the routing split bit for bit, the
features to float32 log1p, the MFMA GEMM and the MLP against the numpy reference (scoring
logits within 2e-2 absolute of an unrounded float32 forward pass; training activations and
gradients against the bf16-rounded mirror), and the routed top-k bit for bit given the same admitted cells."""
import numpy as np
import pytest

import oracle
from oracle import router as ref
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def clustered(n, L, seed, frac=0.6, sigma=0.3, nclump=8):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (nclump, 3))
    clump = centres[rng.integers(0, nclump, n)] + rng.normal(0, sigma, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < frac)[:, None], clump, bg)
    pos = np.mod(pos, L).astype(np.float32)
    pos[pos >= L] = 0.0            # float32 rounding can reach L itself
    return pos


def test_sample_counts_and_features_match_reference():
    import torch
    L, dc = 100.0, 1.0
    pos = clustered(400_000, L, 3)
    counts = torch.zeros(100 ** 3, dtype=torch.int32, device="cuda")
    # two calls with running particle indices equal one call on the whole stream
    csk.sample_counts(dev(pos[:150_000]), dc, L, 17, counts, index0=0)
    csk.sample_counts(dev(pos[150_000:]), dc, L, 17, counts, index0=150_000)
    want = ref.sample_counts(pos, dc, L, 17)
    got = counts.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    cells = np.unique(np.nonzero(want)[0]).astype(np.int64)[:5000]
    feat = csk.cell_features(counts, dc, L, dev(cells)).cpu().numpy()
    assert np.allclose(feat, ref.features(want, 100, cells), rtol=2e-7, atol=0)
    # the same pass with the touched-cell bitmap: bits mark exactly the nonzero cells, the
    # listing from the bitmap equals the reference, and clearing empties both
    counts.zero_()
    bitmap = torch.zeros((100 ** 3 + 31) // 32, dtype=torch.int32, device="cuda")
    csk.sample_counts(dev(pos), dc, L, 17, counts, bitmap=bitmap)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), want)
    bits = np.unpackbits(bitmap.cpu().numpy().view(np.uint8), bitorder="little")[:100 ** 3]
    assert np.array_equal(bits.astype(bool), want > 0)
    for mc in (1, 2, 4):
        got = csk.cell_list(counts, mc, bitmap=bitmap).cpu().numpy()
        assert np.array_equal(got, ref.cell_list(want, mc))
    csk.cells_clear(counts, bitmap)
    assert not counts.any().item() and not bitmap.any().item()


@pytest.mark.parametrize("M,N,K,trans_a,trans_b", [(16, 16, 16, False, False), (37, 64, 27, False, True),
                                                   (64, 64, 300, True, False), (5, 3, 2, True, True),
                                                   (200, 48, 64, False, False)])
def test_mfma_gemm_matches_numpy(M, N, K, trans_a, trans_b):
    # C = A B on bf16-rounded operands with fp32 sums, through the strided MFMA kernel that
    # the training step uses for every layer
    import torch
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.normal(size=(M, K)).astype(np.float32)
    B = rng.normal(size=(K, N)).astype(np.float32)
    Ad = dev(A.T.copy() if trans_a else A)
    Bd = dev(B.T.copy() if trans_b else B)
    Cd = torch.empty((M, N), dtype=torch.float32, device="cuda")
    sa = (1, M) if trans_a else (K, 1)
    sb = (1, K) if trans_b else (N, 1)
    for beta in (0.0, 1.0):
        Cd.fill_(7.0)
        csk.gemm_bf16(M, N, K, Ad, sa, Bd, sb, Cd, (N, 1), beta)
        want = ref.bf16(A).astype(np.float64) @ ref.bf16(B).astype(np.float64) + (7.0 if beta else 0.0)
        assert np.allclose(Cd.cpu().numpy(), want, rtol=1e-5, atol=2e-4)


def he_uniform_params(seed):
    """The documented initialisation of csk_mlp_create: He-uniform weights from the
    SplitMix64 sequence of the seed (W1, W2, w3 in turn; padding inputs zero), zero biases."""
    u = (oracle.splitmix64(seed, 64 * 32 + 64 * 64 + 64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    w = {"W1": (2 * u[:2048] - 1) * np.sqrt(6 / 27), "W2": (2 * u[2048:6144] - 1) * np.sqrt(6 / 64),
         "w3": (2 * u[6144:] - 1) * np.sqrt(6 / 64), "b1": np.zeros(64), "b2": np.zeros(64), "b3": np.zeros(1)}
    w = {k: v.astype(np.float32) for k, v in w.items()}
    w["W1"] = w["W1"].reshape(64, 32)
    w["W1"][:, 27:] = 0
    return ref.pack(w)


def test_mlp_initialisation_follows_its_recipe():
    m = csk.MLP(seed=5, max_batch=16)
    assert np.array_equal(m.params(), he_uniform_params(5))
    m.close()


def test_mlp_logits_and_gradients_match_reference():
    import torch
    rng = np.random.default_rng(8)
    w = ref.unpack(rng.normal(0, 0.25, ref.N_PARAMS).astype(np.float32))
    w["W1"][:, 27:] = 0
    p = ref.pack(w)
    m = csk.MLP(seed=5, max_batch=512)
    m.set_params(p)
    assert np.array_equal(m.params(), p)
    x = np.zeros((700, 32), np.float32)
    x[:, :27] = np.log1p(rng.poisson(3.0, (700, 27))).astype(np.float32)
    # scoring carries every operand as a hi + lo bf16 pair: the logits follow the unrounded
    # float32 forward pass, far inside the required 2e-2
    z = m.forward(dev(x)).cpu().numpy()                   # two chunks of at most 512 rows
    zr = ref.forward_fp32(p, x)
    assert np.max(np.abs(z - zr)) < 2e-2                   # the required tolerance
    assert np.max(np.abs(z - zr)) < 2e-3 * max(1.0, float(np.max(np.abs(zr))))
    y = (rng.random(512) < 0.3).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.train_step(dev(x[:512]), dev(y), 1e-3, loss)
    g = m.grads()
    gr = ref.gradients(p, x[:512], y)
    assert np.allclose(g, gr, rtol=2e-3, atol=1e-6)
    zr512 = ref.forward(p, x[:512])[0].astype(np.float64)
    want_loss = np.mean(np.maximum(zr512, 0) - zr512 * y + np.log1p(np.exp(-np.abs(zr512))))
    assert abs(loss.item() - want_loss) < 1e-4
    m.close()


def test_mlp_learns_a_separable_rule():
    # the training kernels descend: label = (feature 13 > 1) is learned to high accuracy
    import torch
    rng = np.random.default_rng(1)
    x = np.zeros((8192, 32), np.float32)
    x[:, :27] = rng.random((8192, 27)) * 2
    y = (x[:, 13] > 1.0).astype(np.float32)
    m = csk.MLP(seed=2, max_batch=1024)
    xd, yd = dev(x), dev(y)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for epoch in range(30):
        for b in range(0, 8192, 1024):
            m.train_step(xd[b:b + 1024], yd[b:b + 1024], 3e-3, loss)
        losses.append(loss.item())
    acc = ((m.forward(xd).cpu().numpy() > 0) == (y > 0.5)).mean()
    assert losses[-1] < 0.5 * losses[0] and acc > 0.95, (losses[0], losses[-1], acc)
    m.close()


def test_route_split_and_routed_topk_match_oracle():
    import torch
    L, delta, factor = 50.0, 0.25, 4          # fine 200^3, coarse 50^3
    pos = clustered(300_000, L, 9, frac=0.8, sigma=0.2)
    G, Gc = 200, 50
    k_all = oracle.keys(pos, delta, L)
    ix, iy, iz = k_all // np.uint64(G * G), (k_all // np.uint64(G)) % np.uint64(G), k_all % np.uint64(G)
    ck = ((ix // np.uint64(4)) * np.uint64(Gc) + iy // np.uint64(4)) * np.uint64(Gc) + iz // np.uint64(4)
    cu, cc = np.unique(ck, return_counts=True)
    admitted = np.sort(cu[np.argsort(-cc, kind="stable")[:40]]).astype(np.int64)   # 40 busiest coarse cells
    slots = 1 << 13
    tkeys = torch.full((slots,), -1, dtype=torch.int64, device="cuda")
    tcounts = torch.zeros(slots, dtype=torch.int32, device="cuda")
    rest = torch.empty((len(pos), 3), dtype=torch.float32, device="cuda")
    rcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    cut = 123_457                              # two calls: the table adds up, the rest appends
    csk.route_split(dev(pos[:cut]), delta, L, factor, dev(admitted), tkeys, tcounts, rest, rcount, err)
    csk.route_split(dev(pos[cut:]), delta, L, factor, dev(admitted), tkeys, tcounts, rest, rcount, err)
    torch.cuda.synchronize()
    assert err.item() == 0
    tk_ref, tc_ref, rest_ref = ref.route(pos, delta, L, factor, admitted.astype(np.uint64))
    tk = tkeys.cpu().numpy().view(np.uint64)
    tc = tcounts.cpu().numpy()
    full = tk != np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(tk[full])
    assert np.array_equal(tk[full][order], tk_ref) and np.array_equal(tc[full][order], tc_ref)
    nrest = int(rcount.item())
    assert nrest == len(rest_ref)
    assert np.array_equal(rest[:nrest].cpu().numpy(), rest_ref)    # stream order kept
    # the rest goes to a sketch; the top-k merges the table's exact counts with its estimates
    w, seed, theta, k = 9973, 4, 3, 400
    s = csk.Sketch(5, w, seed)
    s.update(rest[:nrest], delta, L)
    s.collect(rest[:nrest], delta, L, theta)
    keys, est, rc = csk.topk_with_table(s, tkeys, tcounts, k)
    M_ref, _ = oracle.sketch(rest_ref, 5, w, seed, delta, L, threads=8)
    assert np.array_equal(s.counters().cpu().numpy(), M_ref)
    kr, er = ref.topk_routed(tk_ref, tc_ref, M_ref, oracle.hash_tables(seed, 5), rest_ref, delta, L, theta, k)
    assert keys.cpu().numpy().view(np.uint64).tolist() == kr
    assert est.cpu().numpy().tolist() == er
    s.close()


@pytest.mark.parametrize("n", [0, 1, 777, 300_000])
def test_exact_counts_and_table_topk_match_oracle(n):
    import torch
    L, delta = 50.0, 0.25
    pos = clustered(n, L, 11 + n, frac=0.7, sigma=0.15)
    if n > 10:
        pos[5] = (3 * L, 1.0, 1.0)             # beyond the periodic wrap (|p| < 2L): skipped and flagged
    tk, tc = csk.new_table(1 << 20)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    cut = n // 3                               # two calls add into one table
    csk.exact_counts(dev(pos[:cut]), delta, L, tk, tc, err)
    csk.exact_counts(dev(pos[cut:]), delta, L, tk, tc, err)
    torch.cuda.synchronize()
    assert err.item() == (1 if n > 10 else 0)
    uniq, cnt = oracle.histogram(oracle.keys(pos, delta, L))
    keys = tk.cpu().numpy().view(np.uint64)
    full = keys != np.uint64(2 ** 64 - 1)
    order = np.argsort(keys[full])
    assert np.array_equal(keys[full][order], uniq) and np.array_equal(tc.cpu().numpy()[full][order], cnt)
    for k in (1, 100, 5000, len(uniq) + 5):
        gk, gc = csk.table_topk(tk, tc, k)
        rk, rc = oracle.topk_exact(uniq, cnt, k)
        assert gk.cpu().numpy().view(np.uint64).tolist() == rk.tolist()
        assert gc.cpu().numpy().tolist() == rc.tolist()


def test_exact_counts_flag_a_full_table():
    import torch
    pos = clustered(5000, 50.0, 2)
    tk, tc = csk.new_table(16)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    csk.exact_counts(dev(pos), 0.25, 50.0, tk, tc, err)
    torch.cuda.synchronize()
    assert err.item() == 2 and (tk.cpu().numpy() != -1).all()


def test_cell_list_and_labels_match_reference():
    import torch
    rng = np.random.default_rng(5)
    counts = np.where(rng.random(10 ** 6) < 0.02, rng.integers(1, 9, 10 ** 6), 0).astype(np.uint32)
    cd = dev(counts.view(np.int32))
    for mc in (1, 3, 9):
        got = csk.cell_list(cd, mc).cpu().numpy()
        assert np.array_equal(got, ref.cell_list(counts, mc))
    part = csk.cell_list(cd, 1, cap=1000).cpu().numpy()          # only the first cap are written
    assert np.array_equal(part, ref.cell_list(counts, 1)[:1000])
    assert csk.cell_list(dev(np.zeros(1000, np.int32)), 1).numel() == 0
    words = np.packbits(counts > 0, bitorder="little").view(np.uint32)   # 10^6 cells: whole words
    bm = dev(words.view(np.int32))
    for mc in (1, 3, 9):
        assert np.array_equal(csk.cell_list(cd, mc, bitmap=bm).cpu().numpy(), ref.cell_list(counts, mc))
    assert np.array_equal(csk.cell_list(cd, 2, cap=777, bitmap=bm).cpu().numpy(), ref.cell_list(counts, 2)[:777])
    buf = torch.empty(10, dtype=torch.int64, device="cuda")         # a caller's buffer grows as needed
    assert np.array_equal(csk.cell_list(cd, 3, out=buf).cpu().numpy(), ref.cell_list(counts, 3))
    # labels of coarse cells (mesh 100, factor 4 of the fine mesh 400) from fine keys
    cells = ref.cell_list(counts, 1)
    fine = rng.choice(400 ** 3, 3000, replace=False).astype(np.int64)
    fine[:50] = ref.parents(fine[:50], 400, 4) * 0     # a few keys share the first parent
    got = csk.cell_labels(dev(cells), dev(fine), 0.25, 100.0, 4).cpu().numpy()
    assert np.array_equal(got, ref.labels(cells, fine.astype(np.uint64), 400, 4))
    assert got.sum() > 0


@pytest.mark.parametrize("A", [1, 100, 512, 5003])
def test_route_admit_matches_reference(A):
    rng = np.random.default_rng(A)
    m = 5000
    cells = rng.choice(2 ** 40, m, replace=False).astype(np.int64)
    z = (rng.integers(-400, 400, m) / 64).astype(np.float32)    # many exact ties
    z[:10] = 0.0
    z[10:20] = -0.0
    z[20] = np.float32(3e38)
    z[21] = np.float32(-3e38)
    got = csk.route_admit(dev(cells), dev(z), A).cpu().numpy()
    assert np.array_equal(got, ref.admit(cells, z, A))


@pytest.mark.parametrize("n,na,factor", [(1, 3, 4), (8191, 0, 4), (8193, 17, 2), (2_000_000, 512, 4)])
def test_route_split_edges_match_oracle(n, na, factor):
    # ragged tiles, no admitted cells, another factor, and the largest admitted set
    import torch
    L, delta = 50.0, 0.25
    G = 200
    pos = clustered(n, L, 20 + na, frac=0.8, sigma=0.2)
    Gc = G // factor
    ck = ref.parents(oracle.keys(pos, delta, L), G, factor)
    cu, cc = np.unique(ck, return_counts=True)
    admitted = np.sort(cu[np.argsort(-cc, kind="stable")[:na]]).astype(np.int64)
    slots = 1 << 16
    tkeys, tcounts = csk.new_table(slots)
    rest = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    rcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    csk.route_split(dev(pos), delta, L, factor, dev(admitted), tkeys, tcounts, rest, rcount, err)
    torch.cuda.synchronize()
    assert err.item() == 0
    tk_ref, tc_ref, rest_ref = ref.route(pos, delta, L, factor, admitted.astype(np.uint64))
    tk = tkeys.cpu().numpy().view(np.uint64)
    full = tk != np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(tk[full])
    assert np.array_equal(tk[full][order], tk_ref)
    assert np.array_equal(tcounts.cpu().numpy()[full][order], tc_ref)
    assert int(rcount.item()) == len(rest_ref)
    assert np.array_equal(rest[:len(rest_ref)].cpu().numpy(), rest_ref)


def test_bitmap_bits_beyond_the_cells_are_ignored():
    # 1000 cells (the last bitmap word has 24 bits past the end, all set here): listing and
    # clearing touch only real cells; the counters sit at the front of a larger buffer whose
    # tail must stay untouched
    # (a bitmap at a 16-byte boundary takes the vector loads, one a word past it the scalar ones)
    import torch
    for off in (0, 1):
        buf = torch.full((1024,), 7, dtype=torch.int32, device="cuda")
        counts = buf[:1000]
        counts.zero_()
        counts[[3, 500, 999]] = torch.tensor([2, 5, 1], dtype=torch.int32, device="cuda")
        words = np.zeros(32, dtype=np.uint32)
        for c in (3, 500, 999):
            words[c // 32] |= np.uint32(1 << (c % 32))
        words[31] |= np.uint32(0xFFFFFF00)              # bits of cells 1000 .. 1023
        store = torch.zeros(32 + off, dtype=torch.int32, device="cuda")
        store[off:] = dev(words.view(np.int32))
        bm = store[off:]
        assert csk.cell_list(counts, 1, bitmap=bm).cpu().numpy().tolist() == [3, 500, 999]
        assert csk.cell_list(counts, 2, bitmap=bm).cpu().numpy().tolist() == [3, 500]
        csk.cells_clear(counts, bm)
        torch.cuda.synchronize()
        assert not counts.any().item() and not bm.any().item()
        assert (buf[1000:] == 7).all().item()


def test_trained_router_logits_match_the_fp32_reference():
    # the MLP trained on real features (two other-seed snapshots of the plain-at-scale
    # recipe, cut down) scores a third snapshot's cells; its split-bf16 logits stay within the
    # required 2e-2 of an unrounded float32 CPU forward pass on the same weights
    import torch
    import workloads
    from paper_1711_00975_amd.router import Router
    wl = workloads.SCALE.with_(L=250.0, n_halo=1 << 14)
    n = 1 << 22
    r = Router(wl.delta, wl.L, max_batch=4096)
    try:
        for seed in (2, 3):
            pos = workloads.DeviceGenerator(wl.with_(seed=seed)).generate(0, n)
            r.add_snapshot(pos, 2000, 1 << 24)
        info = r.train(epochs=3)
        assert info["positives"] > 0
        pos = workloads.DeviceGenerator(wl.with_(seed=1)).generate(0, n)
        cells, x = r.features(pos)
        z = r.mlp.forward(x).cpu().numpy()
        zr = ref.forward_fp32(r.mlp.params(), x.cpu().numpy())
        print("cells", len(z), "max |z - z_fp32|", float(np.max(np.abs(z - zr))), flush=True)
        assert len(z) > 1000
        assert np.max(np.abs(z - zr)) < 2e-2
    finally:
        r.close()
