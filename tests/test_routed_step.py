"""GPU parity of the routed step without host synchronization: the device-count listing
(csk_cell_list_async), the fused features + fp32 scoring (csk_route_score), admission over a
device count (csk_route_admit_async), the split fused into the rest sketch's update
(csk_sketch_update_routed: counters and exact table bit for bit against the oracle's route
followed by Sec. 2.2 Add of the rest), the merged top-k without a host readback
(csk_topk_with_table_async), and the whole step eagerly and replayed in a HIP graph."""
import numpy as np
import pytest

import oracle
from oracle import router as ref
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu

INT32_MIN = csk.INT32_MIN


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def clustered(n, L, seed, frac=0.7, sigma=0.2, nclump=10):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (nclump, 3))
    clump = centres[rng.integers(0, nclump, n)] + rng.normal(0, sigma, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < frac)[:, None], clump, bg)
    pos = np.mod(pos, L).astype(np.float32)
    pos[pos >= L] = 0.0
    return pos


def random_params(seed):
    rng = np.random.default_rng(seed)
    w = ref.unpack(rng.normal(0, 0.25, ref.N_PARAMS).astype(np.float32))
    return ref.pack(w)


def busiest(pos, delta, L, G, factor, na):
    ck = ref.parents(oracle.keys(pos, delta, L), G, factor)
    cu, cc = np.unique(ck, return_counts=True)
    return np.sort(cu[np.argsort(-cc, kind="stable")[:na]]).astype(np.int64)


def test_cell_list_async_matches_reference():
    import torch
    rng = np.random.default_rng(15)
    counts = np.where(rng.random(10 ** 6) < 0.02, rng.integers(1, 9, 10 ** 6), 0).astype(np.uint32)
    cd = dev(counts.view(np.int32))
    words = np.packbits(counts > 0, bitorder="little").view(np.uint32)
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    wd = dev(words.view(np.int32))
    padded = torch.zeros(wd.numel() + 1, dtype=torch.int32, device="cuda")
    padded[1:] = wd                                      # a bitmap one word past a 16-byte boundary
    for bm in (None, wd, padded[1:]):
        for mc, cap in ((1, 30_000), (3, 50), (9, 1 << 16)):
            out = torch.full((cap,), -7, dtype=torch.int64, device="cuda")
            csk.cell_list_async(cd, out, total, mc, bitmap=bm)
            want = ref.cell_list(counts, mc)
            torch.cuda.synchronize()
            assert int(total.item()) == len(want)
            got = out.cpu().numpy()
            k = min(cap, len(want))
            assert np.array_equal(got[:k], want[:k])
            assert (got[k:] == -7).all()                       # nothing written past the list
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    csk.cell_list_async(dev(np.zeros(1000, np.int32)), out, total)
    torch.cuda.synchronize()
    assert int(total.item()) == 0


def test_route_score_matches_the_fp32_forward_pass():
    import torch
    L, dc = 100.0, 1.0
    Gc = 100
    pos = clustered(2_000_000, L, 3)
    counts = torch.zeros(Gc ** 3, dtype=torch.int32, device="cuda")
    csk.sample_counts(dev(pos), dc, L, 5, counts)
    cells = csk.cell_list(counts, 1)
    m = cells.numel()
    assert m > 5000
    p = random_params(7)
    mlp = csk.MLP(seed=1)
    mlp.set_params(p)
    cap = m + 100
    buf = torch.zeros(cap, dtype=torch.int64, device="cuda")
    buf[:m] = cells
    z = torch.full((cap,), float("nan"), dtype=torch.float32, device="cuda")
    cut = m - 333                                              # only the first *m cells are scored
    mdev = torch.tensor([cut], dtype=torch.int64, device="cuda")
    csk.route_score(mlp, counts, dc, L, buf, mdev, z)
    torch.cuda.synchronize()
    zc = z.cpu().numpy()
    cnp = cells.cpu().numpy()
    x = ref.features(counts.cpu().numpy().view(np.uint32), Gc, cnp[:cut])
    zr = ref.forward_fp32(p, x)
    # every layer sums at most 64 fp32 products: within a few hundred ulps of the logit scale
    assert np.max(np.abs(zc[:cut] - zr)) <= 1e-4 * max(1.0, float(np.max(np.abs(zr))))
    assert np.isnan(zc[cut:]).all()
    # and the model's own matrix-core forward pass (split bf16) agrees with it
    zm = mlp.forward(csk.cell_features(counts, dc, L, cells[:cut])).cpu().numpy()
    assert np.max(np.abs(zm - zr)) < 2e-3 * max(1.0, float(np.max(np.abs(zr))))
    mlp.close()


@pytest.mark.parametrize("A,m", [(1, 5000), (100, 5000), (512, 5000), (700, 300), (64, 0)])
def test_route_admit_async_matches_reference(A, m):
    import torch
    rng = np.random.default_rng(A + m)
    cap = 6000
    cells = np.zeros(cap, dtype=np.int64)
    cells[:cap] = rng.choice(2 ** 40, cap, replace=False)
    z = (rng.integers(-400, 400, cap) / 64).astype(np.float32)    # many exact ties
    z[:10] = 0.0
    z[10:20] = -0.0
    z[20] = np.float32(3e38)
    z[21] = np.float32(-3e38)
    admitted = torch.full((A,), -5, dtype=torch.int64, device="cuda")
    na = torch.full((1,), 99999, dtype=torch.int32, device="cuda")
    mdev = torch.tensor([m], dtype=torch.int64, device="cuda")
    csk.route_admit_async(dev(cells), dev(z), mdev, A, admitted, na)
    torch.cuda.synchronize()
    want = ref.admit(cells[:m], z[:m], A)
    assert int(na.item()) == len(want)
    assert np.array_equal(admitted.cpu().numpy()[:len(want)], want)


# (d, w, L, delta, factor, na, n, plan): the general bin kernel (the default, or asked for)
# and the sort-word kernel on the row tables (asked for), each
# with each hash form (w not a power of two; a power of two) and each mesh form
# (power-of-two ratio G / L, general, exact ratio 3), another factor, the direct update for
# d != 5 and when asked for, no admitted cell, the most admitted cells, ragged and empty
# streams
ROUTED = [
    (5, (1 << 22) - 39322, 100.0, 0.25, 4, 512, 2_000_003, "sortword"),
    (5, 1 << 22, 100.0, 0.25, 4, 100, 1_000_000, "sortword"),
    (5, (1 << 22) - 39322, 100.0, 0.25, 4, 512, 2_000_003, "general"),
    (5, 9973 * 7, 50.0, 0.25, 4, 40, 300_001, "sortword"),
    (5, 1 << 16, 123.456, 0.123456, 4, 40, 200_000, "sortword"),
    (5, 1 << 16, 100.0, 1.0 / 3.0, 3, 40, 200_000, "sortword"),
    (5, 1 << 16, 50.0, 0.25, 4, 0, 100_000, "sortword"),
    (5, 1 << 16, 50.0, 0.25, 4, 5, 0, "sortword"),
    (5, 9973 * 7, 50.0, 0.25, 4, 40, 300_001, "auto"),
    (5, 1 << 16, 50.0, 0.25, 4, 40, 250_000, "auto"),
    (5, 1 << 15, 64.0, 0.25, 2, 100, 200_000, "auto"),
    (5, 1 << 16, 123.456, 0.123456, 4, 40, 200_000, "auto"),
    (5, 1 << 16, 100.0, 1.0 / 3.0, 3, 40, 200_000, "auto"),
    (5, 1 << 16, 50.0, 0.25, 4, 0, 100_000, "auto"),
    (5, 1 << 16, 50.0, 0.25, 4, 17, 8193, "auto"),
    (5, 1 << 16, 50.0, 0.25, 4, 512, 1_000_000, "auto"),
    (3, 12_345, 50.0, 0.25, 4, 30, 150_000, "auto"),
    (5, 1 << 16, 50.0, 0.25, 4, 30, 150_000, "direct"),
    (5, 1 << 16, 50.0, 0.25, 4, 5, 0, "auto"),
]


@pytest.mark.parametrize("d,w,L,delta,factor,na,n,plan", ROUTED)
def test_update_routed_matches_route_then_add(d, w, L, delta, factor, na, n, plan):
    import torch
    print("routed update", d, w, L, delta, factor, na, n, plan, flush=True)
    G = int(round(L / delta))
    pos = clustered(n, L, 40 + na + d, frac=0.8)
    admitted = busiest(pos, delta, L, G, factor, na) if n else np.arange(na, dtype=np.int64) * 7
    seed = 11
    s = csk.Sketch(d, w, seed)
    if plan == "direct":
        s.set_update_plan(csk.CSK_UPDATE_DIRECT, 0)
    elif plan == "general":
        s.set_update_tiling(csk.CSK_BIN_GENERAL)
    elif plan == "sortword":
        s.set_update_tiling(csk.CSK_BIN_SORT_WORD)
    slots = 1 << 16
    tk, tc = csk.new_table(slots)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    adm = torch.full((max(na, 1),), -1, dtype=torch.int64, device="cuda")
    adm[:na] = dev(admitted) if na else adm[:0]
    nadev = torch.tensor([na], dtype=torch.int32, device="cuda")
    pd = dev(pos) if n else torch.empty((0, 3), dtype=torch.float32, device="cuda")
    csk.update_routed(s, pd, delta, L, factor, adm, nadev, tk, tc, err)
    torch.cuda.synchronize()
    assert err.item() == 0
    tk_ref, tc_ref, rest_ref = ref.route(pos, delta, L, factor, admitted.astype(np.uint64))
    M_ref, _ = oracle.sketch(rest_ref, d, w, seed, delta, L, threads=8)
    assert np.array_equal(s.counters().cpu().numpy(), M_ref)
    keys = tk.cpu().numpy().view(np.uint64)
    full = keys != np.uint64(2 ** 64 - 1)
    order = np.argsort(keys[full])
    assert np.array_equal(keys[full][order], tk_ref)
    assert np.array_equal(tc.cpu().numpy()[full][order], tc_ref)
    s.close()


def test_update_routed_flags_too_many_admitted_cells():
    # *na above what the exclusion serves (factor 4: 512 cells) is clamped and flagged
    import torch
    L, delta, factor = 50.0, 0.25, 4
    pos = clustered(50_000, L, 2)
    admitted = busiest(pos, delta, L, 200, factor, 600)
    s = csk.Sketch(5, 1 << 16, 3)
    tk, tc = csk.new_table(1 << 16)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    nadev = torch.tensor([len(admitted)], dtype=torch.int32, device="cuda")
    csk.update_routed(s, dev(pos), delta, L, factor, dev(admitted), nadev, tk, tc, err)
    torch.cuda.synchronize()
    assert err.item() == 4
    used = admitted[:512]          # the first 512 of the list are excluded, as documented
    tk_ref, tc_ref, rest_ref = ref.route(pos, delta, L, factor, used.astype(np.uint64))
    M_ref, _ = oracle.sketch(rest_ref, 5, 1 << 16, 3, delta, L, threads=8)
    assert np.array_equal(s.counters().cpu().numpy(), M_ref)
    s.close()


def _oracle_step(pos, r, cells_dev, logits_dev, m, w_rest, seed, theta, k):
    """The oracle's routed step on the GPU's scored cells: admission by the same fp32 logits
    (a decision taken in one precision on both sides), then route, Add and the merged top-k."""
    cells = cells_dev.cpu().numpy()[:m]
    z = logits_dev.cpu().numpy()[:m]
    admitted = ref.admit(cells, z, r.max_admit)
    tk, tc, rest = ref.route(pos, r.delta, r.L, r.factor, admitted.astype(np.uint64))
    M, _ = oracle.sketch(rest, 5, w_rest, seed, r.delta, r.L, threads=8)
    kr, er = ref.topk_routed(tk, tc, M, oracle.hash_tables(seed, 5), rest, r.delta, r.L, theta, k)
    return admitted, M, kr, er


def test_routed_step_eager_and_in_a_hip_graph():
    import torch
    from paper_1711_00975_amd.router import Router, RoutedStep
    L, delta = 100.0, 0.25
    pos = clustered(1_500_000, L, 21, frac=0.75, sigma=0.3, nclump=40)
    r = Router(delta, L, delta_c=1.0, table_slots=1 << 16, max_admit=64)
    r.mlp.set_params(random_params(3))
    w_rest, seed, theta, k = 50_021, 9, 4, 300
    rest = csk.Sketch(5, w_rest, seed)
    step = RoutedStep(r, rest, k, max_cells=1 << 18)
    pd = dev(pos)
    try:
        print("routed step eager", flush=True)
        step.run(pd, theta)
        torch.cuda.synchronize()
        m = int(step.m.item())
        assert 100 < m <= step.cells.numel()
        # the scored cells are the oracle's listing of the oracle's sample
        counts = ref.sample_counts(pos, 1.0, L, r.sample_seed)
        assert np.array_equal(step.cells.cpu().numpy()[:m], ref.cell_list(counts, r.min_count))
        admitted, M, kr, er = _oracle_step(pos, r, step.cells, step.logits, m, w_rest, seed, theta, k)
        na = int(step.na.item())
        assert na == len(admitted) == 64
        assert np.array_equal(step.admitted.cpu().numpy()[:na], admitted)
        assert np.array_equal(rest.counters().cpu().numpy(), M)
        keys, est, partial = step.result()
        assert keys.cpu().numpy().view(np.uint64).tolist() == kr
        assert est.cpu().numpy().tolist() == er
        assert step.err.item() == 0
        want = (keys.cpu().numpy().copy(), est.cpu().numpy().copy())
        print("routed step graph", flush=True)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step.run(pd, theta)
        for rep in range(3):
            rest.update(pd[:1000], delta, L)        # eager work between replays
            step.out.zero_()
            step.na.fill_(-1)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            keys, est, _ = step.result()
            assert np.array_equal(keys.cpu().numpy(), want[0]), rep
            assert np.array_equal(est.cpu().numpy(), want[1]), rep
            assert int(step.na.item()) == 64
            assert np.array_equal(rest.counters().cpu().numpy(), M), rep
        del g
    finally:
        rest.close()
        r.close()
