"""The large combined run's pieces on a 2^24-particle subset, bit for bit against the oracle:
the device generator's stream, the three grids (0.25, 0.5, 1.0) updated as one batch, and the
routing split at the run's mesh."""
import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk
import workloads
from oracle import router as ref

pytestmark = pytest.mark.gpu

N_SUB = 1 << 24


def test_device_generator_follows_the_host_recipe():
    wl = workloads.LARGE
    gen = workloads.DeviceGenerator(wl)
    start, n = 12_345_678_901, 1 << 18          # any chunk: particles depend on (seed, index) only
    got = gen.generate(start, n).cpu().numpy()
    want = wl.generate(start, n)
    same = (got == want).all(axis=1).mean()
    assert same > 0.999, same                    # libm pow / sincos may differ in the last bit
    close = np.abs(got.astype(np.float64) - want).max()
    assert close < 1e-3, close
    assert ((got >= 0) & (got <= wl.L)).all()     # float32 rounding of x < L can reach L, as on the host


def test_three_grids_in_one_batch_match_oracle_on_a_subset():
    wl = workloads.LARGE
    pos = workloads.DeviceGenerator(wl).generate(0, N_SUB)
    host = pos.cpu().numpy()
    deltas = [0.25, 0.5, 1.0]
    sk = [csk.Sketch(wl.d, wl.w, wl.seed) for _ in deltas]
    b = csk.Batch(sk, [N_SUB // 2] * 3, deltas, [wl.L] * 3)
    half = N_SUB // 2                            # two calls, as chunks
    b.update([pos[:half]] * 3)
    b.update([pos[half:]] * 3)
    b.close()
    for s, dd in zip(sk, deltas):
        want, skipped = oracle.sketch(host, wl.d, wl.w, wl.seed, dd, wl.L, threads=8)
        assert skipped == 0
        assert np.array_equal(s.counters().cpu().numpy(), want), dd
        s.close()


def test_batch_rejects_meshes_with_different_floor_paths():
    a, b = csk.Sketch(5, 1 << 16, 1), csk.Sketch(5, 1 << 16, 2)
    with pytest.raises(csk.CskError):
        csk.Batch([a, b], [100, 100], [0.25, 0.3], [3000.0, 3000.0])   # ratio 4 and 10000
    a.close()
    b.close()


def test_routing_split_at_the_large_mesh_matches_oracle():
    import torch
    wl = workloads.LARGE
    n = 1 << 22
    pos = workloads.DeviceGenerator(wl.with_(seed=3)).generate(0, n)
    host = pos.cpu().numpy()
    G = round(wl.L / wl.delta)
    ck = ref.parents(oracle.keys(host, wl.delta, wl.L), G, 4)
    cu, cc = np.unique(ck, return_counts=True)
    admitted = np.sort(cu[np.argsort(-cc, kind="stable")[:512]]).astype(np.int64)
    tk, tc = csk.new_table(1 << 16)
    rest = torch.empty_like(pos)
    rcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    csk.route_split(pos, wl.delta, wl.L, 4, torch.from_numpy(admitted).cuda(), tk, tc, rest, rcount, err)
    torch.cuda.synchronize()
    assert err.item() == 0
    tk_ref, tc_ref, rest_ref = ref.route(host, wl.delta, wl.L, 4, admitted.astype(np.uint64))
    keys = tk.cpu().numpy().view(np.uint64)
    full = keys != np.uint64(2 ** 64 - 1)
    order = np.argsort(keys[full])
    assert np.array_equal(keys[full][order], tk_ref) and np.array_equal(tc.cpu().numpy()[full][order], tc_ref)
    assert int(rcount.item()) == len(rest_ref)
    assert np.array_equal(rest[:len(rest_ref)].cpu().numpy(), rest_ref)
