"""GPU parity of the candidate pass through the field-probe Bloom filter at widths that are
not powers of two (d = 5, w <= 2^24): the filter is keyed by P-bit prefixes of the bucket
input (w <= 2^P < 2w), and a hot bucket enters every prefix that can reach it.  A missed
prefix would drop a candidate, so the top-k (Sec. 2.2 UpdateHeap over the candidates of
Sec. 3.1 item 4) is compared with the oracle's bit for bit, for both variants and for
thresholds from light to heavy, at widths with 1-3 prefixes per bucket."""
import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def clustered(n, L, seed, frac=0.75, sigma=0.12, nclump=24):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, L, (nclump, 3))
    clump = centres[rng.integers(0, nclump, n)] + rng.normal(0, sigma, (n, 3))
    bg = rng.uniform(0, L, (n, 3))
    pos = np.where((rng.random(n) < frac)[:, None], clump, bg)
    pos = np.mod(pos, L).astype(np.float32)
    pos[pos >= L] = 0.0
    return pos


# widths: 9973 * 7 (P = 17), 2^16 + 1 (P = 17, two prefixes per bucket), the router's rest
# width 2^22 - 39 322 (P = 22), 3 * 2^20 + 5 (P = 22), 2^24 - 1 (P = 24), and 2^16 (the
# power-of-two form, one prefix per bucket)
WIDTHS = [9973 * 7, (1 << 16) + 1, (1 << 22) - 39322, 3 * (1 << 20) + 5, (1 << 24) - 1, 1 << 16]


@pytest.mark.parametrize("w", WIDTHS)
@pytest.mark.parametrize("variant", [csk.CSK_VARIANT_COUNT_SKETCH, csk.CSK_VARIANT_COUNT_MIN])
def test_field_filter_topk_matches_oracle(w, variant):
    print("field filter", w, variant, flush=True)
    L, delta, seed, k = 50.0, 0.25, 17, 300
    pos = clustered(1_500_000, L, 5 + w % 97)
    pd = dev(pos)
    s = csk.Sketch(5, w, seed, variant=variant)
    try:
        s.update(pd, delta, L)
        M, _ = oracle.sketch(pos, 5, w, seed, delta, L, variant=variant, threads=8)
        assert np.array_equal(s.counters().cpu().numpy(), M)
        T = oracle.hash_tables(seed, 5)
        for theta in (2, 9, 40, 200):
            s.clear_candidates()
            s.collect(pd, delta, L, theta)
            keys, est, rc = s.topk(k)
            ko, eo, st = oracle.topk_sketch(M, T, pos, delta, L, theta, k, variant=variant)
            got = keys.cpu().numpy().view(np.uint64)
            assert np.array_equal(got, ko), (w, variant, theta)
            assert np.array_equal(est.cpu().numpy(), eo), (w, variant, theta)
            assert (rc == csk.CSK_W_INCOMPLETE) == (st == oracle.W_INCOMPLETE), (w, variant, theta)
    finally:
        s.close()
