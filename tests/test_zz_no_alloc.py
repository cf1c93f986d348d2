"""The no-allocation update (csk_sketch_update_noalloc) against csk_sketch_update.

Both entry points add the same stream to a handle of the same seed; the counters are
integer results of one fully specified computation, so they must agree bit for bit
after every call.  The scratch is shared by every call on the device and keeps the
last call's contents, so the second call is smaller than the first: stale tokens of
the first call must not leak into the second.
"""
import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("d,w,L,delta", [(5, 1 << 20, 1000.0, 0.25), (5, 1 << 16, 100.0, 0.1),
                                         (3, 100_003, 123.456, 0.123456)])
def test_noalloc_update_matches_update_on_two_calls(d, w, L, delta):
    print("noalloc vs update", d, w, L, delta, flush=True)
    p1 = _clustered(3_000_000, L, 11)
    p2 = _clustered(400_000, L, 12)
    ref = csk.Sketch(d, w, 5)
    na = csk.Sketch(d, w, 5)
    try:
        t1, t2 = _dev(p1), _dev(p2)
        ref.update(t1, delta, L)
        na.update_noalloc(t1, delta, L)
        a1, b1 = ref.counters().cpu().numpy(), na.counters().cpu().numpy()
        assert np.array_equal(a1, b1), "first call: counters differ"
        ref.update(t2, delta, L)
        na.update_noalloc(t2, delta, L)
        a2, b2 = ref.counters().cpu().numpy(), na.counters().cpu().numpy()
        assert np.array_equal(a2, b2), "second (smaller) call: counters differ"
        assert not np.array_equal(a1, a2)
    finally:
        ref.close()
        na.close()


def test_noalloc_update_matches_oracle_on_a_fresh_handle():
    print("noalloc vs oracle", flush=True)
    d, w, L, delta = 5, 1 << 16, 100.0, 0.1
    pos = _clustered(250_000, L, 21)
    s = csk.Sketch(d, w, 3)
    try:
        s.update_noalloc(_dev(pos), delta, L)
        M = s.counters().cpu().numpy()
    finally:
        s.close()
    Mo, skipped = oracle.sketch(pos, d, w, 3, delta, L)
    assert skipped == 0
    assert np.array_equal(M, Mo)


def test_noalloc_update_refuses_a_stream_beyond_its_scratch():
    print("noalloc refusal", flush=True)
    d, w, L, delta = 5, 1 << 20, 1000.0, 0.25
    s = csk.Sketch(d, w, 5)
    try:
        big = _dev(_clustered(1 << 24, L, 31))
        with pytest.raises(csk.CskError) as ei:
            s.update_noalloc(big, delta, L)
        assert ei.value.code == csk.CSK_E_CAPACITY
        assert not s.counters().cpu().numpy().any(), "a refused call changed the counters"
        # the handle still works, and a stream that fits goes through
        small = _clustered(100_000, L, 32)
        s.update_noalloc(_dev(small), delta, L)
        Mo, _ = oracle.sketch(small, d, w, 5, delta, L)
        assert np.array_equal(s.counters().cpu().numpy(), Mo)
    finally:
        s.close()
