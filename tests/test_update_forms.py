"""Every tiling of the binned update gives the oracle's counters (Sec. 2.2 Add; Alg. 4
Update): the bin kernel forms (general row-interleaved, sort-word on the packed table or on
the row tables), workgroup sizes, rows per LDS pass and prefetch differ only in speed, so
each is checked bit for bit on streams with several tiles per workgroup and a ragged tail,
on the region-overflow path, for the Count-Min variant, for every d the sort-word kernel
serves, and in a batch."""
import numpy as np
import pytest

import oracle
import paper_1711_00975_amd as csk

pytestmark = pytest.mark.gpu

# (form, threads, rows per pass, prefetch)
FORMS = [
    (csk.CSK_BIN_GENERAL, 0, 0, 0),
    (csk.CSK_BIN_SORT_WORD, 1024, 2, 1),
    (csk.CSK_BIN_SORT_WORD, 1024, 3, 1),
    (csk.CSK_BIN_SORT_WORD, 512, 2, 2),
    (csk.CSK_BIN_SORT_WORD, 512, 3, 2),
    (csk.CSK_BIN_SORT_WORD, 512, 3, 1),
    (csk.CSK_BIN_AUTO, 0, 0, 0),
]


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


def _counters(pos, d, w, seed, delta, L, form, variant=0, max_wg=0):
    s = csk.Sketch(d, w, seed, variant)
    try:
        s.set_update_tiling(*form)
        if max_wg:
            s.set_update_plan(csk.CSK_UPDATE_BINNED, max_wg)
        s.update(_dev(pos), delta, L)
        return s.counters().cpu().numpy()
    finally:
        s.close()


@pytest.mark.parametrize("form", FORMS)
def test_forms_multi_tile_ragged_at_the_scale_width(form):
    # w = 2^24 (512 slices per row), 16 workgroups: about 19 tiles each and a ragged last tile
    print("form", form, flush=True)
    n, d, w, L, delta, seed = 2_500_001, 5, 1 << 24, 1000.0, 0.25, 3
    pos = _clustered(n, L, 51, nclump=400, sigma=0.3)
    M = _counters(pos, d, w, seed, delta, L, form, max_wg=16)
    Mo, skipped = oracle.sketch(pos, d, w, seed, delta, L, threads=8)
    assert skipped == 0
    assert np.array_equal(M, Mo)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("d,w,L,delta,variant", [(5, 1 << 16, 100.0, 0.1, 0), (6, 1 << 20, 1000.0, 0.25, 0),
                                                 (7, 1 << 17, 3000.0, 1.0, 1), (8, 1 << 15, 7.0, 0.7, 0),
                                                 (8, 1 << 14, 123.456, 0.123456, 1)])
def test_forms_every_d_and_mesh(form, d, w, L, delta, variant):
    print("form", form, d, w, L, delta, variant, flush=True)
    pos = _clustered(300_007, L, 52 + d)
    M = _counters(pos, d, w, 11, delta, L, form, variant=variant, max_wg=8)
    Mo, _ = oracle.sketch(pos, d, w, 11, delta, L, variant=variant, threads=8)
    assert np.array_equal(M, Mo)
    if variant == 1:
        assert np.all(M.astype(np.int64).sum(axis=1) == len(pos))


@pytest.mark.parametrize("form", FORMS)
def test_forms_one_cell_overflows_regions(form):
    # every particle in one cell: one slice per row takes every token, far above the
    # region capacity, so most tokens take the overflow path
    print("form overflow", form, flush=True)
    n = 300_000
    pos = np.full((n, 3), 12.34, dtype=np.float32)
    M = _counters(pos, 5, 1 << 16, 3, 0.1, 100.0, form)
    Mo, _ = oracle.sketch(pos, 5, 1 << 16, 3, 0.1, 100.0)
    assert np.array_equal(M, Mo)
    assert sorted(np.abs(M).max(axis=1).tolist()) == [n] * 5


def test_tiling_arguments_are_checked():
    s = csk.Sketch(5, 1 << 16, 1)
    try:
        for bad in [(7, 0, 0, 0), (2, 256, 0, 0), (2, 0, 4, 0), (2, 0, 0, 3), (2, 1024, 0, 2)]:
            with pytest.raises(csk.CskError) as ei:
                s.set_update_tiling(*bad)
            assert ei.value.code == csk.CSK_E_INVALID
    finally:
        s.close()


@pytest.mark.parametrize("form", [FORMS[0], FORMS[2], FORMS[4]])
def test_forms_in_a_batch(form):
    # a batch takes the first sketch's tiling for all of its sketches
    print("batch form", form, flush=True)
    import torch
    specs = [(150_000, 1 << 14, 61), (90_001, 1 << 16, 62), (400_000, 1 << 20, 63), (1, 1 << 15, 64)]
    sk = [csk.Sketch(5, w, seed) for _, w, seed in specs]
    try:
        sk[0].set_update_tiling(*form)
        pos = [_clustered(n, 100.0, seed) for n, _, seed in specs]
        b = csk.Batch(sk, [n for n, _, _ in specs], 0.1, 100.0)
        try:
            b.update([_dev(p) for p in pos])
            torch.cuda.synchronize()
        finally:
            b.close()
        for (n, w, seed), s, p in zip(specs, sk, pos):
            Mo, _ = oracle.sketch(p, 5, w, seed, 0.1, 100.0)
            assert np.array_equal(s.counters().cpu().numpy(), Mo), (n, w)
    finally:
        for s in sk:
            s.close()


# The sort-word kernel on the row tables (multiply-high buckets): widths that are not powers
# of two, and powers of two too wide for the packed fields (d = 6: 2^21 > 2^(21 - 1)).
ROW_FORMS = [
    (csk.CSK_BIN_GENERAL, 0, 0, 0),
    (csk.CSK_BIN_SORT_WORD, 1024, 2, 1),
    (csk.CSK_BIN_SORT_WORD, 1024, 3, 1),
    (csk.CSK_BIN_AUTO, 0, 0, 0),
]


@pytest.mark.parametrize("form", ROW_FORMS)
@pytest.mark.parametrize("d,w,L,delta,variant", [(5, 3 * (1 << 20) + 5, 1000.0, 0.25, 0),
                                                 (5, (1 << 24) - 1, 1000.0, 0.25, 1),
                                                 (6, 1 << 21, 123.456, 0.123456, 0),
                                                 (7, 999_999, 100.0, 1.0 / 3.0, 1),
                                                 (8, (1 << 24) - 3, 3000.0, 1.0, 0),
                                                 (5, 9973 * 7, 50.0, 0.25, 0)])
def test_row_table_forms(form, d, w, L, delta, variant):
    print("row form", form, d, w, L, delta, variant, flush=True)
    pos = _clustered(1_200_007, L, 61 + d, nclump=200, sigma=0.3)
    M = _counters(pos, d, w, 13, delta, L, form, variant=variant, max_wg=8)
    Mo, skipped = oracle.sketch(pos, d, w, 13, delta, L, variant=variant, threads=8)
    assert skipped == 0
    assert np.array_equal(M, Mo)


@pytest.mark.parametrize("form", ROW_FORMS[1:3])
def test_row_table_forms_one_cell_overflows_regions(form):
    print("row form overflow", form, flush=True)
    n, w = 300_000, (1 << 21) + 77
    pos = np.full((n, 3), 12.34, dtype=np.float32)
    M = _counters(pos, 5, w, 3, 0.1, 100.0, form)
    Mo, _ = oracle.sketch(pos, 5, w, 3, 0.1, 100.0)
    assert np.array_equal(M, Mo)
    assert sorted(np.abs(M).max(axis=1).tolist()) == [n] * 5
