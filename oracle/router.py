"""CPU reference of the learned router (test infrastructure only).

The router is the second further form of the hot path: a 1 % sample of the stream gives
coarse cell counts; a 27 -> 64 -> 64 -> 1 MLP scores coarse cells from the counts of the
cell and its 26 neighbours; the highest-scored coarse cells are counted exactly and every
other particle is added to a Count Sketch (Sec. 2.2 Add) of the remaining memory.

Plain numpy, float32 where the GPU computes in float32 and with the GPU's bf16 rounding of
matrix operands (round to nearest even), so the comparison measures only summation order.
Nothing here is imported by the product library.
"""
from __future__ import annotations

import numpy as np

import workloads
from . import estimate, keys

SAMPLE_STREAM = 4
SAMPLE_THRESHOLD = 42949672     # floor(0.01 * 2^32)
HIDDEN, FEAT = 64, 32
OFF = {"W1": (0, (64, 32)), "b1": (2048, (64,)), "W2": (2112, (64, 64)), "b2": (6208, (64,)),
       "w3": (6272, (64,)), "b3": (6336, (1,))}
N_PARAMS = 6337


def unpack(p):
    p = np.asarray(p, dtype=np.float32)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in OFF.items()}


def pack(d):
    p = np.zeros(N_PARAMS, dtype=np.float32)
    for k, (o, s) in OFF.items():
        p[o:o + int(np.prod(s))] = np.asarray(d[k], dtype=np.float32).ravel()
    return p


def bf16(x):
    """float32 -> nearest bf16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


# ---------------------------------------------------------------- sample and features

def sample_mask(n, seed, index0=0, threshold=SAMPLE_THRESHOLD):
    """Particle g = index0 + i is sampled when word g of the Philox stream 4 (word g mod 4 of
    counter g / 4) is below threshold."""
    return workloads.philox_words(index0, n, SAMPLE_STREAM, seed) < np.uint32(threshold)


def sample_counts(pos, delta_c, L, seed, index0=0, threshold=SAMPLE_THRESHOLD):
    """Coarse counts (uint32 [G_c^3]) of the sampled, in-domain particles."""
    Gc = int(round(L / delta_c))
    m = sample_mask(len(pos), seed, index0, threshold)
    k = keys(pos[m], delta_c, L)
    return np.bincount(k.astype(np.int64), minlength=Gc ** 3).astype(np.uint32)


def features(counts, Gc, cells):
    """[m][32] float32: log1p counts of each cell's 27 periodic neighbours, (dx, dy, dz)
    lexicographic, then 5 zeros."""
    cells = np.asarray(cells, dtype=np.int64)
    cx, cy, cz = cells // (Gc * Gc), (cells // Gc) % Gc, cells % Gc
    out = np.zeros((len(cells), FEAT), dtype=np.float32)
    q = 0
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nb = (((cx + dx) % Gc) * Gc + (cy + dy) % Gc) * Gc + (cz + dz) % Gc
                out[:, q] = np.log1p(counts[nb].astype(np.float32))
                q += 1
    return out


# ---------------------------------------------------------------- the model

def forward(p, x):
    """Logits and the activations (H1, H2) with the GPU's bf16 operand rounding."""
    w = unpack(p)
    h1 = np.maximum(bf16(x) @ bf16(w["W1"]).T + w["b1"], 0).astype(np.float32)
    h2 = np.maximum(bf16(h1) @ bf16(w["W2"]).T + w["b2"], 0).astype(np.float32)
    z = (bf16(h2) @ bf16(w["w3"]) + w["b3"][0]).astype(np.float32)
    return z, h1, h2


def forward_fp32(p, x):
    """Logits in plain float32 with no bf16 rounding anywhere: the CPU FP32 reference the
    bf16-operand MLP is held to (within 2e-2 absolute)."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float32)
    h1 = np.maximum(x @ w["W1"].T + w["b1"], np.float32(0)).astype(np.float32)
    h2 = np.maximum(h1 @ w["W2"].T + w["b2"], np.float32(0)).astype(np.float32)
    return (h2 @ w["w3"] + w["b3"][0]).astype(np.float32)


def gradients(p, x, y):
    """Gradients of the mean binary cross-entropy, with the GPU's roundings: dz, dw3, db3,
    db2, db1 in float32; dW2, the back-propagated dA1 and dW1 from bf16-rounded operands."""
    w = unpack(p)
    z, h1, h2 = forward(p, x)
    n = len(x)
    dz = ((1.0 / (1.0 + np.exp(-z.astype(np.float64)))) - y) / n
    dz = dz.astype(np.float32)
    g = {"w3": dz @ h2, "b3": np.array([dz.sum()], np.float32)}
    dA2 = np.where(h2 > 0, np.outer(dz, w["w3"]), 0).astype(np.float32)
    g["W2"] = bf16(dA2).T @ bf16(h1)
    g["b2"] = dA2.sum(axis=0)
    dA1 = np.where(h1 > 0, bf16(dA2) @ bf16(w["W2"]), 0).astype(np.float32)
    g["W1"] = bf16(dA1).T @ bf16(x)
    g["b1"] = dA1.sum(axis=0)
    return pack(g)


def forward_loops_exact(p, x):
    """forward_fp32 as explicit float64 loops over neurons, no rounding of any operand (an
    independent check of `forward_fp32` on small inputs)."""
    w = unpack(p)
    W1, W2, w3 = (w[k].astype(np.float64) for k in ("W1", "W2", "w3"))
    out = []
    for row in np.asarray(x, dtype=np.float32).astype(np.float64):
        h1 = [max(0.0, sum(W1[j, k] * row[k] for k in range(FEAT)) + float(w["b1"][j])) for j in range(HIDDEN)]
        h2 = [max(0.0, sum(W2[j, k] * h1[k] for k in range(HIDDEN)) + float(w["b2"][j])) for j in range(HIDDEN)]
        out.append(sum(w3[j] * h2[j] for j in range(HIDDEN)) + float(w["b3"][0]))
    return np.array(out)


def forward_loops(p, x):
    """The same forward pass as explicit float64 loops over neurons (an independent check of
    `forward` on small inputs)."""
    w = unpack(p)
    W1, W2, w3 = (bf16(w[k]).astype(np.float64) for k in ("W1", "W2", "w3"))
    out = []
    for row in np.asarray(x, dtype=np.float32):
        xr = bf16(row).astype(np.float64)
        h1 = np.array([max(0.0, sum(W1[j, k] * xr[k] for k in range(FEAT)) + float(w["b1"][j]))
                       for j in range(HIDDEN)], np.float32)
        h1r = bf16(h1).astype(np.float64)
        h2 = np.array([max(0.0, sum(W2[j, k] * h1r[k] for k in range(HIDDEN)) + float(w["b2"][j]))
                       for j in range(HIDDEN)], np.float32)
        h2r = bf16(h2).astype(np.float64)
        out.append(sum(w3[j] * h2r[j] for j in range(HIDDEN)) + float(w["b3"][0]))
    return np.array(out)


# ---------------------------------------------------------------- routing

def route(pos, delta, L, factor, admitted):
    """(table keys, table counts) of the particles whose coarse parent is admitted, sorted by
    key, and the positions of the rest (stream order)."""
    G = int(round(L / delta))
    k = keys(pos, delta, L)
    assert len(k) == len(pos), "the reference expects an in-domain stream"
    Gc = G // factor
    ix, iy, iz = k // np.uint64(G * G), (k // np.uint64(G)) % np.uint64(G), k % np.uint64(G)
    ck = ((ix // np.uint64(factor)) * np.uint64(Gc) + iy // np.uint64(factor)) * np.uint64(Gc) + iz // np.uint64(factor)
    adm = np.isin(ck, np.asarray(admitted, dtype=np.uint64))
    tk, tc = np.unique(k[adm], return_counts=True)
    return tk, tc.astype(np.int64), pos[~adm]


def topk_routed(table_keys, table_counts, M_rest, T_rest, rest_pos, delta, L, theta, k, variant=0):
    """Top-k of the routed pair: candidates are the table's keys (their exact counts) and the
    distinct cells of the rest whose sketch estimate is >= theta, ordered by (value desc,
    key asc)."""
    items = [(-int(c), int(kk)) for kk, c in zip(table_keys, table_counts)]
    rk = np.unique(keys(rest_pos, delta, L))
    if len(rk):
        e = estimate(M_rest, T_rest, rk, variant)
        items += [(-int(v), int(kk)) for kk, v in zip(rk, e) if v >= theta]
    items.sort()
    return [kk for _, kk in items[:k]], [-v for v, _ in items[:k]]


# ---------------------------------------------------------------- training labels and admission

def cell_list(counts, min_count=1):
    """Cells (int64, ascending) whose count is at least min_count."""
    return np.flatnonzero(np.asarray(counts) >= min_count).astype(np.int64)


def parents(fine_keys, G, factor):
    """Coarse parent keys (mesh G / factor) of fine keys of the mesh G."""
    k = np.asarray(fine_keys, dtype=np.uint64)
    G64, f, Gc = np.uint64(G), np.uint64(factor), np.uint64(G // factor)
    ix, iy, iz = k // (G64 * G64), (k // G64) % G64, k % G64
    return (((ix // f) * Gc + iy // f) * Gc + iz // f).astype(np.int64)


def labels(cells, fine_keys, G, factor):
    """float32 1 where the coarse cell is the parent of one of the fine keys, else 0."""
    return np.isin(np.asarray(cells, dtype=np.int64), parents(fine_keys, G, factor)).astype(np.float32)


def admit(cells, logits, A):
    """The min(A, m) cells of highest logit, ties by smaller key, returned in ascending
    key order (the routing split takes a sorted list)."""
    c = np.asarray(cells, dtype=np.int64)
    z = np.asarray(logits, dtype=np.float64)          # -0.0 and +0.0 compare equal
    order = np.lexsort((c, -z))
    return np.sort(c[order[:A]])


def exact_topk(pos, delta, L, k):
    """(keys, counts) of the k heaviest cells of the stream by (count desc, key asc)."""
    from . import histogram, topk_exact
    uniq, cnt = histogram(keys(pos, delta, L))
    return topk_exact(uniq, cnt, k)
