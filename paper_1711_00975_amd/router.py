"""The learned router in front of a Count Sketch.

A 1 % sample of the stream gives coarse cell counts (cells of side delta_c, each the
parent of factor^3 fine cells).  A 27 -> 64 -> 64 -> 1 MLP scores every coarse cell from
the log counts of the cell and its 26 neighbours.  The highest-scored coarse cells are
admitted and every particle inside them is counted exactly in a small device hash table.
All other particles go to a Count Sketch (Sec. 2.2 Add) whose width is cut so that the
table and the sketch together take no more memory than the plain sketch they replace.
The top-k merges the two: an admitted key takes its exact count, every other key takes
its sketch estimate (the median of Sec. 2.2 Estimate).

Training labels come from the exact top-k of other snapshots: a coarse cell is positive
when one of its fine cells is among the exact k heaviest.

Every arithmetic step runs in the library's kernels.  torch holds the device buffers, and
its indexing shuffles training rows into minibatches.
"""
from __future__ import annotations

import math

from . import (FEAT, MLP, Sketch, cell_features, cell_labels, cell_list, cell_list_async, cell_list_workspace_bytes,
               cells_clear, exact_counts, new_table, route_admit, route_admit_async, route_admit_workspace_bytes,
               route_score, route_split, route_update_workspace_bytes, sample_counts, table_topk, topk_with_table,
               topk_with_table_async, update_routed)

TABLE_BYTES_PER_SLOT = 12     # 8-byte key + 4-byte count


def rest_width(w_plain: int, d: int, table_slots: int) -> int:
    """Width of the rest sketch such that table + rest sketch <= a plain d x w_plain sketch."""
    return w_plain - math.ceil(table_slots * TABLE_BYTES_PER_SLOT / (4 * d))


class Router:
    def __init__(self, delta: float, L: float, delta_c: float = 1.0, table_slots: int = 1 << 16,
                 max_admit: int = 512, min_count: int = 2, sample_seed: int = 1, model_seed: int = 1,
                 max_batch: int = 4096):
        import torch
        self.delta, self.L, self.delta_c = delta, L, delta_c
        G, Gc = round(L / delta), round(L / delta_c)
        if G % Gc:
            raise ValueError("the coarse mesh must nest in the fine one")
        self.factor = G // Gc
        self.Gc = Gc
        self.table_slots, self.min_count, self.sample_seed = table_slots, min_count, sample_seed
        self.max_admit = min(max_admit, table_slots // (2 * self.factor ** 3))
        self.counts = torch.zeros(Gc ** 3, dtype=torch.int32, device="cuda")
        self.bitmap = torch.zeros((Gc ** 3 + 31) // 32, dtype=torch.int32, device="cuda")
        self.mlp = MLP(seed=model_seed, max_batch=max_batch)
        self.cells = torch.empty(1 << 20, dtype=torch.int64, device="cuda")
        self.X, self.Y = [], []

    # ---- the sample pre-pass and features
    def features(self, pos):
        """(coarse cells with >= min_count sampled particles, their features)."""
        sample_counts(pos, self.delta_c, self.L, self.sample_seed, self.counts, bitmap=self.bitmap)
        cells = cell_list(self.counts, self.min_count, out=self.cells, bitmap=self.bitmap)
        if cells.data_ptr() != self.cells.data_ptr():      # the buffer grew
            self.cells = cells
        x = cell_features(self.counts, self.delta_c, self.L, cells)
        cells_clear(self.counts, self.bitmap)              # back to empty for the next stream
        return cells, x

    # ---- training
    def add_snapshot(self, pos, k: int, exact_slots: int):
        """Labels from the exact top-k of this snapshot; keeps its rows for training."""
        import torch
        tk, tc = new_table(exact_slots)
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        exact_counts(pos, self.delta, self.L, tk, tc, err)
        top, _ = table_topk(tk, tc, k)
        if err.item() & 2:
            raise RuntimeError("exact table too small for the snapshot")
        del tk, tc
        cells, x = self.features(pos)
        y = cell_labels(cells, top, self.delta, self.L, self.factor)
        self.X.append(x)
        self.Y.append(y)
        return {"rows": int(cells.numel()), "positives": int(y.sum().item())}

    def train(self, epochs: int = 4, batch: int = 4096, lr: float = 2e-3, seed: int = 1):
        import torch
        X, Y = torch.cat(self.X), torch.cat(self.Y)
        n = X.shape[0]
        gen = torch.Generator(device="cpu").manual_seed(seed)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        hist = []
        for _ in range(epochs):
            perm = torch.randperm(n, generator=gen).cuda()
            tot, steps = 0.0, 0
            for b in range(0, n, batch):
                idx = perm[b:b + batch]
                self.mlp.train_step(X.index_select(0, idx).contiguous(), Y.index_select(0, idx).contiguous(), lr,
                                    loss)
                tot += loss  # stays on the device until the epoch ends
                steps += 1
            hist.append(float((tot / steps).item()))
        return {"rows": n, "positives": int(Y.sum().item()), "epochs": epochs, "loss": hist}

    # ---- inference and routing
    def admit(self, pos):
        cells, x = self.features(pos)
        z = self.mlp.forward(x)
        return route_admit(cells, z, self.max_admit)

    def split(self, pos, admitted, table_keys, table_counts, rest, rest_count, err):
        route_split(pos, self.delta, self.L, self.factor, admitted, table_keys, table_counts, rest, rest_count, err)

    def close(self):
        self.mlp.close()


class RoutedStep:
    """One routed step with no host synchronization, on buffers held here:

    sample -> coarse-cell listing (device count) -> features and fp32 logits (one kernel)
    -> admission of the best max_admit cells (device count) -> update of the rest sketch
    with the admitted cells' particles counted in the exact table instead (no rest stream
    is written) -> candidate pass of the rest sketch over the whole stream -> merged top-k.

    Every call only enqueues kernels, so that after one eager run (which sizes the
    libraries' scratch) the step can be captured in a HIP graph and replayed."""

    def __init__(self, router: Router, rest: Sketch, k: int, max_cells: int = 1 << 20):
        import torch
        dev = "cuda"
        self.r, self.rest, self.k = router, rest, k
        self.cells = torch.empty(max_cells, dtype=torch.int64, device=dev)
        self.m = torch.zeros(1, dtype=torch.int64, device=dev)
        self.logits = torch.empty(max_cells, dtype=torch.float32, device=dev)
        self.admitted = torch.empty(router.max_admit, dtype=torch.int64, device=dev)
        self.na = torch.zeros(1, dtype=torch.int32, device=dev)
        self.table_keys, self.table_counts = new_table(router.table_slots)
        self.err = torch.zeros(1, dtype=torch.int32, device=dev)
        self.keys = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
        self.est = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        self.out = torch.zeros(2, dtype=torch.int32, device=dev)
        u8 = torch.uint8
        self.list_ws = torch.empty(cell_list_workspace_bytes(router.counts.numel()), dtype=u8, device=dev)
        self.admit_ws = torch.empty(route_admit_workspace_bytes(max_cells, router.max_admit), dtype=u8, device=dev)
        self.update_ws = torch.empty(route_update_workspace_bytes(router.factor, router.table_slots), dtype=u8,
                                     device=dev)

    def admit(self, pos):
        r = self.r
        sample_counts(pos, r.delta_c, r.L, r.sample_seed, r.counts, bitmap=r.bitmap)
        cell_list_async(r.counts, self.cells, self.m, r.min_count, bitmap=r.bitmap, workspace=self.list_ws)
        route_score(r.mlp, r.counts, r.delta_c, r.L, self.cells, self.m, self.logits)
        cells_clear(r.counts, r.bitmap)
        route_admit_async(self.cells, self.logits, self.m, r.max_admit, self.admitted, self.na,
                          workspace=self.admit_ws)

    def update(self, pos):
        r = self.r
        self.table_keys.fill_(-1)
        self.table_counts.zero_()
        self.rest.reset()
        update_routed(self.rest, pos, r.delta, r.L, r.factor, self.admitted, self.na, self.table_keys,
                      self.table_counts, self.err, workspace=self.update_ws)

    def select(self, pos, theta):
        r = self.r
        self.rest.collect(pos, r.delta, r.L, theta)
        topk_with_table_async(self.rest, self.table_keys, self.table_counts, self.k, self.keys, self.est, self.out)

    def run(self, pos, theta):
        self.admit(pos)
        self.update(pos)
        self.select(pos, theta)

    def result(self):
        """(keys, estimates, status) after the stream has synchronized: status 0, or 1 when
        fewer than k keys came from a partial candidate set."""
        n, partial = (int(v) for v in self.out.cpu())
        return self.keys[:n], self.est[:n], partial


def routed_topk(sketch: Sketch, table_keys, table_counts, k: int):
    return topk_with_table(sketch, table_keys, table_counts, k)


__all__ = ["Router", "RoutedStep", "rest_width", "routed_topk", "TABLE_BYTES_PER_SLOT", "FEAT"]
