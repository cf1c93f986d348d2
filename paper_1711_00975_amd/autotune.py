"""Autotuner for the update kernels.

Every update plan gives the same counters (the binned update and the global-atomic
update add the same +-1s, Sec. 2.2 Add), so tuning only chooses speed.  The axes:

* where the increments are privatised: LDS tiles of 2^15 counters fed by a token
  partition (the binned update), or nowhere (one device-scope atomic per row and
  particle: fastest for short streams into narrow rows);
* for the binned update, the bin kernel's form and tiling: the general row-interleaved
  kernel with a cap of 64..256 workgroups, or the sort-word kernel with 1024 threads and
  2 or 3 rows per LDS pass, or 512 threads with the next tile's positions prefetched;
* per batch shape: the bin kernel form and the number of bin workgroups shared out
  among the sketches.

A per-XCD L2 copy of the counters is not an axis: its atomics (performed in the issuing
XCD's L2) are measured by bench.py's ceilings and are orders of magnitude slower than LDS
adds at these stream sizes.

Results are cached as JSON, keyed by the device (name, architecture, compute units),
in ``$CSK_AUTOTUNE_CACHE`` or ``~/.cache/csk_autotune.json``.
"""
from __future__ import annotations

import json
import math
import os

from . import (CSK_BIN_AUTO, CSK_BIN_GENERAL, CSK_BIN_SORT_WORD, CSK_UPDATE_BINNED, CSK_UPDATE_DIRECT, Batch,
               CskError, Sketch)


def _plan(mode, max_wg=0, form=CSK_BIN_AUTO, threads=0, rows=0, prefetch=0):
    return {"mode": mode, "max_wg": max_wg, "form": form, "threads": threads, "rows": rows, "prefetch": prefetch}


UPDATE_CANDIDATES = [
    _plan(CSK_UPDATE_DIRECT),
    _plan(CSK_UPDATE_BINNED, 64, CSK_BIN_GENERAL),
    _plan(CSK_UPDATE_BINNED, 128, CSK_BIN_GENERAL),
    _plan(CSK_UPDATE_BINNED, 256, CSK_BIN_GENERAL),
    _plan(CSK_UPDATE_BINNED, 256, CSK_BIN_SORT_WORD, 1024, 2, 1),
    _plan(CSK_UPDATE_BINNED, 256, CSK_BIN_SORT_WORD, 1024, 3, 1),
    _plan(CSK_UPDATE_BINNED, 256, CSK_BIN_SORT_WORD, 512, 3, 2),
]
BATCH_BUDGETS = [256, 512, 1024, 2048]
BATCH_FORMS = [_plan(CSK_UPDATE_BINNED, 0, CSK_BIN_GENERAL), _plan(CSK_UPDATE_BINNED, 0, CSK_BIN_SORT_WORD, 1024, 3, 1)]


def plan_key(p: dict) -> str:
    return "{mode}:{max_wg}:{form}:{threads}:{rows}:{prefetch}".format(**p)


def set_plan(sketch: Sketch, p: dict) -> None:
    """Apply a plan; plans cached before the tiling axes existed take the automatic tiling."""
    sketch.set_update_plan(p["mode"], p["max_wg"])
    sketch.set_update_tiling(p.get("form", CSK_BIN_AUTO), p.get("threads", 0), p.get("rows", 0), p.get("prefetch", 0))


def default_cache_path() -> str:
    return os.environ.get("CSK_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                             "csk_autotune.json"))


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def size_class(w: int, n: int) -> str:
    """Width and stream size rounded to powers of two."""
    return f"w{round(math.log2(max(w, 1)))}_n{round(math.log2(max(n, 1)))}"


def batch_class(d: int, widths, counts) -> str:
    return f"batch_d{d}_m{len(widths)}_n{round(math.log2(max(1, sum(counts))))}"


class Tuner:
    """The cache: {device key: {class: plan}} with plans {"mode", "max_wg", "form",
    "threads", "rows", "prefetch", "ms"} for one sketch and {"wg_budget", "form", ..., "ms"}
    for a batch."""

    def __init__(self, path: str | None = None, device: str | None = None):
        self.path = path or default_cache_path()
        self.device = device
        self.data = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def _dev(self) -> str:
        if self.device is None:
            self.device = device_key()
        return self.device

    def lookup(self, cls: str):
        return self.data.get(self._dev(), {}).get(cls)

    def record(self, cls: str, plan: dict) -> None:
        self.data.setdefault(self._dev(), {})[cls] = plan

    def save(self) -> None:
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    # ---- one sketch
    def tune_update(self, d: int, w: int, n: int, delta: float = 0.1, L: float = 100.0, reps: int = 5,
                    seed: int = 1) -> dict:
        """Time every update plan on a uniform stream of n particles; record the fastest."""
        import torch
        gen = torch.Generator(device="cuda").manual_seed(seed)
        pos = torch.rand((max(n, 1), 3), generator=gen, device="cuda", dtype=torch.float32) * L
        s = Sketch(d, w, seed)
        times, plans = {}, {}
        for p in UPDATE_CANDIDATES:
            try:
                set_plan(s, p)
            except CskError:                              # a form this sketch cannot take
                continue
            s.update(pos, delta, L)                       # warm-up (sizes the scratch)
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.update(pos, delta, L)
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1))
            times[plan_key(p)] = best
            plans[plan_key(p)] = p
        s.close()
        key = min(times, key=times.get)
        plan = dict(plans[key], ms=times[key], all_ms=times)
        self.record(size_class(w, n), plan)
        return plan

    def apply(self, sketch: Sketch, n: int) -> bool:
        """Set the tuned plan of sketch's (w, n) class if there is one."""
        plan = self.lookup(size_class(sketch.w, n))
        if plan is None:
            return False
        set_plan(sketch, plan)
        return True

    # ---- a batch
    def tune_batch(self, sketches, positions, delta: float, L: float, reps: int = 3) -> dict:
        """Time the batched update with each bin kernel form and workgroup budget; record the
        fastest and leave its form set on the first sketch (a batch takes that sketch's)."""
        counts = [int(p.shape[0]) for p in positions]
        times, forms = {}, {}
        for f in BATCH_FORMS:
            try:
                set_plan(sketches[0], f)
            except CskError:                              # a form this batch cannot take
                continue
            for budget in BATCH_BUDGETS:
                key = f"{budget}:{f['form']}"
                times[key] = self._time_batch(sketches, positions, counts, delta, L, budget, reps)
                forms[key] = f
        key = min(times, key=times.get)
        set_plan(sketches[0], forms[key])
        plan = dict(forms[key], wg_budget=int(key.split(":")[0]), ms=times[key], all_ms=times)
        self.record(batch_class(sketches[0].d, [s.w for s in sketches], counts), plan)
        return plan

    @staticmethod
    def _time_batch(sketches, positions, counts, delta, L, budget, reps):
        import torch
        b = Batch(sketches, counts, delta, L, wg_budget=budget)
        b.update(positions)
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.update(positions)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        b.close()
        return best

    def batch_budget(self, sketches, counts) -> int:
        """The tuned budget of this batch shape (0: none), its bin kernel form set on the first
        sketch."""
        plan = self.lookup(batch_class(sketches[0].d, [s.w for s in sketches], counts))
        if not plan:
            return 0
        if "form" in plan:
            set_plan(sketches[0], plan)
        return plan["wg_budget"]
