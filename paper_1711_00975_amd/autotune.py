"""Autotuner for the update kernels.

Every update plan gives the same counters (the binned update and the global-atomic
update add the same +-1s, Sec. 2.2 Add), so tuning only chooses speed:

* per (w, n) class of one sketch: the LDS-binned update with a cap of 32..256 bin
  workgroups, or one global atomic per row and particle (fastest for short streams);
* per batch shape: the number of bin workgroups shared out among the sketches.

Results are cached as JSON, keyed by the device (name, architecture, compute units),
in ``$CSK_AUTOTUNE_CACHE`` or ``~/.cache/csk_autotune.json``.
"""
from __future__ import annotations

import json
import math
import os

from . import CSK_UPDATE_BINNED, CSK_UPDATE_DIRECT, Batch, Sketch

UPDATE_CANDIDATES = [(CSK_UPDATE_BINNED, 32), (CSK_UPDATE_BINNED, 64), (CSK_UPDATE_BINNED, 128),
                     (CSK_UPDATE_BINNED, 256), (CSK_UPDATE_DIRECT, 0)]
BATCH_BUDGETS = [256, 512, 1024, 2048]


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
    """The cache: {device key: {class: plan}} with plans {"mode", "max_wg", "ms"} for one
    sketch and {"wg_budget", "ms"} for a batch."""

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
        times = {}
        for mode, wg in UPDATE_CANDIDATES:
            s.set_update_plan(mode, wg)
            s.update(pos, delta, L)                       # warm-up (sizes the scratch)
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.update(pos, delta, L)
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1))
            times[f"{mode}:{wg}"] = best
        s.close()
        key = min(times, key=times.get)
        mode, wg = (int(x) for x in key.split(":"))
        plan = {"mode": mode, "max_wg": wg, "ms": times[key], "all_ms": times}
        self.record(size_class(w, n), plan)
        return plan

    def apply(self, sketch: Sketch, n: int) -> bool:
        """Set the tuned plan of sketch's (w, n) class if there is one."""
        plan = self.lookup(size_class(sketch.w, n))
        if plan is None:
            return False
        sketch.set_update_plan(plan["mode"], plan["max_wg"])
        return True

    # ---- a batch
    def tune_batch(self, sketches, positions, delta: float, L: float, reps: int = 3) -> dict:
        """Time the batched update with each workgroup budget; record the fastest."""
        import torch
        counts = [int(p.shape[0]) for p in positions]
        times = {}
        for budget in BATCH_BUDGETS:
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
            times[str(budget)] = best
        budget = int(min(times, key=times.get))
        plan = {"wg_budget": budget, "ms": times[str(budget)], "all_ms": times}
        self.record(batch_class(sketches[0].d, [s.w for s in sketches], counts), plan)
        return plan

    def batch_budget(self, sketches, counts) -> int:
        plan = self.lookup(batch_class(sketches[0].d, [s.w for s in sketches], counts))
        return plan["wg_budget"] if plan else 0
