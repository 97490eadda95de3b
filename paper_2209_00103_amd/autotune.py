"""Autotuner for the batched mode: picks each array's first-bucket size.

The first bucket F changes how many buckets an array allocates and how often an
insertion tile crosses a bucket boundary, so it changes speed and memory, never
contents (the result depends only on the inputs and the LFVector count V, which
the tuner never touches).  For every size class (octave of the target element
count) the tuner times the batched phases -- four insertion rounds, r/w and
flatten -- of a probe array of the class's representative size for each
candidate F in 2^6 .. 2^14 whose predicted capacity stays within twice the live
elements, and keeps the fastest.  Results are cached as JSON keyed by
(GPU architecture, element size, size class).

The launch shape is tuned too, where it is a free knob: the insertion kernel's
is fixed by design (one wavefront per 4096-thread tile is the unit of work,
whatever the array), but the r/w and flatten launches run a persistent grid
whose workgroup count (256 threads each) trades tail imbalance against
per-workgroup overhead; ``tune_grid`` times the candidates on the batch itself.
"""
from __future__ import annotations

import json
import os

CANDIDATES = tuple(1 << k for k in range(6, 15))
GRID_CANDIDATES = (0, 8192, 16384, 32768, 65536, 131072)  # 0: the library's default shape
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ggarray", "autotune.json")


def _nbuckets(F: int, s: int) -> int:
    """Buckets an LFVector of s elements holds: smallest k with F (2^k - 1) >= s."""
    k = 0
    while F * ((1 << k) - 1) < s:
        k += 1
    return k


def predicted_ratio(n: int, V: int, F: int, rounds: list[int]) -> float:
    """Capacity / live elements after the rounds, from the thread -> LFVector rule
    (contiguous chunks of ceil(n_r / V) threads, every thread inserting once)."""
    sizes = [0] * V
    for n_r in rounds:
        if n_r == 0:
            continue
        chunk = -(-n_r // V)
        for v in range(V):
            lo = v * chunk
            sizes[v] += max(0, min(chunk, n_r - lo))
    live = sum(sizes)
    cap = sum(F * ((1 << _nbuckets(F, s)) - 1) for s in sizes)
    return cap / live if live else 1.0


def size_class(n: int) -> int:
    return max(0, int(n).bit_length() - 1)


class AutoTuner:
    def __init__(self, vectors_for, rounds_for, elem_bytes: int = 4, cache_path: str | None = None):
        self.vectors_for = vectors_for
        self.rounds_for = rounds_for
        self.elem_bytes = elem_bytes
        self.cache_path = cache_path or os.environ.get("GGARRAY_AUTOTUNE_CACHE", DEFAULT_CACHE)
        self.cache = {}
        if os.path.exists(self.cache_path):
            try:
                with open(self.cache_path) as f:
                    self.cache = json.load(f)
            except (OSError, ValueError):
                self.cache = {}

    def _key(self, cls: int) -> str:
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        return f"{arch}|e{self.elem_bytes}|c{cls}"

    def allowed(self, n: int) -> list[int]:
        V, rounds = self.vectors_for(n), self.rounds_for(n)
        ok = [F for F in CANDIDATES if predicted_ratio(n, V, F, rounds) <= 2.0]
        return ok or [CANDIDATES[0]]

    def first_bucket(self, n: int) -> int:
        cls = size_class(n)
        key = self._key(cls)
        if key not in self.cache:
            self.cache[key] = self._tune(cls)
            self._save()
        F = int(self.cache[key])
        allowed = self.allowed(n)
        return F if F in allowed else max(allowed)

    def _save(self):
        try:
            os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
        except OSError:
            pass

    def _tune(self, cls: int) -> int:
        import torch

        from paper_2209_00103_amd import ggarray as G

        n = (1 << cls) + (1 << cls) // 2
        V, rounds = self.vectors_for(n), self.rounds_for(n)
        best, best_ms = None, None
        pool = G.Pool(max(64 << 20, 8 * n * self.elem_bytes + (4 << 20)))
        try:
            for F in self.allowed(n):
                a = G.GGArray(pool, self.elem_bytes, V, F)
                b = G.Batch([a])
                out = torch.empty(sum(rounds), dtype=torch.int32 if self.elem_bytes == 4 else torch.int64,
                                  device="cuda")
                gens = [G.make_gen(G.GEN_KEYED, seed=1, round=r) for r in range(len(rounds))]

                def phase():
                    b.shrink(1, 1)
                    for r, n_r in enumerate(rounds):
                        b.insert_gen(gens[r], [n_r])
                    b.rw(G.ADD1)
                    b.flatten_into(out)

                phase()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                times = []
                for _ in range(5):
                    e0.record()
                    phase()
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                ms = min(times)
                if best_ms is None or ms < best_ms:
                    best, best_ms = F, ms
                b.close()
                a.close()
        finally:
            pool.close()
        return best

    def tune_grid(self, batch, out, total_elems: int) -> int:
        """Workgroups of the batch's r/w + flatten launches: the fastest of
        GRID_CANDIDATES on this batch (r/w x+1 then flatten into out; 0 is the
        library's default shape), cached by (architecture, element size, octave of
        the batch's element count).  Leaves the batch's contents changed by the r/w
        passes."""
        import torch

        from paper_2209_00103_amd import ggarray as G

        key = self._key(size_class(total_elems)).replace("|c", "|grid") + f"|n{batch.n}"
        if key not in self.cache:
            best, best_ms = None, None
            for g in GRID_CANDIDATES:
                batch.set_grid(g)
                batch.rw(G.ADD1)
                batch.flatten_into(out)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                times = []
                for _ in range(5):
                    e0.record()
                    batch.rw(G.ADD1)
                    batch.flatten_into(out)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                ms = min(times)
                if best_ms is None or ms < best_ms:
                    best, best_ms = g, ms
            self.cache[key] = best
            self._save()
        g = int(self.cache[key])
        batch.set_grid(g)
        return g
