"""Autotuner of the codec's launch parameters.

The parameters are those that change how the work is cut, never a byte of
the output (block size B does change the stream, so it is tuned per
workload and reported with the result):

* block size B (section 2.1: the unit of independent coding);
* sub-block index stride S (it also picks the decoder: the wave-staged table
  decoder for S <= 128, the per-lane line ring above);
* the encode tile, ``hc_tuning.encode_tile_loads`` (16-byte loads per
  thread; 0 = the library's rule).

Work-group sizes are fixed by the kernels' design (256 threads, occupancy
set by each kernel's LDS), so they are not searched.

``Autotuner.tune`` measures a caller-supplied step over the candidates (the
lowest time wins) and caches the winner per (device architecture, device
name, workload key) in a JSON file, so a later run on the same kind of
device and workload takes it without measuring.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Iterable, List, Optional, Tuple

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1107_1525_amd", "autotune.json")


def device_key(torch) -> str:
    """Architecture and name of the current device (what a tuning depends on)."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or "unknown-arch"
    return f"{arch}|{p.name}|{p.multi_processor_count}cu"


def candidate_key(c: Dict) -> str:
    return ",".join(f"{k}={c[k]}" for k in sorted(c))


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None):
        self.cache_path = cache_path or os.environ.get("HC_AUTOTUNE_CACHE", DEFAULT_CACHE)

    def _load(self) -> Dict:
        try:
            with open(self.cache_path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}

    def _store(self, cache: Dict) -> None:
        d = os.path.dirname(self.cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def lookup(self, device: str, workload: str) -> Optional[Dict]:
        return self._load().get(device, {}).get(workload)

    def tune(self, device: str, workload: str, candidates: Iterable[Dict], measure: Callable[[Dict], float],
             force: bool = False) -> Tuple[Dict, List[Dict], bool]:
        """Returns (best candidate, measured table, taken from the cache).
        measure(candidate) -> seconds (lower is better); a candidate whose
        measurement raises is recorded with its error and never chosen."""
        if not force:
            hit = self.lookup(device, workload)
            if hit is not None:
                return dict(hit["best"]), list(hit.get("table", [])), True
        table: List[Dict] = []
        best, best_t = None, float("inf")
        for c in candidates:
            row = {"candidate": dict(c)}
            try:
                t = float(measure(dict(c)))
                row["seconds"] = t
                if t < best_t:
                    best, best_t = dict(c), t
            except Exception as e:  # a candidate the device or data cannot run
                row["error"] = f"{type(e).__name__}: {e}"
            table.append(row)
        if best is None:
            raise RuntimeError("autotune: no candidate could be measured")
        cache = self._load()
        cache.setdefault(device, {})[workload] = {"best": best, "table": table}
        self._store(cache)
        return best, table, False
