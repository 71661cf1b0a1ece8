"""Tile-size autotuner for the grouped-GEMM projection.

The plan splits every output block (and every intermediate of a two-sided
record) into square tiles of 16 or 32 rows/columns, picked by the largest
block dimension through a small table ``(bounds, tiles)``: blocks with
max(rows, cols) <= bounds[c] get tiles[c].  This module times the projection
of a given workload for a set of candidate tables (HIP events on the launch
stream), keeps the fastest, and stores it in ``tiles_gfx950.json`` keyed by
precision and workload size class.  ``Plan(..., tiles="auto")`` applies the
stored table when one exists for its key.

    python -m paper_1309_5571_amd.autotune --workload hubbard_m2048 --prec f64

The paper picks a CPU/GPU workload split per matrix size from a
configuration file; this plays the same role for tile shapes on one GPU.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Sequence, Tuple

import numpy as np

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_gfx950.json")

CANDIDATES: List[Tuple[Tuple[int, ...], Tuple[int, ...]]] = [
    ((1 << 30,), (16,)),
    ((1 << 30,), (32,)),
    ((16, 1 << 30), (16, 32)),
    ((32, 1 << 30), (16, 32)),
    ((64, 1 << 30), (16, 32)),
    ((128, 1 << 30), (16, 32)),
]


def size_class(problems) -> str:
    """Workload class by the largest sector dimension over all members."""
    dmax = 0
    for p in problems:
        dmax = max(dmax, int(np.max(p.left.dims)), int(np.max(p.right.dims)))
    if dmax <= 48:
        return "dmax<=48"
    if dmax <= 200:
        return "dmax<=200"
    return "dmax>200"


def key_of(problems, prec: str) -> str:
    return f"{prec}|{size_class(problems)}"


def load_table(key: str):
    if not os.path.exists(TABLE_PATH):
        return None
    with open(TABLE_PATH) as f:
        tab = json.load(f)
    ent = tab.get("entries", {}).get(key)
    if not ent:
        return None
    return tuple(ent["bounds"]), tuple(ent["tiles"])


def tune(problems, prec: str = "f64", reps: int = 50, candidates: Sequence = CANDIDATES) -> Dict:
    """Time every candidate table on this workload; return results and the best."""
    import torch

    from . import Plan, set_tile_table

    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    results = []
    try:
        for bounds, tiles in candidates:
            set_tile_table(bounds, tiles)
            plan = Plan(problems, prec=prec, tiles=None)
            psi = torch.randn(plan.n, dtype=torch.float64, device=plan.device)
            y = torch.empty_like(psi)
            for _ in range(5):
                plan.project_raw(psi, prec=prec, out=y)
            s = torch.cuda.current_stream(plan.device)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                plan.project_raw(psi, prec=prec, out=y)
            e1.record(s)
            e1.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            results.append({"bounds": list(bounds), "tiles": list(tiles), "us": t * 1e6,
                            "tflops": plan.flop / t * 1e-12})
            plan.close()
    finally:
        set_tile_table((), ())
    best = min(results, key=lambda r: r["us"])
    return {"key": key_of(problems, prec), "best": best, "results": results}


def save(result: Dict, path: str = TABLE_PATH) -> None:
    tab = {"arch": "gfx950", "entries": {}}
    if os.path.exists(path):
        with open(path) as f:
            tab = json.load(f)
    b = result["best"]
    tab["entries"][result["key"]] = {"bounds": b["bounds"], "tiles": b["tiles"], "us": b["us"]}
    with open(path, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)


def main():
    import argparse
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import gen

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="all", choices=["all", "heisenberg_m1024", "hubbard_m2048",
                                                         "j1j2_m1024", "batched_64"])
    ap.add_argument("--prec", default="all", choices=["all", "f64", "f32", "bf16"])
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--save", action="store_true")
    ap.add_argument("--table", default=TABLE_PATH, help="where --save writes the table")
    a = ap.parse_args()
    loads = {"heisenberg_m1024": lambda: [gen.config(2)], "hubbard_m2048": lambda: [gen.config(3)],
             "j1j2_m1024": lambda: [gen.config(5)], "batched_64": lambda: gen.config(4)}
    names = list(loads) if a.workload == "all" else [a.workload]
    precs = ["f64", "f32", "bf16"] if a.prec == "all" else [a.prec]
    for nm in names:
        probs = loads[nm]()
        for pr in precs:
            r = tune(probs, pr, reps=a.reps)
            print(json.dumps({"workload": nm, **r}), flush=True)
            if a.save:
                save(r, a.table)


if __name__ == "__main__":
    main()
