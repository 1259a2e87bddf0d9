"""Autotuners: a graph's work-split parameters for a template (tune) and for a batched
multi-template count (tune_multi), chosen by measurement.

The paper's load balancing (Section 3.3, Algorithm 4) partitions the neighbour lists of high-degree
vertices into tasks of a fixed size and reports that the task size matters (its Fig. 11 sweeps it).
Here the same knobs are the hub threshold tau (rows with more than tau neighbours are cut) and the
chunk size c (neighbours per task of a cut row). `tune` times one colouring of the plan under a
small grid of (tau, c) around the library's default and keeps the fastest. Every candidate counts
the same colouring; counts are checked against each other (exact below 2^53, 1e-12 relative above:
the chunking changes only the summation order of the cut rows).

Records are keyed by what decides the choice: the device, k, the passive row widths of the plan's
splits, and the graph's size and degree profile (log2 of the mean and of the largest degree). A
record cache can be kept in a JSON file and reused by later runs.

tune_multi does the same for the batched path (a multi-template packed count of B colourings):
the degree split, then the tile row of the packed kernels (cc_tuning.packed_tile: how many
colourings of a neighbour's row a wavefront reads per pass).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, field

import numpy as np

from . import Graph, Plan, Workspace, colour, count

TWO53 = float(2 ** 53)


@dataclass
class TuneRecord:
    hub_threshold: int
    chunk: int
    ms: float                                   # mean milliseconds per colouring of the choice
    default_ms: float                           # the library default's, same measurement
    timings: dict = field(default_factory=dict)  # "tau,c" -> ms


def default_chunk(nnz: int) -> int:
    """The library's automatic chunk size (cc_tuning.chunk = 0)."""
    return 2048 if nnz >= (1 << 28) else 512


def candidates(nnz: int, max_degree: int) -> list[tuple[int, int]]:
    """(tau, c) pairs: chunk sizes of half, one and two times the default (multiples of 64), each
    with tau at one, two and four chunks; tau values at or above the largest degree cut no row and
    collapse into one candidate. The default (2c, c) comes first."""
    c0 = default_chunk(nnz)
    out = [(2 * c0, c0)]
    for c in sorted({max(64, c0 // 2 // 64 * 64), c0, 2 * c0}):
        for m in (1, 2, 4):
            tau = m * c
            if tau > max_degree:
                tau = max(max_degree, c)
            if (tau, c) not in out:
                out.append((tau, c))
    return out


def record_key(plan: Plan, n: int, nnz: int, max_degree: int, device: str) -> str:
    widths = [math.comb(plan.k - 1, p - 1) for (_, _, p) in plan.splits]
    mean = nnz / max(n, 1)
    return json.dumps({"device": device, "k": plan.k, "passive_widths": widths, "n": n, "nnz": nnz,
                       "log2_mean_degree": int(math.floor(math.log2(mean))) if mean >= 1 else -1,
                       "log2_max_degree": int(math.floor(math.log2(max_degree))) if max_degree >= 1 else -1},
                      sort_keys=True)


def _agree(a: float, b: float) -> bool:
    if a < TWO53 and b < TWO53:
        return a == b
    return abs(a - b) <= 1e-12 * max(a, b)


def tune(plan: Plan, row_ptr, col, seed: int = 1, repeats: int = 2, cache_path: str | None = None,
         trust: bool = False) -> TuneRecord:
    """Time one colouring of `plan` on the CSR (row_ptr int64, col int32, device tensors) under each
    candidate (tau, c); return the fastest as a TuneRecord (cached in `cache_path` if given).
    The first graph preparation validates the CSR unless `trust`; the others skip it."""
    import torch
    n = row_ptr.numel() - 1
    nnz = col.numel()
    degrees = (row_ptr[1:] - row_ptr[:-1]) if n > 0 else row_ptr[:0]
    max_degree = int(degrees.max().item()) if n > 0 else 0
    device = torch.cuda.get_device_name(row_ptr.device)
    key = record_key(plan, n, nnz, max_degree, device)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return TuneRecord(**cache[key])
    ws = Workspace()
    timings: dict[str, float] = {}
    ref = None
    validated = trust
    C = None
    for tau, c in candidates(nnz, max_degree):
        G = Graph(row_ptr, col, hub_threshold=tau, chunk=c, trust=validated)
        validated = True
        if C is None:
            C = colour(G, plan.k, seed=seed, first_iter=0, B=1)
        X = count(plan, G, C, workspace=ws)  # warm-up, and the value every candidate must agree on
        torch.cuda.synchronize()
        x = float(X.cpu()[0])
        if ref is None:
            ref = x
        elif not _agree(x, ref):
            raise RuntimeError(f"tau={tau} c={c}: count {x!r} differs from {ref!r}")
        t0 = time.perf_counter()
        for _ in range(repeats):
            count(plan, G, C, workspace=ws, out=X)
        torch.cuda.synchronize()
        timings[f"{tau},{c}"] = (time.perf_counter() - t0) * 1e3 / repeats
        del G
    best = min(timings, key=timings.get)
    tau, c = (int(v) for v in best.split(","))
    c0 = default_chunk(nnz)
    rec = TuneRecord(hub_threshold=tau, chunk=c, ms=timings[best], default_ms=timings[f"{2 * c0},{c0}"],
                     timings=timings)
    if cache_path:
        cache[key] = asdict(rec)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return rec


@dataclass
class MultiTuneRecord:
    hub_threshold: int
    chunk: int
    packed_tile: int                            # 0 = the library's automatic tile
    ms: float                                   # milliseconds of one multi-template count, the choice
    default_ms: float                           # the library default's, same measurement
    timings: dict = field(default_factory=dict)  # "tau,c,tile" -> ms


def multi_record_key(plans, n: int, nnz: int, max_degree: int, B: int, device: str) -> str:
    widths = sorted({math.comb(p.k - 1, q - 1) for p in plans for (_, _, q) in p.splits})
    mean = nnz / max(n, 1)
    return json.dumps({"device": device, "k": plans[0].k, "templates": len(plans), "B": B,
                       "passive_widths": widths, "n": n, "nnz": nnz,
                       "log2_mean_degree": int(math.floor(math.log2(mean))) if mean >= 1 else -1,
                       "log2_max_degree": int(math.floor(math.log2(max_degree))) if max_degree >= 1 else -1},
                      sort_keys=True)


TILES = (0, 128, 512)


def tune_multi(plans, row_ptr, col, B: int, seed: int = 1, repeats: int = 2, cache_path: str | None = None,
               trust: bool = False) -> MultiTuneRecord:
    """The batched path's parameters by measurement (the task-size sweep of Section 3.3 / Fig. 11
    applied to a multi-template packed count of B colourings): first the degree split (tau, c) over
    candidates() with the automatic tile, then the tile row (packed_tile in TILES) at the best
    (tau, c). Every candidate counts the same colourings and must agree with the first (exact below
    2^53, 1e-12 relative above); the fastest is returned (and cached in `cache_path`)."""
    import torch
    from . import Multi
    n = row_ptr.numel() - 1
    nnz = col.numel()
    degrees = (row_ptr[1:] - row_ptr[:-1]) if n > 0 else row_ptr[:0]
    max_degree = int(degrees.max().item()) if n > 0 else 0
    device = torch.cuda.get_device_name(row_ptr.device)
    key = multi_record_key(plans, n, nnz, max_degree, B, device)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return MultiTuneRecord(**cache[key])
    multi = Multi(plans)
    ws = Workspace()
    timings: dict[str, float] = {}
    state = {"ref": None, "validated": trust, "C": None}

    def run(tau, c, tile):
        G = Graph(row_ptr, col, hub_threshold=tau, chunk=c, packed_tile=tile, trust=state["validated"])
        state["validated"] = True
        if state["C"] is None:
            state["C"] = colour(G, plans[0].k, seed=seed, first_iter=0, B=B)
        X = multi.count(G, state["C"], workspace=ws)
        torch.cuda.synchronize()
        x = X.cpu().numpy().ravel()
        if state["ref"] is None:
            state["ref"] = x
        elif not all(_agree(float(a), float(b)) for a, b in zip(x, state["ref"])):
            raise RuntimeError(f"tau={tau} c={c} tile={tile}: counts differ from the first candidate's")
        t0 = time.perf_counter()
        for _ in range(repeats):
            multi.count(G, state["C"], workspace=ws, out=X)
        torch.cuda.synchronize()
        timings[f"{tau},{c},{tile}"] = (time.perf_counter() - t0) * 1e3 / repeats
        del G

    for tau, c in candidates(nnz, max_degree):
        run(tau, c, 0)
    best = min(timings, key=timings.get)
    tau, c, _ = (int(v) for v in best.split(","))
    for tile in TILES[1:]:
        run(tau, c, tile)
    best = min(timings, key=timings.get)
    tau, c, tile = (int(v) for v in best.split(","))
    c0 = default_chunk(nnz)
    rec = MultiTuneRecord(hub_threshold=tau, chunk=c, packed_tile=tile, ms=timings[best],
                          default_ms=timings[f"{2 * c0},{c0},0"], timings=timings)
    if cache_path:
        cache[key] = asdict(rec)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return rec
