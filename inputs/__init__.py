"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds input generation only: graphs (Erdos-Renyi, R-MAT, cycles, stars, cliques),
tree templates (Pruefer sequences, all non-isomorphic trees of a size) and explicit colour arrays
drawn with numpy's PCG64. It contains none of the colour-coding arithmetic: no sub-template
tables, no colour-set ranks, no counting. Both the oracle and the GPU path consume what it
returns; neither side's code is imported here.

Graph format everywhere: CSR with ``row_ptr`` int64[n+1] and ``col`` int32[nnz], rows sorted,
no self-loops, no duplicates, symmetric (undirected graph stored in both directions).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")

# SplitMix64 finaliser constants (Steele, Lea, Flood 2014) and the two stream multipliers.
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_G = np.uint64(0x9E3779B97F4A7C15)
_H = np.uint64(0xD1B54A32D192ED03)

RMAT_ABC = (0.57, 0.19, 0.19)


_GPU_LIB_PATH = os.path.join(_HERE, "libgen_gpu.so")


def build(force: bool = True) -> str:
    """Compile inputs/gen.c into inputs/libgen.so (gcc, OpenMP) and inputs/gen_gpu.hip into
    inputs/libgen_gpu.so (hipcc, gfx950)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    gsrc = os.path.join(_HERE, "gen_gpu.hip")
    if force or not os.path.exists(_GPU_LIB_PATH) or os.path.getmtime(_GPU_LIB_PATH) < os.path.getmtime(gsrc):
        tmp = _GPU_LIB_PATH + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, gsrc], stderr=subprocess.DEVNULL)
        os.replace(tmp, _GPU_LIB_PATH)
    return _LIB_PATH


@lru_cache(maxsize=1)
def _gpu_lib():
    if not os.path.exists(_GPU_LIB_PATH):
        raise RuntimeError(f"{_GPU_LIB_PATH} is not built; run inputs.build()")
    L = ctypes.CDLL(_GPU_LIB_PATH)
    P, U64, I64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64
    L.gen_gpu_count.argtypes = [ctypes.c_int, U64, P, U64, P, P]
    L.gen_gpu_scatter.argtypes = [ctypes.c_int, U64, P, U64, P, P, P]
    L.gen_gpu_sort_small.argtypes = [P, P, I64, P, P, P]
    L.gen_gpu_sort_large.argtypes = [P, P, ctypes.c_int, P, P, I64, P, P]
    L.gen_gpu_compact.argtypes = [P, P, P, I64, P, P]
    return L


def rmat_graph_gpu(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC, device="cuda",
                   bitmap_budget: int = 4 << 30):
    """The same R-MAT graph as rmat_graph(), built on the GPU; returns (row_ptr, col) torch tensors
    (int64, int32) on `device`."""
    import torch
    L = _gpu_lib()
    dev = torch.device(device)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    k8 = np.array(rmat_params(scale, *abc, seed), dtype=np.uint64)
    n = 1 << scale
    E = edge_factor << scale

    def chk(rc, what):
        if rc != 0:
            raise RuntimeError(f"{what}: hip error {rc}")

    deg = torch.zeros(n, dtype=torch.int32, device=dev)
    chk(L.gen_gpu_count(scale, E, k8.ctypes.data, seed, deg.data_ptr(), st), "count")
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(deg.to(torch.int64), 0)
    cursor = off[:-1].clone()
    raw_n = int(off[-1].item())
    raw = torch.empty(max(raw_n, 1), dtype=torch.int32, device=dev)
    chk(L.gen_gpu_scatter(scale, E, k8.ctypes.data, seed, cursor.data_ptr(), raw.data_ptr(), st), "scatter")
    del cursor
    uniq = torch.zeros(n, dtype=torch.int32, device=dev)
    small = torch.nonzero((deg > 0) & (deg <= 4096)).view(-1).to(torch.int32)
    large = torch.nonzero(deg > 4096).view(-1).to(torch.int32)
    chk(L.gen_gpu_sort_small(off.data_ptr(), small.data_ptr(), small.numel(), raw.data_ptr(), uniq.data_ptr(), st),
        "sort small rows")
    words = (n + 31) // 32
    group = max(1, min(4096, bitmap_budget // (words * 4), large.numel()))
    if large.numel():
        bitmaps = torch.empty(group * words, dtype=torch.int32, device=dev)
        for g0 in range(0, large.numel(), group):
            rows = large[g0:g0 + group].contiguous()
            bitmaps.zero_()
            chk(L.gen_gpu_sort_large(off.data_ptr(), rows.data_ptr(), rows.numel(), raw.data_ptr(),
                                     bitmaps.data_ptr(), words, uniq.data_ptr(), st), "sort large rows")
        del bitmaps
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(uniq.to(torch.int64), 0)
    col = torch.empty(max(int(row_ptr[-1].item()), 1), dtype=torch.int32, device=dev)
    chk(L.gen_gpu_compact(off.data_ptr(), row_ptr.data_ptr(), raw.data_ptr(), n, col.data_ptr(), st), "compact")
    nnz = int(row_ptr[-1].item())
    torch.cuda.synchronize(dev)
    del raw
    return row_ptr, col[:nnz]


@lru_cache(maxsize=1)
def _lib():
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gen_rmat_build.restype = ctypes.c_void_p
    lib.gen_rmat_build.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.gen_rmat_fill.restype = ctypes.c_int
    lib.gen_rmat_fill.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.gen_free.restype = None
    lib.gen_free.argtypes = [ctypes.c_void_p]
    lib.gen_rmat_params.restype = None
    lib.gen_rmat_params.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_uint64, ctypes.c_void_p]
    lib.gen_rmat_draws.restype = ctypes.c_int
    lib.gen_rmat_draws.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


# ----------------------------------------------------------------------------------------------
# CSR helpers
# ----------------------------------------------------------------------------------------------

def csr_from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Undirected edge list (m, 2) -> symmetric, sorted, de-duplicated CSR without self-loops."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    key = np.unique(both[:, 0] * np.int64(n) + both[:, 1])
    src = key // n
    dst = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    return row_ptr, dst.astype(np.int32)


def degrees(row_ptr: np.ndarray) -> np.ndarray:
    return np.diff(row_ptr)


def check_csr(row_ptr: np.ndarray, col: np.ndarray) -> None:
    """Raise ValueError unless the CSR is a simple, symmetric, sorted undirected graph."""
    n = len(row_ptr) - 1
    if row_ptr[0] != 0 or row_ptr[-1] != len(col) or np.any(np.diff(row_ptr) < 0):
        raise ValueError("bad row offsets")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    c = col.astype(np.int64)
    if len(c) and (c.min() < 0 or c.max() >= n):
        raise ValueError("column out of range")
    if np.any(src == c):
        raise ValueError("self-loop")
    key = src * n + c
    if np.any(np.diff(key) <= 0):
        raise ValueError("rows not strictly increasing (unsorted or duplicate)")
    rkey = np.sort(c * n + src)
    if not np.array_equal(rkey, key):
        raise ValueError("not symmetric")


# ----------------------------------------------------------------------------------------------
# Graph families
# ----------------------------------------------------------------------------------------------

def er_graph(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Uniform simple graph G(n, m): m distinct undirected edges, no self-loops (PCG64 draws)."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    rng = np.random.default_rng(seed)
    seen = np.zeros(0, dtype=np.int64)
    while len(seen) < m:
        need = m - len(seen)
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        ok = u != v
        a = np.minimum(u, v)[ok]
        b = np.maximum(u, v)[ok]
        key = a * n + b
        allk = np.concatenate([seen, key])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        seen = allk[first][:m]
    edges = np.stack([seen // n, seen % n], axis=1)
    return csr_from_edges(n, edges)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def rmat_params(scale: int, a: float, b: float, c: float, seed: int) -> list[int]:
    with np.errstate(over="ignore"):
        s = np.array([seed + 1, seed + 2, seed + 3, seed + 4], dtype=np.uint64)
        m = _mix64(s)
    return [int(np.floor(a * 4294967296.0)), int(np.floor((a + b) * 4294967296.0)),
            int(np.floor((a + b + c) * 4294967296.0)), int(m[0]) | 1, int(m[1]), int(m[2]) | 1,
            int(m[3]), (scale + 1) // 2]


def rmat_draws_np(scale: int, a: float, b: float, c: float, seed: int, e0: int, count: int):
    """numpy twin of the C edge draw (before de-duplication); returns (src, dst, keep)."""
    ta, tb, tc, p1, q1, p2, q2, shift = rmat_params(scale, a, b, c, seed)
    with np.errstate(over="ignore"):
        e = np.arange(e0, e0 + count, dtype=np.uint64)
        base = _mix64(np.uint64(seed) + _G * (e + np.uint64(1)))
        s = np.zeros(count, dtype=np.uint64)
        d = np.zeros(count, dtype=np.uint64)
        for lvl in range(scale):
            r = _mix64(base + _H * np.uint64(lvl + 1)) >> np.uint64(32)
            bs = (r >= np.uint64(tb)).astype(np.uint64)
            bd = (((r >= np.uint64(ta)) & (r < np.uint64(tb))) | (r >= np.uint64(tc))).astype(np.uint64)
            s = (s << np.uint64(1)) | bs
            d = (d << np.uint64(1)) | bd
        mask = np.uint64((1 << scale) - 1)

        def perm(x):
            x = (x * np.uint64(p1) + np.uint64(q1)) & mask
            x ^= x >> np.uint64(shift)
            x = (x * np.uint64(p2) + np.uint64(q2)) & mask
            x ^= x >> np.uint64(shift)
            return x

        s = perm(s)
        d = perm(d)
    return s.astype(np.uint32), d.astype(np.uint32), (s != d).astype(np.uint8)


def rmat_graph_np(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC):
    """Pure numpy R-MAT (small scales only; the C builder is the fast path)."""
    a, b, c = abc
    count = edge_factor << scale
    s, d, keep = rmat_draws_np(scale, a, b, c, seed, 0, count)
    keep = keep.astype(bool)
    edges = np.stack([s[keep].astype(np.int64), d[keep].astype(np.int64)], axis=1)
    return csr_from_edges(1 << scale, edges)


def rmat_graph(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC, threads: int = 0):
    """R-MAT graph (C builder, OpenMP): n = 2^scale, sorted symmetric simple CSR."""
    a, b, c = abc
    lib = _lib()
    n = ctypes.c_int64()
    nnz = ctypes.c_int64()
    h = lib.gen_rmat_build(scale, edge_factor, a, b, c, seed, threads, ctypes.byref(n), ctypes.byref(nnz))
    if not h:
        raise MemoryError("R-MAT build failed")
    try:
        row_ptr = np.empty(n.value + 1, dtype=np.int64)
        col = np.empty(max(nnz.value, 1), dtype=np.int32)[: nnz.value]
        lib.gen_rmat_fill(h, row_ptr.ctypes.data, col.ctypes.data, threads)
    finally:
        lib.gen_free(h)
    return row_ptr, col


def path_graph(n: int):
    return csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle_graph(n: int):
    return csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def star_graph(m: int):
    """K_{1,m}: centre 0, leaves 1..m."""
    return csr_from_edges(m + 1, [(0, i) for i in range(1, m + 1)])


def clique_graph(n: int):
    return csr_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


# ----------------------------------------------------------------------------------------------
# Tree templates
# ----------------------------------------------------------------------------------------------

def pruefer_decode(seq, k: int) -> np.ndarray:
    """Tree on vertices 0..k-1 from a Pruefer sequence of length k-2; returns (k-1, 2) int32."""
    if k == 1:
        return np.zeros((0, 2), dtype=np.int32)
    if k == 2:
        return np.array([[0, 1]], dtype=np.int32)
    seq = list(int(x) for x in seq)
    degree = [1] * k
    for x in seq:
        degree[x] += 1
    import heapq
    leaves = [i for i in range(k) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for x in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, x))
        degree[x] -= 1
        if degree[x] == 1:
            heapq.heappush(leaves, x)
    u = heapq.heappop(leaves)
    w = heapq.heappop(leaves)
    edges.append((u, w))
    return np.array(edges, dtype=np.int32)


def pruefer_tree(k: int, seed: int) -> np.ndarray:
    """Uniform random labelled tree on k vertices (seeded Pruefer sequence)."""
    rng = np.random.default_rng(seed)
    seq = rng.integers(0, k, size=max(k - 2, 0))
    return pruefer_decode(seq, k)


def path_tree(k: int) -> np.ndarray:
    return np.array([(i, i + 1) for i in range(k - 1)], dtype=np.int32).reshape(-1, 2)


def star_tree(k: int) -> np.ndarray:
    return np.array([(0, i) for i in range(1, k)], dtype=np.int32).reshape(-1, 2)


def _rooted_trees(n: int):
    """All rooted unlabelled trees with n vertices as canonical nested tuples (sorted children)."""
    return _rooted_cache(n)


@lru_cache(maxsize=None)
def _rooted_cache(n: int):
    if n == 1:
        return [()]
    out = []
    # children multiset of total size n-1, as non-increasing sequence of canonical subtrees
    ordered = []  # (size, tree) in a fixed total order
    for sz in range(1, n):
        for t in _rooted_cache(sz):
            ordered.append((sz, t))
    idx = {x: i for i, x in enumerate(ordered)}

    def gen(remaining, max_i, acc):
        if remaining == 0:
            out.append(tuple(sorted(acc)))
            return
        for i in range(min(max_i, len(ordered) - 1), -1, -1):
            sz, t = ordered[i]
            if sz <= remaining:
                acc.append(t)
                gen(remaining - sz, i, acc)
                acc.pop()

    gen(n - 1, len(ordered) - 1, [])
    del idx
    return sorted(set(out))


def _tuple_to_edges(t):
    edges = []
    counter = [0]

    def walk(node):
        me = counter[0]
        for ch in node:
            counter[0] += 1
            c = counter[0]
            edges.append((me, c))
            walk(ch)

    walk(t)
    return edges


def _unrooted_canon(k: int, edges) -> str:
    """Canonical string of an unrooted tree (centre-rooted AHU encoding); used only to de-duplicate."""
    adj = [[] for _ in range(k)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    if k <= 2:
        return str(k)
    deg = [len(a) for a in adj]
    layer = [i for i in range(k) if deg[i] == 1]
    left = k
    removed = [False] * k
    while left > 2:
        nxt = []
        for x in layer:
            removed[x] = True
            left -= 1
            for y in adj[x]:
                if not removed[y]:
                    deg[y] -= 1
                    if deg[y] == 1:
                        nxt.append(y)
        layer = nxt
    centres = [i for i in range(k) if not removed[i]]

    def enc(x, p):
        return "(" + "".join(sorted(enc(y, x) for y in adj[x] if y != p)) + ")"

    return min(enc(c, -1) for c in centres)


def all_trees(k: int) -> list[np.ndarray]:
    """All non-isomorphic (unlabelled, unrooted) trees on k vertices, each as a (k-1, 2) edge array."""
    seen = {}
    for t in _rooted_trees(k):
        e = _tuple_to_edges(t)
        key = _unrooted_canon(k, e)
        if key not in seen:
            seen[key] = np.array(e, dtype=np.int32).reshape(-1, 2)
    return [seen[key] for key in sorted(seen)]


# ----------------------------------------------------------------------------------------------
# Explicit colourings (passed to both sides as inputs)
# ----------------------------------------------------------------------------------------------

def colours(n: int, k: int, seed: int) -> np.ndarray:
    """Uniform colouring of n vertices with k colours (uint8), PCG64 draws."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, k, size=n, dtype=np.uint8) if n else np.zeros(0, dtype=np.uint8)


def colour_batch(n: int, k: int, seed: int, count: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, k, size=(count, n), dtype=np.uint8)
