"""Guaranteed relative error of the FP64 counts, from the summation structure of the kernels.

Every quantity of the dynamic program (Section 2.1, Eq. 1) is a sum of products of non-negative
integers. For such sums the standard first-order bound holds: if a term passes through L rounded
additions on its way into the result and carries a relative error e_t itself, the computed sum has
relative error at most max(e_t) + L u, u = 2^-53; a product of two computed factors has relative
error at most e_a + e_b + u. Per split of the partition (Eq. 1 in its distributive form):

  N(v, Q) = sum_u P(u, .)        e_N <= e_P + L_nbr u
  O(v, S) = sum A(v, S1) N(v, Q) e_O <= e_A + e_N + (L_split + 1) u      (a >= 2)
  O(v, S) = N(v, .)              e_O  = e_N                               (a = 1, a copy)

so the error of the root counts is the sum of the local terms over every split of the partition
(a shared table counts once per use), and the total X adds the root reduction's L_red u. Single
vertices are exact, and so are neighbour sums of single vertices (p = 1: integer counts below
2^53).

L_nbr and L_split follow the kernels' fixed orders:
  * plain light rows: a neighbour's row joins a run of at most 64 equal-colour neighbours of one
    64-entry block (<= 63 additions), and each block folds at most p runs into one entry of N
    (a set Q of p colours receives one run per colour of Q), so L = 63 + p ceil(tau / 64);
  * plain chunks of cut rows: the same with the chunk size c instead of tau, then the chunk
    partials of the row in the blocked order (16, 16, rest: blocked_sum in the device code);
  * packed rows: every entry receives its neighbours' terms one by one in CSR order
    (L = tau - 1 for light rows, c - 1 per chunk), then the same blocked chunk sum;
  * the combine: each output adds its C(s-1, p) products in the blocked order; outputs narrower
    than 32 entries spread their pairs over 64 / G lane groups and add the groups' sums by a
    log2(64 / G) shuffle tree.
"""
from __future__ import annotations

import math

U = 2.0 ** -53


def blocked_len(n: int) -> int:
    """Roundings a term passes through in blocked_sum over n terms (runs of 16, groups of 16 runs,
    then the groups in order)."""
    if n <= 1:
        return 0
    runs = math.ceil(n / 16)
    groups = math.ceil(n / 256)
    return (min(n, 16) - 1) + (min(runs, 16) - 1) + (groups - 1)


def _pow2_at_least(x: int) -> int:
    g = 1
    while g < x:
        g <<= 1
    return g


def split_terms(k: int, s: int, a: int, p: int, *, hub_threshold: int, chunk: int, max_degree: int,
                packed: bool) -> dict:
    """L_nbr and L_split of one split (see the module docstring)."""
    Ws = math.comb(k - 1, s - 1)
    npairs = math.comb(s - 1, p)
    has_hubs = max_degree > hub_threshold
    light_deg = min(hub_threshold, max_degree)
    chunks = math.ceil(max_degree / chunk) if has_hubs else 0
    if p == 1:
        l_light = l_chunk = 0  # integer counts: exact
    elif packed:
        l_light = max(light_deg - 1, 0)
        l_chunk = chunk - 1
    else:
        l_light = 63 + p * math.ceil(light_deg / 64)
        l_chunk = 63 + p * math.ceil(chunk / 64)
    l_nbr = l_light
    if has_hubs and p >= 2:
        l_nbr = max(l_nbr, l_chunk + blocked_len(chunks))
    if a == 1:
        l_split = 0
    elif packed or Ws >= 32:
        l_split = blocked_len(npairs) + 1
    else:
        G = _pow2_at_least(Ws)
        parts = 64 // G
        l_split = blocked_len(math.ceil(npairs / parts)) + int(math.log2(parts)) + 1
    return {"s": s, "a": a, "p": p, "L_nbr": l_nbr, "L_split": l_split, "local": l_nbr + l_split}


def packed_kernel_split(k: int, s: int, a: int, p: int) -> bool:
    """Whether a packed count runs the split on packed rows (every per-colouring width <= 64)."""
    W = lambda t: math.comb(k - 1, t - 1)  # noqa: E731
    return (p < 2 or W(p) <= 64) and W(a) <= 64 and W(s) <= 64


def reduce_len(n: int, packed: bool) -> int:
    """Roundings of a root count in the total X (k_reduce_* kernels)."""
    if n <= 1:
        return 0
    if packed:
        blocks = min(1024, max(1, math.ceil(n / 1024)))
        per = math.ceil(n / blocks)
        return blocked_len(math.ceil(per / 4)) + 3 + blocked_len(blocks)
    blocks = min(1024, max(1, math.ceil(n / 8192)))
    per = math.ceil(n / blocks)
    return (math.ceil(per / 256) - 1) + 8 + (math.ceil(blocks / 256) - 1) + 8


def bound(k: int, splits, ids, *, n: int, max_degree: int, hub_threshold: int, chunk: int,
          path: str = "plain") -> dict:
    """Relative error bound of every table entry at the root and of X.

    splits: (s, a, p) per split in execution order; ids: (act, pas, out) table ids per split
    (-1: a single vertex, out -2: the root). path: "plain" or "packed"."""
    err = {}
    rows = []
    root_e = 0.0
    for (s, a, p), (act, pas, out) in zip(splits, ids):
        packed = path == "packed" and packed_kernel_split(k, s, a, p)
        t = split_terms(k, s, a, p, hub_threshold=hub_threshold, chunk=chunk, max_degree=max_degree,
                        packed=packed)
        e = (err[act] if act >= 0 else 0) + (err[pas] if pas >= 0 else 0) + t["local"]
        t["e_out_u"] = e
        rows.append(t)
        if out >= 0:
            err[out] = e
        else:
            root_e = e
    red = reduce_len(n, path == "packed")
    return {"splits": rows, "root_u": root_e, "X_u": root_e + red, "reduce_L": red,
            "root_rel": root_e * U, "X_rel": (root_e + red) * U}


def plan_bound(plan, graph_info: dict, path: str = "plain") -> dict:
    """bound() for a Plan (paper_1804_09764_amd.Plan) on a prepared graph (Graph.info)."""
    ids = []
    for i in range(plan.info.n_splits):
        m = plan.split_maps(i)
        ids.append((m["act"], m["pas"], m["out"]))
    return bound(plan.k, plan.splits, ids, n=graph_info["n"], max_degree=graph_info["max_degree"],
                 hub_threshold=graph_info["hub_threshold"], chunk=graph_info["chunk"], path=path)
