"""bench.py's host-side pieces, on the CPU: the refusal of several GPUs, the byte models' relations,
the request generator of the serving leg, and the two rocprofv3 summarisers (synthetic CSV files
in rocprofv3's column layout) that write the committed profiles."""
import csv
import json
import math
import os
import subprocess
import sys
import types

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N, NNZ = 8388608, 3595472962  # R-MAT scale 23, edge factor 256


def test_refuses_several_gpus():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


@pytest.mark.parametrize("split", [(7, 1, 6), (6, 1, 5), (12, 7, 5), (5, 3, 2), (3, 1, 2), (2, 1, 1), (4, 3, 1)])
def test_byte_models_are_ordered(split):
    """Per launch: the method's needed entries <= the 128-byte lines holding them; every array once
    (compulsory) <= the lines when the passive rows are wide. p = 1 reads no passive rows."""
    k = 12
    s, a, p = split
    m = bench.method_bytes(k, s, a, p, N, NNZ)
    lines = bench.loaded_bytes(k, s, a, p, N, NNZ)
    assert m <= lines
    if p == 1:
        assert m == lines
        assert m < bench.split_bytes(k, s, a, p, N, NNZ)
    # the passive term of the method: (k-1)/k of the entries read C(k-2, p-1) doubles
    if p >= 2:
        per_vertex = 8 * (N + 1) + N + 8 * N * math.comb(k - 1, s - 1) + (8 * N * math.comb(k - 1, a - 1) if a >= 2 else 0)
        passive = m - 5 * NNZ - per_vertex
        assert abs(passive - 8 * math.comb(k - 2, p - 1) * NNZ * (k - 1) / k) <= 1e-6 * passive


def test_projected_rows_read_fewer_lines_than_stored_rows():
    # the headline's dominant split: 16 lines of needed entries instead of 21.7 per neighbour row
    k, s, a, p = 12, 7, 1, 6
    stored = bench.loaded_bytes(k, s, a, p, N, NNZ)
    projected = bench.loaded_bytes_projected(k, s, a, p, N, NNZ, 4)
    assert projected < stored
    assert bench.method_bytes(k, s, a, p, N, NNZ) < projected


def test_packed_model_at_one_colouring_matches_the_stored_row_model():
    k, s, a, p = 7, 4, 1, 3
    n, nnz = 262144, 7609396
    one = bench.method_bytes_packed(k, s, a, p, n, nnz, 1)
    assert abs(one - bench.method_bytes(k, s, a, p, n, nnz)) < 1.0
    assert bench.packed_kernel_split(k, s, a, p)
    assert not bench.packed_kernel_split(12, 7, 1, 6)


def test_requests_are_seeded_and_rate_independent():
    pool = bench.SERVE_POOL
    a = bench.make_requests(50, pool, seed=9, rate=0, b_range=(8, 16), max_scale=20, large=0.1)
    b = bench.make_requests(50, pool, seed=9, rate=5.0, b_range=(8, 16), max_scale=20, large=0.1)
    assert [(r.rid, r.graph_id, r.B, r.k) for r in a] == [(r.rid, r.graph_id, r.B, r.k) for r in b]
    assert all(r.arrival == 0.0 for r in a)
    arrivals = [r.arrival for r in b]
    assert arrivals == sorted(arrivals) and arrivals[0] > 0
    assert all(pool[r.graph_id][0] <= 20 for r in a)
    assert all(8 <= r.B <= 16 or bench.LARGE_B[0] <= r.B <= bench.LARGE_B[1] for r in a)
    assert all(5 <= r.k <= 12 for r in a)


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_stats_table(tmp_path, capsys):
    d = tmp_path / "prof"
    _write_csv(str(d / "x" / "head_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs"], [
        ["void cc::(anonymous namespace)::k_split<4, 0>(cc::StepParams)", 12, 3000000000],
        ["cc::k_hub_finish(cc::StepParams)", 4, 4000000],
        ["void cc::k_project<true>(double const*, long)", 3, 60000000],
    ])
    args = types.SimpleNamespace(stats_dir=str(d), title="t", command="c", workload=bench.DEFAULT_WORKLOAD)
    bench.summarize_stats(args)
    out = capsys.readouterr().out
    assert "| k_split<4, 0> | 12 | 3000.00 | 250.000 |" in out
    assert "| k_project<true> | 3 | 60.00 | 20.000 |" in out
    assert "| k_hub_finish | 4 | 4.00 | 1.000 |" in out


def test_summarize_pmc_sums_the_dominant_split(tmp_path, monkeypatch):
    """Two colourings of a three-split count; the dominant split (1) runs a copy and two kernels.
    FETCH_SIZE of a 1 GiB copy reads half its bytes (factor 2), WRITE_SIZE all of them (factor 1)."""
    seq = [["k_edge_colours", -1], ["k_split", 0], ["k_project", 1], ["k_split", 1], ["k_hub_finish", 1],
           ["k_split", 2], ["k_reduce_blocks", -1], ["k_reduce_final", -1]]
    dm = tmp_path / "dmap.json"
    json.dump({"sequence": seq, "dominant_split": 1}, open(dm, "w"))
    gib_kib = float(1 << 30) / 1024.0
    header = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]

    def rows(counter, copy_kib, per_kernel):
        out, i = [], 0
        for _ in range(3):  # three copies of the calibration; the middle value is used
            i += 1
            out.append([i, "__amd_rocclr_copyBuffer", counter, copy_kib])
        for _ in range(2):
            for name, split in seq:
                i += 1
                out.append([i, f"void cc::{name}<4, 0>(cc::StepParams)", counter, per_kernel(name, split)])
        return out

    fetch = lambda name, split: 100.0 if split == 1 else 7.0  # noqa: E731
    write = lambda name, split: 10.0 if split == 1 else 3.0  # noqa: E731
    _write_csv(str(tmp_path / "f" / "a_counter_collection.csv"), header, rows("FETCH_SIZE", gib_kib / 2, fetch))
    _write_csv(str(tmp_path / "w" / "a_counter_collection.csv"), header, rows("WRITE_SIZE", gib_kib, write))
    out = tmp_path / "pmc.json"
    args = types.SimpleNamespace(fetch_dir=str(tmp_path / "f"), write_dir=str(tmp_path / "w"), dispatch_map=str(dm),
                                 copy_bytes=float(1 << 30), workload=bench.DEFAULT_WORKLOAD, command="c", out=str(out))
    bench.summarize_pmc(args)
    res = json.load(open(out))
    assert res["colourings"] == 2 and res["split_index"] == 1
    assert res["fetch_kib_per_colouring"] == 300.0 and res["write_kib_per_colouring"] == 30.0
    assert res["copy_fetch_factor"] == 2.0 and res["copy_write_factor"] == 1.0
    assert res["traffic_bytes_per_launch"] == 300.0 * 1024 * 2 + 30.0 * 1024
    assert res["kernels"] == ["k_hub_finish", "k_project", "k_split"]


def test_reference_plan_model_on_the_3_path():
    """The 3-path rooted at its centre: splits (2, 1, 1) then (3, 2, 1); the combine's multiply-adds
    per vertex are C(3,2) C(2,1) + C(3,3) C(3,2) = 9, and the CSEU units per edge 1 + 1 = 2."""
    import inputs
    r = bench.reference_plan_model(inputs.path_tree(3), nnz=10, colourings=2, seconds=1.0)
    assert sorted(tuple(x) for x in r["splits"]) == [(2, 1, 1), (3, 2, 1)]
    assert r["combine_fma_per_vertex"] == 9
    assert r["units_per_edge"] == 2
    assert r["paper_model_ops_per_s"] == 10 * 9 * 2
