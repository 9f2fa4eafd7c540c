"""Host checks of bench.py's accounting (no GPU): the algorithmic bytes the
roofline divides by, the index widths they assume, the committed counter
entries, and the single-GPU guard."""
import json
import pathlib
import subprocess
import sys

import bench

ROOT = pathlib.Path(__file__).resolve().parents[1]


def test_algorithmic_bytes_of_the_512_projector():
    # A of the 512^2 workload: 120,155,712 nonzeros, 261,000 rays x 262,144
    # pixels, 32-bit columns (n > 65536), window of ell + 1 = 3 w-vectors.
    # Written out: values + columns, row pointers, z once, w once, window once.
    nnz, m, n = 120155712, 261000, 262144
    want = 12 * nnz + 4 * (m + 1) + 8 * n + 8 * m + 8 * m * 3
    assert want == 1453361700
    assert bench.spmv_bytes(nnz, m, n, m, 3, bench.index_bytes(n, "CSR-stream")) == want


def test_sixteen_bit_columns_only_where_the_kernels_read_them():
    assert bench.index_bytes(65536, "CSR-stream") == 2
    assert bench.index_bytes(65536, "SELL-64") == 2
    assert bench.index_bytes(65537, "CSR-stream") == 4
    assert bench.index_bytes(4096, "wave/row") == 4
    # 10 bytes per nonzero instead of 12, the rest unchanged
    assert (bench.spmv_bytes(1000, 10, 20, 10, 2, 2) + 2 * 1000
            == bench.spmv_bytes(1000, 10, 20, 10, 2, 4))


def test_committed_counter_entries_are_consistent():
    entries = json.loads((ROOT / "profiles" / "traffic.json").read_text())
    entries = entries if isinstance(entries, list) else [entries]
    assert entries
    for tr in entries:
        for k, total in tr["bytes_per_launch"].items():
            assert total == tr["read_bytes_per_launch"][k] + tr["write_bytes_per_launch"][k]
        assert tr["fetch_scale"] > 0 and tr["write_scale"] > 0
        if tr["workload"] == "ct512_sparse":
            # the operator stream alone exceeds the last-level cache: HBM reads
            # cannot fall below the algorithmic bytes, and are within 1.3x
            alg = bench.spmv_bytes(120155712, 261000, 262144, 261000, 3, 4)
            assert alg <= tr["read_bytes_per_launch"]["spmv_A"] <= 1.3 * alg


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
