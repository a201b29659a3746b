"""Host-side configuration that the GPU runs depend on, checked on the CPU.

- bench.py is a one-GPU benchmark: any other GPU count is refused with a JSON
  error line and a nonzero exit, before anything touches a device.
- Every entry of the autotuner's tuning.json is usable: its key names the
  precision, solver and nested grid list of the workload it was measured on,
  and its values lie in the ranges mlsgd_set_tuning accepts.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("gpus", ["2", "8"])
def test_bench_refuses_more_than_one_gpu(gpus):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", gpus],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == int(gpus)


def test_tuning_entries_are_usable():
    sys.path.insert(0, ROOT)
    from paper_2606_09291_amd import inputs
    prec_code = {"fp64": 0, "mixed": 1, "mixed_bf16": 2}
    with open(os.path.join(ROOT, "paper_2606_09291_amd", "tuning.json")) as fh:
        table = json.load(fh)
    assert table
    for key, entry in table.items():
        arch, p, s, grids = key.split(":")
        assert arch == "gfx950"
        grid = [int(n) for n in grids.split("x")]
        # nested 2^m + 1 grids, each twice the one before
        for a, b in zip(grid, grid[1:]):
            assert b - 1 == 2 * (a - 1)
        assert all(((n - 1) & (n - 2)) == 0 and n >= 5 for n in grid)
        w = inputs.WORKLOADS[entry["workload"]]
        assert list(w.grid_n) == grid
        assert int(p[1:]) == prec_code[w.precision]
        assert int(s[1:]) == (0 if w.solver == "cg" else 1)
        t = entry["tuning"]
        assert t["smoother"] in (0, 1, 2)
        assert 1 <= t["sweeps"] <= 8
        assert 0.0 < t["omega"] < 2.0
        assert 0.0 < t["cheb_lo"] < 1.0
        assert t["tile_y"] in (4, 8, 16)
        assert 8 <= t["xchunk"] <= 1024
        assert t["cache"] in (0, 1)
        assert entry["ms"] > 0


def test_roofline_counts_algorithmic_bytes_only():
    """The bench's roofline record for the fused post-smoothing pass divides
    the algorithmic bytes (x and b read, x'' written, the coarse correction at
    one eighth of a point: 25 B per interior point in FP64; the coefficient at
    0 B, since the method regenerates it) by the live average launch time;
    the coefficient cache it reads on top is reported apart."""
    sys.path.insert(0, ROOT)
    import bench
    pts = 16 * 127 ** 3
    tm = {"ms": 2.0 * 0.5, "launches": 2, "bytes": 2 * 25.0 * pts}
    r = bench.roofline(tm, 2, 129, "fp64")
    assert r["algorithmic_bytes_per_point"] == 25.0
    assert r["interior_points_per_launch"] == pytest.approx(pts)
    assert r["achieved"] == pytest.approx(25.0 * pts / 0.5e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["coefficient_cache_bytes_per_launch"] == pytest.approx(8.0 * pts)
    rm = bench.roofline({"ms": 1.0, "launches": 1, "bytes": 12.5 * pts}, 2, 129, "mixed")
    assert rm["algorithmic_bytes_per_point"] == 12.5
    assert rm["coefficient_cache_bytes_per_launch"] == pytest.approx(4.0 * pts)
