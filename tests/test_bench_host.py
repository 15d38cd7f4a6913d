"""Host-side logic of the benchmark script: stored HBM-counter lookups and
the single-GPU contract (no GPU needed)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _records():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


def test_traffic_lookup_matches_configuration_and_source(monkeypatch):
    recs = _records()
    assert recs
    # the box and general-mesh kernels are hashed from different sources
    assert bench.kernel_source_hash(False) != bench.kernel_source_hash(True)
    for r in recs:
        gen = r.get("general", False)
        monkeypatch.setattr(bench, "kernel_source_hash", lambda general=False, r=r: r["source"])
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"], general=gen) == r
        # counters of the monatomic gas never stand in for the (F, G) pair
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"], 2.0, general=gen) is None
        # nor for another precision / scheme pair without its own record
        other = [x for x in recs if x["workload"] == r["workload"] and x["precision"] == 1 - r["precision"]
                 and x["rk"] == r["rk"]]
        if not other:
            assert bench.measured_traffic(r["workload"], 1 - r["precision"], r["rk"], general=gen) is None
        # a changed kernel source invalidates the stored counters
        monkeypatch.setattr(bench, "kernel_source_hash", lambda general=False: "0" * 16)
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"], general=gen) is None


def test_traffic_records_are_at_least_algorithmic():
    # counted HBM bytes below the bytes the stage must move would mean a
    # miscalibrated counter scale
    for r in _records():
        assert r["bytes_per_launch"] >= 0.95 * r["algorithmic_bytes_per_launch"]


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode != 0
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_byte_models():
    """Unfused per-DOF traffic of a p = 3 stage: FP64 SSP 56 B, FP32 SSP 28 B,
    FP32 low-storage 32 B; the fused stage kernel's algorithmic bytes averaged
    over the stages of a long call: FP64 SSP 4.17 values (33.3 B), FP32
    low-storage 4.83 values (19.3 B), the FP32 deviation storage the same
    (FP32 state and traces)."""
    import bench
    assert bench.unfused_bytes_per_dof(3, 0, 0) == 56.0
    assert bench.unfused_bytes_per_dof(3, 1, 0) == 28.0
    assert bench.unfused_bytes_per_dof(3, 1, 1) == 32.0
    n = 1000
    assert abs(bench.stage_bytes(3, 0, 0, n) / (3 * n) - 8 * 25 / 6) < 1e-2
    assert abs(bench.stage_bytes(3, 1, 1, n) / (3 * n) - 4 * 29 / 6) < 1e-2
    assert abs(bench.stage_bytes(3, 2, 1, n) / (3 * n) - 4 * 29 / 6) < 1e-2


def test_operator_flop_models():
    # p = 3 (N = 4): per direction 4 multiply-adds of the derivative, one of the
    # metric scaling, one of the lifting, and a quarter of the line's trace
    # (4 multiply-adds) and jump (2 flops): 14.5 flops, 43.5 over 3 directions;
    # dense: 3 x 64 derivative + 96 lifting + 96 interpolation multiply-adds
    assert bench.fr_operator_flops_per_dof(3) == 43.5
    assert bench.fr_dense_flops_per_dof(3) == 768.0
    assert bench.fr_dense_flops_per_dof(1) == 2.0 * (3 * 8 + 2 * 24)


@pytest.mark.parametrize("t,p", [(1, 1), (1, 2), (1, 3), (2, 3)])
def test_mixed_operator_row_counts_match_the_oracle_operators(t, p):
    """The mixed-mesh flop model counts, per solution point, the operator
    entries the kernel reads.  Prisms: the pairs of points on one layer
    (in-plane derivatives, side-face lifting) or one column (axial
    derivative, end-face lifting), found here from the oracle's point
    coordinates; every nonzero entry of the oracle's operators lies among
    them.  Tetrahedra: dense rows, an upper bound of the nonzeros."""
    import bench
    from oracle import mixed as M
    R = M.ref_element([M.HEX, M.PRISM, M.TET][t], p)
    x = R.x
    lift = np.concatenate([fc["lift"] for fc in R.faces], axis=1)
    assert lift.shape[1] == bench.MIXED_SIZES[p][t][1]
    tol_d = 1e-12 * max(np.abs(d).max() for d in R.D)
    tol_l = 1e-12 * np.abs(lift).max()
    if t == 1:
        same_z = np.abs(x[:, None, 2] - x[None, :, 2]) < 1e-12
        same_xy = np.all(np.abs(x[:, None, :2] - x[None, :, :2]) < 1e-12, axis=2)
        pats = [same_z, same_z, same_xy]
        cols = []
        for fc in R.faces:
            end = len(fc["verts"]) == 3
            for node in fc["nodes"]:
                cols.append((same_xy if end else same_z)[:, node])
        lpat = np.stack(cols, axis=1)
        for d, pat in zip(R.D, pats):
            assert np.all(np.abs(d[~pat]) < tol_d)
        assert np.all(np.abs(lift[~lpat]) < tol_l)
        assert sum(int(pt.sum()) for pt in pats) + int(lpat.sum()) == R.ns * bench.mixed_row_madds(t, p)
    else:
        nz = sum(int((np.abs(d) > tol_d).sum()) for d in R.D) + int((np.abs(lift) > tol_l).sum())
        assert nz <= R.ns * bench.mixed_row_madds(t, p) == R.ns * (3 * R.ns + lift.shape[1])
