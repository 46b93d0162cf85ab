"""Host logic of bench.py (no GPU): the algorithmic byte model of the fused stage call, the count of
same-level faces per axis that sizes the halo copies, and the readers of the committed counter
summaries with their digest and workload guards."""
import os
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2406_11626_amd import ccz4  # noqa: E402


def fake_ctx(n0, bc, ids):
    return types.SimpleNamespace(n0=tuple(n0), bc=bc, ids=np.array(ids, dtype=np.int32))


def faces_by_brute_force(n0, bc, ids):
    """The same count from the definition, through dense per-level occupancy arrays."""
    count = [0, 0, 0]
    levels = {}
    for lev, i, j, k in ids:
        n = [v * 3 ** lev for v in n0]
        grid = levels.setdefault(lev, np.zeros(n[::-1], bool))
        grid[k, j, i] = True
    for lev, grid in levels.items():
        for a in range(3):
            ax = 2 - a
            for d in (-1, 1):
                shifted = np.roll(grid, -d, axis=ax)
                if bc != ccz4.BC_PERIODIC:  # no wrap: the row rolled past the edge has no neighbour
                    idx = [slice(None)] * 3
                    idx[ax] = -1 if d > 0 else 0
                    shifted[tuple(idx)] = False
                count[a] += int((grid & shifted).sum())
    return count


def test_same_level_faces_uniform_meshes():
    ids = [(0, i, j, k) for k in range(16) for j in range(16) for i in range(16)]
    assert bench.same_level_faces_per_axis(fake_ctx((16, 16, 16), ccz4.BC_SOMMERFELD, ids)) == [7680] * 3
    ids = [(0, i, j, k) for k in range(3) for j in range(2) for i in range(1)]
    # periodic: every leaf has both neighbours along every axis (itself along x)
    assert bench.same_level_faces_per_axis(fake_ctx((1, 2, 3), ccz4.BC_PERIODIC, ids)) == [12, 12, 12]


@pytest.mark.parametrize("bc", [ccz4.BC_SOMMERFELD, ccz4.BC_PERIODIC])
def test_same_level_faces_on_a_refined_mesh_match_brute_force(bc):
    """Two refined level-0 cubes (27 level-1 leaves each), one of them split again in a corner: the
    coarse-fine faces are not counted, the faces inside each refined block are."""
    n0 = (4, 3, 2)
    refined = {(1, 1, 0), (2, 1, 1)}
    ids = [(0, i, j, k) for k in range(2) for j in range(3) for i in range(4) if (i, j, k) not in refined]
    fine = [(1, 3 * i + a, 3 * j + b, 3 * k + c) for (i, j, k) in sorted(refined)
            for c in range(3) for b in range(3) for a in range(3)]
    split = fine.pop(0)
    ids += fine
    ids += [(2, 3 * split[1] + a, 3 * split[2] + b, 3 * split[3] + c)
            for c in range(3) for b in range(3) for a in range(3)]
    got = bench.same_level_faces_per_axis(fake_ctx(n0, bc, ids))
    assert got == faces_by_brute_force(n0, bc, ids)
    assert all(v > 0 for v in got)


def test_stage_bytes_closed_forms():
    """Per interior cell: Q_s halo-inclusive (58 evolved slots x 3 cell-vectors + K_0) plus the
    stream of the stage; per pushed face 243 cells x 59 slots; per Sommerfeld face the ghost update."""
    cv = 8 * 59
    qs = 8 * (58 * 3 + 1)
    for s, stream in ((0, 3), (1, 4), (2, 4), (3, 2)):
        assert bench.stage_bytes(s, 1, 0) == qs + stream * cv
    assert bench.stage_bytes(1, 0, 1) == 243 * cv
    assert bench.stage_bytes(1, 0, 0, 3) == pytest.approx(3 * 243 * cv * (4 / 3 + 5))
    assert bench.stage_bytes(3, 0, 0, 1) == pytest.approx(243 * cv * (4 / 3 + 3))
    mean = sum(bench.stage_bytes(s, 1, 0) for s in range(4)) / 4
    assert mean == 2934


def write_record(path, **rec):
    with open(path, "w") as f:
        f.write("# a counter summary\n\nsome text\n\n")
        for k, v in rec.items():
            f.write(f"- {k}: {v}\n")


def test_profile_readers_guard_digest_and_workload(tmp_path, monkeypatch):
    digest = bench.kernel_source_digest()
    t, fl = tmp_path / "traffic.md", tmp_path / "ops.md"
    monkeypatch.setattr(bench, "traffic_file", lambda config: str(t))
    monkeypatch.setattr(bench, "flops_file", lambda config: str(fl))
    assert bench.measured_traffic(2) is None and bench.measured_fp64_ops(2) == (None, None)
    write_record(t, hbm_bytes_per_launch=2.5e10, source_sha256=digest, workload_config=2)
    write_record(fl, fp64_ops_per_stage_launch=2.75e10, fp64_ops_per_rhs_launch=2.6e10, source_sha256=digest,
                 workload_config=2)
    assert bench.measured_traffic(2) == 2.5e10
    assert bench.measured_fp64_ops(2) == (2.75e10, 2.6e10)
    assert bench.measured_traffic(3) is None  # another workload
    write_record(t, hbm_bytes_per_launch=2.5e10, source_sha256="0" * 64, workload_config=2)
    assert bench.measured_traffic(2) is None  # the kernels changed since the counters were taken
    r = bench.fp64_rate(2.75e10, 5.5)
    assert r["achieved"] == pytest.approx(5.0) and r["frac"] == pytest.approx(5.0 / 78.6)
    assert bench.fp64_rate(None, 5.5) is None


def test_committed_profiles_parse():
    """The committed summaries carry the fields the readers take (whatever their digest)."""
    import glob
    files = [(p, ("hbm_bytes_per_launch",)) for p in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))]
    files += [(p, ("fp64_ops_per_stage_launch", "fp64_ops_per_rhs_launch"))
              for p in glob.glob(os.path.join(ROOT, "profiles", "*_fp64_ops.md"))]
    assert files
    for path, keys in files:
        rec = {}
        with open(path) as fh:
            lines = fh.read().splitlines()
        for ln in lines:
            if ln.startswith("- ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                rec[k.strip()] = v.strip()
        for k in keys + ("source_sha256", "workload_config"):
            assert k in rec, (path, k)
        for k in keys:
            assert float(rec[k]) > 0
