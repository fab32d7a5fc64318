"""The timeline metrics P1, P2, P3 (Sec. 5): interval arithmetic pinned to a
brute-force count over unit cells, a hand-worked timeline, and the reader of
rocprofv3 CSV traces on a small synthetic trace with rocprofv3's columns."""
import numpy as np
import pytest

from paper_1901_06798_amd import timeline as T


def cells(intervals, n):
    """Unit cells [k, k + 1] covered by integer intervals (brute force)."""
    cov = np.zeros(n, dtype=bool)
    for a, b in intervals:
        cov[int(a):int(b)] = True
    return cov


def random_intervals(rng, k, n):
    out = []
    for _ in range(k):
        a = int(rng.integers(0, n - 1))
        b = int(rng.integers(a, n))
        out.append((a, b))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_union_and_difference_match_a_cell_count(seed):
    rng = np.random.default_rng(seed)
    n = 60
    A = random_intervals(rng, 7, n)
    B = random_intervals(rng, 5, n)
    assert T.measure(A) == cells(A, n).sum()
    assert T.measure(A + B) == (cells(A, n) | cells(B, n)).sum()
    assert T.measure(T.difference(A, B)) == (cells(A, n) & ~cells(B, n)).sum()
    # merged intervals are disjoint and sorted
    m = T.merge(A)
    assert all(m[i][1] < m[i + 1][0] for i in range(len(m) - 1))
    assert T.clip(A, 10, 20) == [(max(a, 10), min(b, 20)) for a, b in A if min(b, 20) > max(a, 10)]


def test_metrics_of_a_hand_worked_timeline():
    # run [0, 10]: GPU busy [0, 4], CPU busy [3, 6], copies [5, 8] and [9, 10]
    # -> P1 = 4/10, P2 = 3/10; copies outside computation [6, 8] and [9, 10]: P3 = 3/10
    p = T.p_metrics([(0, 4)], [(3, 6)], [(5, 8)], [(9, 10)], (0, 10))
    assert p["P1"] == pytest.approx(0.4) and p["P2"] == pytest.approx(0.3)
    assert p["P3"] == pytest.approx(0.3)
    # events outside the run are clipped; overlapping events count once
    p = T.p_metrics([(-5, 2), (1, 3), (9, 20)], [], [], [], (0, 10))
    assert p["P1"] == pytest.approx(0.4) and p["P2"] == 0.0 and p["P3"] == 0.0
    with pytest.raises(ValueError):
        T.p_metrics([], [], [], [], (3, 3))


def write(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            f.write(",".join(f'"{v}"' if isinstance(v, str) else str(v) for v in r) + "\n")


def test_reader_of_rocprof_csv(tmp_path):
    write(tmp_path / "run_marker_api_trace.csv",
          ["Domain", "Function", "Process_Id", "Thread_Id", "Correlation_Id", "Start_Timestamp",
           "End_Timestamp"],
          [["MARKER_CORE_RANGE_API", "serve warm-up", 1, 1, 1, 0, 50],
           ["MARKER_CORE_RANGE_API", "serve 200 GB", 1, 1, 2, 100, 200],
           ["MARKER_CORE_RANGE_API", "host: admit", 1, 1, 3, 100, 120],
           ["MARKER_CORE_RANGE_API", "host: enqueue", 1, 1, 4, 130, 150]])
    write(tmp_path / "run_memory_copy_trace.csv",
          ["Kind", "Direction", "Stream_Id", "Source_Agent_Id", "Destination_Agent_Id",
           "Correlation_Id", "Start_Timestamp", "End_Timestamp"],
          [["MEMORY_COPY", "MEMORY_COPY_HOST_TO_DEVICE", 0, "Agent 0", "Agent 1", 5, 115, 125],
           ["MEMORY_COPY", "MEMORY_COPY_DEVICE_TO_HOST", 0, "Agent 1", "Agent 0", 6, 185, 195],
           ["MEMORY_COPY", "MEMORY_COPY_DEVICE_TO_DEVICE", 0, "Agent 1", "Agent 1", 7, 160, 170]])
    write(tmp_path / "run_kernel_trace.csv",
          ["Kind", "Agent_Id", "Queue_Id", "Kernel_Name", "Correlation_Id", "Start_Timestamp",
           "End_Timestamp"],
          [["KERNEL_DISPATCH", "Agent 1", 1, "k", 8, 10, 40],
           ["KERNEL_DISPATCH", "Agent 1", 1, "k", 9, 140, 180],
           ["KERNEL_DISPATCH", "Agent 1", 1, "k", 10, 170, 190]])
    p = T.from_rocprof(str(tmp_path), "serve 200 GB")
    # run [100, 200]: GPU [140, 190] = 50; CPU [100, 120] + [130, 150] = 40;
    # copies [115, 125] and [185, 195] outside computation: [120, 125] and [190, 195]
    assert p["P1"] == pytest.approx(0.5) and p["P2"] == pytest.approx(0.4)
    assert p["P3"] == pytest.approx(0.1)
    assert p["h2d"] == 1 and p["d2h"] == 1 and p["host_ranges"] == 2
    assert p["span_ms"] == pytest.approx(100e-6)
    with pytest.raises(ValueError):
        T.from_rocprof(str(tmp_path), "serve 1 GB")
