"""Host logic of bench.py (no GPU): the calls of a chunked step."""
import bench


def test_chunk_slices_cover_every_shower_once_within_the_call_size():
    for n, chunk in ((1_000_000, 2000), (10, 3), (5, 5), (5, 7), (1, 1)):
        calls = bench.chunk_slices(n, chunk)
        assert all(0 < m <= chunk for _, m in calls)
        covered = [i for s0, m in calls for i in range(s0, s0 + m)] if n < 100 else None
        if covered is not None:
            assert covered == list(range(n))
        assert sum(m for _, m in calls) == n
        assert all(calls[k][0] + calls[k][1] == calls[k + 1][0] for k in range(len(calls) - 1))
    assert bench.chunk_slices(0, 4) == []


def test_oracle_baseline_runs_in_host_processes():
    """The all-core leg of the CPU baseline: worker processes each take every
    k-th shower of the sample and report what they did in the time given."""
    import numpy as np
    from paper_2202_05012_amd import workloads
    w = workloads.WORKLOADS["e10_normal_5planes_1k"]
    geom = workloads.geometry(w)
    ids = np.arange(40)
    n1, s1, t1 = bench.oracle_sample_rate(w, geom, ids, 1, 0.2, False)
    n2, s2, t2 = bench.oracle_sample_rate(w, geom, ids, 2, 0.5, False)
    assert n1 > 0 and s1 > 0 and t1 >= 0.2
    assert n2 > 0 and s2 > 0 and t2 >= 0.5
