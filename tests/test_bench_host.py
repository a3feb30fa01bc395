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
