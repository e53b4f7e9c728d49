"""Host-side tests of the automatic tile-row choice (ccl_wave_plan_rows).

For 2D the library picks the rows per tile that minimise
rounds x streamed rows, where a K-chunk launch of a depth-T kernel runs
sum_k ceil(rows_k / r) * strips waves in ceil(waves / slots) rounds, and
each wave streams r + 2T rows rounded up to whole loop bodies (3 rows for
the in-place T = 1 update, 12 for float32 at T > 1).  Here that cost is
evaluated for every admissible r by brute force and compared with the
library's choice; slots come from ccl_wave_slots, so the test holds with
or without a device.  No kernel is launched.
"""
import pytest

import paper_2505_06022_amd as ccl


def _strip_width(T, nv=4):
    overlap = nv * ((T + nv - 1) // nv)
    return 64 * nv - 2 * overlap


def _cost_table(ny, nx, K, T, slots):
    strips = -(-nx // _strip_width(T))
    chunk_rows = [(k + 1) * ny // K - k * ny // K for k in range(K)]
    granule = 3 if T == 1 else 12
    lo, hi = max(8, T), max(max(chunk_rows), 8)
    table = {}
    for r in range(lo, hi + 1):
        waves = sum(-(-rows // r) for rows in chunk_rows) * strips
        rounds = -(-waves // slots)
        streamed = -(-(r + 2 * T) // granule) * granule
        table[r] = (rounds, rounds * streamed)
    return table


@pytest.mark.parametrize("shape,K", [((8192, 8192), 4), ((1000, 3000), 3), ((77, 300), 1),
                                     ((4096, 640), 16), ((300, 20000), 2)])
@pytest.mark.parametrize("T", [1, 2, 5, 8])
def test_plan_rows_minimises_rounds_times_streamed(shape, K, T):
    slots = ccl.ccl_wave_slots(2, T)
    assert slots >= 1
    r = ccl.ccl_wave_plan_rows(ccl.make_tune_config(shape, K, T))
    table = _cost_table(shape[0], shape[1], K, T, slots)
    assert r in table, f"rows {r} outside [{min(table)}, {max(table)}]"
    best = min(c for _, c in table.values())
    rounds, cost = table[r]
    assert cost == best, f"{shape} K={K} T={T}: rows {r} cost {cost}, best {best}"
    # among the rows that fit in the same number of rounds, the fewest
    assert all(table[q][0] > rounds for q in table if q < r)


@pytest.mark.parametrize("T", [1, 4, 8])
def test_plan_rows_keeps_an_explicit_choice(T):
    assert ccl.ccl_wave_plan_rows(ccl.make_tune_config((8192, 8192), 4, T, 32)) == 32


@pytest.mark.parametrize("shape,K,T", [((768, 768, 768), 8, 1), ((768, 768, 768), 8, 7),
                                       ((40, 36, 130), 3, 4), ((97, 64, 64), 1, 8)])
def test_plan_planes_within_the_chunk(shape, K, T):
    z = ccl.ccl_wave_plan_rows(ccl.make_tune_config(shape, K, T))
    zmax = max((k + 1) * shape[0] // K - k * shape[0] // K for k in range(K))
    assert 4 <= z <= max(zmax, 4)


def test_plan_rows_rejects_malformed_configs():
    with pytest.raises(ccl.CclError):
        ccl.ccl_wave_plan_rows(ccl.make_tune_config((16, 16), 17, 2))  # more chunks than rows
    with pytest.raises(ccl.CclError):
        ccl.ccl_wave_plan_rows(ccl.make_tune_config((16, 16), 1, 9))   # T above the maximum
    with pytest.raises(ccl.CclError):
        ccl.ccl_wave_plan_rows(ccl.make_tune_config((0, 16), 1, 2))    # empty extent
