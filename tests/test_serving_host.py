"""Host-side serving logic on the CPU: footprints come from exact sector
dimensions (character formula) that match the oracle's enumeration."""
import pytest

import oracle
from paper_2308_16712_amd import serve
from workloads import configs


@pytest.mark.parametrize("sec", [configs.ring_symmetric(12, 0, 1, 1), configs.ring_symmetric(14, 7, -1, -1),
                                 configs.ring_symmetric(13, 2, 0, 0), configs.square_j1j2(4, 3),
                                 configs.ring16_u1()], ids=lambda s: s.name)
def test_sector_dimension_matches_oracle(sec):
    assert serve.sector_dimension(sec) == oracle.count_basis(oracle.Problem(sec))


def test_serving_trace_config_dimensions():
    trace = configs.serving_trace(count=40)
    dims = {r.sector.name.split("_j2")[0]: serve.sector_dimension(r.sector) for r in trace}
    assert dims.get("square6x6", 15804956) == 15804956
    assert dims.get("ring36_k0_r1_z1", 63068876) == 63068876
    assert dims.get("square6x4", 15578) == 15578


def test_footprint_grows_with_krylov_dimension():
    sec = configs.ring_symmetric(20, 0, 1, 1)
    assert serve.footprint_bytes(sec, 200) > serve.footprint_bytes(sec, 50) > 0


def test_records_summary():
    st = serve.ServeStats()
    for k in range(10):
        st.records.append(serve.Record(k, "x", 1, arrival=0.0, done=0.01 * (k + 1)))
    st.makespan = 0.1
    s = st.summary()
    assert s["requests"] == 10 and abs(s["throughput_rps"] - 100.0) < 1e-9
    assert 50.0 <= s["p50_ms"] <= 60.0 and s["p99_ms"] <= 100.0
