"""The cost model's TDI shape (terms, delay groups, links per delay) against
the oracle's term lists, and the bench's traffic-record bookkeeping."""
import json
from collections import Counter

import pytest

from oracle import tdi_terms
from paper_2204_06633_amd import costs


@pytest.mark.parametrize("gen", [1, 2])
def test_tdi_shape_matches_the_term_lists(gen):
    terms = tdi_terms.michelson_terms(gen)
    direct = [t for t in terms if len(t.path) == 1]
    delayed = [t for t in terms if len(t.path) > 1]

    def delay_key(t):       # multiset of arms (receiver, emitter) the chain sums
        return tuple(sorted(Counter(zip(t.path[:-1], t.path[1:])).items()))

    groups = {delay_key(t) for t in delayed}
    shape = costs.TDI_SHAPE[gen]
    assert shape["direct"] == len(direct)
    assert shape["delayed"] == len(delayed)
    assert shape["groups"] == len(groups)
    links_per_group = sum(sum(n for _, n in g) for g in groups) / len(groups)
    assert shape["mean_links"] == pytest.approx(links_per_group)


def test_recorded_traffic_needs_matching_sources(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    srcs = ("forward_kernels.hpp",)
    assert bench.recorded_traffic("tdi_1yr", srcs) is None            # no record
    rec = {"bytes_per_launch": 123.0, "source_hash": "not-the-sources"}
    (prof / "traffic_tdi_1yr.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda names: "the-sources")
    assert bench.recorded_traffic("tdi_1yr", srcs) is None            # stale record
    rec["source_hash"] = "the-sources"
    (prof / "traffic_tdi_1yr.json").write_text(json.dumps(rec))
    assert bench.recorded_traffic("tdi_1yr", srcs) == 123.0


def test_lane_op_model_matches_the_stated_counts():
    """The FP64 lane-op model: projection 9 x 5N + 9 x 2N + 320, TDI-2 36 x 5N
    + 42 N (weights shared by `share` templates), sky 9 x 19 N + 420."""
    assert costs.lane_ops_projection(25) == 9 * 130 + 9 * 52 + 320 == 1958
    assert costs.lane_ops_tdi(25, 2) == 36 * 130 + 42 * 26 == 5772
    assert costs.lane_ops_tdi(25, 2, share=2) == 36 * 65 + 42 * 26
    assert costs.lane_ops_tdi(25, 1) == 15 * 130 + 18 * 26
    assert costs.lane_ops_sky(25) == 9 * 19 * 26 + 420
    assert costs.LANE_OPS_PEAK == pytest.approx(3.93216e13)
