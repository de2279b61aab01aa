"""Host logic of the benchmark's counter-traffic figures: a committed
counter summary is used only for the kernel sources and the variant it was
taken with, and its totals follow from its per-kernel counts."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(name):
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        return json.load(fh)


def test_spmv_summary_totals_follow_from_counts():
    d = _load("spmv_xslice_pmc.json")
    known = d["copy_known_kib_each_way"]
    assert known == 16 * bench.SPMV_COPY_DOUBLES / 2 / 1024
    for key, e in d["variants"].items():
        tot = 0.0
        for k in ("k_xs_products", "k_xs_reduce"):
            c = e[k]
            assert c["fetch_bytes"] == pytest.approx(c["fetch_kib_raw"] * e["fetch_scale"] * 1024)
            assert c["write_bytes"] == pytest.approx(c["write_kib_raw"] * e["write_scale"] * 1024)
            tot += c["fetch_bytes"] + c["write_bytes"]
        assert e["traffic_bytes_per_spmv"] == pytest.approx(tot)
        # the copy reads back its known bytes after scaling: FETCH_SIZE
        # counts about half of a copy's reads on this part, WRITE_SIZE all
        assert 1.9 < e["fetch_scale"] < 2.1 and 0.9 < e["write_scale"] < 1.1


def test_jacobi_summary_totals_follow_from_counts():
    d = _load("jacobi_512_pmc.json")
    assert d["fetch_bytes_per_launch"] == pytest.approx(
        d["fetch_kib_per_launch_raw"] * d["fetch_scale"] * 1024)
    assert d["write_bytes_per_launch"] == pytest.approx(
        d["write_kib_per_launch_raw"] * d["write_scale"] * 1024)
    assert d["traffic_bytes_per_launch"] == pytest.approx(
        d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"])
    assert d["min_traffic_bytes_per_launch"] == 16 * 512 ** 3
    assert d["traffic_bytes_per_launch"] >= d["min_traffic_bytes_per_launch"]


def test_gates_refuse_other_variants_and_sources(monkeypatch):
    d = _load("spmv_xslice_pmc.json")
    key = next(iter(d["variants"]))
    current = bench.source_digest(bench.SPMV_SOURCES) == d["source_sha256"]
    got = bench.spmv_pmc_traffic(key)
    assert got == (d["variants"][key]["traffic_bytes_per_spmv"] if current else None)
    assert bench.spmv_pmc_traffic("family=12 bx=64 by=0") is None
    assert bench.pmc_traffic("family=0 bx=1 by=1") is None
    # another kernel source: no summary applies
    monkeypatch.setattr(bench, "source_digest", lambda names: "0" * 64)
    assert bench.spmv_pmc_traffic(key) is None
    assert bench.pmc_traffic(_load("jacobi_512_pmc.json")["variant"]) is None
    for prof in _load("batch_graph_pmc.json")["profiles"]:
        assert bench.batch_pmc_traffic(prof["autotuned_candidates"]) is None


def test_batch_summaries_match_their_tiles():
    d = _load("batch_graph_pmc.json")
    current = bench.source_digest(bench.BATCH_SOURCES) == d["source_sha256"]
    seen = set()
    for prof in d["profiles"]:
        key = tuple(prof["autotuned_candidates"][3:])
        assert key not in seen  # one summary per tile pair of the large buckets
        seen.add(key)
        assert prof["traffic_bytes_per_replay"] == pytest.approx(
            prof["fetch_bytes_per_replay"] + prof["write_bytes_per_replay"])
        assert prof["traffic_bytes_per_replay"] >= prof["min_traffic_bytes_per_replay"]
        got = bench.batch_pmc_traffic([0, 0, 0] + list(key))
        assert got == (prof["traffic_bytes_per_replay"] if current else None)
    assert bench.batch_pmc_traffic([0, 0, 0, -1, -1]) is None
