"""Host-side parts of the autotuner: workload keys and the JSON cache."""
import json

import pytest


def test_workload_key_buckets():
    from paper_2107_12672_amd import autotune as at, ddvr as d
    k1 = at.workload_key("gfx950", d.ABSORPTION, "bf16", 0, 512, 256, "V", d.PASS_FUSED)
    k2 = at.workload_key("gfx950", d.ABSORPTION, "bf16", 7, 400, 200, "V", d.PASS_FUSED)
    assert k1 == k2 == "gfx950|ao|bf16|R0|img512|grid256|V|pass2"
    k3 = at.workload_key("gfx950", d.EMISSION_ABSORPTION, "f16", 20, 1024, 512, "V+TF+step",
                         d.PASS_ADJOINT)
    assert k3 == "gfx950|ea|f16|R32|img1024|grid512|V+TF+step|pass1"


def test_class_keys_are_distinct_and_candidates_valid():
    """Every tuned class has its own key, and every candidate set holds only
    launch shapes the library accepts (all fields, valid ranges)."""
    from paper_2107_12672_amd import autotune as at, ddvr as d
    keys = [at.c1_key("gfx950"), at.c2_key("gfx950"), at.c4_key("gfx950"),
            at.color_key("gfx950", "bf16", 512, 256),
            at.workload_key("gfx950", d.ABSORPTION, "bf16", 0, 512, 256, "V", d.PASS_FUSED)]
    assert len(set(keys)) == len(keys)
    assert keys[0] == "gfx950|ao|f32|R0|img64|grid32|V|pass2"
    assert keys[1] == "gfx950|ea|f32|R16|img256|grid128|V+TF+cam+step|pass2"
    for cands in (at.default_candidates(), at.uneven_candidates(), at.small_candidates(),
                  at.color_candidates()):
        assert cands
        for c in cands:
            assert set(c) == set(d.TUNING_DEFAULT)
            assert c["waves"] in (1, 2, 4) and 64 <= c["lds_cap"] <= 16384
            assert 4 <= c["slab_k"] <= c["slab_kmax"] <= 4096
            assert c["slab_axis"] in (0, 1) and 0 <= c["lane_map"] <= 3


def test_cache_roundtrip_and_apply(tmp_path):
    from paper_2107_12672_amd import autotune as at, ddvr as d
    path = str(tmp_path / "cache.json")
    assert at.lookup("k", path) is None
    t = dict(d.TUNING_DEFAULT, waves=2, lds_cap=4096)
    at.save_cache({"k": {"tuning": t, "ms": 1.0}, "bad": {"tuning": {"waves": 2}}}, path)
    assert at.lookup("k", path) == t
    assert at.lookup("bad", path) is None          # incomplete entries are ignored
    old = d.get_tuning()
    try:
        assert at.apply("k", path)
        assert d.get_tuning() == t
        assert not at.apply("missing", path)
        assert d.get_tuning() == t
    finally:
        d.set_tuning(**old)
    json.load(open(path))
