"""The tuning table (paper_1406_7416_amd/tuning.json, written by the offline sweep in
paper_1406_7416_amd/tune.py) and the header the build generates from it."""
import json
import os

import pytest

from paper_1406_7416_amd import build as B
from paper_1406_7416_amd import tune

HERE = os.path.dirname(os.path.abspath(__file__))


def test_committed_table_names_known_classes_and_parameters():
    t = B.load_tuning()
    assert t["classes"], "empty tuning table"
    for key, params in t["classes"].items():
        d, N, prec = key.split(",")
        assert int(d) in (2, 3) and 1 <= int(N) <= 9 and prec in ("fp32", "fp64")
        assert set(params) <= set(B.TUNE_KEYS)
        assert params.get("pred_tb", 256) in (64, 128, 256, 512)
        assert 1 <= params.get("sub_wps", 2) <= 4 and params.get("corr_cpb", 4) in (1, 2, 4, 8)
    # every chosen value is one the sweep measured: the fastest of its stage, or the defaults
    # when they are within the stored margin of it
    for key, m in t.get("measured", {}).items():
        cls, group = key.rsplit(":", 1)
        ms = m["ms_per_step"]
        best = min(range(len(ms)), key=lambda i: ms[i])
        if ms[0] <= t.get("margin", 1.0) * ms[best]:
            best = 0
        names = {"predictor": ("pred_tb", "pred_wps"), "corrector_detect": ("corr_cpb",),
                 "subcell": ("sub_wps",)}[group]
        assert [t["classes"][cls][n] for n in names] == m["options"][best]
    assert t["classes"] == tune.choose(t["measured"])


def test_header_overrides_only_named_parameters():
    h = B.tuning_header({"classes": {"2,5,fp32": {"sub_wps": 4}, "3,3,fp64": {"pred_tb": 128, "corr_cpb": 2}}})
    assert "template <> struct Tune<2, 5, true> : TuneDefault<2, 5, true> {" in h
    assert "static constexpr int sub_wps = 4;" in h
    assert "template <> struct Tune<3, 3, false> : TuneDefault<3, 3, false> {" in h
    assert h.count("static constexpr") == 3
    with pytest.raises(ValueError):
        B.tuning_header({"classes": {"2,5,fp32": {"warp_size": 32}}})


def test_sweep_variants_cover_the_defaults_first():
    v0 = tune.variant_table(0)["classes"]
    for key, params in v0.items():
        d, N, prec = key.split(",")
        f32 = prec == "fp32"
        assert params["pred_tb"] == 256 and params["pred_wps"] == (4 if f32 else 2)
        assert params["corr_cpb"] == 4
    for i in range(tune.NVAR):
        for key, params in tune.variant_table(i)["classes"].items():
            N = int(key.split(",")[1])
            assert params["corr_cpb"] <= 4 or N <= 3
