"""The paper's own timing figures are mutually consistent (context numbers).

The benchmark compares against these numbers only as context; this check
keeps the transcription of Table 1 honest: the fits must reproduce the
timings the paper quotes in prose to within 20 %, and the ratios of the cubic
coefficients must give the quoted CPU-core equivalents to within 10 %.
"""

import json
import os

FIX = os.path.join(os.path.dirname(__file__), "golden", "table1_cubic_fits.json")


def test_table1_reproduces_quoted_timings():
    d = json.load(open(FIX))
    for q in d["quoted"]:
        f = d["fits"][q["device"]]
        n = q["n"]
        y = f["a3"] * n ** 3 + f["a2"] * n ** 2 + f["a1"] * n + f["a0"]
        assert abs(y - q["seconds"]) / q["seconds"] < 0.20, (q, y)


def test_core_equivalents():
    d = json.load(open(FIX))
    cpu = d["fits"]["i9_13th_gen_1thread"]["a3"]
    for dev in ("RTX4070_laptop", "A100_80GB"):
        ratio = cpu / d["fits"][dev]["a3"]
        assert abs(ratio - d["core_equivalents"][dev]) / d["core_equivalents"][dev] < 0.10, ratio
