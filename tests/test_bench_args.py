"""bench.py's step defaults (CPU only; nothing is run).

A whole sliced permanent (the 48 x 48 workload: minutes per step) is timed
once by default, and a checkpoint, which resumes one permanent, allows only
that single step: further steps would resume a complete checkpoint and time
no work.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def parse(argv, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
    a = bench.parse()
    return a.steps, a.warmup


def test_defaults(monkeypatch):
    assert parse([], monkeypatch) == (5, 1)  # the 40 x 40 complex workload, ~4 s a step
    assert parse(["--workload", "c3"], monkeypatch) == (5, 1)
    assert parse(["--workload", "c2"], monkeypatch) == (20, 3)
    assert parse(["--workload", "c8"], monkeypatch) == (3, 1)
    assert parse(["--workload", "c5", "--terms-log2", "30"], monkeypatch) == (20, 3)
    assert parse(["--workload", "c5"], monkeypatch) == (1, 0)
    assert parse(["--slices", "4"], monkeypatch) == (1, 0)
    assert parse(["--workload", "c5", "--checkpoint", "ck.jsonl"], monkeypatch) == (1, 0)
    assert parse(["--steps", "5", "--warmup", "0"], monkeypatch) == (5, 0)
    assert parse(["--steps", "20", "--warmup", "5"], monkeypatch) == (20, 5)


@pytest.mark.parametrize("argv", [["--workload", "c5", "--checkpoint", "c", "--steps", "2"],
                                  ["--workload", "c5", "--checkpoint", "c", "--warmup", "1"],
                                  ["--steps", "0"], ["--warmup", "-1"],
                                  ["--workload", "c6", "--n", "47"],
                                  ["--workload", "c6", "--n", "66"],
                                  ["--workload", "dense", "--n", "65"]])
def test_rejected(argv, monkeypatch):
    with pytest.raises(SystemExit):
        parse(argv, monkeypatch)


def test_traffic_lines_parse():
    """Every TRAFFIC line of the committed counter summaries names a kernel, a
    source hash and two byte counts; kernel names may hold spaces."""
    import re
    pdir = os.path.join(ROOT, "profiles")
    seen = 0
    for fn in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, fn)) as fh:
            for line in fh:
                if not line.startswith("TRAFFIC "):
                    continue
                kv = bench.parse_traffic_line(line)
                assert set(kv) == {"kernel", "src", "fetch_bytes", "write_bytes"}, (fn, kv)
                assert int(kv["fetch_bytes"]) > 0 and int(kv["write_bytes"]) > 0
                assert re.fullmatch(r"[0-9a-f]{16}", kv["src"])
                seen += 1
    assert seen >= 4


def test_oracle_check_int01_sign_and_coverage():
    """The 0/1 check turns Ryser's subset sum, (-1)^n per(A), into per(A)
    before comparing, and refuses a sample that is not the whole permanent.
    A planted sign error in the comparison would fail one of the two n."""
    import numpy as np
    import oracle
    from types import SimpleNamespace
    oracle.build(force=False)
    for n, seed in ((7, 2), (8, 1)):
        A = (np.random.default_rng(seed).random((n, n)) < 0.6).astype(np.uint8)
        per = oracle.brute(A)
        raw = oracle.ryser_range(A, 0, 1 << n)
        good = bench.oracle_check("int01", n, None, SimpleNamespace(exact=per), 1 << n, raw)
        assert good["checked"] and good["exact_match"]
        bad = bench.oracle_check("int01", n, None, SimpleNamespace(exact=per + 1), 1 << n, raw)
        assert bad["checked"] and not bad["exact_match"]
        part = bench.oracle_check("int01", n, None, SimpleNamespace(exact=per), 1 << (n - 1), raw)
        assert not part["checked"]


def test_complex_rel_err_formula():
    """complex_rel_err measures |g - want| / |want| on the double-double parts
    exactly: a known perturbation of each part gives the known error, and a
    result equal to the oracle's gives 0."""
    import math
    from types import SimpleNamespace
    from oracle import CPair, Pair
    want = CPair(Pair(3.0, 2.0 ** -60), Pair(-4.0, 0.0))
    same = SimpleNamespace(re_hi=3.0, re_lo=2.0 ** -60, im_hi=-4.0, im_lo=0.0)
    assert bench.complex_rel_err(same, want) == 0.0
    off = SimpleNamespace(re_hi=3.0, re_lo=2.0 ** -60 + 3e-9, im_hi=-4.0, im_lo=4e-9)
    assert math.isclose(bench.complex_rel_err(off, want), 5e-9 / 5.0, rel_tol=1e-9)


def test_more_than_one_gpu_refused(monkeypatch, capsys):
    """The benchmark measures one GPU: --gpus above 1 ends with a message
    (and exit status 2) before anything touches a device."""
    import json
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
