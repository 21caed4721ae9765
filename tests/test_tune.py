"""The tuner's host side: its size classes cover 129 ... 2^20 without gaps,
its record of the built-in rule matches the rule the library applies without
a table row, and the table it writes has one row per class in ascending
order (the library takes the first row with n <= n_max)."""
import re

from paper_2202_10042_amd import tune


def test_classes_cover_the_range():
    cl = tune.classes()
    assert cl[0][0] == 128 and cl[-1][1] == 1 << 20
    assert all(a[1] == b[0] for a, b in zip(cl, cl[1:]))
    assert all(lo < hi for lo, hi in cl)


def test_rule_record():
    assert tune.rule_config("f32", 4096) == (16, 256)
    assert tune.rule_config("f32", 5000) == (8, 1024)
    assert tune.rule_config("f32", 9000) == (16, 0)
    assert tune.rule_config("f64", 2048) == (8, 256)
    assert tune.rule_config("f64", 8192) == (8, 1024)
    assert tune.rule_config("f64", 8193) == (8, 0)


def test_written_table(tmp_path):
    rows = []
    for dt in ("f64", "f32"):
        for lo, hi in tune.classes():
            n = (lo + hi) // 2
            rows.append({"dtype": dt, "n_lo": lo, "n_max": hi, "n": n, "instances": 8,
                         "best": tune.rule_config(dt, n), "best_shared": (8, 0),
                         "rule": tune.rule_config(dt, n),
                         "us_per_instance_iteration": {
                             f"{r}x{nt}": 1.0 for r, nt in [tune.rule_config(dt, n), (8, 0)]}})
    p = tmp_path / "t.h"
    tune.write_table(rows, str(p))
    body = p.read_text()
    got = re.findall(r"\{(\d), (\d+), (\d+), (\d+), (\d+)\}", body)
    assert len(got) == len(rows)
    for dt in ("0", "1"):
        nmax = [int(g[1]) for g in got if g[0] == dt]
        assert nmax == sorted(nmax) and nmax[-1] == 1 << 20
