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


def test_read_table_round_trip(tmp_path):
    rows = tune.read_table()
    for dt in ("f64", "f32"):
        mine = [r for r in rows if r["dtype"] == dt]
        assert mine[0]["n_lo"] == 128 and mine[-1]["n_max"] == 1 << 20
        assert all(a["n_max"] == b["n_lo"] for a, b in zip(mine, mine[1:]))
    p = tmp_path / "t.h"
    tune.write_table(rows, str(p))
    again = tune.read_table(str(p))
    assert [(r["dtype"], r["n_max"], r["best"], r["best_shared"]) for r in again] == \
        [(r["dtype"], r["n_max"], r["best"], r["best_shared"]) for r in rows]


def test_instance_config_and_cut_offs():
    rows = [{"dtype": "f64", "n_lo": 128, "n_max": 2048, "best": (8, 256), "best_shared": (8, 0)},
            {"dtype": "f64", "n_lo": 2048, "n_max": 8192, "best": (8, 1024),
             "best_shared": (8, 0)},
            {"dtype": "f64", "n_lo": 8192, "n_max": 1 << 20, "best": (8, 0),
             "best_shared": (8, 0)}]
    assert tune.instance_config(rows, "f64", 3000, 1e-2) == (8, 1024)
    assert tune.instance_config(rows, "f64", 3000, 1e-2, cut=2048) == (8, 0)
    assert tune.instance_config(rows, "f64", 1000, 1e-2, cut=2048) == (8, 256)
    # h/eps beyond the binary64 bound for runs of 8: runs of 1, shared
    assert tune.instance_config(rows, "f64", 200, 1e-6) == (1, 0)
    cut = tune.apply_cuts(rows, {"f64": 2048})
    assert [r["best"] for r in cut] == [(8, 256), (8, 0), (8, 0)]
    assert tune.run_length_bound("f32", 4.0) == 16 and tune.run_length_bound("f32", 4.1) == 8
    assert tune.run_length_bound("f32", 20.0) == 4 and tune.run_length_bound("f32", 21.0) == 1


def test_shipped_table_keeps_residents_within_one_chunk():
    # the request server runs every request in shared launches with the batched
    # solve's run length; a resident instance equals a one-chunk shared launch
    # bit for bit only when its workgroup is one chunk (256 threads)
    for r in tune.read_table():
        rr, nt = r["best"]
        assert nt in (0, 256), r
