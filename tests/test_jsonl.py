"""JSON Lines export of the per-step records (write_jsonl / read_jsonl and the
Run / Batch exporters)."""
import io
import json
import math

import pytest

import paper_2102_06611_amd as pa


def _strict(line):
    def no_constant(name):
        raise ValueError("non-standard JSON constant %s" % name)
    return json.loads(line, parse_constant=no_constant)


def _same(a, b):
    if isinstance(a, float) and isinstance(b, float) and math.isnan(a) and math.isnan(b):
        return True
    return a == b and type(a) is type(b)


def test_roundtrip_keeps_values_order_and_nonfinite_numbers(tmp_path):
    recs = [
        {"step": 0, "R_i": 100, "beta": 0.0, "sum_E": -(2 ** 62), "e": -1.25, "r_eff_E": math.inf,
         "err_e": math.nan, "jk_cov_e": -math.inf},
        {"step": 1, "R_i": 101, "beta": 0.1, "sum_E": 12345678901234, "e": 1e-300,
         "r_eff_E": 42.5, "err_e": 0.0, "jk_cov_e": -0.0},
    ]
    path = tmp_path / "r.jsonl"
    assert pa.write_jsonl(recs, str(path), L=8, seed=7, resample="nearest") == 2
    lines = path.read_text().splitlines()
    assert len(lines) == 2
    for line, rec in zip(lines, recs):
        obj = _strict(line)  # strict JSON: no bare NaN / Infinity
        assert list(obj)[:3] == ["L", "seed", "resample"]
        assert list(obj)[3:] == list(rec)
    back = pa.read_jsonl(str(path))
    for got, rec in zip(back, recs):
        assert got["L"] == 8 and got["seed"] == 7 and got["resample"] == "nearest"
        for k, v in rec.items():
            assert _same(got[k], v), (k, got[k], v)
    # open file objects work both ways, and an empty iterable writes nothing
    buf = io.StringIO()
    assert pa.write_jsonl(iter(recs), buf) == 2
    buf.seek(0)
    assert len(pa.read_jsonl(buf)) == 2
    assert pa.write_jsonl([], str(tmp_path / "empty.jsonl")) == 0
    assert pa.read_jsonl(str(tmp_path / "empty.jsonl")) == []


@pytest.mark.gpu
def test_run_and_batch_exports_match_observables(tmp_path):
    import torch
    from workloads import linear_schedule
    torch.cuda.set_device(0)
    betas = linear_schedule(0.44, 5)
    run = pa.Run(8, 200, betas, 2, 99, "nearest", "msc64")
    run.run(5)
    path = tmp_path / "run.jsonl"
    assert run.export_jsonl(str(path)) == 6
    back = pa.read_jsonl(str(path))
    for i, got in enumerate(back):
        want = run.observables(i)
        assert got["L"] == 8 and got["R"] == 200 and got["seed"] == 99
        for k, v in want.items():
            assert _same(got[k], v), (i, k, got[k], v)
    assert run.export_jsonl(str(path), first=2, last=3) == 2
    assert [r["step"] for r in pa.read_jsonl(str(path))] == [2, 3]
    run.close()

    specs = [dict(L=8, R=130, theta=1, seed=5, betas=betas, resample="multinomial"),
             dict(L=16, R=70, theta=2, seed=6, betas=betas, layout="int8")]
    b = pa.Batch(specs)
    b.run(3)
    bpath = tmp_path / "batch.jsonl"
    assert b.export_jsonl(str(bpath)) == 2 * 4
    back = pa.read_jsonl(str(bpath))
    for got in back:
        want = b.observables(got["run"], got["step"])
        assert got["L"] == specs[got["run"]]["L"]
        for k, v in want.items():
            assert _same(got[k], v), (got["run"], k, got[k], v)
    assert [(r["run"], r["step"]) for r in back] == [(r, i) for r in range(2) for i in range(4)]
    b.close()
