"""The benchmark's JSONL output: each run appends its per-step records and
then its result line, one JSON object per line (CPU only; no GPU call)."""
import json
import os
import sys
import types

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_emit_appends_records_then_result(tmp_path, capsys):
    path = tmp_path / "runs.jsonl"
    args = types.SimpleNamespace(jsonl=str(path))
    bench.emit({"metric": "m", "value": 1.5}, args, [{"step": 0, "ms": 2.0}, {"step": 1, "ms": 3.0}])
    bench.emit({"metric": "m", "value": 2.5}, args)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert lines == [{"step": 0, "ms": 2.0}, {"step": 1, "ms": 3.0},
                     {"metric": "m", "value": 1.5}, {"metric": "m", "value": 2.5}]
    printed = capsys.readouterr().out.splitlines()
    assert [json.loads(x)["value"] for x in printed] == [1.5, 2.5]


def test_emit_without_jsonl_only_prints(tmp_path, capsys):
    bench.emit({"metric": "m", "value": 1.0}, types.SimpleNamespace(jsonl=None))
    assert json.loads(capsys.readouterr().out)["value"] == 1.0
    assert list(tmp_path.iterdir()) == []
