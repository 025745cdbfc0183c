"""Command-line front end: argument handling (CPU) and one short sweep (GPU)."""
import json

import pytest


def test_codes_lists_presets(capsys):
    from paper_1204_0334_amd.__main__ import main
    assert main(["codes"]) == 0
    out = capsys.readouterr().out
    assert "qc36_p3060" in out and "cc36_p512" in out and "table2_D" in out


def test_unknown_code_and_missing_p():
    from paper_1204_0334_amd.__main__ import main
    with pytest.raises(SystemExit):
        main(["sweep", "--code", "nope", "--ebn0", "1.0"])
    with pytest.raises(SystemExit):
        main(["sweep", "--shifts", "x.json", "--ebn0", "1.0"])


@pytest.mark.gpu
def test_sweep_resumes_from_log(tmp_path, capsys):
    from paper_1204_0334_amd.__main__ import main
    log = tmp_path / "s.jsonl"
    args = ["sweep", "--code", "qc36_p64", "--ebn0", "1.0", "--iters", "10", "--gamma", "256",
            "--min-errors", "20", "--max-frames", "4096", "--log", str(log)]
    assert main(args) == 0
    first = [json.loads(x) for x in capsys.readouterr().out.splitlines() if x.startswith("{")]
    lines = log.read_text().splitlines()
    assert main(args) == 0                      # finished point: read back, not run again
    second = [json.loads(x) for x in capsys.readouterr().out.splitlines() if x.startswith("{")]
    assert log.read_text().splitlines() == lines
    assert first == second and first[0]["frames"] > 0
