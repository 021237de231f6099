"""The benchmark's command-line contract, run in-process: a request for more
than one GPU exits with a message before any device work (no GPU needed), and
on the GPU one short run prints one JSON line with the metric, the roofline of
the dominant kernel and the configuration."""
import json
import sys

import pytest

import bench


def run_main(argv, capsys):
    old = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        code = 0
        try:
            bench.main()
        except SystemExit as e:
            code = e.code
    finally:
        sys.argv = old
    out = capsys.readouterr()
    return code, out.out, out.err


def test_more_than_one_gpu_exits_with_a_message(capsys):
    code, out, err = run_main(["--gpus", "2"], capsys)
    assert code not in (0, None)
    assert "single GPU" in err
    assert out.strip() == ""


@pytest.mark.gpu
def test_short_run_prints_the_contract_line(capsys):
    code, out, err = run_main(["--positions", "512", "--steps", "4", "--warmup", "1", "--no-cpu-baseline",
                               "--no-learned-init"], capsys)
    assert code in (0, None), err[-2000:]
    lines = [l for l in out.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert abs(d["value"] - d["config"]["global_batch"] / (d["ms_per_step"] * 1e-3)) <= 1e-2 * d["value"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] in ("hbm", "mfma", "alu") and 0 < rf["frac"] < 1
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-3


@pytest.mark.gpu
def test_default_line_carries_learned_init(capsys):
    """The default line's learned-init block (metric 2), with a tiny training
    set: iterations and seconds to the target from both starts."""
    code, out, err = run_main(["--positions", "512", "--steps", "2", "--warmup", "1", "--no-cpu-baseline",
                               "--objects", "40", "--epochs", "2", "--iterations", "30"], capsys)
    assert code in (0, None), err[-2000:]
    d = json.loads([l for l in out.splitlines() if l.strip()][-1])
    blk = d["learned_init"]
    for side in ("learned_init", "plain_init"):
        assert set(blk[side]) >= {"iterations", "seconds"}, blk[side]
    assert blk["training"]["pairs"] == 40 * 64 and blk["training"]["seconds"] > 0
