"""The benchmark's output contract: one JSON line holding the fields a run is
read by (throughput, configuration, roofline of the dominant pass, CPU
baseline), and a refusal of more than one GPU.  bench.main runs in this
process (no child process is started from a process that uses the GPU)."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

TOP_KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline")
ROOF_KEYS = ("bound", "achieved", "peak", "unit", "frac", "traffic")


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    out = capsys.readouterr()
    assert out.out.strip() == ""
    assert "one GPU" in out.err


@pytest.mark.gpu
def test_json_line_of_a_short_run(capsys):
    argv = ["--size", "2048", "--steps", "1", "--warmup", "0", "--no-cpu", "--no-ttt", "--no-batch", "--no-unet",
            "--no-psnr", "--no-dict"]
    assert bench.main(argv) in (0, None)
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.strip()]
    assert len(lines) == 1, lines
    d = json.loads(lines[0])
    for k in TOP_KEYS:
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"].startswith("two-step solve, 2048x2048")
    ro = d["roofline"]
    for k in ROOF_KEYS:
        assert k in ro, k
    assert ro["bound"] in ("hbm", "alu")
    assert ro["unit"] == ("GB/s" if ro["bound"] == "hbm" else "TFLOP/s")
    assert 0 < ro["frac"] < 1
    assert ro["frac"] == pytest.approx(ro["achieved"] / ro["peak"], rel=1e-12)
    assert d["cpu_baseline"] is None  # --no-cpu


def test_unet_forward_roofline_counts_every_layer():
    """The network's per-layer roofline at 4096^2: the MFMA work is the 14
    convolutions' 2 P cout kpad (K padded to 32), the bytes at least every
    convolution's bf16 input and output, and the time at least the larger of
    the two totals over their peaks."""
    from paper_2406_18356_amd import unet_layers

    n = 4096
    flops, nbytes, secs = bench.unet_forward_roofline(n)
    lay = unet_layers(32, 4)
    lvl = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0]
    want = sum(2.0 * ((n * n) >> (2 * j)) * co * kpad for (ci, co, kpad), j in zip(lay, lvl))
    assert flops == pytest.approx(want, rel=1e-12)
    outs = sum(((n * n) >> (2 * j)) * co * 2 for (ci, co, kpad), j in zip(lay, lvl))
    assert nbytes > 2 * outs  # every output written once and read at least once
    assert secs >= max(flops / (bench.BF16_MFMA_TFLOPS * 1e12), nbytes / (bench.HBM_PEAK_GBS * 1e9))
