"""The one-workload-per-process entry point the profiler commands use
(`python -m paper_1110_4623_amd.run ...`): each workload prints its JSON line."""

import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT, announce

pytestmark = pytest.mark.gpu

CASES = [
    ["barrier", "--kind", "xcd", "--nwg", "256", "--rounds", "100"],
    ["barrier", "--kind", "default", "--nwg", "32", "--rounds", "100"],
    ["mutex", "--kind", "cohort", "--nwg", "256", "--total", "4096"],
    ["sem", "--kind", "xcd_chain", "--nwg", "256", "--total", "4096", "--K", "32"],
    ["sem", "--kind", "chain", "--nwg", "256", "--total", "4096", "--K", "32", "--data"],
    ["copy", "--bytes", str(1 << 24)],
    ["micro", "--op", "ld", "--T", "4096", "--nwg", "64", "--ops", "4"],
    ["serve", "--rate", "1e5", "--n", "2000"],
]


@pytest.mark.parametrize("args", CASES, ids=lambda a: "-".join(a[:3]))
def test_run_prints_one_json_line(args):
    announce("run.py", " ".join(args))
    env = dict(os.environ, SP_NO_TORCH="1")
    p = subprocess.run([sys.executable, "-u", "-m", "paper_1110_4623_amd.run", *args], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [json.loads(l) for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1 and lines[0]["what"] == args[0]
    if "--data" in args:
        assert lines[0]["data_sum"] == 4096
    if args[0] == "barrier":
        assert lines[0]["kind"] == ("central" if "32" in args else "xcd")
        assert lines[0]["us_per_round"] > 0
