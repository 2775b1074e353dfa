"""Host-side parts of bench.py: the profile summaries name the commands that
produced them, and those commands are the ones bench.py writes."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _code_block(path):
    lines = open(path).read().splitlines()
    a = lines.index("```")
    b = lines.index("```", a + 1)
    return lines[a + 1:b]


def test_traffic_summary_commands_match_writer():
    path = os.path.join(ROOT, "profiles", "hbm_traffic_u64_uniform_2p28.md")
    cmds = _code_block(path)
    folders = cmds[-1].split("--traffic-summary", 1)[1].split()
    assert len(folders) == 4
    assert bench.traffic_commands(*folders) == cmds


def test_from_root_keeps_absolute_paths():
    assert bench._from_root("/abs/dir") == "/abs/dir"
    assert bench._from_root("rel/dir") == "$R/rel/dir"


def test_gpu_count_above_one_is_refused(capsys):
    old = sys.argv
    sys.argv = ["bench.py", "--gpus", "2"]
    try:
        assert bench.main() == 2
    finally:
        sys.argv = old
    assert "one GPU" in capsys.readouterr().err
