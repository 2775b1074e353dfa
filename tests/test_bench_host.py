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


def _stats_csv(path):
    with open(path, "w") as f:
        f.write("Name,Calls,TotalDurationNs,AverageNs,Percentage\n")
        f.write('"void ips::k_lds_bitonic<ips::TQuartet, 512u>(x)",6,6000000,1000000,60.0\n')
        f.write('"void ips::k_permute<ips::TQuartet, 256u>(x)",6,4000000,666666.7,40.0\n')


def test_kernel_stats_summary_names_the_traced_command(tmp_path, capsys):
    csv_path = str(tmp_path / "kq_kernel_stats.csv")
    _stats_csv(csv_path)
    assert bench.kernel_stats_summary(csv_path, "--workload sweep --only quartet") == 0
    out = capsys.readouterr().out
    assert out.startswith("# Kernel time, generator sweep: quartet\n")
    assert "-o kq -- python3 $R/bench.py --workload sweep --only quartet`" in out
    assert f'--kernel-stats-summary {csv_path} --trace-args "--workload sweep --only quartet"' in out
    assert "| 6 | 6000.0 | 1000.0 | 60.00 |" in out
    assert bench.kernel_stats_summary(csv_path) == 0
    out = capsys.readouterr().out
    assert out.startswith("# Kernel time, u64 Uniform n=2^28, IPS4o samplesort\n")
    assert "--trace-args" not in out


def test_committed_kernel_time_profiles_name_their_commands():
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if not name.startswith("kernel_time_"):
            continue
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        traced = txt.split("-- python3 $R/bench.py ", 1)[1].split("`", 1)[0]
        table = txt.split("table from `python3 bench.py --kernel-stats-summary ", 1)[1].split("`", 1)[0]
        if traced != "--steps 3 --warmup 1 --no-cpu --no-radix":
            assert table.endswith(f'--trace-args "{traced}"'), name
