"""bench.py's command line without a GPU: more than one GPU is refused with
a message (the library runs one code on one GPU) before anything is
measured, and every option is documented; the traffic figure and the
committed kernel summaries belong to the current round-kernel source."""
import os
import subprocess
import sys

ROOT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    out = r.stdout + r.stderr
    assert "one GPU only" in out and "--gpus 2" in out
    assert not any(line.startswith("{") for line in r.stdout.splitlines())  # no result line


def test_every_option_has_help():
    r = run("--help")
    assert r.returncode == 0
    lines = r.stdout.split("options:", 1)[1].splitlines()
    opts = [l.strip() for l in lines if l.strip().startswith("--")]
    assert len(opts) >= 18
    for i, l in enumerate(lines):
        s = l.strip()
        if s.startswith("--"):
            # help on the same line, or on the next, indented deeper
            same = len(s.split()) > 2 or (len(s.split()) == 2 and not s.split()[1].isupper())
            nxt = i + 1 < len(lines) and lines[i + 1].startswith(" " * 20) and not lines[i + 1].strip().startswith("-")
            assert same or nxt, s


def test_traffic_figure_and_profiles_match_the_kernel_source():
    """The line's HBM traffic and the committed rocprofv3 summaries were taken
    on one version of the round kernel: the sources must still hash to it, and
    the summaries must name that hash (and the traffic summary the same bytes)."""
    code = ("import bench, json; print(json.dumps([bench.kernel_fingerprint(), bench.TRAFFIC['fingerprint'], "
            "bench.TRAFFIC['bytes_per_launch']]))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    import json
    now, taken, nbytes = json.loads(r.stdout.strip().splitlines()[-1])
    assert now == taken, "round.hip or kernels.hpp changed since the traffic counters were taken"
    prof = os.path.join(ROOT, "profiles")
    for name in ("round_kernel_config3_every_word_hbm_traffic.md", "round_kernel_config3_every_word_kernel_trace.md",
                 "round_kernel_config3_kernel_trace.md", "round_kernel_config3_counters.md"):
        with open(os.path.join(prof, name)) as fh:
            text = fh.read()
        assert now in text, name
    with open(os.path.join(prof, "round_kernel_config3_every_word_hbm_traffic.md")) as fh:
        assert str(nbytes) in fh.read()
