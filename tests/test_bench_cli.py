"""bench.py's command line without a GPU: more than one GPU is refused with
a message (the library runs one code on one GPU) before anything is
measured, and every option is documented."""
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
