"""CPU checks of the benchmark's command line: the JSON line is measured on
one GPU, so a request for several exits at once with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_profile_summaries_name_their_commands():
    # every committed summary states the command that produced it
    prof = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(prof)):
        text = open(os.path.join(prof, f)).read()
        assert "rocprofv3" in text or "python" in text, f
