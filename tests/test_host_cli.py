"""Host-side behaviour that needs no GPU: bench.py refuses more than one GPU, and
the package fails loudly (ImportError) when the HIP library has not been built,
instead of falling back to any CPU path."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable] + args, cwd=ROOT, env=e, capture_output=True, text=True, timeout=120)


def test_bench_refuses_several_gpus():
    r = _run(["bench.py", "--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_bench_refuses_a_multi_rank_launch():
    r = _run(["bench.py"], env={"WORLD_SIZE": "4"})
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_missing_library_raises_instead_of_falling_back():
    code = ("from paper_2012_11430_amd import _lib\n"
            "_lib.LIB_PATH = '/nonexistent/libprony.so'\n"
            "try:\n"
            "    _lib.load()\n"
            "except ImportError as e:\n"
            "    print('raised', 'is missing' in str(e))\n")
    r = _run(["-c", code])
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "raised True"
