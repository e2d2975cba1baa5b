"""bench.py's host-side contract (no GPU): more than one GPU is refused with
a message, and the digest that gates the reported HBM traffic ignores
comments but not code."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_digest_sees_code_not_comments():
    import bench
    a = "int f(int x) {  // doubles x\n  return 2 * x; /* twice */\n}\n"
    b = "/* helper */\nint f(int x) {\n\n  return 2 * x;   // the same\n}\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert len(bench.source_digest()) == 16
