"""Host-side checks of the benchmark's contract that need no GPU: more than one GPU is refused
with a message (one GPU's path only), and the algorithmic byte counts the roofline uses."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_training_step():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    n, U, C, nvert = 1 << 20, 1_820_000, 10, 128 ** 3
    alg = b.algorithmic_bytes(n, U, C, nvert)
    # the adjoint with Adam: 12 B query + 16 B upstream per query, master/m/v read and written
    assert alg["backward_adam"] == n * 28 + nvert * C * 24
    assert alg["forward_loss"] == n * 32 + U * C * 4


def test_kernel_hash_ignores_comments_only():
    import bench

    a = 'int f(int x) { return x + 1; } // one\n/* two */ const char* s = "a // b /* c */";\n'
    b = '/* other words */ int f(int x)\n{\n    return x + 1;  // changed\n}\nconst char* s = "a // b /* c */";\n'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "a // b /* c */";\n'
    assert bench.strip_comments(a) == bench.strip_comments(b)
    assert bench.strip_comments(a) != bench.strip_comments(c)
    assert '"a // b /* c */"' in bench.strip_comments(a)
