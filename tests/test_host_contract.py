"""Host-side contract checks that need no GPU: the product path refuses to
run without its HIP library (there is no CPU fallback), and the benchmark
refuses a multi-GPU request instead of reporting a single-GPU figure."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(code_or_args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable] + code_or_args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


def test_binding_fails_loudly_without_the_library():
    code = ("from paper_2210_07501_amd import lbm\n"
            "try:\n"
            "    lbm.load()\n"
            "except RuntimeError as e:\n"
            "    print('refused:', e)\n"
            "else:\n"
            "    raise SystemExit('loaded a library that does not exist')\n")
    r = run(["-c", code], {"LBM_LIBRARY": os.path.join(ROOT, "no_such_dir", "liblbm.so")})
    assert r.returncode == 0, r.stderr
    assert "refused:" in r.stdout and "not built" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    r = run(["bench.py", "--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
