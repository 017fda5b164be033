"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run on its own pins (tests/oracle_sanitize_test.c):
no memory error, no undefined behaviour, every pin holds."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitize_test"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-ffp-contract=off", "-Wall", "-Wextra",
                    os.path.join(ROOT, "oracle", "fractal_oracle.c"),
                    os.path.join(ROOT, "tests", "oracle_sanitize_test.c"),
                    "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "oracle sanitized pins ok" in out.stdout
