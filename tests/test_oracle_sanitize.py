"""The oracle's C part under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

tests/oracle_sanitize_main.c drives every entry point of oracle/sc_oracle.c on a small
sector (M = 8, 3 + 2 electrons, the full sector of 1568 determinants and a 300-determinant
subset); built with -fsanitize=address,undefined and no recovery, any out-of-bounds access,
leak or undefined operation ends the run with an error.  The run also checks that the two
dense-H routes agree and that the per-key w_a / H_aa routine reproduces the P listing.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_c_under_asan_ubsan():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_sanitize")
        cmd = [gcc, "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               os.path.join(ROOT, "oracle", "sc_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
               "-o", exe, "-lm"]
        b = subprocess.run(cmd, capture_output=True, text=True)
        if b.returncode != 0 and ("asan" in b.stderr.lower() or "ubsan" in b.stderr.lower()):
            pytest.skip("sanitizer runtime not available: " + b.stderr.strip()[-200:])
        assert b.returncode == 0, b.stderr
        env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        print(r.stdout, r.stderr[-2000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert r.stdout.startswith("OK")
