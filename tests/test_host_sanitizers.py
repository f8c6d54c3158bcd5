"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the C oracle (gcc): encode / decode round trips, thresholds checked row by row
  against counts of the uncompressed words, random word sequences fed to the decoder;
* the library's host code (hipcc; the sanitizers on the host side only, the device
  code built as usual and never run): the registration-time validation and index
  builder on well-formed and corrupted streams, the output bound, the variant codes,
  and the selector's model-file reader on valid, truncated and corrupted files.

Both harnesses live in tests/csrc/ and exit non-zero on the first wrong result;
either sanitizer aborts the run on the first error it finds.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1402_4466_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fno-sanitize-recover=all"]


def _run(exe, cwd):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], cwd=cwd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", *SAN, "-o", exe,
                    os.path.join(ROOT, "tests", "csrc", "oracle_sanitize_check.c"),
                    os.path.join(ROOT, "oracle", "ewah_oracle.c")], check=True)
    _run(exe, str(tmp_path))


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = []
    for src in ("thr_tile.hip", "select.hip", "mlp.hip", "selector.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run([HIPCC, *flags, "-c", "-o", o, os.path.join(CSRC, src)], check=True,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        objs.append(o)
    main = str(tmp_path / "main.o")
    subprocess.run([HIPCC, *flags, "-c", "-o", main, os.path.join(ROOT, "tests", "csrc", "host_sanitize_check.cpp")],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    exe = str(tmp_path / "host_san")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", exe, *objs, main], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    _run(exe, str(tmp_path))
