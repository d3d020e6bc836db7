"""The FP64 oracle and the host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU needed).

* The oracle's C source and a driver that calls every entry point on small
  ragged volumes (tests/native/oracle_exercise.c) are built with gcc and
  ``-fsanitize=address,undefined``; any invalid access, leak or undefined
  operation aborts the run.
* The library's host code (argument checks, workspace carving, contexts,
  batches) is rebuilt with the sanitizers on its host pass only and linked
  with the library's other objects and a driver
  (tests/native/abi_host_checks.c) that makes every host-answered call.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, "%s\n%s%s" % (" ".join(cmd), p.stdout, p.stderr)
    return p


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_exercise")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "oracle", "disc_oracle.c"), os.path.join(NATIVE, "oracle_exercise.c"), "-lm",
          "-o", exe])
    p = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle exercise: ok" in p.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_abi_host_checks_under_sanitizers(tmp_path):
    from paper_1204_6295_amd import build

    objdir = build.OBJDIR
    if not os.path.isdir(objdir) or not any(f.endswith(".o") for f in os.listdir(objdir)):
        build.build()
    others = sorted(os.path.join(objdir, f) for f in os.listdir(objdir)
                    if f.endswith(".o") and f != "disc_api.o")
    # sanitizers on the host pass only: the device code is built as usual
    host_san = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "disc_api.o")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops"] + host_san + ["-I" + os.path.join(ROOT, "include"),
                                                      "-I" + build.CSRC, "-c",
                                                      os.path.join(build.CSRC, "disc_api.hip"), "-o", api])
    main = str(tmp_path / "main.o")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"), "-c",
          os.path.join(NATIVE, "abi_host_checks.c"), "-o", main])
    exe = str(tmp_path / "abi_host_checks")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined", main, api] + others +
         ["-o", exe])
    p = _run([exe], env=SAN_ENV, timeout=300)
    assert "abi host checks: ok" in p.stdout
