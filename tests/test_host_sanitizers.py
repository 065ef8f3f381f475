"""The host code of libdrot.so under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The host translation units (drot_host.hip, drot_batch.hip, drot_mlp.hip)
are compiled with the sanitizers on the host side only (`-Xarch_host
-fsanitize=...`); the kernel launchers of drot_kernels.hip are replaced by
stubs that fail (tests/abi_sanitize_stubs.cpp: nothing here reaches a
launch, and building the sweep's many kernel variants would take minutes).
They are linked with tests/abi_sanitize_driver.cpp and run: every C-ABI
entry point's argument validation, the static-scratch size check of
drot_solve_noalloc, context-less calls and the warm-start network's checks,
with the sanitizers watching for out-of-bounds accesses, use after free and
undefined behaviour."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_11738_amd", "csrc")
# (source, compile host code only)
SOURCES = [(os.path.join(CSRC, "drot_host.hip"), False), (os.path.join(CSRC, "drot_batch.hip"), True),
           (os.path.join(CSRC, "drot_mlp.hip"), False),
           (os.path.join(ROOT, "tests", "abi_sanitize_stubs.cpp"), True),
           (os.path.join(ROOT, "tests", "abi_sanitize_driver.cpp"), True)]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not found")


def test_abi_validation_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", *SAN,
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src, host_only in SOURCES:
        obj = str(tmp_path / (os.path.basename(src).split(".")[0] + ".o"))
        cmd = [hipcc, *common, *(["--offload-host-only"] if host_only else []), "-x", "hip",
               "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT)))
        objs.append(obj)
    for cmd, pr in procs:
        out = pr.communicate()[0].decode(errors="replace")
        assert pr.returncode == 0, " ".join(cmd) + "\n" + out
    exe = str(tmp_path / "driver")
    link = subprocess.run([hipcc, "--offload-arch=gfx950", *SAN, *objs, "-o", exe],
                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    assert link.returncode == 0, link.stdout.decode(errors="replace")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(res.stdout[-3000:], res.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in res.stderr
    assert "runtime error" not in res.stderr
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("0 failures")
