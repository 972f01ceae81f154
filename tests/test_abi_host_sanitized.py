"""The C ABI's argument validation under the host AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/abi_host_check.hip calls every entry point with invalid arguments
(zero, negative and overflowing sizes, inconsistent dimensions, NULL pointers,
unknown modes) on a plain host context and checks that each returns its error
status with a message before any GPU work.  rif_api.hip (the validation layer)
and the check are built with the host sanitizers (-Xarch_host keeps them off
the GPU code) and linked against the library's other objects as built; no GPU
is needed or touched.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2012_15662_amd")
CSRC = os.path.join(PKG, "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _objects():
    """The library's objects except the ABI layer's, building them if needed."""
    from paper_2012_15662_amd import build as b
    objdir = os.path.join(PKG, "_build")
    srcs = [s for s in b.sources() if os.path.basename(s) != "rif_api.hip"]
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    stale = any(not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(s) for s, o in zip(srcs, objs))
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    newest_hdr = max(os.path.getmtime(h) for h in hdrs)
    if stale or any(os.path.getmtime(o) < newest_hdr for o in objs):
        b.build()
    return objs


def test_abi_validation_under_host_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    from paper_2012_15662_amd import build as b
    flags = [f for f in b.HIPFLAGS if f not in ("-shared", "-O3")] + ["-O1", "-g"] + SAN
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    api_o = str(tmp_path / "rif_api.o")
    chk_o = str(tmp_path / "abi_host_check.o")
    exe = str(tmp_path / "abi_host_check")
    for src, obj in ((os.path.join(CSRC, "rif_api.hip"), api_o),
                     (os.path.join(ROOT, "tests", "abi_host_check.hip"), chk_o)):
        r = subprocess.run([hipcc, *flags, *inc, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
    link = [hipcc, "--offload-arch=gfx950", *SAN, api_o, chk_o, *_objects(), "-o", exe,
            "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert " 0 failures" in r.stdout
