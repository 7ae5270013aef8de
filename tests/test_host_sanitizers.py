"""The host part of the library (descriptor validation and the plan geometry:
sensor cells, window tables, spreading lists, sweep segments) built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on seeded
descriptors, valid and invalid, by tests/sanitize/geometry_check.cpp. The
kernel launchers are replaced by stand-ins (tests/sanitize/kernel_stubs.cpp),
so nothing here needs or touches a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1501_02946_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")

pytestmark = pytest.mark.slow


def _tool(name):
    for cand in (os.path.join("/opt/rocm/bin", name), os.path.join("/opt/rocm/llvm/bin", name), shutil.which(name)):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip(f"{name} not found")


def test_validation_and_geometry_under_asan_ubsan(tmp_path):
    hipcc = _tool("hipcc")
    clang = _tool("clang++")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    # host code only is instrumented: each sanitizer flag applies to the host pass
    san_host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in (os.path.join(CSRC, "capi.cpp"), os.path.join(HERE, "kernel_stubs.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", *san_host, *inc, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
        objs.append(obj)
    drv = str(tmp_path / "geometry_check.o")
    r = subprocess.run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", *inc, "-c", os.path.join(HERE, "geometry_check.cpp"),
                        "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    exe = str(tmp_path / "geometry_check")
    r = subprocess.run([clang, "-fsanitize=address,undefined", *objs, drv, "-L/opt/rocm/lib", "-lamdhip64",
                        "-Wl,-rpath,/opt/rocm/lib", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "checked" in r.stdout
