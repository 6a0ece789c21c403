"""The host half of the library (program builders and the plan compiler,
every source but the HIP kernels) built with AddressSanitizer and
UndefinedBehaviorSanitizer, with stub device entry points, and driven through
the C ABI by tests/sanitize/host_driver.cpp.  The driver replays one scenario
with the k-th host allocation made to fail, for a sweep of k: every call must
then return HBC_OK or HBC_ENOMEM, and the leak checker must find nothing at
exit."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_14780_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("api.cpp", "plan.cpp", "cubed_sphere.cpp", "consumer.cpp")]
TEST_SOURCES = [os.path.join(ROOT, "tests", "sanitize", f) for f in ("device_stubs.cpp", "host_driver.cpp")]
FLAGS = ["-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _sanitizers_usable(tmp):
    src = os.path.join(tmp, "probe.cpp")
    with open(src, "w") as f:
        f.write("int main() { return 0; }\n")
    r = subprocess.run(["g++", "-fsanitize=address,undefined", src, "-o", os.path.join(tmp, "probe")],
                       capture_output=True)
    return r.returncode == 0


def test_host_library_under_asan_ubsan_with_allocation_failures(tmp_path):
    if shutil.which("g++") is None or not _sanitizers_usable(str(tmp_path)):
        pytest.skip("g++ with the address and undefined-behaviour sanitizers is not available")
    srcs = HOST_SOURCES + TEST_SOURCES
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]

    def compile_one(k):
        return subprocess.run(["g++", *FLAGS, "-c", srcs[k], "-o", objs[k]], capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        for k, r in enumerate(ex.map(compile_one, range(len(srcs)))):
            assert r.returncode == 0, srcs[k] + "\n" + r.stderr[-4000:]
    exe = str(tmp_path / "host_driver")
    r = subprocess.run(["g++", *FLAGS, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    words = r.stdout.split()
    injected = int(words[words.index("injected") + 1])
    assert injected > 1000, r.stdout
