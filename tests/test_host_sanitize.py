"""The library's host octree under AddressSanitizer and
UndefinedBehaviorSanitizer: the octree source and a driver
(tests/native/octree_driver.cpp) are built with g++ alone (host code only, no
GPU code is involved) and run; any invalid access, leak or undefined
behaviour ends the run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_octree_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "octree_asan")
    srcs = [os.path.join(ROOT, "paper_1009_4975_amd", "csrc", "octree.cpp"),
            os.path.join(ROOT, "tests", "native", "octree_driver.cpp")]
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
             "-fsanitize=address,undefined"]
    r = subprocess.run(["g++", *flags, f"-I{os.path.join(ROOT, 'include')}", *srcs, "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
