"""The host code of libdwt2 under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

A copy of the library is built with both sanitizers on the host side only
(device code is compiled as usual), and the host-side test files run against
it in a child process with the sanitizer runtime preloaded; any report fails
the test.  This covers argument validation with garbage values (enum values
outside their enumerators, sizes near the limits), the batch planner, the
server's argument checks and the tuning table's text import and export.
Skipped where a GPU device node exists, so that nothing here runs beside a
GPU job's own environment.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

from paper_1605_00561_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["test_abi_host.py", "test_batch_host.py", "test_server_host.py",
              "test_tune_host.py"]


def _runtime():
    hits = sorted(glob.glob(os.path.join(os.path.dirname(build.HIPCC), "..", "llvm", "lib",
                                         "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    return os.path.realpath(hits[-1]) if hits else None


def _libstdcxx():
    out = subprocess.run(["g++", "-print-file-name=libstdc++.so.6"], capture_output=True,
                         text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_host_code_is_sanitizer_clean(tmp_path):
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present: the sanitizer run is a CPU-container check")
    rt, cxx = _runtime(), _libstdcxx()
    if not (os.path.exists(build.HIPCC) and rt and cxx):
        pytest.skip("hipcc, the clang ASan runtime or libstdc++ not found")
    pkg = tmp_path / "pkg"
    shutil.copytree(os.path.join(ROOT, "include"), pkg / "include")
    src_pkg = os.path.join(ROOT, "paper_1605_00561_amd")
    shutil.copytree(os.path.join(src_pkg, "csrc"), pkg / "paper_1605_00561_amd" / "csrc")
    for f in glob.glob(os.path.join(src_pkg, "*.py")):
        shutil.copy(f, pkg / "paper_1605_00561_amd")
    shutil.copytree(os.path.join(ROOT, "tests"), pkg / "tests",
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__", "*.so"))
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = [f for f in build.CFLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer",
                                                       "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = [f.replace(os.path.join(ROOT, "include"), str(pkg / "include"))
             .replace(build.CSRC, str(pkg / "paper_1605_00561_amd" / "csrc")) for f in flags]
    objs = []
    for src in build.SOURCES:
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([build.HIPCC, *flags, *san, "-c",
                        str(pkg / "paper_1605_00561_amd" / "csrc" / src), "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    lib = str(pkg / "paper_1605_00561_amd" / "libdwt2.so")
    subprocess.run([build.HIPCC, "--offload-arch=gfx950", "-shared", *san, "-shared-libsan", *objs,
                    "-o", lib, "-pthread"], check=True, capture_output=True)
    # the oracle's own library is built by its package on import, in the copy
    logs = tmp_path / "san"
    env = dict(os.environ)
    env.update(ASAN_OPTIONS=f"detect_leaks=0:halt_on_error=1:log_path={logs}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={logs}",
               LD_PRELOAD=f"{rt}:{cxx}", PYTHONPATH=str(pkg))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-k", "not single_hip_runtime", *[f"tests/{t}" for t in HOST_TESTS]],
                       cwd=pkg, env=env, capture_output=True, text=True, timeout=800)
    reports = sorted(glob.glob(str(logs) + "*"))
    text = "".join(open(p).read() for p in reports)
    assert r.returncode == 0 and not reports, (r.stdout[-3000:], r.stderr[-3000:], text[-4000:])
    assert " passed" in r.stdout
