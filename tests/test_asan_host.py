"""The library's host code under AddressSanitizer (CPU only).

The four host sources (planning, argument checks, the batch layer with its
graph cache and autotuner, the server, kernel timing) are compiled again with
ASan on hipcc's host pass, linked with the unchanged kernel object into a
separate library, and driven by tests/asan/driver.c through the C ABI: every
host-only entry point and every argument check that fails before the device
is touched, over a range of column sizes and tunings.  A second run of the
driver reads past a heap buffer of its own, which ASan must report, so that
a run with the sanitizer silently off cannot pass.  The GPU code is built
without the sanitizer (GPU ASan is not available for these kernels here)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_15034_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_2609_15034_amd", "_build", "fd_kernels.o")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SOURCES = ("fd_host.cpp", "fd_batch.cpp", "fd_server.cpp", "fd_profile.cpp")


def _asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in os.listdir(base):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.a")
        if os.path.exists(p):
            return p
    return None


@pytest.fixture(scope="module")
def asan_driver(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG) and _asan_runtime()):
        pytest.skip("hipcc, clang or the clang ASan runtime is not installed")
    if not os.path.exists(KOBJ):
        pytest.skip("kernel object not built (run the package build first)")
    d = tmp_path_factory.mktemp("asan")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address"]
    procs, objs = [], []
    for src in HOST_SOURCES:
        obj = str(d / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for pr, src in zip(procs, HOST_SOURCES):
        out, _ = pr.communicate()
        assert pr.returncode == 0, (src, out[-4000:])
    lib = str(d / "libfd_asan.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs, KOBJ])
    exe = str(d / "driver")
    subprocess.check_call([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "asan", "driver.c"),
                           "-o", exe, "-L" + str(d), "-lfd_asan", "-Wl,-rpath," + str(d)])
    return exe


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23")
    return subprocess.run([exe, *args], capture_output=True, text=True, timeout=300, env=env)


def test_host_entry_points_clean_under_asan(asan_driver):
    r = _run(asan_driver)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr


def test_asan_is_live(asan_driver):
    r = _run(asan_driver, "planted")
    assert r.returncode == 23, (r.returncode, r.stdout, r.stderr[-2000:])
    assert "heap-buffer-overflow" in r.stderr
