"""Host-only C++ checks, built with g++ and the address/undefined-behaviour (and thread)
sanitizers: the serving arena, the serving scheduler against a fake executor, and the host
core of the library (descriptor checks, footprints, workspace sizes, device-less errors)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_randomised(tmp_path):
    exe = tmp_path / "arena_test"
    src = os.path.join(HERE, "native", "arena_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "arena ok" in out.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_is_plain_c_and_links(tmp_path):
    """include/slsht.h compiles as strict C99 (-pedantic), and a C program that calls the
    library through it links against libslsht.so (nothing is run: no GPU needed)."""
    root = os.path.dirname(HERE)
    lib_dir = os.path.join(root, "paper_1207_5558_amd")
    if not os.path.exists(os.path.join(lib_dir, "libslsht.so")):
        from paper_1207_5558_amd import build
        build.build()
    hdr = tmp_path / "header_only.c"
    hdr.write_text('#include "slsht.h"\nint main(void) { slsht_desc d = {0}; '
                   'return slsht_validate(&d) == SLSHT_OK; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(root, "include"), "-fsyntax-only", str(hdr)], check=True)
    exe = tmp_path / "abi_forward"
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror",
                    "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                    "-I", "/opt/rocm/include", os.path.join(HERE, "native", "abi_forward.c"),
                    "-o", str(exe), "-L", lib_dir, "-lslsht", "-L", "/opt/rocm/lib",
                    "-lamdhip64"], check=True)
    assert exe.exists()


ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1207_5558_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build_run(tmp_path, name, srcs, flags, args=(), env=None, extra=()):
    exe = tmp_path / name
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", *flags,
                    "-I", os.path.join(ROOT, "include"), *srcs, *extra, "-lpthread",
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=600,
                         env={**os.environ, **(env or {})})
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_fake_executor_sanitized(tmp_path):
    """Admission order and budget, the bound on passing a blocked head, ETOOBIG, failures in
    preparation / launch / on the device (FAILED with EINVAL / EDEVICE), cancellation of a
    queued request, grouping, shutdown with work queued, and a threaded run; ASan + UBSan."""
    out = _build_run(tmp_path, "sched_asan", [os.path.join(HERE, "native", "sched_test.cpp")],
                     SAN)
    for line in ("order/budget/release ok", "bypass bound ok", "too big / failures ok",
                 "cancel/grouping/shutdown ok", "threads ok", "sched ok"):
        assert line in out, out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_threads_tsan(tmp_path):
    """The threaded scheduler run (worker thread, four submitting and releasing threads)
    under ThreadSanitizer."""
    out = _build_run(tmp_path, "sched_tsan", [os.path.join(HERE, "native", "sched_test.cpp")],
                     ["-fsanitize=thread"], args=("threads",),
                     env={"TSAN_OPTIONS": "halt_on_error=1"})
    assert "threads ok" in out, out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="g++ or the HIP runtime not available")
def test_host_core_sanitized(tmp_path):
    """slsht_api.cpp, slsht_server.cpp and slsht_geom.cpp built with g++ under ASan + UBSan
    (device launchers stubbed): random descriptors through validate / footprint /
    coupling_size, the workspace sizes, and the device-less error returns."""
    srcs = [os.path.join(HERE, "native", "host_api_test.cpp"),
            os.path.join(HERE, "native", "device_stubs.cpp"),
            os.path.join(CSRC, "slsht_api.cpp"), os.path.join(CSRC, "slsht_server.cpp"),
            os.path.join(CSRC, "slsht_geom.cpp")]
    out = _build_run(tmp_path, "host_api", srcs,
                     SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"],
                     extra=("-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"))
    assert "host api ok" in out, out
