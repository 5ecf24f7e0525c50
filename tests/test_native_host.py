"""Host-only C++ checks, built with g++ and the address/undefined-behaviour sanitizers."""
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
