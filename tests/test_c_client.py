"""The C ABI used from C: include/*.h compile as strict C99 (and as C++), and
a plain C program (tests/c_abi_client.c, no Python or torch in its process)
runs a query through the library and checks every node's meet count against
the oracle's, bit for bit."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
PKG = os.path.join(ROOT, "paper_2304_04015_amd")
ORACLE = os.path.join(ROOT, "oracle")
CLIENT = os.path.join(HERE, "c_abi_client.c")

needs_gcc = pytest.mark.skipif(not shutil.which("gcc"), reason="gcc not present")


def _build_client(tmp_path) -> str:
    for lib in (os.path.join(PKG, "libsimrank.so"), os.path.join(ORACLE, "liboracle.so")):
        if not os.path.exists(lib):
            pytest.fail(f"{lib} is missing: build first (__graft_entry__.build())")
    exe = str(tmp_path / "c_abi_client")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", INCLUDE,
                    CLIENT, "-o", exe, "-L", PKG, "-lsimrank", "-L", ORACLE, "-loracle",
                    f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ORACLE}"],
                   check=True, capture_output=True, text=True, timeout=120)
    return exe


@needs_gcc
@pytest.mark.parametrize("header", ["simrank.h", "simrank_roofline.h"])
def test_headers_compile_as_c99_and_cpp(header, tmp_path):
    src = tmp_path / "inc.c"
    src.write_text(f'#include "{header}"\nint main(void) {{ return 0; }}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                    "-I", INCLUDE, str(src)], check=True, capture_output=True, timeout=60)
    if shutil.which("g++"):
        subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++",
                        "-I", INCLUDE, str(src)], check=True, capture_output=True, timeout=60)


@needs_gcc
def test_c_client_builds(tmp_path):
    assert os.path.exists(_build_client(tmp_path))


@needs_gcc
@pytest.mark.gpu
@pytest.mark.parametrize("n,R", [(3000, 1500), (517, 3001)])
def test_c_client_counts_equal_oracle(n, R, tmp_path):
    exe = _build_client(tmp_path)
    env = dict(os.environ)
    r = subprocess.run([exe, str(n), str(R)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "c_abi_client ok" in r.stdout
