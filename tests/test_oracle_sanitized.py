"""The C oracle and the plain-C ABI client built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only, gcc).  The oracle runs under the
sanitizers on a small R-MAT graph with nodes without in-edges (plain counts
and their work, pool sizes and stitched counts, stratified weighted sums,
walk tables) and must finish cleanly with results equal to the unsanitized
library's; the client must compile and link cleanly with the same flags."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2304_04015_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")
ORACLE_SRC = os.path.join(ROOT, "oracle", "simrank_oracle.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

needs_gcc = pytest.mark.skipif(not shutil.which("gcc"), reason="gcc not present")


def _write_graph(g, path):
    with open(path, "wb") as f:
        f.write(np.int32(g.n).tobytes())
        f.write(np.int64(g.m).tobytes())
        f.write(np.ascontiguousarray(g.in_off, np.int32).tobytes())
        f.write(np.ascontiguousarray(g.in_src, np.int32).tobytes())


def _sanitizer_works(tmp_path) -> bool:
    probe = tmp_path / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", *SAN, str(probe), "-o", str(tmp_path / "probe")],
                       capture_output=True, text=True)
    return r.returncode == 0


@needs_gcc
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if not _sanitizer_works(tmp_path):
        pytest.skip("gcc has no sanitizer runtime here")
    exe = str(tmp_path / "driver")
    subprocess.run(["gcc", "-std=c11", "-Wall", *SAN, "-ffp-contract=off", DRIVER, ORACLE_SRC,
                    "-o", exe, "-lm"], check=True, capture_output=True, text=True, timeout=120)
    g = inputs.rmat_in(8, 6 << 8, seed=9)
    assert (g.in_degree() == 0).any()
    s = int(np.argmax(g.in_degree()))
    gp = str(tmp_path / "g.bin")
    _write_graph(g, gp)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, gp, str(s)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    rows = {}
    for line in r.stdout.splitlines():
        name, *vals = line.split()
        rows[name] = np.array([int(v) for v in vals], dtype=np.int64)
    want, work = O.meet_counts_plain(g, s, 0x51, 0.6, 32, 300, with_work=True)
    assert np.array_equal(rows["plain"], want) and np.array_equal(rows["work"], work)
    P = O.pool_sizes(g, 1.0)
    assert np.array_equal(rows["stitched"], O.meet_counts_stitched(g, s, 0x52, 0x53, 0.6, 32, 4,
                                                                    P, 200))
    SP = O.strat_params(g.n, 0.6, 0.1, z=400.0, phi=8)
    assert np.array_equal(rows["strat"].astype(np.uint64), O.strat_sums(g, s, 0x54, SP))
    i = np.arange(64)
    paths, _ = O.walk_table_plain(g, 0x55, 0.6, 32, (i * 7) % g.n, i)
    assert np.array_equal(rows["walks"], paths.ravel())
    assert want.sum() > 300


@needs_gcc
def test_c_client_builds_with_sanitizers(tmp_path):
    if not _sanitizer_works(tmp_path):
        pytest.skip("gcc has no sanitizer runtime here")
    pkg = os.path.join(ROOT, "paper_2304_04015_amd")
    orc = os.path.join(ROOT, "oracle")
    for lib in (os.path.join(pkg, "libsimrank.so"), os.path.join(orc, "liboracle.so")):
        if not os.path.exists(lib):
            pytest.fail(f"{lib} is missing: build first (__graft_entry__.build())")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", *SAN,
                    "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "c_abi_client.c"),
                    "-o", str(tmp_path / "client"), "-L", pkg, "-lsimrank", "-L", orc, "-loracle",
                    f"-Wl,-rpath,{pkg}", f"-Wl,-rpath,{orc}"],
                   check=True, capture_output=True, text=True, timeout=120)
