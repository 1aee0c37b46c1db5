"""The host packer under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (tests/pack_driver.cpp) built with g++ packs a small mesh in every record
layout and curve order and validates corrupted copies; any out-of-bounds access,
use after free, leak or undefined operation ends the run with an error."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_02309_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "pack_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "pack_driver.cpp"), os.path.join(CSRC, "pack.cpp"), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        if "asan" in res.stderr.lower() or "sanitize" in res.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + res.stderr[-300:])
        raise AssertionError(res.stderr)
    return out


def test_pack_under_sanitizers(driver, tmp_path):
    from synth import kuhn_mesh
    m = kuhn_mesh(5, jitter=0.1, seed=3, spheres=[[0.5, 0.5, 0.5, 0.3], [0.2, 0.3, 0.7, 0.15]])
    path = str(tmp_path / "mesh.bin")
    with open(path, "wb") as fh:
        fh.write(np.array([m.n_points, m.n_tets], np.int64).tobytes())
        fh.write(np.ascontiguousarray(m.points, np.float32).tobytes())
        fh.write(np.ascontiguousarray(m.tets, np.int32).tobytes())
        fh.write(np.ascontiguousarray(m.nbrs, np.int32).tobytes())
        fh.write(np.ascontiguousarray(m.cflag, np.uint8).tobytes())
    # verify_asan_link_order=0: the sanitizer runtime need not come first when the
    # environment preloads other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    lines = res.stdout.splitlines()
    assert lines[-1] == "done"
    packs = [l for l in lines if l.startswith("pack ")]
    assert len(packs) == 9 and all(" rc 0 " in l for l in packs), packs
    # the constrained-face count does not depend on layout or curve
    assert len({l.split(" ntri ")[1].split()[0] for l in packs}) == 1
    bad = [l for l in lines if l.startswith("bad ")]
    assert len(bad) == 5 and all(" rc -2:" in l for l in bad), bad
