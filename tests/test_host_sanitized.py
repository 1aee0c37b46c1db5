"""Host C/C++ under AddressSanitizer and UndefinedBehaviorSanitizer, built with
the system compilers into stand-alone drivers: the library's mesh packer
(tests/pack_driver.cpp: every record layout and curve order, corrupted meshes)
and the oracle's walk (tests/oracle_driver.c: traces and locations, compared
with the oracle as the tests load it).  Any out-of-bounds access, use after
free, leak or undefined operation ends a run with an error."""
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
    assert len(packs) == 16 and all(" rc 0 " in l for l in packs), packs
    # the constrained-face count does not depend on layout or curve
    assert len({l.split(" ntri ")[1].split()[0] for l in packs}) == 1
    # region order (sfc 3): as many regions as the flood fill finds (inside the
    # spheres and outside: more than one), each stored as one contiguous run
    for l in packs:
        f = l.split()
        regions, flood, runs = int(f[f.index("regions") + 1]), int(f[f.index("flood") + 1]), int(
            f[f.index("runs") + 1])
        assert flood >= 2
        if " sfc 3 " in l:
            assert regions == flood == runs, l
        else:
            assert regions == 0 and runs > flood, l
    bad = [l for l in lines if l.startswith("bad ")]
    assert len(bad) == 5 and all(" rc -2:" in l for l in bad), bad


@pytest.fixture(scope="module")
def oracle_driver(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("asan_oracle") / "oracle_driver")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "oracle_driver.c"), os.path.join(ROOT, "oracle", "walk.c"),
           "-o", out, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise AssertionError(res.stderr)
    return out


def test_oracle_under_sanitizers(oracle_driver, tmp_path):
    import oracle
    from synth import kuhn_mesh, random_interior_rays, pinhole_rays
    m = kuhn_mesh(6, jitter=0.1, seed=4, spheres=[[0.5, 0.5, 0.5, 0.3]])
    om = oracle.OracleMesh.from_kuhn(m)
    o1, d1 = random_interior_rays(1500, seed=8)
    o2, d2, _ = pinhole_rays((0.5, 0.5, 0.05), 16, 16, 60.0)
    o = np.concatenate([o1, o2]).astype(np.float32)
    d = np.concatenate([d1, d2]).astype(np.float32)
    n = o.shape[0]
    rng = np.random.default_rng(9)
    tm = rng.uniform(0.05, 0.6, n).astype(np.float32)
    sf = np.full(n, -1, np.int32)
    # some rays leave from a constrained face: the origin is a point on that face
    tv = om.tri_verts
    k = np.arange(0, n, 7)
    f = rng.integers(0, tv.shape[0], k.size)
    w = rng.dirichlet([1, 1, 1], k.size)
    o[k] = np.einsum("ij,ijk->ik", w, m.points[tv[f]].astype(np.float64)).astype(np.float32)
    sf[k] = f
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as fh:
        fh.write(np.array([m.n_points, m.n_tets, n], np.int64).tobytes())
        for a, dt in ((m.points, np.float32), (m.tets, np.int32), (m.nbrs, np.int32), (m.cflag, np.uint8),
                      (o, np.float32), (d, np.float32), (tm, np.float32), (sf, np.int32)):
            fh.write(np.ascontiguousarray(a, dt).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([oracle_driver, inp, outp], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0 and res.stdout.strip() == "done", res.stdout[-2000:] + res.stderr[-4000:]
    raw = open(outp, "rb").read()
    off = 0

    def take(dt, cnt):
        nonlocal off
        a = np.frombuffer(raw, dt, cnt, off)
        off += a.nbytes
        return a

    for kw in (dict(), dict(tmax=tm, start_face=sf)):
        ref = om.trace(o, d, **kw)
        assert np.array_equal(take(np.int32, n), ref["tri"])
        assert np.array_equal(take(np.float64, n), ref["t"], equal_nan=True)
        assert np.array_equal(take(np.float64, 2 * n).reshape(n, 2), ref["bary"], equal_nan=True)
        assert np.array_equal(take(np.int32, n), ref["steps"])
    assert np.array_equal(take(np.int32, n), om.locate(o))
    assert off == len(raw)
