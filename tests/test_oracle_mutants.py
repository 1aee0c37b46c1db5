"""The oracle's pins must catch plausible mistakes: each mutant below plants one
(a dropped term, a flipped sign, a wrong index, a swapped operand) in a copy of
the oracle's C source; the pin suite in test_oracle.py is then run against that
build in a subprocess and must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "walk.c")

MUTANTS = {
    "exit_face_wrong_slot": ("if (det2(q[3], q[2]) >= 0.0) return 1;",
                             "if (det2(q[3], q[2]) >= 0.0) return 2;"),
    "det_sign": ("return a[0] * b[1] - a[1] * b[0];", "return a[0] * b[1] + a[1] * b[0];"),
    "dot_dropped_term": ("return a.x * b.x + a.y * b.y + a.z * b.z;", "return a.x * b.x + a.y * b.y;"),
    "next_wrong_slot": ("nxt = m->nbrs[4 * (int64_t)tet + j];", "nxt = m->nbrs[4 * (int64_t)tet + (j ^ 1)];"),
    "bary_wrong_vertex": ("bary[0] = l[ord[1]] / sum;", "bary[0] = l[ord[0]] / sum;"),
    "t_wrong_operand": ("tt = vdot(nf, vsub(A0, F.o)) / vdot(nf, F.d);",
                        "tt = vdot(nf, vsub(A1, F.o)) / vdot(nf, F.d) * 1.0001;"),
    "onb_sign": ("b2->x = b; b2->y = sgn + n.y * n.y * a;", "b2->x = b; b2->y = sgn - n.y * n.y * a;"),
    "early_out_too_soon": ("if (dmin > tm)", "if (dmin > 0.5 * tm)"),
    "locate_stops_early": ("if (j < 0 || s >= 1.0) return t;", "if (j < 0 || s >= 0.5) return t;"),
    "start_face_wrong_side": ("start = ((side > 0.0) == (dn > 0.0)) ? ta : tb;",
                              "start = ((side > 0.0) != (dn > 0.0)) ? ta : tb;"),
    "mirror_id": ("m->face_tri[4 * (int64_t)nb + mirror] = id;",
                  "m->face_tri[4 * (int64_t)nb + mirror] = id + 1 < (int32_t)nflag ? id + 1 : id;"),
    # the start-face branch must put the face in counter-clockwise order (in the
    # located branch the outward-ordered exit face already is, so no mutant there)
    # the fallback that answers rays whose walk reaches the step cap (closest hit by
    # its definition) and the front/back tets of a hit
    "fallback_tie_to_latest": ("if (t < bt - 1e-12 || (fabs(t - bt) <= 1e-12 && f < best)) {",
                               "if (t < bt + 1e-12) {"),
    "fallback_keeps_start_face": ("if (f == exclude) continue;", ""),
    "fallback_hit_behind_origin": ("!(t > 0.0) || t > tm", "!(t > -1e-3) || t > tm"),
    "fallback_front_back_swapped": ("tets2[0] = ta_ahead ? tb : ta;", "tets2[0] = ta_ahead ? ta : tb;"),
    "walk_front_back_swapped": ("tets2[0] = cur; tets2[1] = nxt;", "tets2[0] = nxt; tets2[1] = cur;"),
    # a walk that leaves its ray (a vertex on the ray, zero determinants decided by
    # rounding) must be caught and answered by the definition
    "lost_walk_not_caught": ("if (face_misses_ray(q, m->extent)) {", "if (0) {"),
    "lost_walk_test_sign": ("if (det2(a, b) < -tol) return 1;", "if (det2(b, a) < -tol) return 1;"),
    "ccw_not_enforced": ("            if (o2 < 0.0) {\n                int32_t ti = a[1]; a[1] = a[2]; a[2] = ti;\n                double t0 = q[1][0], t1 = q[1][1];\n                q[1][0] = q[2][0]; q[1][1] = q[2][1]; q[2][0] = t0; q[2][1] = t1;\n            }\n            nxt = start;",
                         "            nxt = start;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: " + name
    mut = tmp_path / "walk.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                           str(mut), "-o", str(lib), "-lm"])
    env = dict(os.environ, TETRT_ORACLE_LIB=str(lib))
    rc = subprocess.call([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle.py")],
                         env=env, cwd=ROOT, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    assert rc != 0, "the pins did not catch mutant " + name
