"""The oracle's pins catch plausible mistakes.

Each mutant is a copy of oracle/oracle.c with one planted mistake (a dropped
term, a wrong sign, a transposed operand, a swapped index, an off-by-one, an
interval end flipped); it is built into a temporary library and the oracle pin
tests (test_oracle_mt, test_oracle_closest, test_oracle_grad) are run against
it in a child process.  Every mutant must make at least one pin fail, and the
unmodified source must pass the same harness.  CPU only; the shipped oracle is
never touched.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = [os.path.join(HERE, f) for f in ("test_oracle_mt.py", "test_oracle_closest.py",
                                         "test_oracle_grad.py", "test_oracle_closest_point.py",
                                         "test_oracle_sah.py")]

MUTANTS = [
    ("edge e2 reversed", "v3 e2 = v3_sub(p2, p0);", "v3 e2 = v3_sub(p0, p2);"),
    ("edge e1 reversed", "v3 e1 = v3_sub(p1, p0);", "v3 e1 = v3_sub(p0, p1);"),
    ("cross x operands transposed", "r.x = fmaf(a.y, b.z, -(a.z * b.y));",
     "r.x = fmaf(a.z, b.y, -(a.y * b.z));"),
    ("dot drops the z term", "return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x));",
     "return fmaf(a.y, b.y, a.x * b.x);"),
    ("origin offset reversed", "v3 S = v3_sub(o, p0);", "v3 S = v3_sub(p0, o);"),
    ("second cross product transposed", "v3 Q = cross_fma(S, e1);", "v3 Q = cross_fma(e1, S);"),
    ("u and v swapped", "*u_out = U * inv;\n    *v_out = V * inv;", "*u_out = V * inv;\n    *v_out = U * inv;"),
    ("edges exclusive", "U + V <= adet", "U + V < adet"),
    ("t = 0 accepted", "T > 0.0f &&", "T >= 0.0f &&"),
    ("tmax exclusive", "T <= adet * tmax", "T < adet * tmax"),
    ("sign of T not folded", "float T = sign_xor(dot_fma(e2, Q), s);", "float T = dot_fma(e2, Q);"),
    ("t scaled from U", "*t_out = T * inv;", "*t_out = U * inv;"),
    ("ties to the highest id", "return ta < tb || (ta == tb && ia < ib);",
     "return ta < tb || (ta == tb && ia > ib);"),
    ("slab entry plane from the wrong side", "float first = neg[a] ? n->hi[a] : n->lo[a];",
     "float first = neg[a] ? n->lo[a] : n->hi[a];"),
    ("right child never visited", "            stack[sp++] = n->right;\n", ""),
    ("last triangle of a leaf skipped", "k < n->first + n->count; k++", "k < n->first + n->count - 1; k++"),
    ("gradient: dL/dd sign", "gr[3] = -t * lam.x;", "gr[3] = t * lam.x;"),
    ("gradient: vertex weights of p1, p2 swapped", "double w[3] = { 1.0 - u - v, u, v };",
     "double w[3] = { 1.0 - u - v, v, u };"),
    ("gradient: Cramer column transposed", "ab = d3_cross(a, b);", "ab = d3_cross(b, a);"),
    ("closest point: edge p1p2 never considered",
     "    cp_consider(q, p0, e1, e2, 1.0 - s12, s12, &bd2, &bu, &bv);\n", ""),
    ("closest point: normal-equation numerator transposed", "double s = (c * r1 - b * r2) / det",
     "double s = (c * r2 - b * r1) / det"),
    ("closest point: segment parameter not clamped at 1", "return s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);",
     "return s < 0.0 ? 0.0 : s;"),
    ("closest point: barycentrics swapped on edge p1p2", "cp_consider(q, p0, e1, e2, 1.0 - s12, s12,",
     "cp_consider(q, p0, e1, e2, s12, 1.0 - s12,"),
    ("closest point: stationary point kept outside the triangle", "if (s >= 0.0 && t >= 0.0 && s + t <= 1.0)",
     "if (s >= 0.0 && t >= 0.0)"),
    ("closest point: radius exclusive", "b->d1 <= (double)r2", "b->d1 < (double)r2"),
    ("closest point: ties to the highest id", "return da < db || (da == db && ia < ib);",
     "return da < db || (da == db && ia > ib);"),
    ("closest point: BVH culls with the best instead of the runner-up",
     "double bound = b.d2 + ldexp(b.d2, -30) + abs_margin;",
     "double bound = b.d1 + ldexp(b.d1, -30) + abs_margin;"),
    ("closest point: box gap below the box measured from the upper plane",
     "if (qq[a] < nd->lo[a]) g = nd->lo[a] - qq[a];", "if (qq[a] < nd->lo[a]) g = nd->hi[a] - qq[a];"),
    ("SAH: right side weighted by the left count", "half_area(&rs[k + 1]) * (float)nr;",
     "half_area(&rs[k + 1]) * (float)nl;"),
    ("SAH: ties to the higher split", "if (cost < best_cost) { best_cost = cost;",
     "if (cost <= best_cost) { best_cost = cost;"),
    ("SAH: partition not stable", "for (int64_t i = t.first; i < t.first + t.count; i++) if (!side[i]) tmp[w++] = perm[i];",
     "for (int64_t i = t.first + t.count - 1; i >= t.first; i--) if (!side[i]) tmp[w++] = perm[i];"),
    ("SAH: fallback rounds the left half up", "nl = t.count / 2;", "nl = (t.count + 1) / 2;"),
    ("SAH: right child one node early", "right = t.node + (int32_t)(2 * nl);",
     "right = t.node + (int32_t)(2 * nl) - 1;"),
    ("SAH: right side starts at the split bin", "int64_t nr = rn[k + 1];", "int64_t nr = rn[k];"),
    ("SAH: area drops a face pair", "return (dx * dy + dy * dz) + dz * dx;", "return dx * dy + dy * dz;"),
]


# Planted mistakes in the oracle's Python part (oracle/__init__.py), run
# against the collapse and SAH pins.
PY_PINS = [os.path.join(HERE, f) for f in ("test_oracle_collapse.py", "test_oracle_sah.py")]
PY_SRC = os.path.join(ROOT, "oracle", "__init__.py")
PY_MUTANTS = [
    ("collapse: a subtree of exactly leaf_size stays interior", "if count <= leaf_size:",
     "if count < leaf_size:"),
    ("collapse: right child one node early", "stack.append(i + 2 * nl)",
     "stack.append(i + 2 * nl - 1)"),
    ("collapse: right subtree emitted before the left",
     "stack.append(i + 2 * nl)\n        stack.append(i + 1)",
     "stack.append(i + 1)\n        stack.append(i + 2 * nl)"),
]


def _build(tmp, tag, text):
    c = os.path.join(tmp, f"{tag}.c")
    so = os.path.join(tmp, f"{tag}.so")
    with open(c, "w") as fh:
        fh.write(text)
    sys.path.insert(0, ROOT)
    import oracle
    cmd = ["gcc", *oracle.CFLAGS, c, "-o", so, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return so


def _run_pins(so):
    env = dict(os.environ, ORACLE_TEST_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = open(SRC).read()
    jobs = [("original", src)]
    for i, (name, old, new) in enumerate(MUTANTS):
        assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
        jobs.append((f"m{i:02d}", src.replace(old, new)))
    libs = {tag: _build(str(tmp_path), tag, text) for tag, text in jobs}
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        res = dict(zip(libs, ex.map(_run_pins, libs.values())))
    rc, out = res["original"]
    assert rc == 0, "the unmodified oracle must pass its pins:\n" + out
    survivors = [name for i, (name, _, _) in enumerate(MUTANTS) if res[f"m{i:02d}"][0] == 0]
    assert not survivors, f"mistakes no pin catches: {survivors}"


def _run_py_pins(pkg_dir):
    import oracle
    env = dict(os.environ, ORACLE_PY_DIR=pkg_dir, ORACLE_TEST_LIB=oracle.LIB_PATH,
               OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PY_PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_every_planted_python_mistake_fails_a_pin(tmp_path):
    sys.path.insert(0, ROOT)
    import oracle
    oracle.lib()
    src = open(PY_SRC).read()
    jobs = [("original", src)]
    for i, (name, old, new) in enumerate(PY_MUTANTS):
        assert src.count(old) == 1, f"mutation site not unique or missing: {name}"
        jobs.append((f"p{i:02d}", src.replace(old, new)))
    dirs = {}
    for tag, text in jobs:
        d = tmp_path / tag / "oracle"
        d.mkdir(parents=True)
        (d / "__init__.py").write_text(text)
        dirs[tag] = str(tmp_path / tag)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        res = dict(zip(dirs, ex.map(_run_py_pins, dirs.values())))
    rc, out = res["original"]
    assert rc == 0, "the unmodified oracle must pass its pins:\n" + out
    survivors = [name for i, (name, _, _) in enumerate(PY_MUTANTS) if res[f"p{i:02d}"][0] == 0]
    assert not survivors, f"mistakes no pin catches: {survivors}"
