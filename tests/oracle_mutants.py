"""Planted mistakes in the CPU oracles, each of which their pins must catch.

Every mutant is one textual change to a copy of oracle/oracle.c (it must
match exactly once).  The copy is compiled like the oracle itself, and
tests/test_oracle_pins.py runs against it (CVX_ORACLE_LIB points the binding
at the mutant); a mutant is caught when that run fails.  Run as a script for
a report, or through tests/test_oracle_mutants.py.

The one oracle branch no pin reaches is listed in UNPINNED: the clamp that
keeps a rounded exit point from lying behind the entry point; no ray of the
pins (nor of the workloads) needs it, so removing it changes nothing they
check.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("octant bit order", "oct |= (uint32_t)b << k;", "oct |= (uint32_t)b << (2 - k);"),
    ("mid-plane tie to the wrong side", "(q[k] == mid && d[k] > 0.0)", "(q[k] == mid && d[k] < 0.0)"),
    ("transmittance factor", "double Tn = T * exp(-kap * len);",
     "double Tn = T * exp(-0.5 * kap * len);"),
    ("length not in leaf units", "double len = (tex - t) / h;", "double len = (tex - t);"),
    ("exit at the farthest plane", "if (tk < tex) {", "if (tex == INFINITY || tk > tex) {"),
    ("kappa scale", "*kappa = half_to_double(h);", "*kappa = 2.0 * half_to_double(h);"),
    ("stop rule on T", "if (use_stop && 1.0 - T >= alpha_stop) break;",
     "if (use_stop && T >= alpha_stop) break;"),
    ("inner/outer face swapped", "bit == (d[kx] > 0.0 ? 0 : 1);", "bit == (d[kx] > 0.0 ? 1 : 0);"),
    ("pixel corner instead of centre", "u = (2.0 * ((double)x + 0.5)", "u = (2.0 * ((double)x + 0.0)"),
    ("half-float exponent bias", "ldexp((double)(m + 1024), e - 25)",
     "ldexp((double)(m + 1024), e - 24)"),
    ("colour scale", "c[0] = (double)p[0] / 255.0;", "c[0] = (double)p[0] / 256.0;"),
    ("negative start parameter kept", "double t0 = tin > 0.0 ? tin : 0.0, t1 = tout;",
     "double t0 = tin, t1 = tout;"),
    ("direction not normalised", "for (int k = 0; k < 3; ++k) d[k] = d[k] / n;",
     "for (int k = 0; k < 3; ++k) d[k] = d[k] / (n > 0.0 ? 1.0 : n);"),
    ("face band at exit points only",
     "if (!(k == ent_axis && s == ent_side) && fabs(q[k] - P) < eps_face)",
     "if (0 && fabs(q[k] - P) < eps_face)"),
    ("face band at entry points only",
     "if (!(k == kx && s == xs) && fabs(qx[k] - P) < eps_face)",
     "if (0 && fabs(qx[k] - P) < eps_face)"),
    ("payload bytes", "16.0 + 8.0 * res->n_leaves", "16.0 + 4.0 * res->n_leaves"),
    ("descent byte count", "if (dep > prev_depth) res->n_descent += dep - prev_depth;",
     "if (dep > prev_depth) res->n_descent += 1;"),
    ("canvas exit test", "(d[kx] > 0.0 && Xe >= Rd)", "(d[kx] > 0.0 && Xe >= 0.75 * Rd)"),
    ("entry side", "sin_side = d[k] > 0.0 ? 0 : 1;", "sin_side = d[k] > 0.0 ? 1 : 0;"),
    ("termination-ambiguity band", "fabs((1.0 - T) - alpha_stop) < 1e-5",
     "fabs((1.0 - T) - alpha_stop) < 1e-9"),
    ("length sum in leaf units", "res->sum_len += len * h;", "res->sum_len += len;"),
]

# Planted mistakes in the stroke oracle (oracle/stroke.py, Python): the
# mutated source is executed into the module before its pins run.
STROKE_SRC = os.path.join(ROOT, "oracle", "stroke.py")
STROKE_PINS = os.path.join(ROOT, "tests", "test_stroke_oracle.py")
STROKE_MUTANTS = [
    ("split while the edge is at least radius / k",
     "if e > hmin and d < max_depth:\n            split.add(cell)",
     "if e >= hmin and d < max_depth:\n            split.add(cell)"),
    ("split at the max depth", "if e > hmin and d < max_depth:\n            split.add(cell)",
     "if e > hmin and d <= max_depth:\n            split.add(cell)"),
    ("overlap includes touching at distance r",
     "if _outside(lo, e, box) or not any(_box_dist2(lo, e, s) < s[3] * s[3] for s in stamps):\n"
     "            out[cell] = pay",
     "if _outside(lo, e, box) or not any(_box_dist2(lo, e, s) <= s[3] * s[3] for s in stamps):\n"
     "            out[cell] = pay"),
    ("centre on the sphere does not take the stroke",
     "if any(_centre_dist2(lo, e, s) <= s[3] * s[3] for s in stamps):\n"
     "            out[cell] = paint(pay, fmt, e, rgb, sigma, radius)\n        else:",
     "if any(_centre_dist2(lo, e, s) < s[3] * s[3] for s in stamps):\n"
     "            out[cell] = paint(pay, fmt, e, rgb, sigma, radius)\n        else:"),
    ("colour mix weights swapped", "q[ch] = m * rgb[ch] + (1.0 - m) * q[ch]",
     "q[ch] = (1.0 - m) * rgb[ch] + m * q[ch]"),
    ("stroke optical depth not per leaf edge", "kb = sigma * e / radius", "kb = sigma / radius"),
    ("optical depths not added", "q[3] = kb + kc", "q[3] = max(kb, kc)"),
    ("child keeps the parent's optical depth (F64)",
     "return (pay[0], pay[1], pay[2], pay[3] * 0.5)", "return (pay[0], pay[1], pay[2], pay[3])"),
    ("child optical depth quartered (RGBA8)", "np.float32(_f16_value(pay[4])) * np.float32(0.5)",
     "np.float32(_f16_value(pay[4])) * np.float32(0.25)"),
    ("leaf centre taken at the corner", "c = [lo[k] + 0.5 * e - s[k] for k in range(3)]",
     "c = [lo[k] - s[k] for k in range(3)]"),
    ("box distance negative inside", "v = max(max(lo[k] - s[k], 0.0), s[k] - (lo[k] + e))",
     "v = max(lo[k] - s[k], s[k] - (lo[k] + e))"),
    ("opacity byte from twice the optical depth",
     "a = int(np.rint(255.0 * (1.0 - math.exp(-kap))))\n    return (_byte(col[0])",
     "a = int(np.rint(255.0 * (1.0 - math.exp(-2.0 * kap))))\n    return (_byte(col[0])"),
    ("merged leaf keeps the child's optical depth",
     "return (child[0], child[1], child[2], child[3] * 2.0)",
     "return (child[0], child[1], child[2], child[3])"),
]

UNPINNED = [
    ("exit point kept behind the entry point",
     "if (d[k] > 0.0 && qx[k] < q[k]) qx[k] = q[k];", ""),
]


def mutate(text, old, new):
    if text.count(old) != 1:
        raise ValueError(f"mutant text found {text.count(old)} times: {old!r}")
    return text.replace(old, new)


def run_one(name, old, new, workdir):
    """Compiles the mutant and runs the pins against it; returns (name,
    caught, detail)."""
    src = mutate(open(SRC).read(), old, new)
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    c_path = os.path.join(workdir, tag + ".c")
    so_path = os.path.join(workdir, tag + ".so")
    with open(c_path, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-pthread", "-o", so_path, c_path, "-lm"])
    env = dict(os.environ, CVX_ORACLE_LIB=so_path)
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return name, r.returncode != 0, (lines[0] if lines else r.stdout.strip().splitlines()[-1])


def run_all(mutants=MUTANTS, workers=None):
    workers = workers or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory() as d, cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda m: run_one(m[0], m[1], m[2], d), mutants))


_STROKE_BOOT = """
import sys
sys.path.insert(0, {root!r})
import oracle.stroke as m
exec(compile(open({path!r}).read(), {path!r}, "exec"), m.__dict__)
import pytest
sys.exit(pytest.main([{pins!r}, "-x", "-q", "-p", "no:cacheprovider"]))
"""


def run_one_stroke(name, old, new, workdir):
    src = mutate(open(STROKE_SRC).read(), old, new)
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    path = os.path.join(workdir, tag + ".py")
    with open(path, "w") as f:
        f.write(src)
    boot = _STROKE_BOOT.format(root=ROOT, path=path, pins=STROKE_PINS)
    r = subprocess.run([sys.executable, "-c", boot], cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return name, r.returncode != 0, (lines[0] if lines else r.stdout.strip().splitlines()[-1])


def run_all_stroke(mutants=STROKE_MUTANTS, workers=None):
    workers = workers or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory() as d, cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda m: run_one_stroke(m[0], m[1], m[2], d), mutants))


if __name__ == "__main__":
    res = run_all()
    for name, caught, detail in res:
        print(f"{'caught' if caught else 'MISSED'}  {name}: {detail}")
    for name, caught, detail in run_all(UNPINNED):
        print(f"{'caught' if caught else 'unpinned'}  {name}: {detail}")
    res_s = run_all_stroke()
    for name, caught, detail in res_s:
        print(f"{'caught' if caught else 'MISSED'}  stroke: {name}: {detail}")
    sys.exit(0 if all(c for _, c, _ in res + res_s) else 1)
