"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/mcs_oracle.c (a
dropped term, a wrong sign or index, a transposed operand, a wrong
comparison), builds it, and runs the pin file that should catch it with the
broken library in place of the real one.  A case passes when that pin run
fails.  This is how the pins are shown to pin something: an oracle that can
be broken without a pin noticing is not checked.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mcs_oracle.c")

# (name, text in mcs_oracle.c, replacement, pin file expected to fail)
MUTATIONS = [
    ("cross product sign",
     "double r0 = a[1] * b[2] - a[2] * b[1];", "double r0 = a[2] * b[1] - a[1] * b[2];",
     "test_oracle_gradient_fd.py"),
    ("trilinear corner sign",
     "dG[0] += val * (2 * a - 1) * w[1][b] * w[2][c];", "dG[0] += val * (1 - 2 * a) * w[1][b] * w[2][c];",
     "test_oracle_likelihood.py"),
    ("transposed corner index",
     "size_t idx = (size_t)(i0[0] + a) + (size_t)g->nx * ((size_t)(i0[1] + b)",
     "size_t idx = (size_t)(i0[0] + b) + (size_t)g->nx * ((size_t)(i0[1] + a)",
     "test_oracle_likelihood.py"),
    ("resampling >= for >",
     "while (i < N && !(cdf[i] > uk)) ++i;", "while (i < N && !(cdf[i] >= uk)) ++i;",
     "test_oracle_weights_resample.py"),
    ("transposed V", "V[e] = (e % 4 == 0 ? 1.0 : 0.0) + a * K[e] + b * K2[e];",
     "V[e] = (e % 4 == 0 ? 1.0 : 0.0) - a * K[e] + b * K2[e];", "test_oracle_se3.py"),
    ("ESS without the square", "S2 += w * w;", "S2 += w;", "test_oracle_weights_resample.py"),
    ("dropped half-voxel offset", "u[a] = (v[a] + t[a] - g->o[a]) / g->h - 0.5;",
     "u[a] = (v[a] + t[a] - g->o[a]) / g->h;", "test_oracle_likelihood.py"),
    ("R for R^T in the gradient", "mat3T_vec(R, A, gr);", "mat3_vec(R, A, gr);",
     "test_oracle_gradient_fd.py"),
    ("swapped composition order", "quat_mul(qa, qb, q);", "quat_mul(qb, qa, q);", "test_oracle_step.py"),
    ("quaternion product sign",
     "r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];",
     "r[1] = a[0] * b[1] + a[1] * b[0] - a[2] * b[3] + a[3] * b[2];", "test_oracle_se3.py"),
    ("weights from the post-step likelihood", "        if (post_eval) {\n            eval_pose(",
     "        if (1) {\n            eval_pose(", "test_oracle_filter_step.py"),
    ("resampled poses not gathered",
     "memcpy(poses_out + 7 * (size_t)k, cur + 7 * (size_t)ancestors[k], 7 * sizeof(double));",
     "memcpy(poses_out + 7 * (size_t)k, cur + 7 * (size_t)k, 7 * sizeof(double));",
     "test_oracle_filter_step.py"),
    ("neighbour ties to the larger index", "if (best < 0 || d < bd) { bd = d; best = k; }",
     "if (best < 0 || d <= bd) { bd = d; best = k; }", "test_oracle_keyframes.py"),
    ("face allowance misses the lower cell", "const int cell_off[4] = {-1, -1, 0, 0};",
     "const int cell_off[4] = {0, -1, 0, 0};", "test_oracle_filter_step.py"),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_the_mutation(tmp_path, name, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: %r" % old
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", str(lib), str(mutant), "-lm"], check=True)
    env = dict(os.environ, MCS_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pins)], env=env, cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode != 0, "%s: %s passed against the mutated oracle\n%s" % (name, pins, r.stdout[-2000:])
    # Caught by a failed check, not by a library that would not load.
    assert "OSError" not in r.stdout and ("AssertionError" in r.stdout or "assert " in r.stdout), r.stdout[-2000:]
