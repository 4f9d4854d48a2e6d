"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a wider
stencil window, a window that crosses into the next subgrid, swapped outputs
of the bin finder, the lower subgrid on a threshold tie, a wrong slope rule, a
dropped basis term, a transposed value index), builds it with gcc into a
temporary directory, and runs the pin tests against that build in a child
process (ORACLE_LIB_OVERRIDE).  The pins pass on an unaltered copy and must
fail on every altered one.  Nothing here touches the GPU library.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pdf_oracle.c")
PINS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
        os.path.join(ROOT, "tests", "test_oracle_stencil_locate.py")]

# (name, text in the source, replacement)
MUTATIONS = [
    ("stencil_window_one_knot_wider", "for (int i = ix - 1; i <= ix + 2; ++i) {",
     "for (int i = ix - 1; i <= ix + 3; ++i) {"),
    ("stencil_window_crosses_subgrid", "if (k < 0 || k >= ns)", "if (k < 0 || k >= ns + 1)"),
    ("locate_swaps_subgrid_and_bin", "s[p] = b;\n        iq[p] = c;",
     "s[p] = c;\n        iq[p] = b;"),
    ("threshold_tie_takes_lower_subgrid", "if (g->q2[g->q_off[k]] <= q2)",
     "if (g->q2[g->q_off[k]] < q2)"),
    ("interior_slope_not_halved", "return 0.5 * (dl + dr);", "return 0.5 * dl + dr;"),
    ("basis_term_h11_dropped", "h[2] * y1 + h[3] * dz * m1;", "h[2] * y1;"),
    ("x_and_q_index_transposed",
     "const double *col = g->xf + (long)f * g->n_x * nq + off + k;   /* stride nq along x */",
     "const double *col = g->xf + (long)f * g->n_x * nq + (off + k) * g->n_x;"),
]


def _build(src_text: str, out_dir: str, name: str) -> str:
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-o", so, c, "-lm", "-lpthread"], check=True)
    return so


def _run_pins(lib: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=300)


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def test_pins_pass_on_unaltered_copy(source, tmp_path):
    r = _run_pins(_build(source, str(tmp_path), "unaltered"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_fail_on_planted_mistake(source, tmp_path, name, old, new):
    assert source.count(old) == 1, "mutation target not found once: " + name
    r = _run_pins(_build(source.replace(old, new), str(tmp_path), name))
    assert r.returncode != 0, "no pin caught " + name
