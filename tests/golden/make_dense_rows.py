"""Write the dense-row fixtures: seeded rows of the dense Galerkin EFIE matrix
(Sec. 2, Eq. 1-3) times a seeded vector, computed by the oracle alone.

    python tests/golden/make_dense_rows.py [case ...]

Each fixture (``dense_rows_<case>.json``) holds the mesh recipe, the vector's
seed, the sampled rows (canonical RWG order) and the values (Z x)[rows].  The
values are the plain definition of the product NESA approximates, so a product
of any NESA operator of the same mesh compared on these rows measures its
truncation error.  Only ``oracle`` and ``synth`` are imported.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import efie  # noqa: E402

# case -> (mesh recipe evaluated against synth, number of rows, row seed, vector seed)
CASES = {
    "sphere201720": ("synth.icosphere(82, 4.0)", 64, 11, 0),
    "aircraft959364": ("synth.aircraft_like(3)", 24, 12, 0),
}


def body_cases(n=4):
    """Four bodies of the uneven family (seed 4), indices 0..3."""
    return {"body4_%d" % i: ("synth.body_family(%d, seed=4)[%d][:2]" % (i + 1, i), 32, 20 + i, 100 + i)
            for i in range(n)}


CASES.update(body_cases())


def make(case):
    recipe, nrows, row_seed, x_seed = CASES[case]
    t0 = time.time()
    v, t = eval(recipe, {"synth": synth})
    m = efie.RWG(v, t)
    rows = np.sort(np.random.default_rng(row_seed).choice(m.n, nrows, replace=False))
    x = synth.complex_normal(m.n, x_seed)
    y = efie.z_block(m, rows, np.arange(m.n)) @ x
    out = {"mesh": recipe, "n": int(m.n), "x": "synth.complex_normal(n, %d)" % x_seed,
           "rows": rows.tolist(), "y_re": y.real.tolist(), "y_im": y.imag.tolist()}
    path = os.path.join(HERE, "dense_rows_%s.json" % case)
    with open(path, "w") as f:
        json.dump(out, f)
    print("%s: n = %d, %d rows, %.1f s -> %s" % (case, m.n, nrows, time.time() - t0, path))


def load(case):
    with open(os.path.join(HERE, "dense_rows_%s.json" % case)) as f:
        d = json.load(f)
    return d["mesh"], d["n"], np.array(d["rows"]), np.array(d["y_re"]) + 1j * np.array(d["y_im"])


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        make(c)
