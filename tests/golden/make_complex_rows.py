"""Write tests/golden/complex_rows.npz: oracle values of (H X)[rows, :16] for the
complex Bloch workload (24^3 cells, degree 7, k = (0.25, 0.1, 0) 2 pi / 28,
128 atoms x 9 projectors), X = the first 16 seeded columns of
paper_2512_08571_amd.inputs.  Calls only the CPU oracle and the input
generators; run from the repository root:  python tests/golden/make_complex_rows.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import operator as op  # noqa: E402
from oracle.mesh import Mesh as OMesh  # noqa: E402
from paper_2512_08571_amd import inputs  # noqa: E402


def main():
    t0 = time.time()
    s = inputs.make_system("complex")
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint)
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors)
    X = inputs.make_vectors(s, cols=range(16))
    rng = np.random.default_rng(6)
    p = om.p
    pick = [0, p - 1, p, p + 1, om.M[0] * p + p // 2, (om.M[0] * om.M[1]) * p + om.M[0] * p + p, om.m - 1]
    pick += list(rng.integers(0, om.m, 24)) + list(rng.choice(P.tocoo().row, 8))
    rows = np.unique(np.array(pick) % om.m)
    Y = op.apply_rows(om, vl, vg, X, rows, P, h)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "complex_rows.npz")
    np.savez(out, rows=rows, y=Y, cols=np.arange(16))
    print(f"wrote {out}: {len(rows)} rows x 16 columns in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
