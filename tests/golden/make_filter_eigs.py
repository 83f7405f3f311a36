"""Write tests/golden/filter_eigs.npz: the FP64 oracle's Ritz values of the
mixed-precision filter workload, the reference of the precision gate.

The procedure is Alg. 3 with the Alg. 4 filter (M = D, the lumped mass), the
bounds rule of oracle.eigen.chfsi (10 Lanczos steps on D^-1/2 H D^-1/2 from
the workload's seeded start vector; Rayleigh-Ritz of the seeded start block;
pass 1 from the Lanczos interval and the free-electron cut, later passes from
the previous Ritz interval), filter degree 40, 3 outer passes, on the Mid
operator (16^3 cells, p = 6, n_q = 7, GGA, 32 atoms x 4 projectors) with
512 start vectors, H applied by the oracle's cell-matrix route.  Stores all
512 Ritz values (ascending) and the bounds of each pass.

Calls only the CPU oracle and the input generators (about an hour and ~40 GB
of host memory on 8 cores); run from the repository root:
    python tests/golden/make_filter_eigs.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import eigen  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle.mesh import Mesh as OMesh  # noqa: E402
from paper_2512_08571_amd import inputs  # noqa: E402

DEGREE, OUTER, LANCZOS = 40, 3, 10


def main():
    t0 = time.time()
    s = inputs.make_system("filter")
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint)
    pts = om.quad_points()
    vl, vg = inputs.eval_vloc(s, pts), inputs.eval_vgga(s, pts)
    P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors)
    Hop = op.cm_operator(om, vl, vg, P, h, batch=256)
    Dv = op.lumped_mass(om)
    X0 = inputs.make_vectors(s, seed_offset=0)
    v0 = inputs.lanczos_start(s)
    del pts
    print(f"set-up {time.time() - t0:.0f} s: {om.m} DoFs x {X0.shape[1]} vectors", flush=True)
    calls = [0]

    def counted(X):
        calls[0] += 1
        if calls[0] % 10 == 0:
            print(f"  H X call {calls[0]} at {time.time() - t0:.0f} s", flush=True)
        return Hop(X)

    lam, X, log = eigen.chfsi(counted, Dv, X0, v0, om.volume, outer=OUTER, degree=DEGREE,
                              lanczos_steps=LANCZOS)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "filter_eigs.npz")
    bounds = np.array([[g["lmin"], g["lT"], g["lmax"]] for g in log])
    np.savez(out, ritz=np.asarray(lam), bounds=bounds, degree=DEGREE, outer=OUTER, lanczos_steps=LANCZOS,
             ndofs=om.m, nvec=X0.shape[1])
    print(f"wrote {out}: {len(lam)} Ritz values, lowest {lam[0]:.12f}, 400th {lam[399]:.12f}, "
          f"{calls[0]} H X calls in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
