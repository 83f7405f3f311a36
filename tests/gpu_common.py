"""Shared set-up for the GPU parity tests: the same seeded arrays feed both sides."""
import numpy as np

from oracle import operator as op
from oracle.mesh import Mesh as OMesh
from paper_2512_08571_amd import inputs


def oracle_side(s, with_P=True):
    om = OMesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint)
    pts = om.quad_points()
    vl = inputs.eval_vloc(s, pts)
    vg = inputs.eval_vgga(s, pts)
    P = h = None
    if with_P and s.projectors:
        P, h = op.projector_matrix(om, inputs.positions_array(s), s.projectors)
    return om, vl, vg, P, h


def lib_side(s, vl, vg, device=0):
    from paper_2512_08571_amd import fehx
    m = fehx.Mesh(s.lattice, s.ncell, s.degree, s.nq, s.kpoint, device=device)
    m.set_potential(vl, vg)
    if s.projectors:
        m.set_projectors(inputs.positions_array(s), s.projectors)
    return m


def to_dev(X, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(X))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
