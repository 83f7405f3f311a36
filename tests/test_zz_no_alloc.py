"""fe_apply_H_noalloc (the application for callers that cannot allocate)
against fe_apply_H, through the C-ABI: two calls in a row on the shared
static scratch, the second with a smaller input, each equal to fe_apply_H bit
for bit (the same kernels in the same order) and the first to the oracle at
1e-12; a call whose projector workspace exceeds the scratch is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import operator as op  # noqa: E402
from paper_2512_08571_amd import fehx, inputs  # noqa: E402

from gpu_common import lib_side, oracle_side, rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _pair(s):
    om, vl, vg, P, h = oracle_side(s)
    return om, vl, vg, P, h, lib_side(s, vl, vg)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_equals_apply_twice(prec):
    big = inputs.make_custom(np.diag([8.0, 7.5, 8.5]), (4, 3, 4), 4, 5, kpoint=(0.25, -0.1, 0.2), nvec=24,
                             seed=31, natoms=6, pset="spd", rc=3.0)
    small = inputs.make_custom(np.diag([6.5, 7.0, 6.0]), (3, 3, 2), 3, 4, kpoint=(0.0, 0.0, 0.0), nvec=5,
                               seed=32, natoms=3, pset="sp", rc=2.5)
    cdt = {"f64": (torch.complex128, torch.float64), "f32": (torch.complex64, torch.float32)}[prec]
    for idx, s in enumerate((big, small)):          # the second call has a smaller input
        om, vl, vg, P, h, m = _pair(s)
        X = inputs.make_vectors(s)
        Xd = to_dev(X, cdt[0] if s.is_complex else cdt[1])
        Ya, Yb = torch.full_like(Xd, 7.0), torch.full_like(Xd, -3.0)
        print(f"noalloc case {idx} prec {prec} ndofs {m.ndofs} nvec {s.nvec}", flush=True)
        m.apply(Xd, Ya, prec)
        m.apply_noalloc(Xd, Yb, prec)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb), f"case {idx}: noalloc differs from fe_apply_H"
        if idx == 0 and prec == "f64":
            want = op.apply_sparse(op.assemble_H(om, vl, vg), X, P, h)
            assert rel(Yb.cpu().numpy(), want) < 1e-12
        m.close()


def test_noalloc_refuses_oversized_workspace():
    # 64 atoms x 4 projectors, at least one node chunk per atom:
    # (64 x 10 + 256) x 4800 lanes x 8 bytes > 32 MiB of scratch
    s = inputs.make_custom(np.diag([8.0, 8.0, 8.0]), (4, 4, 4), 4, 5, nvec=4800, seed=33, natoms=64,
                           pset="sp", rc=3.0)
    _, vl, vg, _, _ = oracle_side(s, with_P=False)
    m = lib_side(s, vl, vg)
    Xd = torch.zeros((m.ndofs, s.nvec), dtype=torch.float64, device="cuda")
    Yd = torch.empty_like(Xd)
    with pytest.raises(fehx.FeError) as e:
        m.apply_noalloc(Xd, Yd)
    assert e.value.code == -1 and "scratch" in str(e.value)
    m.apply(Xd, Yd)                                  # the allocating entry point still serves it
    torch.cuda.synchronize()
    assert float(Yd.abs().max()) == 0.0
    m.close()
