"""The Python binding validates every tensor before it reaches the C-ABI
(which takes the row count from the mesh and the element type from the
precision argument): wrong dtype, row count, layout, device or vector length
raises ValueError and no library call is made.  Host-only meshes and CPU
tensors, so no GPU is needed."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2512_08571_amd import fehx  # noqa: E402

pytestmark = pytest.mark.skipif(not os.path.exists(fehx.LIB_PATH), reason="library not built")


@pytest.fixture(scope="module", params=[False, True], ids=["real", "complex"])
def mesh(request):
    k = (0.2, 0.0, 0.0) if request.param else (0.0, 0.0, 0.0)
    m = fehx.Mesh(np.diag([6.0, 6.0, 6.0]), (2, 2, 2), 2, 3, kpoint=k, device=-1)
    yield m
    m.close()


@pytest.fixture
def no_library_calls(monkeypatch):
    """Any call into the library through the binding fails the test."""
    L = fehx.lib()

    class Guard:
        def __getattr__(self, name):
            if name.startswith("fe_") and name not in ("fe_last_error",):
                raise AssertionError(f"library call {name} made with an invalid argument")
            return getattr(L, name)

    monkeypatch.setattr(fehx, "lib", lambda: Guard())


def _good(mesh, prec="f64", nvec=4):
    dt = fehx._dtypes(prec, mesh.is_complex)
    shape = (mesh.ndofs, nvec, 2) if (prec == "bf16" and mesh.is_complex) else (mesh.ndofs, nvec)
    return torch.zeros(shape, dtype=dt)


def test_apply_rejects_wrong_dtype(mesh, no_library_calls):
    X = _good(mesh, "f32")
    with pytest.raises(ValueError, match="dtype"):
        mesh.apply(X, _good(mesh, "f32"), "f64")      # float32 block with the FP64 default
    with pytest.raises(ValueError, match="dtype"):
        mesh.apply(_good(mesh, "f64"), _good(mesh, "f64"), "bf16")


def test_apply_rejects_wrong_rows_and_layout(mesh, no_library_calls):
    dt = fehx._dtypes("f64", mesh.is_complex)
    short = torch.zeros((mesh.ndofs - 1, 4), dtype=dt)
    with pytest.raises(ValueError, match="rows"):
        mesh.apply(short, _good(mesh), "f64")
    with pytest.raises(ValueError, match="rows"):
        fehx._check_block(mesh, short, "f64", "Y")
    flat = torch.zeros(mesh.ndofs * 4, dtype=dt)
    with pytest.raises(ValueError, match="block"):
        mesh.apply(flat, _good(mesh), "f64")
    with pytest.raises(ValueError, match="unknown precision"):
        mesh.apply(_good(mesh), _good(mesh), "f16")


def test_apply_rejects_host_tensors(mesh, no_library_calls):
    with pytest.raises(ValueError, match="mesh is on"):
        mesh.apply(_good(mesh), _good(mesh), "f64")
    with pytest.raises(ValueError, match="mesh is on"):
        mesh.apply_mass(_good(mesh, "f32"), _good(mesh, "f32"), "f32")


def test_apply_rejects_nvec_beyond_the_block(mesh, no_library_calls, monkeypatch):
    # pretend the tensors are on the mesh's device so that only nvec is wrong
    monkeypatch.setattr(fehx, "_check_block", lambda *a: None)
    with pytest.raises(ValueError, match="nvec"):
        mesh.apply(_good(mesh, nvec=4), _good(mesh, nvec=3), "f64", nvec=4)


def test_solver_entry_points_need_fp64_blocks(mesh, no_library_calls):
    lam = torch.zeros(4, dtype=torch.float64)
    X32 = _good(mesh, "f32")
    with pytest.raises(ValueError, match="dtype"):
        mesh.cheb_filter(X32, lam, 8, -1.0, 1.0, 5.0, inner="f32")
    with pytest.raises(ValueError, match="dtype"):
        mesh.rayleigh_ritz(X32, lam)
    with pytest.raises(ValueError, match="dtype"):
        mesh.chfsi(X32, torch.zeros(mesh.ndofs, dtype=torch.float64))
    with pytest.raises(ValueError, match="inner precision"):
        mesh.cheb_filter(_good(mesh), lam, 8, -1.0, 1.0, 5.0, inner="fp8")


def test_solver_vectors_checked(mesh, no_library_calls, monkeypatch):
    monkeypatch.setattr(fehx, "_check_block", lambda *a: None)
    X = _good(mesh, nvec=4)
    with pytest.raises(ValueError, match="at least 4"):
        mesh.cheb_filter(X, torch.zeros(3, dtype=torch.float64), 8, -1.0, 1.0, 5.0)
    with pytest.raises(ValueError, match="dtype"):
        mesh.rayleigh_ritz(X, torch.zeros(4, dtype=torch.float32))
    vdt = torch.complex128 if mesh.is_complex else torch.float64
    with pytest.raises(ValueError, match="at least"):
        mesh.lanczos(torch.zeros(mesh.ndofs - 1, dtype=vdt))
    wrong = torch.float64 if mesh.is_complex else torch.complex128
    with pytest.raises(ValueError, match="dtype"):
        mesh.lanczos(torch.zeros(mesh.ndofs, dtype=wrong))
    with pytest.raises(ValueError, match="mesh is on"):
        mesh.lanczos(torch.zeros(mesh.ndofs, dtype=vdt))


def test_batch_apply_checks_each_block(mesh, no_library_calls):
    with pytest.raises(ValueError, match="one X and one Y"):
        fehx.batch_apply([mesh], [_good(mesh)], [], "f64")
    with pytest.raises(ValueError, match=r"X\[0\]"):
        fehx.batch_apply([mesh], [_good(mesh, "f32")], [_good(mesh)], "f64")


def test_library_refuses_overlapping_blocks():
    """fe_apply_H refuses X and Y that share an element (FE_EINVAL) and accepts
    disjoint column windows of one array; a host-only mesh then stops at
    FE_ESTATE.  The pointers are never dereferenced (no device here)."""
    import ctypes
    m = fehx.Mesh(np.diag([6.0, 6.0, 6.0]), (2, 2, 2), 2, 3, device=-1)
    L = fehx.lib()
    base, ld, nv = 1 << 40, 16, 8

    def call(x_off, y_off, nvec=nv, ldy=ld):
        return L.fe_apply_H(m._h, ctypes.c_void_p(base + 8 * x_off), ld, ctypes.c_void_p(base + 8 * y_off), ldy,
                            nvec, fehx.FE_F64, None)
    assert call(0, 0) == -1                       # the same block
    assert call(0, 3) == -1                       # windows [0, 8) and [3, 11) share columns
    assert call(0, 8) == -4                       # disjoint windows [0, 8) and [8, 16) of one array
    assert call(8, 0) == -4
    assert call(0, 5 * ld + 9) == -1              # window [9, 17) wraps into the next row's [0, 1)
    assert call(0, m.ndofs * ld) == -4            # Y after X
    assert call(0, 8, ldy=24) == -1               # interleaving with another leading dimension
    m.close()
