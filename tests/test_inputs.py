"""Host-side checks of the seeded input generators (no method arithmetic)."""
import numpy as np

from paper_2512_08571_amd import inputs


def test_column_subsets_are_reproducible():
    s = inputs.make_system("tiny")
    X = inputs.make_vectors(s)
    Xs = inputs.make_vectors(s, cols=[5, 2])
    assert np.array_equal(X[:, [5, 2]], Xs)
    assert X.min() >= -1 and X.max() <= 1 and X.shape == (4096, 8)


def test_systems_match_the_workload_recipes():
    t = inputs.make_system("tiny")
    assert t.ndofs == 16 ** 3 and len(t.centres) == 4 and t.gga_coef is None
    m = inputs.make_system("mid")
    assert m.ndofs == 884736 and len(m.projectors) == 128 and m.nvec == 256
    f = inputs.make_system("filter")
    assert f.nvec == 512 and np.array_equal(f.atoms, m.atoms)
    c = inputs.make_system("complex")
    assert c.is_complex and len(c.projectors) == 128 * 9 and c.ndofs == (24 * 7) ** 3


def test_fields_are_periodic_and_positive():
    s = inputs.make_system("mid")
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 20, (50, 3))
    for shift in np.eye(3) * 20.0:
        assert np.allclose(inputs.eval_vloc(s, x), inputs.eval_vloc(s, x + shift), atol=1e-14)
        assert np.allclose(inputs.eval_vgga(s, x), inputs.eval_vgga(s, x + shift), atol=1e-14)
    assert np.all(inputs.eval_vgga(s, x) > 0)
    assert np.all(inputs.eval_vloc(s, x) < 0)
