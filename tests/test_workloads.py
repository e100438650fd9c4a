"""Sanity of the seeded input generators (mesh, coefficient field, sources)."""
import numpy as np

import workloads as W


def test_kuhn_mesh_volume_and_conformity():
    for n, jit in [(3, 0.0), (4, 0.2)]:
        xyz, tets = W.kuhn_mesh(n, jitter=jit, seed=0)
        assert xyz.shape == ((n + 1) ** 3, 3) and tets.shape == (6 * n ** 3, 4)
        x = xyz[tets]
        vol = np.einsum("ij,ij->i", x[:, 1] - x[:, 0], np.cross(x[:, 2] - x[:, 0], x[:, 3] - x[:, 0])) / 6
        assert abs(np.abs(vol).sum() - 1.0) < 1e-12
        # every interior face is shared by exactly two tets, boundary faces lie on the cube faces
        faces = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]],
                                        tets[:, [0, 1, 2]]]), axis=1)
        uniq, cnt = np.unique(faces, axis=0, return_counts=True)
        assert set(cnt) <= {1, 2}
        bf = xyz[uniq[cnt == 1]]
        on_face = np.any(np.all(np.isclose(bf, 0.0), axis=1) | np.all(np.isclose(bf, 1.0), axis=1), axis=1)
        assert np.all(on_face)
        assert (cnt == 1).sum() == 12 * n * n


def test_jitter_is_seeded_and_bounded():
    a, _ = W.kuhn_mesh(5, jitter=0.2, seed=0)
    b, _ = W.kuhn_mesh(5, jitter=0.2, seed=0)
    c, _ = W.kuhn_mesh(5)
    assert np.array_equal(a, b)
    assert np.max(np.abs(a - c)) <= 0.2 / 5 + 1e-15
    bnd = np.any((c == 0) | (c == 1), axis=1)
    assert np.array_equal(a[bnd], c[bnd])


def test_grf_statistics():
    xyz, tets = W.kuhn_mesh(16)
    g = W.grf_log_kappa(xyz, tets, seed=1)
    assert g.shape == (tets.shape[0],)
    assert 1.0 < g.std() < 4.0
    assert np.array_equal(g, W.grf_log_kappa(xyz, tets, seed=1))


def test_sources():
    p = np.random.default_rng(0).uniform(size=(100, 3))
    assert np.allclose(W.manufactured_f(p), 3 * np.pi ** 2 * W.manufactured_u(p))
    f0 = W.fourier_f(0)
    assert np.array_equal(f0(p), W.fourier_f(0)(p)) and not np.array_equal(f0(p), W.fourier_f(1)(p))
    edge = np.array([[0.0, 0.3, 0.4], [0.2, 1.0, 0.5]])
    assert np.allclose(f0(edge), 0.0)


def test_fourier_fields_equal_single_sources():
    p = np.random.default_rng(1).uniform(size=(2000, 3))
    rs = [0, 3, 7, 31]
    F = W.fourier_fields(rs)(p)
    assert F.shape == (4, 2000)
    for c, r in enumerate(rs):
        ref = W.fourier_f(r)(p)
        assert np.max(np.abs(F[c] - ref)) < 1e-13 * np.max(np.abs(ref))
