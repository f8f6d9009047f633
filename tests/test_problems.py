"""Input generators: sizes, symmetry, definiteness, determinism."""

import numpy as np

from problems import FVDiffusion, FourierField, config1, config2, tiny


def test_config_sizes_match_stated_workloads():
    c1 = config1()
    assert (c1.n, c1.nnz) == (1024, 4992)
    fv = FVDiffusion(128, 3)
    assert (fv.n, fv.nnz) == (2_097_152, 14_581_760)


def test_fv_matrices_are_symmetric_positive_definite():
    for cfg in (config1(N=12), config2(N=7, steps=3)):
        A = cfg.fv.dense(cfg.matrix_values(2))
        assert np.array_equal(A, A.T)
        assert np.linalg.eigvalsh(A).min() > 0
        # columns sorted within each row
        for i in range(cfg.n):
            c = cfg.colind[cfg.rowptr[i]:cfg.rowptr[i + 1]]
            assert np.all(np.diff(c) > 0) and i in c


def test_fv_constant_coefficient_is_the_scaled_laplacian():
    fv = FVDiffusion(6, 2)
    A = fv.dense(fv.values(np.ones((8, 8))))
    ref = tiny.laplacian_2d(6) / fv.h ** 2
    assert np.allclose(A, ref, rtol=1e-14)


def test_config1_matrix_is_a_uniform_scaling():
    c = config1()
    assert np.allclose(c.matrix_values(7), 1.07 * c.matrix_values(0), rtol=1e-15)


def test_config2_drift_is_a_one_cell_shift():
    c = config2(N=9, steps=4)
    k = c._g
    J = c.steps
    assert np.array_equal(k[:, :, J - 2: J - 2 + 11][:, :, 1:], k[:, :, J - 1: J - 1 + 11][:, :, :-1])


def test_fields_are_seeded_and_unit_variance():
    f1 = FourierField(2, 0.2, 7)
    f2 = FourierField(2, 0.2, 7)
    pts = np.random.Generator(np.random.PCG64(0)).uniform(size=(4000, 2)) * 20
    a, b = f1.at_points(pts), f2.at_points(pts)
    assert np.array_equal(a, b)
    assert 0.7 < a.var() < 1.3
    ax = np.linspace(0, 1, 5)
    g = f1.on_grid(ax, ax)
    X, Y = np.meshgrid(ax, ax)
    assert np.allclose(g, f1.at_points(np.stack([X.ravel(), Y.ravel()], 1)).reshape(5, 5))
