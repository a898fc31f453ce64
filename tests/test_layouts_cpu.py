"""The paper-scale problem descriptions carry the paper's mesh sizes and cross sections
("Benchmark Performance") on the layouts this library defines."""
import numpy as np

from paper_2512_13965_amd import inputs


def test_lattice_problem():
    p = inputs.lattice_problem(16)
    assert (p.nx, p.ny) == (112, 112) and abs(p.L - 7.0 / 112) < 1e-15
    sig_t = p.tau / p.L
    sig_s = sig_t * p.c
    absorber = sig_t > 5
    np.testing.assert_allclose(sig_t[~absorber], 1.0)
    np.testing.assert_allclose(sig_s[~absorber], 1.0)
    np.testing.assert_allclose(sig_t[absorber], 10.0)
    np.testing.assert_allclose(sig_s[absorber], 0.5)
    assert absorber.sum() == 12 * 16 * 16                      # twelve 1 x 1 cm blocks
    assert (p.src_x0, p.src_y0, p.src_nx, p.src_ny, p.src_face) == (48, 48, 16, 16, -1)
    a = absorber.reshape(112, 112)
    assert not a[48:64, 48:64].any()                           # the source block scatters
    np.testing.assert_array_equal(a, a.T)                      # the array is symmetric
    np.testing.assert_array_equal(a, a[::-1, ::-1])


def test_hohlraum_problem():
    p = inputs.hohlraum_problem(112)
    assert (p.nx, p.ny) == (112, 112) and abs(p.L - 1.3 / 112) < 1e-15
    sig_t = p.tau / p.L
    sig_s = sig_t * p.c
    pairs = {(round(a, 6), round(s, 6)) for a, s in zip(sig_t - sig_s, sig_s)}
    assert pairs == {(round(a, 6), round(s, 6)) for a, s in inputs.HOHLRAUM_MATERIALS.values()}
    assert (p.src_x0, p.src_y0, p.src_nx, p.src_ny, p.src_face, p.reflect) == (0, 0, 1, 112, 3, False)
    m = sig_s.reshape(112, 112)
    assert m[56, 56] == 5.0 and sig_t.reshape(112, 112)[56, 56] == 100.0    # blue centre
    assert m[56, 10] == 5.0 and sig_t.reshape(112, 112)[56, 10] == 5.0      # white, near the source
    assert m[0, 56] == 50.0 and m[111, 56] == 50.0 and m[56, 111] == 50.0   # black walls


def test_lattice_problem_with_rectangular_cells():
    p = inputs.lattice_problem(16, 8)
    sq = inputs.lattice_problem(16)
    assert (p.nx, p.ny, p.L, p.Ly) == (112, 56, 1.0 / 16, 1.0 / 8)
    # the same material map sampled at every other row
    np.testing.assert_array_equal((p.c.reshape(56, 112) < 0.5), (sq.c.reshape(112, 112)[::2] < 0.5))
    assert (p.src_x0, p.src_y0, p.src_nx, p.src_ny) == (48, 24, 16, 8)


def test_weight_blobs_of_every_model_kind_round_trip():
    for n_in in (inputs.N_IN, inputs.N_IN_RECT, inputs.N_IN_INTERNAL):
        w = inputs.random_weights(32, 3, n_in=n_in)
        back = inputs.unpack_blob(inputs.pack_blob(w))
        assert back.n_in == n_in and back.W[0].shape == (32, n_in)
        for a, b in zip(w.W + w.b, back.W + back.b):
            np.testing.assert_array_equal(a, b)
