"""The seeded input generator: shapes, determinism, the bilinear design."""
import numpy as np

from inla_synth import THETA0, config_theta_batch, fd_stencil, line_search_points, make_model, uneven_batch


def test_shapes_and_determinism():
    a = make_model(5, 3, 2, seed=7)
    b = make_model(5, 3, 2, seed=7)
    assert a.m == 2 * 25 * 3 and a.n == 25 * 3 + 2
    assert a.A_rowptr.dtype == np.int64 and a.A_col.dtype == np.int32
    assert a.A_rowptr[-1] == a.A_col.size == a.A_val.size
    assert np.array_equal(a.y, b.y) and np.array_equal(a.A_val, b.A_val)


def test_bilinear_rows():
    md = make_model(6, 4, 3, seed=1)
    nst = md.ns * md.nt
    for j in range(0, md.m, 37):
        lo, hi = md.A_rowptr[j], md.A_rowptr[j + 1]
        cols, vals = md.A_col[lo:hi], md.A_val[lo:hi]
        st = cols < nst
        assert st.sum() == 4 and np.all(np.diff(cols) > 0)
        assert abs(vals[st].sum() - 1.0) < 1e-14 and np.all(vals[st] >= 0)
        t = j // (2 * md.ns)
        assert np.all(cols[st] // md.ns == t)
        assert np.array_equal(cols[~st], nst + np.arange(md.nb))


def test_theta_batches():
    st = fd_stencil(THETA0, 1e-3)
    assert st.shape == (9, 4) and np.allclose(st[1] - st[2], [2e-3, 0, 0, 0])
    ls = line_search_points(THETA0, 2209)
    assert ls.shape == (8, 4)
    d = ls - THETA0
    assert np.allclose(np.linalg.matrix_rank(d), 1)
    assert config_theta_batch("c2").shape == (9, 4)
    shapes = uneven_batch(64, build=False)
    assert len(shapes) == 64
    assert {s[0][0] for s in shapes} <= {16, 24, 32}
