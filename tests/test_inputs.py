"""The synthetic input recipe: lid data on every top-boundary node (corners
included), compatible pressure data, and interior-only uniform vertex jitter."""
import numpy as np
import pytest

from paper_2306_06795_amd.inputs import make_problem
from paper_2306_06795_amd.inputs.mesh import rect_mesh


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 3)])
def test_lid_is_ex_on_every_top_node_corners_included(dim, n):
    P = make_problem(dim=dim, n=n, forcing="gaussian", bc="lid", seed=1)
    f0 = P.field0
    top = P.dir0 & (f0 == 0) & (P.b == 1.0)
    # the P2 nodes of the top side are the (2n+1)^(dim-1) points of the h/2 grid on it
    assert int(top.sum()) == (2 * n + 1) ** (dim - 1)
    # every other Dirichlet value is zero: other components, other sides
    other = P.dir0 & ~top
    assert np.all(P.b[other] == 0.0)
    # no Dirichlet pressure rows; the pressure rows carry only the lifted
    # boundary data -B_D u_D, whose sum vanishes (the lid conserves mass)
    assert not np.any(P.dir0 & (f0 == dim))
    assert abs(P.b[f0 == dim].sum()) <= 1e-12 * np.abs(P.b).max()


def test_jitter_moves_interior_vertices_only_by_uniform_offsets():
    n, jit = 64, 0.2
    h = 1.0 / n
    base = rect_mesh(n).verts
    m = rect_mesh(n, jitter=jit, rng=np.random.default_rng(11))
    d = (m.verts - base) / h
    on_bnd = np.any((np.abs(base) < 1e-15) | (np.abs(base - 1.0) < 1e-15), axis=1)
    assert np.all(d[on_bnd] == 0.0)
    di = d[~on_bnd]
    assert di.shape[0] == (n - 1) ** 2
    assert np.all(np.abs(di) <= jit) and np.all(np.abs(di) > 0.0)
    # U(-a, a): mean 0, variance a^2 / 3 (7938 samples: bounds at ~5 standard errors)
    assert abs(di.mean()) < 5 * jit / np.sqrt(3 * di.size)
    assert abs(di.var() / (jit ** 2 / 3) - 1.0) < 0.08
