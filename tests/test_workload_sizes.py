"""The benchmark inputs have the sizes their descriptions state, from closed
forms of each mesh family (not from the generator):

* Taylor-Hood on N x N squares split into two triangles: the P2 nodes are the
  (2N+1)^2 points of the grid of spacing h/2, the P1 pressure nodes the
  (N+1)^2 vertices; 2N^2 triangles; the Dirichlet velocity nodes are the 8N
  boundary points of the fine grid.
* Taylor-Hood on N^3 cubes split into 6 tetrahedra (Kuhn): again the P2 nodes
  are the (2N+1)^3 points of the h/2 grid, pressure (N+1)^3; 6N^3 tetrahedra;
  the Dirichlet nodes are (2N+1)^3 - (2N-1)^3.
* Scott-Vogelius on the Alfeld (barycentric) refinement of N x N squares split
  into two triangles: 3 * 2N^2 cells; vertices (N+1)^2 + 2N^2 (one barycentre
  per coarse triangle); edges 2N(N+1) + N^2 (coarse) + 3 * 2N^2 (new); P2
  nodes = vertices + edges; P1disc pressure = 3 per cell.
"""
import pytest

from paper_2306_06795_amd.inputs import make_config


def _th2d(N):
    nodes = (2 * N + 1) ** 2
    return dict(n_u=2 * nodes, n_p=(N + 1) ** 2, n_dir=2 * 8 * N, n_elem=2 * N * N)


def _th3d(N):
    nodes = (2 * N + 1) ** 3
    return dict(n_u=3 * nodes, n_p=(N + 1) ** 3, n_dir=3 * (nodes - (2 * N - 1) ** 3), n_elem=6 * N ** 3)


def _sv2d(N):
    cells = 3 * 2 * N * N
    verts = (N + 1) ** 2 + 2 * N * N
    edges = 2 * N * (N + 1) + N * N + 3 * 2 * N * N
    return dict(n_u=2 * (verts + edges), n_p=3 * cells, n_dir=2 * 8 * N, n_elem=cells)


@pytest.mark.parametrize("name,want", [("th2d_256", _th2d(256)), ("th3d_32", _th3d(32)),
                                       ("sv2d_128x64", _sv2d(128))])
def test_benchmark_inputs_have_their_stated_sizes(name, want):
    P = make_config(name)
    got = dict(n_u=P.meta["n_u"], n_p=P.n0 - P.meta["n_u"], n_dir=int(P.dir0.sum()), n_elem=P.meta["n_elem"])
    assert got == want
    assert P.n0 == want["n_u"] + want["n_p"]


def test_closed_forms_on_the_small_case():
    # the 16 x 16 Taylor-Hood problem: 2178 velocity and 289 pressure unknowns
    w = _th2d(16)
    assert (w["n_u"], w["n_p"]) == (2178, 289)
    # the 32^3 problem: about 824k velocity and 36k pressure unknowns
    w = _th3d(32)
    assert (w["n_u"], w["n_p"]) == (823875, 35937)
