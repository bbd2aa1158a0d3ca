"""Defaults that the paper fixes, read from a cited fixture."""
import json
import os

from oracle import dc, fgmres
from paper_2306_06795_amd.inputs import make_problem

FACTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_sv_defaults_follow_table4():
    P = make_problem(dim=2, n=2, disc="SV")
    p = dc.default_params(P)
    t = FACTS["sv_dc_all_vanka_structured"]
    assert (p.omega0, p.eta_p, p.eta_u) == (t["omega0"], t["eta_p"], t["eta_u"])


def test_dlsc_degrees_follow_table3():
    P2 = make_problem(dim=2, n=3)
    P3 = make_problem(dim=3, n=2)
    assert tuple(dc.DCPreconditioner(P2, dc.default_params(P2, relax="dlsc", max_coarse=10)).relax[0].deg) == tuple(FACTS["chebyshev_degrees"]["2D"])
    assert tuple(dc.DCPreconditioner(P3, dc.default_params(P3, relax="dlsc", max_coarse=10)).relax[0].deg) == tuple(FACTS["chebyshev_degrees"]["3D"])


def test_fgmres_restart():
    import inspect
    assert inspect.signature(fgmres.fgmres).parameters["restart"].default == FACTS["fgmres"]["restart"]
