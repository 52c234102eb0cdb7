"""GPU parity of the comparison modes on the rest-state locking workloads.

Straight rods at rest (h = 300) for several segment lengths, with the
paper's filter, no filter and culling at 11 and 5 elements; flat sheets at
rest (h = 1000) with the filter and without.  The GPU's active set and
counts must equal the oracle's exactly (and, on the rod, the closed form of
tests/test_oracle_cull.py); energies, gradients and Hessians within the
path's bound.  The paper's filter leaves no pair active at rest at any
resolution; the others lock once the segments are shorter than the
thickness (culling: shorter than h / r).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

MODES = [("filter", 0, 11), ("none", 1, 11), ("cull11", 2, 11), ("cull5", 2, 5)]


def _run(sc, mode, r):
    import paper_2510_10256_amd as bfc
    cs = bfc.ContactScene(sc, filter_mode=mode, cull_radius=r, device=torch.device("cuda:0"))
    cs.run(sc.x)
    g = cs.results()
    cs.close()
    return g


@requires_gpu
@pytest.mark.parametrize("ell", [600.0, 200.0, 100.0, 50.0, 25.0])
def test_rod_at_rest(ell):
    sc = synth.straight_rod(ell, length=10000.0)
    print(f"[locking] rod ell={ell} E={sc.n_edges}", flush=True)
    for name, mode, r in MODES:
        g = _run(sc, mode, r)
        o = oracle.evaluate(sc, mode=1, filter_mode=mode, cull_radius=r)
        compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
        print(ell, name, g["counts"]["n_act"], g["E_total"], float(np.abs(g["g"]).max()), flush=True)
        if mode == 0:
            assert g["counts"]["n_act"] == 0 and g["E_total"] == 0.0 and not np.any(g["g"])
        if mode == 1 and ell < sc.h:
            assert g["counts"]["n_act"] > 0


@requires_gpu
@pytest.mark.parametrize("ell", [2000.0, 700.0, 350.0])
def test_sheet_at_rest(ell):
    sc = synth.flat_sheet(ell, side=8000.0)
    print(f"[locking] sheet ell={ell} V={sc.n_verts}", flush=True)
    for name, mode, r in MODES[:2]:
        g = _run(sc, mode, r)
        o = oracle.evaluate(sc, mode=1, filter_mode=mode)
        compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
        print(ell, name, g["counts"], flush=True)
        if mode == 0:
            assert g["counts"]["n_act"] == 0 and g["E_total"] == 0.0
        elif ell < sc.h:
            assert g["counts"]["n_act"] > 0
