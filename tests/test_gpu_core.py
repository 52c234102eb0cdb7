"""GPU parity of the temporary zero offset (Sec. 3.4) against the oracle.

Scenes that start inside the core: two rods crossing 250 um apart (h 300,
eta 270) and the yarn patch squeezed in z so that its crossings sit closer
than eta.  Sequence: mark at the start; evaluate there (core pairs take
offset 0, nothing is infeasible); move to a configuration where part of the
set is beyond eta (those pairs are released); move back (released pairs are
infeasible again, the rest stays in the set); the line search with the set
(offset 0 in ACCD).  At every stage the GPU's path is compared with the
oracle given the same set, with the bar of the path's parity tests, and the
BF_F_CORE flags, the marked count and the live count must match exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _squeezed_yarn(full=False):
    sc = synth.workload("woven_patch") if full else synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)
    return sc, sc.x * np.array([1.0, 1.0, 0.88])


CASES = {
    "crossing": lambda: (synth.crossing_rods(250.0), synth.crossing_rods(250.0).x,
                         synth.crossing_rods(262.0).x),
    "yarn": lambda: (_squeezed_yarn()[0], _squeezed_yarn()[1], _squeezed_yarn()[0].x * np.array([1, 1, 0.95])),
    "yarn_full": lambda: (_squeezed_yarn(True)[0], _squeezed_yarn(True)[1],
                          _squeezed_yarn(True)[0].x * np.array([1, 1, 0.95])),
}


def _core_keys(res):
    sel = (res["flags"] & 8) != 0
    return set(zip(res["ptype"][sel].tolist(), res["i"][sel].tolist(), res["j"][sel].tolist()))


def _oracle_core_keys(o):
    sel = (o["flags"] & oracle.F_CORE) != 0
    return set(zip(o["ptype"][sel].tolist(), o["i"][sel].tolist(), o["j"][sel].tolist()))


@requires_gpu
@pytest.mark.parametrize("name", list(CASES))
def test_core_set_mark_release_and_line_search(name):
    import paper_2510_10256_amd as bfc
    sc, x0, x1 = CASES[name]()
    print(f"[core] {name} V={sc.n_verts}", flush=True)
    dev = torch.device("cuda:0")
    cs = bfc.ContactScene(sc, device=dev)
    X0 = torch.tensor(x0, dtype=torch.float64, device=dev)
    X1 = torch.tensor(np.ascontiguousarray(x1), dtype=torch.float64, device=dev)
    st = cs.run(X0)
    assert st & bfc.BF_S_INFEASIBLE  # the start is inside the core
    core0 = oracle.core_mark(sc, x0)
    assert len(core0[0]) > 0
    cs.build_candidates(X0)
    cnt = cs.core_mark(X0)
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(core0[0])
    assert cs.status(clear=True) & bfc.BF_S_CORE_OVERFLOW == 0

    def check(x, core, label):
        cs.run(torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev))
        g = cs.results()
        o = oracle.evaluate(sc, x, mode=1, core=core)
        rep = compare(g, o, sc.n_verts, kappa=sc.kappa, tau=1e-10)
        assert _core_keys(g) == _oracle_core_keys(o), label
        live = cs.core_live()
        torch.cuda.synchronize()
        assert int(live.item()) == len(core[0]), label
        print(name, label, g["counts"], "core", len(core[0]), rep, flush=True)
        return g

    # at the start: the marked pairs take offset 0, nothing is infeasible
    g0 = check(x0, core0, "start")
    assert g0["counts"]["n_infeasible"] == 0
    # part of the set moves beyond eta: released
    rel = oracle.core_release(sc, x1, core0)
    assert rel.any()
    core1 = tuple(a[~rel] for a in core0)
    check(x1, core1, "moved")
    # back at the start: the released pairs are infeasible again
    g2 = check(x0, core1, "back")
    assert g2["counts"]["n_infeasible"] > 0 or not (~rel).any()
    # line search from x1 with the remaining set: offset 0 in ACCD
    p = synth.search_direction(sc)
    Xp = torch.tensor(p, dtype=torch.float64, device=dev)
    cs.fit_swept(X1, Xp)
    t, tp, it = cs.max_step(X1, Xp, per_pair=True)
    torch.cuda.synchronize()
    orc = oracle.max_step(sc, x1, p, core=core1)
    n = int(cs.c_n.item())
    tp, it = tp[:n].cpu().numpy(), it[:n].cpu().numpy()
    inset = tp >= 0
    keys = list(zip(cs.c_t[:n].cpu().numpy()[inset].astype(int).tolist(), cs.c_i[:n].cpu().numpy()[inset].tolist(),
                    cs.c_j[:n].cpu().numpy()[inset].tolist()))
    gk = dict(zip(keys, tp[inset].tolist()))
    ok = dict(zip(zip(orc["ptype"].tolist(), orc["i"].tolist(), orc["j"].tolist()), orc["tpair"].tolist()))
    assert set(gk) == set(ok)
    tg = np.array([gk[k] for k in ok])
    to = np.array([ok[k] for k in ok])
    assert np.all(np.abs(tg - to) <= 1e-9 * np.maximum(to, 1e-300))
    assert abs(float(t.item()) - orc["t"]) <= 1e-9 * max(orc["t"], 1e-300)
    cs.core_clear()
    cs.close()
