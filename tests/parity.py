"""Comparison of GPU results with the CPU oracle (test helper).

Tolerance (FP64 path tau = 1e-10, mixed path tau = 1e-5), per active pair p
with band width w = a - eta and mid-band barrier value
b_ref = kappa * (w/2)^2 ln 2:
    |dE|     <= tau (|E| + b_ref)
    |dG|_2   <= tau (|G|_2 + b_ref / w)
    |dH+|_F  <= tau (|H+|_F + b_ref / w^2)
Assembled values use the same bounds summed over the contributing pairs.
The active set (type, i, j, filtered, infeasible) must match exactly.

Where the two sides chose different distance sub-cases for a pair (a pair
on the boundary between regions, where several sub-cases give the same
distance: lattice geometry puts points exactly above vertices and edges),
the energy and gradient are still unique and compared as above; the GPU's
choice must be a valid one (its sub-case's distance equals the minimum to
1e-12) and its Hessian is compared with the oracle's derivatives of that
same sub-case (the one-sided Hessian on the GPU's side of the boundary).
This needs the positions: gpu["x"].
"""
import math

import numpy as np

import oracle


def active_view(res):
    """Active pairs sorted by (ptype, i, j)."""
    act = (res["flags"] & oracle.F_ACTIVE) != 0 if "counts" not in res else np.ones(len(res["i"]), bool)
    idx = np.nonzero(act)[0]
    order = np.lexsort((res["j"][idx], res["i"][idx], res["ptype"][idx]))
    return idx[order]


def compare(gpu, orc, nv, kappa=1.0, tau=1e-10, check_assembly=True, derivs=True):
    report = {}
    oc = oracle.counts(orc)
    gc = gpu["counts"]
    for k in ("n_c", "n_filt", "n_act", "n_infeasible"):
        assert gc[k] == oc[k], f"count {k}: gpu {gc[k]} oracle {oc[k]}"
    gi = active_view(gpu)
    oi = active_view(orc)
    assert len(gi) == len(oi)
    for k in ("ptype", "i", "j"):
        assert np.array_equal(gpu[k][gi], orc[k][oi]), f"active set differs in {k}"
    gfl = gpu["flags"][gi] & 5
    ofl = orc["flags"][oi] & (oracle.F_FILTERED | oracle.F_INFEASIBLE)
    assert np.array_equal(gfl, ofl), "filtered/infeasible flags differ"
    report["code_match"] = float(np.mean(gpu["code"][gi] == orc["code"][oi])) if len(gi) else 1.0
    # candidate superset of the N_c set
    if "cand" in gpu:
        cset = set(map(tuple, gpu["cand"].tolist()))
        nc = list(zip(orc["ptype"].tolist(), orc["i"].tolist(), orc["j"].tolist()))
        missing = [p for p in nc if p not in cset]
        assert not missing, f"{len(missing)} pairs with d < h missing from the candidates"
    if not len(gi):
        return report
    orc = _with_gpu_subcases(gpu, orc, gi, oi, report, kappa)
    a, eta = orc["a"][oi], orc["eta"][oi]
    w = a - eta
    bref = kappa * (w / 2) ** 2 * math.log(2)
    feas = (orc["flags"][oi] & oracle.F_INFEASIBLE) == 0
    Eg, Eo = gpu["E"][gi], orc["E"][oi]
    assert np.all(np.isinf(Eg[~feas])) and np.all(np.isinf(Eo[~feas]))
    dE = np.abs(Eg[feas] - Eo[feas])
    tolE = tau * (np.abs(Eo[feas]) + bref[feas])
    report["E_worst"] = float(np.max(dE / tolE)) if feas.any() else 0.0
    assert np.all(dE <= tolE), f"per-pair energy: worst ratio {report['E_worst']:.3g}"
    if derivs:
        dG = np.linalg.norm(gpu["G"][gi][feas] - orc["G"][oi][feas], axis=1)
        tolG = tau * (np.linalg.norm(orc["G"][oi][feas], axis=1) + bref[feas] / w[feas])
        report["G_worst"] = float(np.max(dG / tolG, initial=0.0))
        assert np.all(dG <= tolG), f"per-pair gradient: worst ratio {report['G_worst']:.3g}"
        dH = np.linalg.norm((gpu["Hpsd"][gi][feas] - orc["Hpsd"][oi][feas]).reshape(-1, 144), axis=1)
        tolH = tau * (np.linalg.norm(orc["Hpsd"][oi][feas].reshape(-1, 144), axis=1) + bref[feas] / w[feas] ** 2)
        report["H_worst"] = float(np.max(dH / tolH, initial=0.0))
        assert np.all(dH <= tolH), f"per-pair Hessian: worst ratio {report['H_worst']:.3g}, " \
                                   f"{int(np.sum(dH > tolH))} pairs"
    if check_assembly and derivs:
        asm = oracle.assemble(orc, nv)
        sig = np.abs(Eo[feas]) + bref[feas]
        if np.all(feas):
            assert abs(gpu["E_total"] - asm["E"]) <= tau * np.sum(sig) + 1e-300, "assembled energy"
        else:
            assert np.isinf(gpu["E_total"]) and np.isinf(asm["E"])
        # per-vertex gradient bound: sum of the contributing pairs' bounds
        gb = np.zeros(nv)
        for s in range(4):
            np.add.at(gb, orc["verts"][oi][feas][:, s], tau * (np.linalg.norm(orc["G"][oi][feas], axis=1)
                                                                + bref[feas] / w[feas]))
        dg = np.linalg.norm(gpu["g"] - asm["g"], axis=1)
        assert np.all(dg <= gb + 1e-300), "assembled gradient"
        assert np.array_equal(gpu["row_ptr"], asm["row_ptr"]), "BSR row pointers"
        assert np.array_equal(gpu["col"], asm["col"]), "BSR columns"
        hb = np.zeros(nv)
        for s in range(4):
            np.add.at(hb, orc["verts"][oi][feas][:, s], tau * (np.linalg.norm(orc["Hpsd"][oi][feas].reshape(-1, 144),
                                                                               axis=1) + bref[feas] / w[feas] ** 2))
        rows = np.repeat(np.arange(nv), np.diff(asm["row_ptr"]))
        dv = np.linalg.norm((gpu["val"] - asm["val"]).reshape(-1, 9), axis=1)
        assert np.all(dv <= hb[rows] + 1e-300), "assembled Hessian blocks"
    return report


def _with_gpu_subcases(gpu, orc, gi, oi, report, kappa):
    """The oracle's results with the pairs whose sub-case differs from the
    GPU's re-derived on the GPU's sub-case, after checking that the GPU's
    sub-case is a valid choice (same distance)."""
    diff = np.nonzero(gpu["code"][gi] != orc["code"][oi])[0]
    report["subcase_ties"] = int(len(diff))
    if not len(diff) or "Hpsd" not in orc:
        return orc
    assert "x" in gpu, f"{len(diff)} pairs with another sub-case and no positions to check them"
    x = np.asarray(gpu["x"], np.float64)
    out = dict(orc)
    out["G"] = orc["G"].copy()
    out["Hpsd"] = orc["Hpsd"].copy()
    for q in diff:
        k = oi[q]
        if orc["flags"][k] & oracle.F_INFEASIBLE:
            continue
        X = x[orc["verts"][k]].reshape(12)
        code = int(gpu["code"][gi[q]])
        D_alt = oracle.case_distance(code, X)[0]
        D_min = orc["d"][k] ** 2
        assert abs(D_alt - D_min) <= 1e-12 * D_min, f"GPU sub-case {code} is not a nearest one"
        r = oracle.pair_barrier_code(code, X, orc["a"][k], orc["eta"][k], kappa=kappa, quad=True)
        out["G"][k] = r["G"]
        out["Hpsd"][k] = r["Hpsd"]
    return out


def compare_assembled(E, g, orc, nv, kappa=1.0, tau=1e-10):
    """The assembled energy and gradient of a step (E, g[V,3]) against the
    oracle's, within the summed per-pair bounds (the serving loop returns
    only these)."""
    asm = oracle.assemble(orc, nv)
    act = (orc["flags"] & oracle.F_ACTIVE) != 0
    feas = act & ((orc["flags"] & oracle.F_INFEASIBLE) == 0)
    w = (orc["a"] - orc["eta"])[feas]
    bref = kappa * (w / 2) ** 2 * math.log(2)
    if np.all(feas == act):
        assert abs(E - asm["E"]) <= tau * np.sum(np.abs(orc["E"][feas]) + bref) + 1e-300, "assembled energy"
    else:
        assert np.isinf(E) and np.isinf(asm["E"])
    gb = np.zeros(nv)
    nG = np.linalg.norm(orc["G"][feas], axis=1)
    for s in range(4):
        np.add.at(gb, orc["verts"][feas][:, s], tau * (nG + bref / w))
    dg = np.linalg.norm(np.asarray(g) - asm["g"], axis=1)
    assert np.all(dg <= gb + 1e-300), "assembled gradient"
    return {"E_ratio": abs(E - asm["E"]) / (tau * np.sum(np.abs(orc["E"][feas]) + bref) + 1e-300)}
