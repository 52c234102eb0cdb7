"""Comparison of GPU results with the CPU oracle (test helper).

Tolerance (FP64 path tau = 1e-10, mixed path tau = 1e-5), per active pair p
with band width w = a - eta and mid-band barrier value
b_ref = kappa * (w/2)^2 ln 2:
    |dE|     <= tau (|E| + b_ref)
    |dG|_2   <= tau (|G|_2 + b_ref / w)
    |dH+|_F  <= tau (|H+|_F + b_ref / w^2)
Assembled values use the same bounds summed over the contributing pairs.
The active set (type, i, j, filtered, infeasible) must match exactly.
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
