"""CPU oracle for barrier-filtered contact evaluation (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2510_10256_amd``); both read the same seeded inputs from ``synth``.

The arithmetic lives in ``oracle.cpp`` (plain C++17, double precision, with
binary128 re-evaluation inside the guard band of each threshold decision).
This module is argument marshalling plus the plain assembly of the per-pair
results (sums over pairs, Sec. 3 and App. A: the global energy, gradient and
Hessian fed to the Newton solve).

Functions whose parity is not pinned by an independent check: none.  The
pins of each function are in ``tests/test_oracle_pins.py`` (distances,
barrier, derivatives, projection, decisions, precompute, rest states),
``tests/test_oracle_assembly.py`` (assembly against finite differences of
the assembled energy and gradient; the binary128 derivative branch against
50-digit arithmetic; exact ties against rational arithmetic),
``tests/test_oracle_accd.py``, ``tests/test_oracle_core.py``,
``tests/test_oracle_cull.py`` and ``tests/test_oracle_friction.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

F_FILTERED, F_ACTIVE, F_INFEASIBLE, F_EXTENDED, F_CORE = 1, 2, 4, 8, 16
PT, EE = 0, 1

# distance sub-case codes (see oracle.cpp): kind of formula per code
CASE_KIND = np.array([0, 0, 0, 1, 1, 1, 2, 0, 0, 0, 0, 1, 1, 1, 1, 3], np.int32)


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (OpenMP, binary128 via libquadmath)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               _SRC, "-o", _SO + ".tmp", "-lquadmath"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Scene(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nv", C.c_int64), ("ne", C.c_int64), ("nt", C.c_int64),
                ("edges", C.c_void_p), ("tris", C.c_void_p), ("ref", C.c_void_p),
                ("h", C.c_double), ("eta", C.c_double), ("kappa", C.c_double),
                ("filter_mode", C.c_int32), ("n_core", C.c_int64), ("core_ptype", C.c_void_p),
                ("core_i", C.c_void_p), ("core_j", C.c_void_p), ("cull_radius", C.c_int32),
                ("refdist", C.c_int32), ("xrest", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        L.orc_precompute.argtypes = [C.POINTER(_Scene), P, P, P, C.c_int32]
        L.orc_precompute.restype = C.c_int32
        L.orc_evaluate.argtypes = [C.POINTER(_Scene), P, C.c_int32, C.c_int32, C.c_int32]
        L.orc_evaluate.restype = C.c_void_p
        L.orc_count.argtypes = [P]
        L.orc_count.restype = C.c_int64
        L.orc_get.argtypes = [P] * 14
        L.orc_free.argtypes = [P]
        L.orc_pair_distance.argtypes = [C.c_int32, P, P, P]
        L.orc_case_distance.argtypes = [C.c_int32, P, P, P, P]
        L.orc_pair_barrier.argtypes = [C.c_int32, P, C.c_double, C.c_double, C.c_double,
                                       P, P, P, P, P, C.c_int32]
        L.orc_pair_barrier_code.argtypes = [C.c_int32, P, C.c_double, C.c_double, C.c_double, P, P, P, P, C.c_int32]
        L.orc_barrier_scalar.argtypes = [C.c_double, C.c_double, C.c_double, P, P, P]
        L.orc_psd_project.argtypes = [C.c_int32, P, P, P]
        L.orc_accd_pair.argtypes = [C.c_int32, P, P, C.c_double, C.c_double, C.c_int32, P, P]
        L.orc_max_step.argtypes = [C.POINTER(_Scene), P, P, C.c_double, C.c_int32, C.c_int32, C.c_int32]
        L.orc_max_step.restype = C.c_void_p
        L.orc_ms_count.argtypes = [P]
        L.orc_ms_count.restype = C.c_int64
        L.orc_ms_get.argtypes = [P] * 8
        L.orc_ms_free.argtypes = [P]
        L.orc_core_release.argtypes = [C.POINTER(_Scene), P, C.c_int64, P, P, P, P]
        L.orc_friction_lag.argtypes = [C.c_int32, P, C.c_double, C.c_double, C.c_double, C.c_double, P, P, P]
        L.orc_friction_pair.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, P, P, P, P]
        L.orc_friction_energy.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double]
        L.orc_friction_energy.restype = C.c_double
        L.orc_friction_batch.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, C.c_double, P, P, P, P, C.c_int32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _scene_struct(scene, filter_mode=0, eta=None, kappa=None, core=None, cull_radius=11):
    keep = []
    edges = np.ascontiguousarray(scene.edges, np.int32)
    tris = np.ascontiguousarray(scene.tris, np.int32)
    ref = np.ascontiguousarray(scene.ref, np.float64)
    keep += [edges, tris, ref]
    cp = ci = cj = None
    n_core = 0
    if core is not None and len(core[0]):
        cp, ci, cj = (np.ascontiguousarray(a, np.int32) for a in core)
        keep += [cp, ci, cj]
        n_core = len(cp)
    refdist = int(getattr(scene, "refdist", 0))
    xrest = None
    if refdist == 1:
        xrest = np.ascontiguousarray(scene.xrest, np.float64)
        assert xrest.shape == (scene.n_verts, 3), "the Euclidean reading needs the rest pose [V,3]"
        keep.append(xrest)
    s = _Scene(0 if scene.kind == "rod" else 1, scene.n_verts, scene.n_edges,
               scene.n_tris if scene.kind == "shell" else 0,
               _p(edges), _p(tris) if tris.size else None, _p(ref),
               float(scene.h), float(scene.eta if eta is None else eta),
               float(scene.kappa if kappa is None else kappa), int(filter_mode), n_core,
               _p(cp), _p(ci), _p(cj), int(cull_radius), refdist, _p(xrest))
    return s, keep


def precompute(scene, filter_mode=0):
    """Components (numbered by smallest vertex) and per-component d_min^2, d_min."""
    s, keep = _scene_struct(scene, filter_mode)
    comp = np.zeros(scene.n_verts, np.int32)
    cap = scene.n_verts
    dmin2 = np.zeros(cap, np.float64)
    dmin = np.zeros(cap, np.float64)
    nc = lib().orc_precompute(C.byref(s), _p(comp), _p(dmin2), _p(dmin), cap)
    return comp, dmin2[:nc].copy(), dmin[:nc].copy()


def evaluate(scene, x=None, mode=1, derivs=True, filter_mode=0, eta=None, kappa=None,
             nthreads=0, core=None, cull_radius=11):
    """Every pair of the universe with d < h, sorted by (ptype, i, j).

    Returns a dict of numpy arrays: ptype, i, j, verts[n,4], code, flags, d, a,
    eta, E, G[n,12], Hraw[n,12,12], Hpsd[n,12,12] (derivative arrays are zero
    for inactive pairs; E is +inf for infeasible active pairs).  core: the
    (ptype, i, j) arrays of pairs under the temporary zero offset (Sec. 3.4;
    pass the ones not released at x, see core_release).  filter_mode: 0 the
    paper's filter (Eq. 4), 1 none, 2 culling of edges of one polyline at most
    cull_radius elements apart (rods).
    """
    x = np.ascontiguousarray(scene.x if x is None else x, np.float64)
    s, keep = _scene_struct(scene, filter_mode, eta, kappa, core, cull_radius)
    L = lib()
    h = L.orc_evaluate(C.byref(s), _p(x), int(mode), int(bool(derivs)), int(nthreads))
    try:
        n = L.orc_count(h)
        out = dict(ptype=np.zeros(n, np.int32), i=np.zeros(n, np.int32), j=np.zeros(n, np.int32),
                   verts=np.zeros((n, 4), np.int32), code=np.zeros(n, np.int32),
                   flags=np.zeros(n, np.int32), d=np.zeros(n), a=np.zeros(n), eta=np.zeros(n),
                   E=np.zeros(n), G=np.zeros((n, 12)))
        if derivs:
            out["Hraw"] = np.zeros((n, 12, 12))
            out["Hpsd"] = np.zeros((n, 12, 12))
        L.orc_get(h, _p(out["ptype"]), _p(out["i"]), _p(out["j"]), _p(out["verts"]),
                  _p(out["code"]), _p(out["flags"]), _p(out["d"]), _p(out["a"]),
                  _p(out["eta"]), _p(out["E"]), _p(out["G"]),
                  _p(out.get("Hraw")), _p(out.get("Hpsd")))
    finally:
        L.orc_free(h)
    return out


def counts(res):
    f = res["flags"]
    return dict(n_c=int(f.size), n_filt=int(((f & F_FILTERED) != 0).sum()),
                n_act=int(((f & F_ACTIVE) != 0).sum()),
                n_infeasible=int(((f & F_INFEASIBLE) != 0).sum()))


def pair_distance(ptype, X):
    X = np.ascontiguousarray(X, np.float64).reshape(12)
    D = np.zeros(1)
    code = np.zeros(1, np.int32)
    lib().orc_pair_distance(int(ptype), _p(X), _p(D), _p(code))
    return float(D[0]), int(code[0])


def case_distance(code, X):
    """(D in double, D in binary128 as hi + lo doubles) for one sub-case formula."""
    X = np.ascontiguousarray(X, np.float64).reshape(12)
    o = np.zeros(3)
    lib().orc_case_distance(int(code), _p(X), _p(o[0:1]), _p(o[1:2]), _p(o[2:3]))
    return float(o[0]), float(o[1]), float(o[2])


def pair_barrier(ptype, X, a, eta, kappa=1.0, quad=False):
    X = np.ascontiguousarray(X, np.float64).reshape(12)
    E = np.zeros(1)
    G = np.zeros(12)
    Hraw = np.zeros((12, 12))
    Hpsd = np.zeros((12, 12))
    code = np.zeros(1, np.int32)
    lib().orc_pair_barrier(int(ptype), _p(X), float(a), float(eta), float(kappa),
                           _p(E), _p(G), _p(Hraw), _p(Hpsd), _p(code), int(bool(quad)))
    return dict(E=float(E[0]), G=G, Hraw=Hraw, Hpsd=Hpsd, code=int(code[0]))


def pair_barrier_code(code, X, a, eta, kappa=1.0, quad=False):
    """pair_barrier with the distance sub-case `code` given instead of
    classified (for pairs at a boundary between sub-cases of equal distance)."""
    X = np.ascontiguousarray(X, np.float64).reshape(12)
    E = np.zeros(1)
    G = np.zeros(12)
    Hraw = np.zeros((12, 12))
    Hpsd = np.zeros((12, 12))
    lib().orc_pair_barrier_code(int(code), _p(X), float(a), float(eta), float(kappa),
                                _p(E), _p(G), _p(Hraw), _p(Hpsd), int(bool(quad)))
    return dict(E=float(E[0]), G=G, Hraw=Hraw, Hpsd=Hpsd, code=int(code))


def barrier_scalar(d, a, eta):
    o = np.zeros(3)
    lib().orc_barrier_scalar(float(d), float(a), float(eta), _p(o[0:1]), _p(o[1:2]), _p(o[2:3]))
    return float(o[0]), float(o[1]), float(o[2])


def psd_project(A):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    Ap = np.zeros_like(A)
    ev = np.zeros(n)
    lib().orc_psd_project(int(n), _p(A), _p(Ap), _p(ev))
    return Ap, ev


def _stencil(res, k):
    """Global vertex ids of the four local slots of active pair(s) k."""
    return res["verts"][k]


def _block(H, r, c):
    """The 3x3 block (local slot r, local slot c) of 12x12 pair matrices (stacked)."""
    return H[..., 3 * r:3 * r + 3, 3 * c:3 * c + 3]


def assemble(res, n_verts, hess="Hpsd"):
    """Plain sums of the active pairs' results (row-major BSR with 3x3 blocks).

    Every active pair contributes its 12-vector to the gradient of its four
    stencil vertices, and all 16 3x3 blocks of its projected Hessian to the
    block pattern of its four stencil vertices.  Returns E, g[V,3] and the BSR
    arrays row_ptr[V+1], col[nnzb], val[nnzb,3,3] with columns sorted per row.
    hess names the per-pair matrices summed ("Hpsd"; "Hraw", the Hessians
    before projection, for the finite-difference pins of this function).
    The sums are numpy scatter-adds over (vertex) and (row vertex, column
    vertex) keys; the same values as pair-by-pair accumulation up to the
    order of the additions.
    """
    act = (res["flags"] & F_ACTIVE) != 0
    feas = act & ((res["flags"] & F_INFEASIBLE) == 0)
    E = float(np.sum(res["E"][act])) if act.any() else 0.0
    g = np.zeros((n_verts, 3))
    idx = np.nonzero(feas)[0]
    if not len(idx):
        return dict(E=E, g=g, row_ptr=np.zeros(n_verts + 1, np.int64), col=np.zeros(0, np.int32),
                    val=np.zeros((0, 3, 3)))
    vs = np.asarray(_stencil(res, idx)).astype(np.int64)  # [n, 4]
    G = res["G"][idx].reshape(-1, 4, 3)
    H = res[hess][idx]
    rows, cols, blks = [], [], []
    for r in range(4):
        np.add.at(g, vs[:, r], G[:, r])
        for c in range(4):
            rows.append(vs[:, r])
            cols.append(vs[:, c])
            blks.append(_block(H, r, c))
    # pair-major order: every key (and its transpose) receives its pairs'
    # blocks in pair order, so the sums are bitwise symmetric
    key = (np.stack(rows, 1) * n_verts + np.stack(cols, 1)).reshape(-1)
    uk, inv = np.unique(key, return_inverse=True)
    val = np.zeros((len(uk), 3, 3))
    np.add.at(val, inv, np.stack(blks, 1).reshape(-1, 3, 3))
    row = uk // n_verts
    row_ptr = np.zeros(n_verts + 1, np.int64)
    np.add.at(row_ptr, row + 1, 1)
    return dict(E=E, g=g, row_ptr=np.cumsum(row_ptr), col=(uk % n_verts).astype(np.int32), val=val)


# ---- line search (Sec. 3.3, last paragraph; App. A) --------------------------

def energy(scene, x, filter_mode=0, eta=None, kappa=None, nthreads=0):
    """Energy-only evaluation at positions x: the sum of the filtered barrier
    over the active pairs (+inf if any active pair is at or inside its
    offset), in the order of the sorted pair list."""
    res = evaluate(scene, x, mode=1, derivs=False, filter_mode=filter_mode, eta=eta, kappa=kappa,
                   nthreads=nthreads)
    act = (res["flags"] & F_ACTIVE) != 0
    return float(np.sum(res["E"][act])) if act.any() else 0.0, res


def accd_pair(ptype, X, P, xi, s=0.1, max_iter=65536):
    """Additive CCD of one pair (4 local vertices X, displacements P, offset
    xi): (t, iterations)."""
    X = np.ascontiguousarray(X, np.float64).reshape(12)
    P = np.ascontiguousarray(P, np.float64).reshape(12)
    t = np.zeros(1)
    it = np.zeros(1, np.int32)
    lib().orc_accd_pair(int(ptype), _p(X), _p(P), float(xi), float(s), int(max_iter), _p(t), _p(it))
    return float(t[0]), int(it[0])


def max_step(scene, x, p, s=0.1, max_iter=65536, mode=1, filter_mode=0, eta=None, nthreads=0, core=None):
    """ACCD over the pairs whose boxes swept from x to x + p are within h,
    each with its filtered offset (eta, or 0 for filtered stencils and for
    the pairs of the core set, Sec. 3.4).

    Returns dict(t=min step (1 if no pair), ptype, i, j, filtered, iters, xi,
    tpair) with the pairs sorted by (ptype, i, j)."""
    x = np.ascontiguousarray(x, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    sc, keep = _scene_struct(scene, filter_mode, eta, core=core)
    L = lib()
    h = L.orc_max_step(C.byref(sc), _p(x), _p(p), float(s), int(max_iter), int(mode), int(nthreads))
    try:
        n = L.orc_ms_count(h)
        out = dict(ptype=np.zeros(n, np.int32), i=np.zeros(n, np.int32), j=np.zeros(n, np.int32),
                   filtered=np.zeros(n, np.int32), iters=np.zeros(n, np.int32), xi=np.zeros(n),
                   tpair=np.zeros(n))
        L.orc_ms_get(h, _p(out["ptype"]), _p(out["i"]), _p(out["j"]), _p(out["filtered"]),
                     _p(out["iters"]), _p(out["xi"]), _p(out["tpair"]))
    finally:
        L.orc_ms_free(h)
    out["t"] = float(out["tpair"].min()) if n else 1.0
    return out


# ---- temporary zero offset (Sec. 3.4) -----------------------------------------

def core_mark(scene, x, filter_mode=0, nthreads=0):
    """Non-stencil pairs inside the core at x (d < h and d <= eta, not
    filtered), as sorted (ptype, i, j) arrays."""
    res = evaluate(scene, x, mode=1, derivs=False, filter_mode=filter_mode, nthreads=nthreads)
    sel = ((res["flags"] & F_INFEASIBLE) != 0) & ((res["flags"] & F_FILTERED) == 0)
    return res["ptype"][sel].copy(), res["i"][sel].copy(), res["j"][sel].copy()


def core_release(scene, x, core, filter_mode=0):
    """Boolean mask over the core pairs: True where the pair is at d > eta at x."""
    x = np.ascontiguousarray(x, np.float64)
    cp, ci, cj = (np.ascontiguousarray(a, np.int32) for a in core)
    s, keep = _scene_struct(scene, filter_mode)
    out = np.zeros(len(cp), np.int32)
    lib().orc_core_release(C.byref(s), _p(x), len(cp), _p(cp), _p(ci), _p(cj), _p(out))
    return out.astype(bool)


# ---- lagged friction (App. A: IPC contact and friction energies) -----------------

def _local(x, verts):
    return np.ascontiguousarray(np.asarray(x, np.float64)[np.asarray(verts)].reshape(12))


def friction_lag(scene, xlag, filter_mode=0, core=None, kappa=None):
    """Lagged friction data of the active pairs at xlag (sorted by (ptype, i,
    j)): lam (kappa |b'(d)|, 0 for infeasible pairs), closest-point weights
    w[n,4] and contact normals n[n,3]; plus the pairs' ptype, i, j, verts."""
    res = evaluate(scene, xlag, mode=1, derivs=False, filter_mode=filter_mode, core=core, kappa=kappa)
    act = (res["flags"] & F_ACTIVE) != 0
    idx = np.nonzero(act)[0]
    kap = float(scene.kappa if kappa is None else kappa)
    lam = np.zeros(len(idx))
    w = np.zeros((len(idx), 4))
    nrm = np.zeros((len(idx), 3))
    L = lib()
    for q, k in enumerate(idx):
        X = _local(xlag, res["verts"][k])
        lo, wo, no = np.zeros(1), np.zeros(4), np.zeros(3)
        L.orc_friction_lag(int(res["code"][k]), _p(X), float(res["d"][k]), float(res["a"][k]),
                           float(res["eta"][k]), kap, _p(lo), _p(wo), _p(no))
        lam[q], w[q], nrm[q] = lo[0], wo, no
    return dict(ptype=res["ptype"][idx], i=res["i"][idx], j=res["j"][idx], verts=res["verts"][idx],
                code=res["code"][idx], lam=lam, w=w, n=nrm)


def friction_eval(lag, x, xlag, mu, eh, derivs=True, nthreads=0):
    """Friction energy (and gradient, Hessian) of every lagged pair at x."""
    n = len(lag["lam"])
    E = np.zeros(n)
    G = np.zeros((n, 12))
    H = np.zeros((n, 12, 12))
    Hp = np.zeros((n, 12, 12))
    L = lib()
    if derivs:
        vt = np.asarray(lag["verts"])
        X = np.ascontiguousarray(np.asarray(x, np.float64)[vt].reshape(n, 12))
        Xl = np.ascontiguousarray(np.asarray(xlag, np.float64)[vt].reshape(n, 12))
        w = np.ascontiguousarray(lag["w"], np.float64)
        nn = np.ascontiguousarray(lag["n"], np.float64)
        lam = np.ascontiguousarray(lag["lam"], np.float64)
        L.orc_friction_batch(n, _p(X), _p(Xl), _p(w), _p(nn), _p(lam), float(mu), float(eh), _p(E), _p(G), _p(H),
                             _p(Hp), int(nthreads))
        return dict(E=E, G=G, H=H, Hpsd=Hp)
    for q in range(n):
        X = _local(x, lag["verts"][q])
        Xl = _local(xlag, lag["verts"][q])
        w = np.ascontiguousarray(lag["w"][q])
        nn = np.ascontiguousarray(lag["n"][q])
        if derivs:
            e = np.zeros(1)
            g = np.zeros(12)
            h = np.zeros((12, 12))
            hp = np.zeros((12, 12))
            L.orc_friction_pair(_p(X), _p(Xl), _p(w), _p(nn), float(lag["lam"][q]), float(mu), float(eh),
                                _p(e), _p(g), _p(h), _p(hp))
            E[q], G[q], H[q], Hp[q] = e[0], g, h, hp
        else:
            E[q] = L.orc_friction_energy(_p(X), _p(Xl), _p(w), _p(nn), float(lag["lam"][q]), float(mu), float(eh))
    return dict(E=E, G=G, H=H, Hpsd=Hp)
