"""ctypes binding of libbfc (argument marshalling only).

Every step of the contact path runs in the library's HIP kernels; this module
allocates the caller-owned device buffers as torch tensors, passes their
pointers and the current HIP stream, and reads results back on request.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libbfc.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("bfc_kernels.hip", "bfc_api.hip", "bfc_serve.hip")]

BF_OK = 0
BF_ROD, BF_SHELL = 0, 1
BF_FP64, BF_MIXED = 0, 1
BF_FILTER_PAPER, BF_FILTER_NONE, BF_FILTER_CULL = 0, 1, 2
BF_REFDIST_PARAM, BF_REFDIST_EUCLID_REST = 0, 1
BF_S_CAND_OVERFLOW, BF_S_ACT_OVERFLOW, BF_S_INFEASIBLE = 1, 2, 4
BF_S_BSR_OVERFLOW, BF_S_CORE_OVERFLOW = 8, 16
BF_S_EIG_NOCONV, BF_S_SCAN_SLOW, BF_S_EXACT_LIMIT = 32, 64, 128
BF_F_FILTERED, BF_F_INFEASIBLE, BF_F_CORE = 1, 4, 8

EXPORTED = ["bf_scene_create", "bf_workspace_bytes", "bf_scene_create_ws", "bf_scene_reserve", "bf_scene_destroy",
            "bf_scene_info", "build_candidates", "filter_pairs", "eval_barrier", "assemble_grad_hess",
            "bf_scene_set_pq", "bf_scene_tune", "bf_batch_create", "bf_batch_step", "bf_batch_info",
            "bf_batch_destroy", "build_candidates_swept", "max_step_accd", "eval_energy", "bf_core_mark",
            "bf_core_live", "bf_core_clear", "friction_lag", "friction_eval", "friction_assemble", "bf_status_word",
            "bf_set_scan_poll_limit", "bf_scene_set_timing", "bf_scene_stage_ms", "eval_energy_noalloc",
            "bf_scene_deferred", "bf_serve_start", "bf_serve_submit", "bf_serve_poll", "bf_serve_info",
            "bf_serve_stop", "bf_last_error"]


def build(verbose: bool = False) -> str:
    """Compile libbfc.so for gfx950 with hipcc (in-tree)."""
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(_ROOT, "include"), *SOURCES, "-o", LIB_PATH + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _packed_index():
    """Packed position of every entry (I, J) of a pair's 12 x 12 Hessian: the
    upper triangle by 3 x 3 blocks, block-row s = block (s, s) as its upper
    triangle, then blocks (s, t > s) row-major; block-rows at 0, 33, 57, 72."""
    off = [0, 33, 57, 72]
    idx = np.zeros((12, 12), np.int64)
    for I in range(12):
        for J in range(12):
            a, b = min(I, J), max(I, J)
            s, i, t, j = a // 3, a % 3, b // 3, b % 3
            idx[I, J] = off[s] + ([j, 2 + j, 5][i] if s == t else 6 + 9 * (t - s - 1) + 3 * i + j)
    return idx


PACKED_INDEX = _packed_index()


def unpack_hessians(Hp):
    """[n, 78] packed upper triangles (FP64, or FP32 from a mixed-precision
    scene) -> [n, 12, 12] symmetric FP64 matrices."""
    return np.asarray(Hp, np.float64)[:, PACKED_INDEX]


class Params(C.Structure):
    _fields_ = [("h", C.c_double), ("eta", C.c_double), ("kappa", C.c_double),
                ("prec", C.c_int32), ("filter", C.c_int32), ("cull_radius", C.c_int32), ("refdist", C.c_int32)]


class MeshDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_verts", C.c_int64), ("n_edges", C.c_int64), ("n_tris", C.c_int64),
                ("edges_h", C.c_void_p), ("tris_h", C.c_void_p), ("ref_h", C.c_void_p), ("ref_pos_h", C.c_void_p)]


class ServeConfig(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("meshes", C.c_void_p), ("params", C.c_void_p), ("cand_cap", C.c_void_p),
                ("act_cap", C.c_void_p), ("bsr_cap", C.c_void_p), ("budget_bytes", C.c_int64), ("slots", C.c_int32),
                ("max_bypass", C.c_int32), ("device", C.c_int32)]


class ServeResult(C.Structure):
    _fields_ = [("done", C.c_int32), ("scene", C.c_int32), ("error", C.c_int32), ("status", C.c_uint32),
                ("E", C.c_double), ("counts", C.c_int64 * 5), ("n_bp", C.c_int64), ("ms", C.c_double),
                ("retries", C.c_int32)]


class Pairs(C.Structure):
    _fields_ = [("i_d", C.c_void_p), ("j_d", C.c_void_p), ("type_d", C.c_void_p), ("cap", C.c_int64),
                ("count_d", C.c_void_p)]


class Active(C.Structure):
    _fields_ = [("p", Pairs), ("code_d", C.c_void_p), ("flags_d", C.c_void_p), ("dist_d", C.c_void_p),
                ("counters_d", C.c_void_p)]


class Local(C.Structure):
    _fields_ = [("E_d", C.c_void_p), ("G_d", C.c_void_p), ("H_d", C.c_void_p), ("cap", C.c_int64)]


class Bsr(C.Structure):
    _fields_ = [("row_ptr_d", C.c_void_p), ("col_d", C.c_void_p), ("val_d", C.c_void_p), ("cap", C.c_int64),
                ("nnzb_d", C.c_void_p)]


class Friction(C.Structure):
    _fields_ = [("lam_d", C.c_void_p), ("w_d", C.c_void_p), ("n_d", C.c_void_p), ("cap", C.c_int64)]


class BatchItem(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("x_d", C.c_void_p), ("cand", Pairs), ("act", Active), ("loc", Local),
                ("E_d", C.c_void_p), ("g_d", C.c_void_p), ("H", Bsr)]


_lib = None


def lib():
    """Load libbfc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.bf_scene_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(Params), C.c_int64, C.c_int64, P,
                                      C.POINTER(P)]
        L.bf_workspace_bytes.argtypes = [C.POINTER(MeshDesc), C.POINTER(Params), C.c_int64, C.c_int64,
                                         C.POINTER(C.c_int64)]
        L.bf_scene_create_ws.argtypes = [C.POINTER(MeshDesc), C.POINTER(Params), C.c_int64, C.c_int64, P,
                                         C.c_int64, P, C.POINTER(P)]
        L.bf_serve_start.argtypes = [C.POINTER(ServeConfig), C.POINTER(P)]
        L.bf_serve_submit.argtypes = [P, C.c_int32, P, P, C.POINTER(C.c_int64)]
        L.bf_serve_poll.argtypes = [P, C.c_int64, C.c_int32, C.POINTER(ServeResult)]
        L.bf_serve_info.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), P, P]
        L.bf_serve_stop.argtypes = [P]
        L.bf_scene_reserve.argtypes = [P, C.c_int64, C.c_int64]
        L.bf_scene_destroy.argtypes = [P]
        L.bf_scene_info.argtypes = [P, P, P, P, P, C.c_int32]
        L.build_candidates.argtypes = [P, P, C.POINTER(Pairs), P]
        L.filter_pairs.argtypes = [P, P, C.POINTER(Pairs), C.POINTER(Active), P]
        L.eval_barrier.argtypes = [P, P, C.POINTER(Active), C.POINTER(Local), P]
        L.assemble_grad_hess.argtypes = [P, C.POINTER(Active), C.POINTER(Local), P, P, C.POINTER(Bsr), P]
        L.bf_scene_set_pq.argtypes = [P, C.c_int32]
        L.bf_scene_tune.argtypes = [P, P, C.POINTER(Pairs), C.c_int32, P, C.POINTER(C.c_int32)]
        L.bf_batch_create.argtypes = [C.POINTER(BatchItem), C.c_int32, C.c_int32, P, C.POINTER(P)]
        L.bf_batch_step.argtypes = [P, P]
        L.bf_batch_info.argtypes = [P, C.POINTER(C.c_int32), P]
        L.bf_batch_destroy.argtypes = [P]
        L.build_candidates_swept.argtypes = [P, P, P, C.POINTER(Pairs), P]
        L.max_step_accd.argtypes = [P, P, P, C.POINTER(Pairs), C.c_double, C.c_int32, P, P, P, P]
        L.eval_energy.argtypes = [P, P, P, P, C.POINTER(Pairs), P, P]
        L.eval_energy_noalloc.argtypes = [P, P, P, P, C.POINTER(Pairs), P, P]
        L.bf_core_mark.argtypes = [P, P, C.POINTER(Pairs), C.c_int64, P, P]
        L.bf_core_live.argtypes = [P, P, P]
        L.bf_core_clear.argtypes = [P]
        L.friction_lag.argtypes = [P, P, C.POINTER(Active), C.POINTER(Friction), P]
        L.friction_eval.argtypes = [P, P, P, C.POINTER(Active), C.POINTER(Friction), C.c_double, C.c_double,
                                    C.c_int32, C.POINTER(Local), P]
        L.friction_assemble.argtypes = [P, C.POINTER(Active), C.POINTER(Local), P, P, C.POINTER(Bsr), P]
        L.bf_status_word.argtypes = [P, C.POINTER(C.c_uint32), C.c_int32]
        L.bf_set_scan_poll_limit.argtypes = [C.c_int32]
        L.bf_scene_set_timing.argtypes = [P, C.c_int32]
        L.bf_scene_stage_ms.argtypes = [P, P]
        L.bf_scene_deferred.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.bf_last_error.restype = C.c_char_p
        for name in EXPORTED[:-1]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, what):
    if rc != BF_OK:
        raise RuntimeError(f"{what} failed ({rc}): {lib().bf_last_error().decode()}")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class ContactScene:
    """One mesh resident on the GPU plus the caller-owned buffers of a step.

    ``step(x)`` enqueues build_candidates -> filter_pairs -> eval_barrier ->
    assemble_grad_hess on the current torch stream.  Capacities start from
    size estimates and grow when the device reports an overflow (``run``
    retries the step; ``step`` never synchronises).
    """

    def __init__(self, scene, prec=BF_FP64, filter_mode=BF_FILTER_PAPER, kappa=None, eta=None, cull_radius=11,
                 cand_cap=None, act_cap=None, bsr_cap=None, device="cuda", own_workspace=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.kind = BF_ROD if scene.kind == "rod" else BF_SHELL
        self.nv, self.ne = scene.n_verts, scene.n_edges
        self.nt = scene.n_tris if self.kind == BF_SHELL else 0
        self.h = float(scene.h)
        self.eta = float(scene.eta if eta is None else eta)
        self.kappa = float(scene.kappa if kappa is None else kappa)
        nprims = self.ne + self.nt + (self.nv if self.kind == BF_SHELL else 0)
        self.cand_cap = int(cand_cap or max(4096, 40 * nprims))
        self.act_cap = int(act_cap or max(4096, 4 * nprims))
        self.bsr_cap = int(bsr_cap or max(4096, 8 * self.act_cap))
        self._edges = np.ascontiguousarray(scene.edges, np.int32)
        self._tris = np.ascontiguousarray(scene.tris, np.int32) if self.nt else None
        self._ref = np.ascontiguousarray(scene.ref, np.float64)
        # reference distance: the scene's reading (rest parameters, or the
        # Euclidean distance at its rest pose xrest)
        self.refdist = int(getattr(scene, "refdist", BF_REFDIST_PARAM))
        self._xrest = (np.ascontiguousarray(scene.xrest, np.float64) if self.refdist == BF_REFDIST_EUCLID_REST
                       else None)
        desc = MeshDesc(self.kind, self.nv, self.ne, self.nt, self._edges.ctypes.data,
                        self._tris.ctypes.data if self.nt else None, self._ref.ctypes.data,
                        self._xrest.ctypes.data if self._xrest is not None else None)
        prm = Params(self.h, self.eta, self.kappa, int(prec), int(filter_mode), int(cull_radius), self.refdist)
        self.prec, self.filter_mode = int(prec), int(filter_mode)
        h = C.c_void_p()
        self.workspace = None
        if own_workspace:
            # the scene's memory in a tensor of ours (bf_workspace_bytes / bf_scene_create_ws)
            nb = C.c_int64(0)
            _check(lib().bf_workspace_bytes(C.byref(desc), C.byref(prm), self.cand_cap, self.act_cap,
                                            C.byref(nb)), "bf_workspace_bytes")
            self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
            _check(lib().bf_scene_create_ws(C.byref(desc), C.byref(prm), self.cand_cap, self.act_cap,
                                            self.workspace.data_ptr(), int(nb.value), C.c_void_p(self._stream()),
                                            C.byref(h)), "bf_scene_create_ws")
        else:
            _check(lib().bf_scene_create(C.byref(desc), C.byref(prm), self.cand_cap, self.act_cap,
                                         C.c_void_p(self._stream()), C.byref(h)), "bf_scene_create")
        self.handle = h
        self.pq = 4
        self._gen = 0       # filter_pairs calls so far (the lagged friction list is tied to one)
        self._fgen = -1
        self._alloc()

    # -- buffers -------------------------------------------------------------
    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _alloc(self):
        t, dev = self.torch, self.device
        z = lambda n, dt: t.zeros(n, dtype=dt, device=dev)
        self.c_i, self.c_j, self.c_t = z(self.cand_cap, t.int32), z(self.cand_cap, t.int32), z(self.cand_cap, t.uint8)
        self.c_n = z(1, t.int64)
        self.a_i, self.a_j, self.a_t = z(self.act_cap, t.int32), z(self.act_cap, t.int32), z(self.act_cap, t.uint8)
        self.a_n = z(1, t.int64)
        self.a_code, self.a_flags = z(self.act_cap, t.uint8), z(self.act_cap, t.uint8)
        self.a_dist = z(self.act_cap, t.float64)
        self.counters = z(4, t.int64)
        # Hessian records in the scene's precision (FP32 for BF_MIXED)
        self.h_dtype = t.float32 if self.prec == BF_MIXED else t.float64
        self.l_E, self.l_G, self.l_H = z(self.act_cap, t.float64), z((self.act_cap, 12), t.float64), \
            z((self.act_cap, 78), self.h_dtype)
        self.E = z(1, t.float64)
        self.g = z((self.nv, 3), t.float64)
        self.row_ptr = z(self.nv + 1, t.int32)
        self.col = z(self.bsr_cap, t.int32)
        self.val = z((self.bsr_cap, 9), t.float64)
        self.nnzb = z(1, t.int64)
        self._cand = Pairs(self.c_i.data_ptr(), self.c_j.data_ptr(), self.c_t.data_ptr(), self.cand_cap,
                           self.c_n.data_ptr())
        self._act = Active(Pairs(self.a_i.data_ptr(), self.a_j.data_ptr(), self.a_t.data_ptr(), self.act_cap,
                                 self.a_n.data_ptr()),
                           self.a_code.data_ptr(), self.a_flags.data_ptr(), self.a_dist.data_ptr(),
                           self.counters.data_ptr())
        self._loc = Local(self.l_E.data_ptr(), self.l_G.data_ptr(), self.l_H.data_ptr(), self.act_cap)
        self._bsr = Bsr(self.row_ptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr(), self.bsr_cap,
                        self.nnzb.data_ptr())

    # -- the four calls -------------------------------------------------------
    def build_candidates(self, x):
        _check(lib().build_candidates(self.handle, _ptr(x), C.byref(self._cand), C.c_void_p(self._stream())),
               "build_candidates")

    def filter_pairs(self, x):
        self._gen += 1
        _check(lib().filter_pairs(self.handle, _ptr(x), C.byref(self._cand), C.byref(self._act),
                                  C.c_void_p(self._stream())), "filter_pairs")

    def eval_barrier(self, x):
        _check(lib().eval_barrier(self.handle, _ptr(x), C.byref(self._act), C.byref(self._loc),
                                  C.c_void_p(self._stream())), "eval_barrier")

    def assemble_grad_hess(self):
        _check(lib().assemble_grad_hess(self.handle, C.byref(self._act), C.byref(self._loc), _ptr(self.E),
                                        _ptr(self.g), C.byref(self._bsr), C.c_void_p(self._stream())),
               "assemble_grad_hess")

    def step(self, x):
        """Enqueue one pass of the whole path on the current stream (no sync)."""
        self.build_candidates(x)
        self.filter_pairs(x)
        self.eval_barrier(x)
        self.assemble_grad_hess()

    # -- line search -----------------------------------------------------------
    def build_candidates_swept(self, x, p):
        """Candidates for the whole segment x -> x + p (enqueued, no sync)."""
        _check(lib().build_candidates_swept(self.handle, _ptr(x), _ptr(p), C.byref(self._cand),
                                            C.c_void_p(self._stream())), "build_candidates_swept")

    def fit_swept(self, x, p, max_tries=4):
        """Grow the candidate capacity until the swept list of (x, p) fits
        (synchronises); returns its length."""
        for _ in range(max_tries):
            self.build_candidates_swept(x, p)
            self.torch.cuda.synchronize(self.device)
            n = int(self.c_n.item())
            if n <= self.cand_cap:
                return n
            self.cand_cap = n + n // 4 + 1024
            _check(lib().bf_scene_reserve(self.handle, self.cand_cap, self.act_cap), "bf_scene_reserve")
            self._alloc()
        raise RuntimeError("swept candidate list kept overflowing")

    def max_step(self, x, p, accd_s=0.1, max_iter=65536, per_pair=False, out=None):
        """Additive CCD step over the swept candidates (run build_candidates_swept
        first).  Returns a device tensor t[1]; with per_pair also the steps of
        the candidates (-1 outside the swept set) and their step counts."""
        t = out if out is not None else self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        tp = it = None
        if per_pair:
            tp = self.torch.zeros(self.cand_cap, dtype=self.torch.float64, device=self.device)
            it = self.torch.zeros(self.cand_cap, dtype=self.torch.int32, device=self.device)
        _check(lib().max_step_accd(self.handle, _ptr(x), _ptr(p), C.byref(self._cand), float(accd_s),
                                   int(max_iter), _ptr(t), _ptr(tp) if per_pair else None,
                                   _ptr(it) if per_pair else None, C.c_void_p(self._stream())), "max_step_accd")
        return (t, tp, it) if per_pair else t

    def eval_energy(self, x, p=None, alpha=None, out=None):
        """Energy alone at x (or at x + alpha p, alpha a device tensor [1]) over
        the current candidates; a device tensor E[1]."""
        E = out if out is not None else self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        _check(lib().eval_energy(self.handle, _ptr(x), _ptr(p) if p is not None else None,
                                 _ptr(alpha) if alpha is not None else None, C.byref(self._cand), _ptr(E),
                                 C.c_void_p(self._stream())), "eval_energy")
        return E

    def eval_energy_noalloc(self, x, p=None, alpha=None, out=None):
        """eval_energy through the allocation-free entry point (its partial
        sums in the library's static device array)."""
        E = out if out is not None else self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        _check(lib().eval_energy_noalloc(self.handle, _ptr(x), _ptr(p) if p is not None else None,
                                         _ptr(alpha) if alpha is not None else None, C.byref(self._cand), _ptr(E),
                                         C.c_void_p(self._stream())), "eval_energy_noalloc")
        return E

    # -- lagged friction (App. A: IPC contact and friction energies) ----------
    def friction_lag(self, xlag):
        """Lagged friction data at xlag for the active list of the last
        filter_pairs (run the step at xlag first).  The lagged list is copied
        into buffers of its own: later steps replace the contact list, the
        friction keeps its pairs until the next friction_lag."""
        t = self.torch
        cap = self.act_cap
        z = lambda shape, dt=t.float64: t.zeros(shape, dtype=dt, device=self.device)
        self.f_i, self.f_j, self.f_t = self.a_i.clone(), self.a_j.clone(), self.a_t.clone()
        self.f_cnt, self.f_code, self.f_flags = self.a_n.clone(), self.a_code.clone(), self.a_flags.clone()
        self.f_dist, self.f_counters = self.a_dist.clone(), self.counters.clone()
        self._fact = Active(Pairs(self.f_i.data_ptr(), self.f_j.data_ptr(), self.f_t.data_ptr(), cap,
                                  self.f_cnt.data_ptr()),
                            self.f_code.data_ptr(), self.f_flags.data_ptr(), self.f_dist.data_ptr(),
                            self.f_counters.data_ptr())
        self.f_lam, self.f_w, self.f_n = z(cap), z((cap, 4)), z((cap, 3))
        self._fr = Friction(self.f_lam.data_ptr(), self.f_w.data_ptr(), self.f_n.data_ptr(), cap)
        self.fl_E, self.fl_G, self.fl_H = z(cap), z((cap, 12)), z((cap, 78), self.h_dtype)
        self._floc = Local(self.fl_E.data_ptr(), self.fl_G.data_ptr(), self.fl_H.data_ptr(), cap)
        self.f_E, self.f_g = z(1), z((self.nv, 3))
        self.f_row_ptr, self.f_col = z(self.nv + 1, t.int32), z(self.bsr_cap, t.int32)
        self.f_val, self.f_nnzb = z((self.bsr_cap, 9)), z(1, t.int64)
        self._fbsr = Bsr(self.f_row_ptr.data_ptr(), self.f_col.data_ptr(), self.f_val.data_ptr(), self.bsr_cap,
                         self.f_nnzb.data_ptr())
        self._xlag = xlag
        self._fgen = self._gen
        _check(lib().friction_lag(self.handle, _ptr(xlag), C.byref(self._fact), C.byref(self._fr),
                                  C.c_void_p(self._stream())), "friction_lag")

    def friction_eval(self, x, mu, eps_vh, accumulate=False):
        """Friction of the lagged pairs at x into their own local buffers
        (fl_E, fl_G, fl_H).  accumulate=True adds it onto the contact terms
        instead (l_E, l_G, l_H), which is only meaningful while the contact
        list is still the lagged one (no filter_pairs since friction_lag)."""
        if accumulate and self._gen != self._fgen:
            raise RuntimeError("friction_eval(accumulate=True): the contact list changed since friction_lag")
        loc = self._loc if accumulate else self._floc
        _check(lib().friction_eval(self.handle, _ptr(x), _ptr(self._xlag), C.byref(self._fact), C.byref(self._fr),
                                   float(mu), float(eps_vh), int(bool(accumulate)), C.byref(loc),
                                   C.c_void_p(self._stream())), "friction_eval")

    def friction_assemble(self):
        """Assemble the friction terms of the last friction_eval over the lagged
        list into f_E, f_g and the block matrix (f_row_ptr, f_col, f_val)."""
        _check(lib().friction_assemble(self.handle, C.byref(self._fact), C.byref(self._floc), _ptr(self.f_E),
                                       _ptr(self.f_g), C.byref(self._fbsr), C.c_void_p(self._stream())),
               "friction_assemble")

    def friction_results(self):
        """Host copies of the lagged list, its friction data and the last
        friction evaluation and assembly (synchronises)."""
        self.torch.cuda.synchronize(self.device)
        n = min(int(self.f_cnt.item()), self.act_cap)
        nb = min(int(self.f_nnzb.item()), self.bsr_cap)
        c = lambda a: a[:n].cpu().numpy()
        return dict(ptype=c(self.f_t).astype(np.int32), i=c(self.f_i), j=c(self.f_j), lam=c(self.f_lam),
                    w=c(self.f_w), n=c(self.f_n), E=c(self.fl_E), G=c(self.fl_G),
                    Hpsd=unpack_hessians(c(self.fl_H)), E_total=float(self.f_E.item()), g=self.f_g.cpu().numpy(),
                    row_ptr=self.f_row_ptr.cpu().numpy().astype(np.int64), col=self.f_col[:nb].cpu().numpy(),
                    val=self.f_val[:nb].cpu().numpy().reshape(-1, 3, 3), nnzb=int(self.f_nnzb.item()))

    # -- temporary zero offset (Sec. 3.4) ------------------------------------
    def core_mark(self, x, cap=None):
        """Mark the non-stencil pairs inside the core at x (uses the current
        candidates: call build_candidates(x) first).  Returns a device int64[1]
        count."""
        cnt = self.torch.zeros(1, dtype=self.torch.int64, device=self.device)
        _check(lib().bf_core_mark(self.handle, _ptr(x), C.byref(self._cand), int(cap or max(64, self.act_cap)),
                                  _ptr(cnt), C.c_void_p(self._stream())), "bf_core_mark")
        return cnt

    def core_live(self):
        cnt = self.torch.zeros(1, dtype=self.torch.int64, device=self.device)
        _check(lib().bf_core_live(self.handle, _ptr(cnt), C.c_void_p(self._stream())), "bf_core_live")
        return cnt

    def core_clear(self):
        _check(lib().bf_core_clear(self.handle), "bf_core_clear")

    def set_pq(self, pq):
        """Threads per broad-phase query (2, 4, 8 or 16)."""
        _check(lib().bf_scene_set_pq(self.handle, int(pq)), "bf_scene_set_pq")
        self.pq = int(pq)

    def tune(self, x, reps=5):
        """Time build_candidates with 2, 4, 8 and 16 threads per query on x and
        keep the fastest (synchronises)."""
        x = self._as_x(x)
        pq = C.c_int32(0)
        _check(lib().bf_scene_tune(self.handle, _ptr(x), C.byref(self._cand), int(reps),
                                   C.c_void_p(self._stream()), C.byref(pq)), "bf_scene_tune")
        self.pq = int(pq.value)
        return self.pq

    def batch_item(self, x):
        """The C-ABI batch item of this scene with positions tensor x (kept
        alive by the caller; a batch reads it at every step)."""
        return BatchItem(self.handle, x.data_ptr(), self._cand, self._act, self._loc, self.E.data_ptr(),
                         self.g.data_ptr(), self._bsr)

    STAGES = ("broad", "narrow", "compact", "eval", "asm_structure", "asm_values")

    def set_timing(self, on=True):
        """Per-stage HIP events around the kernels of each call (eager launches)."""
        _check(lib().bf_scene_set_timing(self.handle, int(bool(on))), "bf_scene_set_timing")

    def stage_ms(self):
        """Durations (ms) of each stage's latest call (synchronises)."""
        ms = np.zeros(len(self.STAGES), np.float32)
        _check(lib().bf_scene_stage_ms(self.handle, ms.ctypes.data), "bf_scene_stage_ms")
        return {k: float(v) for k, v in zip(self.STAGES, ms)}

    def deferred(self):
        """(candidates of the last filter_pairs with a value in FP64's band
        around a threshold, those of them decided in exact arithmetic)."""
        nb, ne = C.c_int64(0), C.c_int64(0)
        _check(lib().bf_scene_deferred(self.handle, C.byref(nb), C.byref(ne)), "bf_scene_deferred")
        return int(nb.value), int(ne.value)

    def status(self, clear=True):
        v = C.c_uint32(0)
        _check(lib().bf_status_word(self.handle, C.byref(v), int(clear)), "bf_status_word")
        return int(v.value)

    def run(self, x, max_tries=4):
        """Step, then grow any overflowing buffer and step again (synchronises)."""
        x = self._as_x(x)
        for _ in range(max_tries):
            self.step(x)
            st = self.status(clear=True)
            over = st & (BF_S_CAND_OVERFLOW | BF_S_ACT_OVERFLOW | BF_S_BSR_OVERFLOW)
            if not over:
                return st
            nc, na, nb = int(self.c_n.item()), int(self.a_n.item()), int(self.nnzb.item())
            grow = False
            if nc > self.cand_cap:
                self.cand_cap = nc + nc // 4 + 1024
                grow = True
            if na > self.act_cap:
                self.act_cap = na + na // 4 + 1024
                grow = True
            if nb > self.bsr_cap or (st & BF_S_ACT_OVERFLOW):
                self.bsr_cap = max(nb + nb // 4 + 1024, 8 * self.act_cap)
                grow = True
            if grow:
                _check(lib().bf_scene_reserve(self.handle, self.cand_cap, self.act_cap), "bf_scene_reserve")
                self._alloc()
        raise RuntimeError("buffers kept overflowing")

    def _as_x(self, x):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.ascontiguousarray(x, np.float64))
        x = x.to(device=self.device, dtype=t.float64).contiguous()
        assert x.shape == (self.nv, 3)
        return x

    # -- results ----------------------------------------------------------------
    def info(self):
        comp = np.zeros(self.nv, np.int32)
        nc = C.c_int32(0)
        _check(lib().bf_scene_info(self.handle, comp.ctypes.data, C.byref(nc), None, None, 0), "bf_scene_info")
        d2 = np.zeros(nc.value)
        d = np.zeros(nc.value)
        _check(lib().bf_scene_info(self.handle, None, None, d2.ctypes.data, d.ctypes.data, nc.value),
               "bf_scene_info")
        return comp, d2, d

    def counts(self):
        c = self.counters.cpu().numpy()
        return dict(n_bp=int(self.c_n.item()), n_c=int(c[0]), n_filt=int(c[1]), n_act=int(c[2]),
                    n_infeasible=int(c[3]), nnzb=int(self.nnzb.item()))

    def results(self):
        """Copy the step's outputs to host numpy arrays (synchronises)."""
        self.torch.cuda.synchronize(self.device)
        na = min(int(self.a_n.item()), self.act_cap)
        nc = min(int(self.c_n.item()), self.cand_cap)
        nb = min(int(self.nnzb.item()), self.bsr_cap)
        Hf = unpack_hessians(self.l_H[:na].cpu().numpy())
        return dict(
            cand=np.stack([self.c_t[:nc].cpu().numpy().astype(np.int32), self.c_i[:nc].cpu().numpy(),
                           self.c_j[:nc].cpu().numpy()], 1),
            ptype=self.a_t[:na].cpu().numpy().astype(np.int32), i=self.a_i[:na].cpu().numpy(),
            j=self.a_j[:na].cpu().numpy(), code=self.a_code[:na].cpu().numpy().astype(np.int32),
            flags=self.a_flags[:na].cpu().numpy().astype(np.int32), d=self.a_dist[:na].cpu().numpy(),
            E=self.l_E[:na].cpu().numpy(), G=self.l_G[:na].cpu().numpy(), Hpsd=Hf,
            E_total=float(self.E.item()), g=self.g.cpu().numpy(),
            row_ptr=self.row_ptr.cpu().numpy().astype(np.int64), col=self.col[:nb].cpu().numpy(),
            val=self.val[:nb].cpu().numpy().reshape(-1, 3, 3), counts=self.counts())

    def close(self):
        if getattr(self, "handle", None):
            lib().bf_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many resident scenes stepped together by one HIP graph launch.

    ``scenes`` are ContactScene objects already sized for their inputs (call
    ``run`` once each); ``xs`` their device position tensors, which the batch
    reads at every step (update them in place).  ``lanes``: concurrent streams
    inside the graph (0: four, the hardware queues a process gets).
    """

    def __init__(self, scenes, xs, lanes=0):
        import torch
        self.torch = torch
        self.scenes, self.xs = list(scenes), list(xs)
        assert len(self.scenes) == len(self.xs) and self.scenes
        items = (BatchItem * len(self.scenes))(*[cs.batch_item(x) for cs, x in zip(self.scenes, self.xs)])
        self._items = items
        h = C.c_void_p()
        st = torch.cuda.current_stream(self.scenes[0].device).cuda_stream
        _check(lib().bf_batch_create(items, len(self.scenes), int(lanes), C.c_void_p(st), C.byref(h)),
               "bf_batch_create")
        self.handle = h
        n = C.c_int32(0)
        lane_of = np.zeros(len(self.scenes), np.int32)
        _check(lib().bf_batch_info(self.handle, C.byref(n), lane_of.ctypes.data), "bf_batch_info")
        self.lanes, self.lane_of = int(n.value), lane_of

    def step(self):
        """One step of every scene: one graph launch on the current stream."""
        st = self.torch.cuda.current_stream(self.scenes[0].device).cuda_stream
        _check(lib().bf_batch_step(self.handle, C.c_void_p(st)), "bf_batch_step")

    def close(self):
        if getattr(self, "handle", None):
            lib().bf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NativeServer:
    """The library's serving loop (bf_serve_*): scenes registered at start,
    requests submitted with host positions, results polled by ticket."""

    def __init__(self, scenes, caps, budget_bytes, slots=4, max_bypass=8, prec=BF_FP64, device=0):
        n = len(scenes)
        self._keep = []
        descs = (MeshDesc * n)()
        prms = (Params * n)()
        for k, sc in enumerate(scenes):
            kind = BF_ROD if sc.kind == "rod" else BF_SHELL
            edges = np.ascontiguousarray(sc.edges, np.int32)
            tris = np.ascontiguousarray(sc.tris, np.int32) if kind == BF_SHELL else None
            ref = np.ascontiguousarray(sc.ref, np.float64)
            refdist = int(getattr(sc, "refdist", BF_REFDIST_PARAM))
            xr = np.ascontiguousarray(sc.xrest, np.float64) if refdist == BF_REFDIST_EUCLID_REST else None
            self._keep += [edges, tris, ref, xr]
            descs[k] = MeshDesc(kind, sc.n_verts, sc.n_edges, sc.n_tris if kind == BF_SHELL else 0,
                                edges.ctypes.data, tris.ctypes.data if tris is not None else None, ref.ctypes.data,
                                xr.ctypes.data if xr is not None else None)
            prms[k] = Params(float(sc.h), float(sc.eta), float(sc.kappa), int(prec), BF_FILTER_PAPER, 11, refdist)
        cc = np.ascontiguousarray([c[0] for c in caps], np.int64)
        ac = np.ascontiguousarray([c[1] for c in caps], np.int64)
        bc = np.ascontiguousarray([c[2] for c in caps], np.int64)
        self._keep += [descs, prms, cc, ac, bc]
        cfg = ServeConfig(n, C.addressof(descs), C.addressof(prms), cc.ctypes.data, ac.ctypes.data, bc.ctypes.data,
                          int(budget_bytes), int(slots), int(max_bypass), int(device))
        h = C.c_void_p()
        _check(lib().bf_serve_start(C.byref(cfg), C.byref(h)), "bf_serve_start")
        self.handle = h
        self.nv = [sc.n_verts for sc in scenes]
        self._grads = {}

    def submit(self, sid, x, grad=False):
        """Queue a request; returns its ticket.  With grad, poll returns the
        gradient as well."""
        x = np.ascontiguousarray(x, np.float64)
        assert x.shape == (self.nv[sid], 3)
        g = np.zeros((self.nv[sid], 3)) if grad else None
        t = C.c_int64(0)
        _check(lib().bf_serve_submit(self.handle, int(sid), x.ctypes.data, g.ctypes.data if grad else None,
                                     C.byref(t)), "bf_serve_submit")
        if grad:
            self._grads[t.value] = g
        return int(t.value)

    def poll(self, ticket, wait=True):
        """None while pending; else a dict of the request's results."""
        r = ServeResult()
        _check(lib().bf_serve_poll(self.handle, int(ticket), int(bool(wait)), C.byref(r)), "bf_serve_poll")
        if not r.done:
            return None
        out = dict(scene=r.scene, error=r.error, status=r.status, E=r.E, n_bp=r.n_bp, ms=r.ms, retries=r.retries,
                   counts=dict(n_c=r.counts[0], n_filt=r.counts[1], n_act=r.counts[2], n_infeasible=r.counts[3],
                               nnzb=r.counts[4]))
        g = self._grads.pop(ticket, None)
        if g is not None:
            out["g"] = g
        return out

    def info(self):
        n, used = C.c_int32(0), C.c_int64(0)
        sz = np.zeros((len(self.nv), 2), np.int64)
        ev = np.zeros(4, np.int64)
        _check(lib().bf_serve_info(self.handle, C.byref(n), C.byref(used), sz.ctypes.data, ev.ctypes.data),
               "bf_serve_info")
        return dict(resident=int(n.value), used=int(used.value), footprint=sz[:, 0].copy(), step=sz[:, 1].copy(),
                    created=int(ev[0]),
                    evicted=int(ev[1]), retried=int(ev[2]), peak_bytes=int(ev[3]))

    def close(self):
        if getattr(self, "handle", None):
            lib().bf_serve_stop(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
