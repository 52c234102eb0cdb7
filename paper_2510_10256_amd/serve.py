"""Serving loop: contact-evaluation requests from many independent scenes.

Requests (scene id + positions) arrive from independent simulations.  A
request is admitted when an execution slot is free and its scene fits the HBM
budget: a scene that is not resident is created on the device (topology, the
filter precompute, the buffers of a step) after the least recently used idle
scenes are evicted to make room.  At most one request per scene is on the
device at a time.  Admitted requests run on their slot's stream and overlap
on the device; a request completes when its energy and counters are back on
the host (gradient and Hessian stay in the scene's device buffers until that
scene's next request).  Requests that arrive while others run are admitted as
soon as a slot and memory free up (continuous batching, no fixed batches).

``Admission`` is the host-side policy and needs no GPU; ``Server`` drives the
library's four calls through ``ContactScene``.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    sid: int                 # scene id
    x: np.ndarray            # [V,3] positions
    t_arrival: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    bypassed: int = 0
    E: float = float("nan")
    counts: dict = field(default_factory=dict)
    retries: int = 0
    g: object = None         # [V,3] gradient on the host (Server(keep_grad=True))


class Admission:
    """Which queued requests start now, and which resident scenes make room.

    FIFO order, except that a request whose scene is busy, or that does not
    fit yet, may be passed by later ones; a request passed ``max_bypass`` times
    blocks every later request until it starts (no starvation of large
    scenes).  Eviction takes idle resident scenes, least recently used first.
    """

    def __init__(self, budget_bytes: int, slots: int, footprint, max_bypass: int = 8):
        self.budget, self.slots, self.footprint, self.max_bypass = int(budget_bytes), int(slots), footprint, max_bypass
        self.resident: OrderedDict[int, int] = OrderedDict()  # sid -> bytes, least recent first
        self.busy: set[int] = set()
        self.queue: deque[Request] = deque()
        self.used = 0

    def arrive(self, req: Request):
        if self.footprint(req.sid) > self.budget:
            raise ValueError(f"scene {req.sid} needs {self.footprint(req.sid)} B, above the budget {self.budget} B")
        self.queue.append(req)

    def plan(self):
        """[(request, create, evict_sids)] to start now, in order."""
        out = []
        free = self.slots - len(self.busy)
        kept = deque()
        blocked = False
        while self.queue:
            req = self.queue.popleft()
            if blocked or free <= 0 or req.sid in self.busy:
                if not blocked and free > 0:
                    req.bypassed += 1
                kept.append(req)
                blocked = blocked or req.bypassed > self.max_bypass
                continue
            need = 0 if req.sid in self.resident else self.footprint(req.sid)
            evict = []
            if need:
                avail = self.budget - self.used
                for s2, b2 in self.resident.items():
                    if avail >= need:
                        break
                    if s2 not in self.busy:
                        evict.append(s2)
                        avail += b2
                if avail < need:
                    req.bypassed += 1
                    kept.append(req)
                    blocked = req.bypassed > self.max_bypass
                    continue
            for s2 in evict:
                self.used -= self.resident.pop(s2)
            if need:
                self.resident[req.sid] = need
                self.used += need
            self.resident.move_to_end(req.sid)
            self.busy.add(req.sid)
            free -= 1
            out.append((req, need > 0, evict))
        self.queue = kept
        return out

    def done(self, req: Request):
        self.busy.discard(req.sid)

    def resize(self, sid: int, nbytes: int):
        """Correct a resident scene's size (e.g. after its buffers grew)."""
        if sid in self.resident:
            self.used += int(nbytes) - self.resident[sid]
            self.resident[sid] = int(nbytes)


def scene_caps(scene):
    """Initial buffer capacities of a scene's step, from its primitive counts:
    candidates 32 per shell primitive (the folded cloth needs 23) and 12 per
    rod edge, active pairs 2 per shell primitive and 1.5 per edge, BSR blocks
    2 per active pair (the cloth needs 1.33).  A step that overflows runs again
    with capacities grown to its counts (the serving loops do this), so dense
    scenes pay one re-run on their first request."""
    nprims = scene.n_edges + (scene.n_tris + scene.n_verts if scene.kind == "shell" else 0)
    shell = scene.kind == "shell"
    cand = max(4096, (32 if shell else 12) * nprims)
    act = max(4096, (2 * nprims if shell else 3 * nprims // 2))
    return cand, act, max(4096, 2 * act)


def scene_bytes(scene, cand, act, bsr, prec=1):
    """Device bytes of a resident scene: the caller buffers of a step plus the
    library's scene workspace (topology, grid, staging, assembly).  Each
    active pair's packed Hessian record is 78 doubles, or 78 floats in the
    mixed mode (prec 1)."""
    nv = scene.n_verts
    nprims = scene.n_edges + (scene.n_tris + nv if scene.kind == "shell" else 0)
    hrec = 78 * (4 if prec == 1 else 8)
    buffers = 9 * cand + act * (4 + 4 + 1 + 1 + 1 + 8 + 8 + 96 + hrec) + bsr * (4 + 72) + nv * 3 * 8 * 2 + 4 * nv
    workspace = (nprims * (24 + 8 + 16 + 16) + 16 * 2 * max(4096, 2 * nprims) + 8 * 4 * (nv + scene.n_edges)
                 + 20 * cand + 80 * act + 20 * nv)
    return int(buffers + workspace)


class Server:
    """Continuous-batching request loop over resident scenes on one GPU."""

    def __init__(self, scenes, budget_bytes=2 << 30, slots=4, prec=None, device="cuda:0", keep_grad=False):
        import torch
        from . import binding as B
        self.torch, self.B = torch, B
        self.scenes = list(scenes)
        self.prec = B.BF_MIXED if prec is None else prec
        self.device = torch.device(device)
        self.caps = [scene_caps(sc) for sc in self.scenes]
        self._bytes = [scene_bytes(sc, *c, prec=self.prec) for sc, c in zip(self.scenes, self.caps)]
        self.adm = Admission(budget_bytes, slots, lambda sid: self._bytes[sid])
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]  # default priority
        vmax = max(sc.n_verts for sc in self.scenes)
        self.stage = [torch.empty((vmax, 3), dtype=torch.float64).pin_memory() for _ in range(slots)]
        self.out_host = [torch.empty(6, dtype=torch.float64).pin_memory() for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.keep_grad = keep_grad
        self.cs = {}        # sid -> ContactScene
        self.graph = {}     # sid -> one-scene Batch (the step captured as a graph)
        self.xdev = {}      # sid -> device positions
        self.running = {}   # slot -> (request, event)
        self.created = 0
        self.evicted = 0

    # -- scene residency ---------------------------------------------------------
    def _create(self, sid):
        sc = self.scenes[sid]
        cand, act, bsr = self.caps[sid]
        cs = self.B.ContactScene(sc, prec=self.prec, cand_cap=cand, act_cap=act, bsr_cap=bsr, device=self.device)
        self.cs[sid] = cs
        self.xdev[sid] = self.torch.tensor(sc.x, dtype=self.torch.float64, device=self.device)
        self._capture(sid)
        self.created += 1

    def _capture(self, sid):
        # buffers are zeroed on the creating stream: finish that before any
        # slot stream touches them, then capture the step as a graph
        self.torch.cuda.current_stream(self.device).synchronize()
        if sid in self.graph:
            self.graph.pop(sid).close()
        self.graph[sid] = self.B.Batch([self.cs[sid]], [self.xdev[sid]], lanes=1)

    def _evict(self, sid):
        self.graph.pop(sid).close()
        cs = self.cs.pop(sid)
        cs.close()
        del self.xdev[sid]
        self.evicted += 1

    # -- request flow --------------------------------------------------------------
    def submit(self, req: Request):
        req.t_arrival = time.perf_counter()
        self.adm.arrive(req)

    def _launch(self, req: Request, slot: int):
        torch = self.torch
        cs, x = self.cs[req.sid], self.xdev[req.sid]
        n = req.x.shape[0]
        st = self.streams[slot]
        stage = self.stage[slot][:n]
        stage.numpy()[:] = req.x
        with torch.cuda.stream(st):
            x.copy_(stage, non_blocking=True)
            self.graph[req.sid].step()
            if self.keep_grad:
                req.g = torch.empty((n, 3), dtype=torch.float64).pin_memory()
                req.g.copy_(cs.g, non_blocking=True)
            o = self.out_host[slot]
            o[:1].copy_(cs.E, non_blocking=True)
            o[1:5].copy_(cs.counters.to(torch.float64), non_blocking=True)
            o[5:6].copy_(cs.nnzb.to(torch.float64), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.running[slot] = (req, ev)

    def pump(self):
        """Start what the policy allows, collect what finished; returns the
        requests completed in this call."""
        done = []
        for slot, (req, ev) in list(self.running.items()):
            if not ev.query():
                continue
            del self.running[slot]
            cs = self.cs[req.sid]
            st = cs.status(clear=True)
            B = self.B
            if st & (B.BF_S_CAND_OVERFLOW | B.BF_S_ACT_OVERFLOW | B.BF_S_BSR_OVERFLOW):
                # grow the scene's buffers to what the device reported, then redo
                cs.run(self.xdev[req.sid])
                self._capture(req.sid)
                self.adm.resize(req.sid, scene_bytes(self.scenes[req.sid], cs.cand_cap, cs.act_cap, cs.bsr_cap,
                                                     prec=self.prec))
                req.retries += 1
                self._launch(req, slot)
                continue
            o = self.out_host[slot].numpy()
            req.E = float(o[0])
            req.counts = dict(n_c=int(o[1]), n_filt=int(o[2]), n_act=int(o[3]), n_infeasible=int(o[4]),
                              nnzb=int(o[5]))
            req.t_done = time.perf_counter()
            self.adm.done(req)
            self.free_slots.append(slot)
            done.append(req)
        for req, create, evict in self.adm.plan():
            for s2 in evict:
                self._evict(s2)
            if create:
                self._create(req.sid)
            req.t_start = time.perf_counter()
            self._launch(req, self.free_slots.pop())
        return done

    def idle(self):
        return not self.running and not self.adm.queue

    def close(self):
        self.torch.cuda.synchronize(self.device)
        for sid in list(self.cs):
            self._evict(sid)


def run_closed_loop(server: Server, make_request, n_requests: int, inflight: int):
    """Keep `inflight` requests waiting or running until n_requests finished;
    returns (completed requests, wall seconds)."""
    done, issued = [], 0
    t0 = time.perf_counter()
    while len(done) < n_requests:
        while issued < n_requests and issued - len(done) < inflight:
            server.submit(make_request(issued))
            issued += 1
        done += server.pump()
    return done, time.perf_counter() - t0


def run_open_loop(server: Server, make_request, arrivals):
    """Submit request k at time arrivals[k] (seconds from the start, open
    loop: arrivals do not wait for completions); returns (completed, wall)."""
    done, k = [], 0
    n = len(arrivals)
    t0 = time.perf_counter()
    while len(done) < n:
        now = time.perf_counter() - t0
        while k < n and arrivals[k] <= now:
            server.submit(make_request(k))
            k += 1
        done += server.pump()
    return done, time.perf_counter() - t0


def poisson_arrivals(rate: float, n: int, seed: int):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def latency_stats(done):
    lat = np.array([r.t_done - r.t_arrival for r in done]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}


def mean_edge_length(scene):
    e = scene.x[scene.edges[:, 1]] - scene.x[scene.edges[:, 0]]
    return float(np.mean(np.linalg.norm(e, axis=1)))


def request_maker(scenes, seed, lbar=None):
    """Requests for uniformly chosen scenes with positions x_base + N(0, (0.01 l)^2)."""
    lbar = lbar or [mean_edge_length(sc) for sc in scenes]

    def make(k):
        rng = np.random.default_rng(seed + 7919 * k)
        sid = int(rng.integers(len(scenes)))
        sc = scenes[sid]
        x = sc.x + rng.normal(0.0, 0.01 * lbar[sid], size=sc.x.shape)
        return Request(rid=k, sid=sid, x=x)

    return make


__all__ = ["Request", "Admission", "Server", "run_closed_loop", "run_open_loop", "poisson_arrivals",
           "latency_stats", "request_maker", "scene_caps", "scene_bytes", "mean_edge_length"]
