"""Serving loop: many independent channel instances on one GPU.

Each request is one wall-modelled channel (its own grid, degree and
viscosity) that asks for a number of enriched velocity-residual applies and
one mixed-precision pressure-Poisson solve to a relative residual of 1e-10.
The loop admits requests in arrival order while a slot is free and their
device-memory footprint fits the budget, keeps every admitted instance's mesh
tables and vectors resident on the device, and advances all instances that
are in their velocity phase together: one batched library call per round
covers every such instance (one launch per degree group and cell class).
Solves run concurrently on worker threads, each on its own HIP stream, so
they overlap with each other and with the batched velocity rounds; the
library calls release the interpreter lock.  A request whose setup or solve
fails is marked failed and its resources are released; the others go on.

Latency is completion minus scheduled arrival on the host monotonic clock.
All compute runs in the HIP library; this module only schedules, allocates
and copies.
"""
from __future__ import annotations

import ctypes
import threading
import time
from collections import deque
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np

from . import Mesh, _lib, apply_velocity_residual_batched, batch_workspace
from .inputs import Request, ServingConfig, draw_inputs, serving_requests


def footprint_bytes(wl, sp) -> int:
    """Device bytes one instance holds while admitted: mesh tables, solve
    workspace, velocity input and output, pressure right-hand side and
    solution (FP64)."""
    L = _lib.lib()
    params = _lib.params_from(wl.mesh)
    mesh_ws = _lib.check(L.dg_mesh_workspace_bytes(ctypes.byref(params)))
    solve_ws = _lib.check(L.dg_solve_workspace_bytes_for(ctypes.byref(params), ctypes.byref(sp)))
    m = wl.mesh
    return int(mesh_ws + solve_ws + 8 * (2 * m.n_vel + 2 * m.n_p))


@dataclass
class Outcome:
    rid: int
    ok: bool
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    latency: float = 0.0
    n_vel: int = 0
    n_p: int = 0
    applies: int = 0
    poisson_applies: int = 0
    outer_its: int = 0
    rel_resid: float = float("nan")
    error: str = ""
    r: object = None           # final velocity residual (kept on request)
    x: object = None           # pressure solution (kept on request)


@dataclass
class _Instance:
    req: Request
    fp: int
    out: Outcome
    stream: object = None
    mesh: Mesh = None
    u: object = None
    r: object = None
    b: object = None
    x: object = None
    ws: object = None
    applies_done: int = 0
    event: object = None


@dataclass
class ServeReport:
    outcomes: list
    makespan: float
    peak_bytes: int
    peak_active: int
    rounds: int

    def ok(self):
        return [o for o in self.outcomes if o.ok]

    def summary(self) -> dict:
        good = self.ok()
        lat = np.array([o.latency for o in good]) if good else np.zeros(1)
        dofs = sum(o.applies * o.n_vel + o.poisson_applies * o.n_p for o in good)
        return {
            "requests": len(self.outcomes), "completed": len(good),
            "failed": len(self.outcomes) - len(good),
            "makespan_s": self.makespan,
            "dofs_per_s": dofs / self.makespan if self.makespan > 0 else 0.0,
            "latency_p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "latency_p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "latency_max_ms": 1e3 * float(lat.max()),
            "peak_admitted_bytes": self.peak_bytes, "peak_active": self.peak_active,
            "velocity_rounds": self.rounds,
            "max_rel_resid": max((o.rel_resid for o in good), default=float("nan")),
        }


class Server:
    """Continuous-batching server for channel-instance requests.

    budget_bytes: device-memory budget for admitted instances.
    slots: most instances admitted at once.
    workers: threads (and HIP streams) for setup and solves.
    keep_results: keep each request's final r and x (device tensors).
    """

    def __init__(self, budget_bytes=32 << 30, slots=64, workers=8, applies=10, solve_kw=None,
                 keep_results=False, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.workers = int(workers)
        self.applies = int(applies)
        kw = dict(rtol=1e-10, mixed=True, max_outer=2000, max_inner=0, cheb_degree=5, multigrid=True,
                  coarse_degree=3)
        kw.update(solve_kw or {})
        self.solve_kw = kw
        self.keep = keep_results
        self._tls = threading.local()
        self.main = torch.cuda.Stream(device=self.device)
        self.batch_ws = batch_workspace(self.slots, self.device)

    def _sp(self):
        k = self.solve_kw
        return _lib.SolveParams(rtol=k["rtol"], max_outer=k["max_outer"], max_inner=k["max_inner"],
                                cheb_degree=k["cheb_degree"], mixed=int(k["mixed"]),
                                multigrid=int(k["multigrid"]), coarse_degree=int(k["coarse_degree"]))

    # -- worker jobs (run on pool threads, each on its own stream) ---------
    def _stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            s = self._tls.stream = self.torch.cuda.Stream(device=self.device)
        return s

    def _setup(self, inst: _Instance):
        torch = self.torch
        wl = inst.req.workload
        inst.stream = self._stream()
        d = draw_inputs(wl)
        with torch.cuda.device(self.device), torch.cuda.stream(inst.stream):
            inst.mesh = Mesh(wl.mesh, tau_w=d["tau"], device=self.device, stream=inst.stream)
            inst.u = torch.from_numpy(d["u"]).to(self.device)
            inst.b = torch.from_numpy(d["p"]).to(self.device)
            inst.r = torch.empty_like(inst.u)
            inst.x = torch.zeros_like(inst.b)
            inst.ws = inst.mesh.solve_workspace(self._sp())
            inst.stream.synchronize()
        return inst

    def _solve(self, inst: _Instance):
        torch = self.torch
        inst.stream = self._stream()
        with torch.cuda.device(self.device), torch.cuda.stream(inst.stream):
            inst.stream.wait_event(inst.event)        # velocity rounds of this instance are done
            try:
                _, st = inst.mesh.solve_poisson(inst.b, inst.x, sp=self._sp(), workspace=inst.ws,
                                                stream=inst.stream)
            finally:
                inst.stream.synchronize()
        return inst, st

    # -- main loop ---------------------------------------------------------
    def run(self, requests, time_scale=1.0) -> ServeReport:
        """Serve `requests` (inputs.Request list, sorted by arrival).  Arrival
        times are multiplied by time_scale (0 = all arrive at once)."""
        torch = self.torch
        sp = self._sp()
        pending = deque(sorted(requests, key=lambda q: q.arrival))
        outcomes = {}
        active_apply = []             # instances in the velocity phase
        used = 0
        n_admitted = 0
        peak_bytes = peak_active = rounds = 0
        futures = {}
        pool = ThreadPoolExecutor(max_workers=self.workers)
        t0 = time.monotonic()

        def release(inst):
            nonlocal used, n_admitted
            used -= inst.fp
            n_admitted -= 1
            if inst.mesh is not None:
                inst.mesh.close()
            inst.mesh = inst.u = inst.b = inst.ws = None
            if not self.keep:
                inst.r = inst.x = None

        try:
            while pending or futures or active_apply:
                now = time.monotonic() - t0
                # admission: arrival order, slot and footprint permitting
                while pending and pending[0].arrival * time_scale <= now and n_admitted < self.slots:
                    q = pending[0]
                    fp = footprint_bytes(q.workload, sp)
                    if fp > self.budget:
                        pending.popleft()
                        outcomes[q.rid] = Outcome(q.rid, False, q.arrival * time_scale, error="footprint above budget")
                        continue
                    if used + fp > self.budget:
                        break
                    pending.popleft()
                    used += fp
                    n_admitted += 1
                    peak_bytes = max(peak_bytes, used)
                    peak_active = max(peak_active, n_admitted)
                    m = q.workload.mesh
                    out = Outcome(q.rid, True, q.arrival * time_scale, admitted=now, n_vel=m.n_vel, n_p=m.n_p)
                    inst = _Instance(q, fp, out)
                    futures[pool.submit(self._setup, inst)] = ("setup", inst)

                # one batched velocity round over every instance in that phase
                if active_apply:
                    with torch.cuda.device(self.device):
                        apply_velocity_residual_batched([i.mesh for i in active_apply], [i.u for i in active_apply],
                                                        [i.r for i in active_apply], workspace=self.batch_ws,
                                                        stream=self.main)
                    rounds += 1
                    still = []
                    for inst in active_apply:
                        inst.applies_done += 1
                        if inst.applies_done >= self.applies:
                            inst.event = torch.cuda.Event()
                            inst.event.record(self.main)
                            futures[pool.submit(self._solve, inst)] = ("solve", inst)
                        else:
                            still.append(inst)
                    active_apply = still

                # collect finished jobs; block only when nothing else can progress
                if futures:
                    timeout = 0.0 if active_apply else None
                    if not active_apply and pending:
                        ahead = pending[0].arrival * time_scale - (time.monotonic() - t0)
                        if ahead > 0:           # next arrival first (a blocked head waits for a completion)
                            timeout = ahead
                    done, _ = wait(list(futures), timeout=timeout, return_when=FIRST_COMPLETED)
                    for f in done:
                        kind, inst = futures.pop(f)
                        err = f.exception()
                        if kind == "setup":
                            if err is not None:
                                inst.out.ok = False
                                inst.out.error = f"setup: {err}"
                                inst.out.done = time.monotonic() - t0
                                outcomes[inst.req.rid] = inst.out
                                release(inst)
                            elif self.applies > 0:
                                active_apply.append(inst)
                            else:
                                inst.event = torch.cuda.Event()
                                inst.event.record(self.main)
                                futures[pool.submit(self._solve, inst)] = ("solve", inst)
                        else:
                            o = inst.out
                            o.done = time.monotonic() - t0
                            o.latency = o.done - o.arrival
                            o.applies = inst.applies_done
                            if err is not None:
                                o.ok = False
                                o.error = f"solve: {err}"
                            else:
                                st = f.result()[1]
                                o.poisson_applies = st.op_applies_f64 + st.op_applies_f32
                                o.outer_its = st.outer_its
                                o.rel_resid = st.rel_resid
                                if self.keep:
                                    o.r, o.x = inst.r, inst.x
                            outcomes[inst.req.rid] = o
                            release(inst)
                elif pending and not active_apply:
                    delay = pending[0].arrival * time_scale - (time.monotonic() - t0)
                    if delay > 0:
                        time.sleep(delay)
            self.main.synchronize()
        finally:
            pool.shutdown(wait=True)
        makespan = time.monotonic() - t0
        return ServeReport([outcomes[k] for k in sorted(outcomes)], makespan, peak_bytes, peak_active, rounds)


def serve(cfg: ServingConfig = ServingConfig(), **server_kw) -> ServeReport:
    """Run the seeded request stream `cfg` through a Server."""
    reqs = serving_requests(cfg)
    return Server(applies=cfg.applies, **server_kw).run(reqs)
