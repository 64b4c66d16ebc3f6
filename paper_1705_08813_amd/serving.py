"""Serving loop: many independent channel instances on one GPU.

Each request is one wall-modelled channel (its own grid, degree and
viscosity) that asks for a number of enriched velocity-residual applies and
one mixed-precision pressure-Poisson solve to a relative residual of 1e-10.
The loop admits requests in arrival order while a slot is free and their
device-memory footprint fits the budget, keeps every admitted instance's mesh
tables and vectors resident on the device, and advances all instances that
are in their velocity phase together: one batched library call per round
covers every such instance (one launch per degree group and cell class).
The instances of one mesh shape that finish their velocity phase in the
same round solve together: one batched solve call advances all of their
pressure solves in lockstep (one launch per iteration step, a mesh leaving
the batch when it converges; the call returns with its slowest mesh, so
only like meshes share a call).  Solve batches run on worker threads, each on
its own HIP stream, so they overlap with each other and with the batched
velocity rounds; the library calls release the interpreter lock.  A request whose setup or solve
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

from . import Mesh, _lib, apply_velocity_residual_batched, batch_workspace, solve_poisson_batched
from .inputs import Request, ServingConfig, draw_inputs, serving_requests


def serving_mesh(wl):
    """The mesh of a request: its operators and solves need no projection-step
    tables, so the instance does not reserve them."""
    return wl.mesh.with_(omit_step_tables=1)


def footprint_bytes(wl, sp) -> int:
    """Device bytes one instance holds while admitted: mesh tables, solve
    workspace, velocity input and output, pressure right-hand side and
    solution (FP64)."""
    L = _lib.lib()
    params = _lib.params_from(serving_mesh(wl))
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
    batch_solves: solve the instances that finish their velocity phase in
        the same round in one batched call (else one solve call each).
    """

    def __init__(self, budget_bytes=32 << 30, slots=64, workers=8, applies=10, solve_kw=None,
                 keep_results=False, device=None, batch_solves=True):
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
        self.batch_solves = bool(batch_solves)
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
            inst.mesh = Mesh(serving_mesh(wl), tau_w=d["tau"], device=self.device, stream=inst.stream)
            inst.u = torch.from_numpy(d["u"]).to(self.device)
            inst.b = torch.from_numpy(d["p"]).to(self.device)
            inst.r = torch.empty_like(inst.u)
            inst.x = torch.zeros_like(inst.b)
            inst.ws = inst.mesh.solve_workspace(self._sp())
            inst.stream.synchronize()
        return inst

    def _batch_ws(self, meshes, sp):
        """The calling worker's descriptor workspace for a batched solve,
        kept between calls and grown (doubling) when a batch needs more."""
        need = int(_lib.check(_lib.lib().dg_solve_batch_workspace_bytes(
            (ctypes.c_void_p * len(meshes))(*[m.handle.value for m in meshes]), len(meshes), ctypes.byref(sp))))
        ws = getattr(self._tls, "bws", None)
        if ws is None or ws.numel() < need:
            size = max(need, 2 * ws.numel() if ws is not None else 0, 8 << 20)
            ws = self._tls.bws = self.torch.empty(size, dtype=self.torch.uint8, device=self.device)
        return ws

    def _solve(self, insts):
        """Solve the instances' pressure problems (one batched call, or one
        call each); returns [(inst, stats or None, error or None)]."""
        torch = self.torch
        stream = self._stream()
        out = []
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            for inst in insts:
                inst.stream = stream
                stream.wait_event(inst.event)         # velocity rounds of this instance are done
            try:
                sp = self._sp()
                # the batched solve needs a coarser multigrid level on every mesh; a lone
                # mesh takes the single call, whose result is bit for bit the same
                batch = [i for i in insts if self.batch_solves and sp.multigrid and len(i.mesh.mg_levels()) >= 2]
                if len(batch) < 2:
                    batch = []
                if batch:
                    meshes = [i.mesh for i in batch]
                    bws = self._batch_ws(meshes, sp)
                    _, stats, codes = solve_poisson_batched(meshes, [i.b for i in batch], [i.x for i in batch],
                                                            sp=sp, workspaces=[i.ws for i in batch], batch_ws=bws,
                                                            stream=stream)
                    for inst, st, code in zip(batch, stats, codes):
                        out.append((inst, st, None if code == 0 else _lib.DgError(code, f"solve status {code}")))
                for inst in insts:
                    if inst in batch:
                        continue
                    try:
                        _, st = inst.mesh.solve_poisson(inst.b, inst.x, sp=sp, workspace=inst.ws, stream=stream)
                        out.append((inst, st, None))
                    except Exception as e:  # noqa: BLE001 (recorded per request)
                        out.append((inst, None, e))
            finally:
                stream.synchronize()
        return out

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
                    still, ready = [], []
                    for inst in active_apply:
                        inst.applies_done += 1
                        if inst.applies_done >= self.applies:
                            inst.event = torch.cuda.Event()
                            inst.event.record(self.main)
                            ready.append(inst)
                        else:
                            still.append(inst)
                    active_apply = still
                    # one solve batch per mesh shape: a batch returns when its slowest
                    # mesh converges, so only like meshes wait for each other
                    groups = {}
                    for inst in ready:
                        m = inst.req.workload.mesh
                        groups.setdefault((m.nx, m.ny, m.nz, m.k_p), []).append(inst)
                    for grp in groups.values():
                        futures[pool.submit(self._solve, grp)] = ("solve", grp)

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
                                futures[pool.submit(self._solve, [inst])] = ("solve", [inst])
                        else:
                            done_at = time.monotonic() - t0
                            results = f.result() if err is None else [(i, None, err) for i in inst]
                            for one, st, e in results:
                                o = one.out
                                o.done = done_at
                                o.latency = o.done - o.arrival
                                o.applies = one.applies_done
                                if e is not None:
                                    o.ok = False
                                    o.error = f"solve: {e}"
                                else:
                                    o.poisson_applies = st.op_applies_f64 + st.op_applies_f32
                                    o.outer_its = st.outer_its
                                    o.rel_resid = st.rel_resid
                                    if self.keep:
                                        o.r, o.x = one.r, one.x
                                outcomes[one.req.rid] = o
                                release(one)
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
