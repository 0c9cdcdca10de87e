"""Continuous-batching request loop for chi^2 (+ gradient) evaluations.

Fitters (MCMC ensembles, gradient optimisers) submit requests against
observations that stay resident on the device; a scheduler thread forms
micro-batches as requests arrive and keeps several of them in flight on
separate HIP streams, so that work submitted while others run overlaps on
the GPU.

 - Admission.  Every request has a device-memory footprint (its model and
   output buffers plus the workspace its calls need).  A micro-batch is
   admitted only while the footprints in flight stay within the HBM budget;
   otherwise it waits until earlier work completes.  A request that cannot
   fit even on an idle device is rejected (MemoryError).
 - Batching.  Queued chi^2-only requests on the same dataset, image grid and
   profile length form one micro-batch, evaluated by one planned batch
   (models and geometry written into the plan's device slots, so the uv data
   is read once for the whole micro-batch).  Gradient requests run the
   adjoint path, one call each, in the micro-batch's stream.
 - Deadlines and cancellation.  A request whose deadline passes while it is
   queued fails with TimeoutError; a cancelled future is dropped.
 - Latency is completion minus arrival on the host clock (time.perf_counter).

The scheduler itself is host logic and takes any executor with the
``footprint / launch / done / collect`` interface; ``GpuExecutor`` is the
HIP one.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    """One chi^2 (and optionally gradient) evaluation of a radial profile."""
    dataset: str
    I: object                      # profile values (numpy array or device tensor)
    Rmin: float
    dR: float
    Nxy: int
    dxy: float
    inc: float = 0.0
    PA: float = 0.0
    dRA: float = 0.0
    dDec: float = 0.0
    grad: bool = False
    deadline: float | None = None  # absolute time.perf_counter() value
    arrival: float = field(default=0.0)
    future: Future | None = field(default=None, repr=False)

    def key(self):
        return (self.dataset, int(self.Nxy), float(self.dxy), int(np.size(self.I)), bool(self.grad))


def _settle(fut: Future, result=None, exc: BaseException | None = None):
    """Resolve a future unless the client cancelled it meanwhile."""
    try:
        if exc is not None:
            fut.set_exception(exc)
        else:
            fut.set_result(result)
    except Exception:  # InvalidStateError: cancelled concurrently
        pass


class Server:
    """Continuous-batching scheduler (see the module docstring)."""

    def __init__(self, executor, max_batch: int = 16, max_inflight: int = 4,
                 hbm_budget: int | None = None, idle_wait: float = 2e-4):
        self.ex = executor
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.budget = hbm_budget if hbm_budget is not None else executor.default_budget()
        self.idle_wait = idle_wait
        self._in = collections.deque()
        self._lock = threading.Lock()
        self._wake = threading.Event()
        self._pending = collections.deque()
        self._inflight = []          # (handle, requests, footprint, stream slot)
        self._free_slots = list(range(self.max_inflight))
        self._used = 0
        self._run = False
        self._thr = None
        self.latencies = []
        self.completed = 0
        self.rejected = 0
        self.expired = 0
        self.batches = 0
        self.peak_used = 0
        self._t_first = None
        self._t_last = None

    # -- client side -------------------------------------------------------
    def submit(self, req: Request) -> Future:
        req.arrival = time.perf_counter()
        req.future = Future()
        with self._lock:
            self._in.append(req)
        self._wake.set()
        return req.future

    def start(self):
        self._run = True
        self._thr = threading.Thread(target=self._loop, name="galario-serve", daemon=True)
        self._thr.start()
        return self

    def stop(self, drain: bool = True, timeout: float = 60.0):
        if drain:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < timeout:
                with self._lock:
                    busy = bool(self._in) or bool(self._pending) or bool(self._inflight)
                if not busy:
                    break
                time.sleep(1e-3)
        self._run = False
        self._wake.set()
        if self._thr is not None:
            self._thr.join(timeout)

    def stats(self) -> dict:
        lat = np.array(self.latencies) * 1e3
        span = (self._t_last - self._t_first) if self._t_first is not None and self._t_last else 0.0
        return {
            "completed": self.completed, "rejected": self.rejected, "expired": self.expired,
            "batches": self.batches,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "evals_per_s": self.completed / span if span > 0 else None,
            "peak_hbm_bytes": self.peak_used, "hbm_budget_bytes": self.budget,
        }

    # -- scheduler ---------------------------------------------------------
    def _loop(self):
        bind = getattr(self.ex, "bind_thread", None)
        if bind is not None:
            bind()
        while self._run:
            progressed = False
            with self._lock:
                while self._in:
                    self._pending.append(self._in.popleft())
            now = time.perf_counter()
            # drop cancelled / expired requests before they take device memory
            if self._pending:
                keep = collections.deque()
                for r in self._pending:
                    if r.future.cancelled():
                        continue
                    if r.deadline is not None and now > r.deadline:
                        _settle(r.future, exc=TimeoutError("deadline passed while queued"))
                        self.expired += 1
                        continue
                    keep.append(r)
                self._pending = keep
            # retire finished micro-batches
            still = []
            for item in self._inflight:
                handle, reqs, fp, slot = item
                if self.ex.done(handle):
                    results = self.ex.collect(handle)
                    t = time.perf_counter()
                    for r, res in zip(reqs, results):
                        _settle(r.future, res)
                        self.latencies.append(t - r.arrival)
                    self.completed += len(reqs)
                    self._t_last = t
                    self._used -= fp
                    self._free_slots.append(slot)
                    progressed = True
                else:
                    still.append(item)
            self._inflight = still
            # admit new micro-batches while slots and memory allow
            while self._pending and self._free_slots:
                head = self._pending[0]
                key = head.key()
                group = [r for r in self._pending if r.key() == key][: self.max_batch]
                fp_one = self.ex.footprint([head])
                if fp_one > self.budget:
                    self._pending.popleft()
                    _settle(head.future, exc=MemoryError(
                        f"request needs {fp_one} bytes of device memory, budget {self.budget}"))
                    self.rejected += 1
                    continue
                while group and self.ex.footprint(group) > self.budget - self._used:
                    group.pop()
                if not group:
                    break              # wait for memory to free up
                fp = self.ex.footprint(group)
                ids = set(id(r) for r in group)
                self._pending = collections.deque(r for r in self._pending if id(r) not in ids)
                slot = self._free_slots.pop()
                try:
                    handle = self.ex.launch(group, slot)
                except Exception as e:  # launch errors go to the callers
                    for r in group:
                        _settle(r.future, exc=e)
                    self._free_slots.append(slot)
                    continue
                if self._t_first is None:
                    self._t_first = time.perf_counter()
                self._inflight.append((handle, group, fp, slot))
                self._used += fp
                self.peak_used = max(self.peak_used, self._used)
                self.batches += 1
                progressed = True
            if not progressed:
                self._wake.wait(self.idle_wait)
                self._wake.clear()


class GpuExecutor:
    """HIP executor: datasets resident in HBM, one stream per in-flight slot,
    planned batches for chi^2-only micro-batches, adjoint calls for gradients."""

    def __init__(self, device=None, dtype=None, max_batch: int = 16, max_inflight: int = 4):
        import torch

        from . import Dataset, profile_batch, Workspace, _lib, _sfx

        self.torch = torch
        self._Dataset, self._profile_batch, self._Workspace = Dataset, profile_batch, Workspace
        self._lib, self._sfx = _lib, _sfx
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.dtype = torch.float64 if dtype is None else dtype
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.datasets = {}
        self._plans = {}            # (key, slot) -> (batch, I slots, geo slots)
        self._ws = {}               # slot -> [Workspace] for gradient calls

    def default_budget(self) -> int:
        free, total = self.torch.cuda.mem_get_info(self.device)
        return int(0.8 * free)

    def bind_thread(self):
        self.torch.cuda.set_device(self.device)

    def add_dataset(self, name, u, v, re, im, w):
        t = lambda a: self.torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype,
                                           device=self.device)
        self.datasets[name] = self._Dataset(t(u), t(v), t(re), t(im), t(w))
        return self.datasets[name]

    def footprint(self, reqs) -> int:
        r = reqs[0]
        el = 8 if self.dtype == self.torch.float64 else 4
        ds = self.datasets[r.dataset]
        if r.grad:
            ws = getattr(self._lib(), "gal_grad_workspace_bytes" + self._sfx(self.dtype))(
                int(r.Nxy), int(ds.M), int(np.size(r.I)))
            return len(reqs) * (int(ws) + 2 * el * int(np.size(r.I)) + 64)
        Nxy = int(r.Nxy)
        spec = (Nxy // 2 + 2) ** 2 * el
        part = 8 * ((ds.M + 1023) // 1024)
        return len(reqs) * (spec + part + el * int(np.size(r.I)) + 64) + 4096

    def _plan(self, key, slot, K):
        pk = (key, slot, K)
        if pk not in self._plans:
            torch = self.torch
            name, Nxy, dxy, Nr, _ = key
            I = torch.zeros((K, Nr), dtype=self.dtype, device=self.device)
            geo = torch.zeros((K, 6), dtype=torch.float64, device=self.device)
            geo[:, 1] = 1.0
            b = self._profile_batch(self.datasets[name], I, geo, Nxy, dxy)
            self._plans[pk] = (b, I, geo)
        return self._plans[pk]

    def launch(self, reqs, slot):
        torch = self.torch
        st = self.streams[slot]
        key = reqs[0].key()
        name, Nxy, dxy, Nr, want_grad = key
        ds = self.datasets[name]
        with torch.cuda.stream(st):
            if not want_grad:
                K = 1
                while K < len(reqs):
                    K *= 2
                b, I, geo = self._plan(key, slot, K)
                Ih = torch.empty((K, Nr), dtype=self.dtype, pin_memory=True)
                gh = torch.empty((K, 6), dtype=torch.float64, pin_memory=True)
                for k in range(K):
                    r = reqs[min(k, len(reqs) - 1)]   # unused slots repeat the last request
                    Ih[k] = torch.as_tensor(np.asarray(r.I) if not torch.is_tensor(r.I)
                                            else r.I.detach().cpu(), dtype=self.dtype)
                    gh[k] = torch.tensor([r.Rmin, r.dR, r.inc, r.PA, r.dRA, r.dDec],
                                         dtype=torch.float64)
                I.copy_(Ih, non_blocking=True)
                geo.copy_(gh, non_blocking=True)
                out = b.chi2()
                host = torch.empty(K, dtype=torch.float64, pin_memory=True)
                host.copy_(out, non_blocking=True)
                keep = (Ih, gh, host)
                outs = [("chi2", host, k) for k in range(len(reqs))]
            else:
                pool = self._ws.setdefault(slot, [])
                while len(pool) < len(reqs):
                    pool.append(self._Workspace(self.device, self.dtype))
                outs, keep = [], []
                for k, r in enumerate(reqs):
                    I = torch.as_tensor(np.asarray(r.I) if not torch.is_tensor(r.I) else r.I,
                                        dtype=self.dtype).to(self.device, non_blocking=True)
                    c2, g = ds.chi2Profile_grad(I, r.Rmin, r.dR, Nxy, dxy, r.inc, r.PA, r.dRA,
                                                r.dDec, ws=pool[k])
                    hc = torch.empty((), dtype=torch.float64, pin_memory=True)
                    hg = torch.empty(g.shape, dtype=g.dtype, pin_memory=True)
                    hc.copy_(c2, non_blocking=True)
                    hg.copy_(g, non_blocking=True)
                    keep.append((I, c2, g))
                    outs.append(("grad", hc, hg))
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, outs, keep)

    def done(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle):
        ev, outs, _ = handle
        ev.synchronize()
        res = []
        for o in outs:
            if o[0] == "chi2":
                res.append((float(o[1][o[2]]), None))
            else:
                res.append((float(o[1]), o[2].numpy().copy()))
        return res
