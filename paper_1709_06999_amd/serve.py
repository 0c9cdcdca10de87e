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
 - Batching.  An executor that evaluates mixed job lists (``mixed_batches``
   true, as ``GpuExecutor``) receives the queue's oldest requests in arrival
   order, whatever their datasets, grids, profile lengths and gradient
   flags: one micro-batch is one batch_exec call (FFTs of equal shape share
   launches, requests on one dataset share its pass over the uv data, the
   gradient requests add the adjoint passes).  Other executors receive
   requests of one key (dataset, grid, profile length, gradient flag).
 - Deadlines and cancellation.  A request whose deadline passes while it is
   queued fails with TimeoutError; a cancelled future is dropped.
 - Latency is completion minus arrival on the host clock (time.perf_counter).

The scheduler itself is host logic and takes any executor with the
``footprint / launch / done / collect`` interface; ``GpuExecutor`` is the
HIP one.
"""
from __future__ import annotations

import collections
import itertools
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
        self.mixed = bool(getattr(executor, "mixed_batches", False))
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
        self.launch_s = 0.0          # host time spent in executor.launch
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

    def reset_stats(self):
        """Start the counters afresh (e.g. after a warm-up phase)."""
        self.latencies = []
        self.completed = self.rejected = self.expired = self.batches = 0
        self.launch_s = 0.0
        self.peak_used = self._used
        self._t_first = None
        self._t_last = None

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
            "host_launch_ms_per_batch": 1e3 * self.launch_s / max(self.batches, 1),
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
                if self.mixed:
                    group = list(itertools.islice(self._pending, self.max_batch))
                else:
                    key = head.key()
                    group = [r for r in self._pending if r.key() == key][: self.max_batch]
                try:
                    fp_one = self.ex.footprint([head])
                except Exception as e:  # a request the executor cannot plan
                    self._pending.popleft()
                    _settle(head.future, exc=e)
                    self.rejected += 1
                    continue
                if fp_one > self.budget:
                    self._pending.popleft()
                    _settle(head.future, exc=MemoryError(
                        f"request needs {fp_one} bytes of device memory, budget {self.budget}"))
                    self.rejected += 1
                    continue
                fp = None
                while group:
                    try:
                        fp = self.ex.footprint(group)
                    except Exception:  # a later member fails alone when it is the head
                        fp = None
                    if fp is not None and fp <= self.budget - self._used:
                        break
                    group.pop()
                if not group:
                    break              # wait for memory to free up
                ids = set(id(r) for r in group)
                self._pending = collections.deque(r for r in self._pending if id(r) not in ids)
                slot = self._free_slots.pop()
                t0 = time.perf_counter()
                try:
                    handle = self.ex.launch(group, slot)
                except Exception as e:  # launch errors go to the callers
                    for r in group:
                        _settle(r.future, exc=e)
                    self._free_slots.append(slot)
                    continue
                self.launch_s += time.perf_counter() - t0
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


def _al(n: int) -> int:
    return (int(n) + 255) & ~255


class _Slot:
    """Pinned host staging of one in-flight slot (models, geometry rows, chi^2
    and gradient outputs), grown on demand.  Host memory only: the device
    buffers of a micro-batch are allocated per launch (see GpuExecutor)."""

    def __init__(self, torch, dtype):
        self.torch, self.dtype = torch, dtype
        self.cap = (0, 0, 0)

    def grow(self, K, n_model, n_grad):
        torch = self.torch
        if K <= self.cap[0] and n_model <= self.cap[1] and n_grad <= self.cap[2]:
            return
        K = max(K, self.cap[0])
        n_model = max(n_model, self.cap[1], 1)
        n_grad = max(n_grad, self.cap[2], 1)
        pin = dict(pin_memory=True)
        self.h_model = torch.empty(n_model, dtype=self.dtype, **pin)
        self.h_geo = torch.empty((K, 6), dtype=torch.float64, **pin)
        self.h_chi2 = torch.empty(K, dtype=torch.float64, **pin)
        self.h_grad = torch.empty(n_grad, dtype=self.dtype, **pin)
        self.cap = (K, n_model, n_grad)


class GpuExecutor:
    """HIP executor: datasets resident in HBM, one stream and pinned staging
    per in-flight slot, one batch_exec call per micro-batch (any mix of
    requests, gradients included).

    Device memory: each micro-batch gets one buffer of exactly
    ``footprint(reqs)`` bytes -- the batch_exec workspace that the library's
    planner computes for its job list, then the models, geometry rows, chi^2
    and gradient outputs -- taken on the slot's stream when it is launched and
    released when its results are collected.  The scheduler's count of bytes
    in flight is therefore the device memory the micro-batches hold."""

    mixed_batches = True

    def __init__(self, device=None, dtype=None, max_batch: int = 16, max_inflight: int = 4):
        import torch

        from . import JOB_PROFILE, Dataset, Workspace, batch_exec, exec_workspace_bytes

        self.torch = torch
        self._Dataset, self._batch_exec, self._JOB_PROFILE = Dataset, batch_exec, JOB_PROFILE
        self._Workspace, self._ws_bytes = Workspace, exec_workspace_bytes
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.dtype = torch.float64 if dtype is None else dtype
        self.el = 8 if self.dtype == torch.float64 else 4
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.slots = [_Slot(torch, self.dtype) for _ in range(max_inflight)]
        self.datasets = {}

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

    def layout(self, reqs):
        """Byte offsets of the parts of a micro-batch's device buffer:
        (workspace bytes, model offset, geo offset, chi2 offset, grad offset,
        total).  The workspace size is the planner's own figure for the
        batch_exec call the launch makes."""
        nr = [int(np.size(r.I)) for r in reqs]
        specs = [(self.datasets[r.dataset], self._JOB_PROFILE, int(r.Nxy), float(r.dxy), n,
                  bool(r.grad)) for r, n in zip(reqs, nr)]
        ws = _al(self._ws_bytes(specs))
        K, n_model = len(reqs), sum(nr)
        n_grad = sum(n for n, r in zip(nr, reqs) if r.grad)
        o_model = ws
        o_geo = o_model + _al(self.el * n_model)
        o_chi2 = o_geo + _al(48 * K)
        o_grad = o_chi2 + _al(8 * K)
        total = o_grad + _al(self.el * max(n_grad, 1))
        return ws, o_model, o_geo, o_chi2, o_grad, total

    def footprint(self, reqs) -> int:
        """Device bytes a micro-batch holds while in flight (exact)."""
        return self.layout(reqs)[-1]

    def launch(self, reqs, slot):
        torch = self.torch
        st, S = self.streams[slot], self.slots[slot]
        K = len(reqs)
        nr = [int(np.size(r.I)) for r in reqs]
        mo = np.concatenate([[0], np.cumsum(nr)]).astype(np.int64)
        n_grad = sum(n for n, r in zip(nr, reqs) if r.grad)
        S.grow(K, int(mo[-1]), n_grad)
        hm, hg = S.h_model.numpy(), S.h_geo.numpy()
        for k, r in enumerate(reqs):
            I = r.I.detach().cpu().numpy() if torch.is_tensor(r.I) else np.asarray(r.I)
            hm[mo[k]:mo[k + 1]] = I
            hg[k] = (r.Rmin, r.dR, r.inc, r.PA, r.dRA, r.dDec)
        ws_b, o_model, o_geo, o_chi2, o_grad, total = self.layout(reqs)
        with torch.cuda.stream(st):
            buf = torch.empty(total, dtype=torch.uint8, device=self.device)
            view = lambda o, n, dt: buf[o:o + n * (8 if dt == torch.float64 else 4)].view(dt)
            d_model = view(o_model, int(mo[-1]), self.dtype)
            d_geo = view(o_geo, 6 * K, torch.float64).view(K, 6)
            d_chi2 = view(o_chi2, K, torch.float64)
            d_grad = view(o_grad, max(n_grad, 1), self.dtype)
            ws = self._Workspace(self.device, torch.float64)
            ws.buf = buf[:ws_b]
            ws.buf[:256].zero_()   # the control block (status flag)
            jobs, grads, goff = [], [], []
            g0 = 0
            for k, r in enumerate(reqs):
                jobs.append({"ds": self.datasets[r.dataset], "kind": self._JOB_PROFILE,
                             "Nxy": int(r.Nxy), "dxy": float(r.dxy),
                             "model": d_model[mo[k]:mo[k + 1]], "geo": d_geo[k]})
                if r.grad:
                    grads.append(d_grad[g0:g0 + nr[k]])
                    goff.append(g0)
                    g0 += nr[k]
                else:
                    grads.append(None)
                    goff.append(-1)
            d_model.copy_(S.h_model[:mo[-1]], non_blocking=True)
            d_geo.copy_(S.h_geo[:K], non_blocking=True)
            self._batch_exec(jobs, grads if n_grad else None, out=d_chi2, ws=ws)
            S.h_chi2[:K].copy_(d_chi2, non_blocking=True)
            if n_grad:
                S.h_grad[:n_grad].copy_(d_grad[:n_grad], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return [ev, S, nr, goff, buf]

    def done(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle):
        ev, S, nr, goff = handle[:4]
        ev.synchronize()
        handle[4] = None   # the micro-batch's device buffer goes back to the allocator
        c, g = S.h_chi2.numpy(), S.h_grad.numpy()
        return [(float(c[k]), None if goff[k] < 0 else g[goff[k]:goff[k] + nr[k]].copy())
                for k in range(len(nr))]
