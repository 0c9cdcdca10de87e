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
import heapq
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
    queued: bool = field(default=False, repr=False)   # waiting in the scheduler's queue

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
        self._deadlines = []         # heap of (deadline, seq, request) of queued requests
        self._seq = itertools.count()
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
        req.queued = True
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
        live = lambda r: r.queued and not r.future.cancelled()
        while self._run:
            progressed = False
            with self._lock:
                while self._in:
                    r = self._in.popleft()
                    self._pending.append(r)
                    if r.deadline is not None:
                        heapq.heappush(self._deadlines, (r.deadline, next(self._seq), r))
            now = time.perf_counter()
            # queued requests whose deadline passed fail before they take device
            # memory (a heap of deadlines: no pass over the whole queue)
            while self._deadlines and self._deadlines[0][0] < now:
                r = heapq.heappop(self._deadlines)[2]
                if live(r):
                    r.queued = False
                    _settle(r.future, exc=TimeoutError("deadline passed while queued"))
                    self.expired += 1
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
            while self._free_slots:
                while self._pending and not live(self._pending[0]):
                    self._pending.popleft().queued = False   # cancelled or expired
                if not self._pending:
                    break
                head = self._pending[0]
                if self.mixed:
                    group = list(itertools.islice((r for r in self._pending if live(r)),
                                                  self.max_batch))
                else:
                    key = head.key()
                    group = list(itertools.islice(
                        (r for r in self._pending if live(r) and r.key() == key), self.max_batch))
                try:
                    fp_one = self.ex.footprint([head])
                except Exception as e:  # a request the executor cannot plan
                    self._pending.popleft().queued = False
                    _settle(head.future, exc=e)
                    self.rejected += 1
                    continue
                if fp_one > self.budget:
                    self._pending.popleft().queued = False
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
                for r in group:
                    r.queued = False
                if self.mixed:         # the group was the queue's head
                    while self._pending and not self._pending[0].queued:
                        self._pending.popleft()
                else:
                    self._pending = collections.deque(r for r in self._pending if r.queued)
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
    """Pinned host staging of one in-flight slot, grown on demand: ``h_in``
    holds the models and geometry rows laid out as in the device buffer,
    ``h_out`` the chi^2 values and gradients, so that each direction is one
    copy.  Host memory only: the device buffer of a micro-batch is allocated
    per launch (see GpuExecutor)."""

    def __init__(self, torch):
        self.torch = torch
        self.cap = (0, 0)

    def grow(self, n_in, n_out):
        torch = self.torch
        if n_in <= self.cap[0] and n_out <= self.cap[1]:
            return
        n_in, n_out = max(n_in, self.cap[0], 256), max(n_out, self.cap[1], 256)
        self.h_in = torch.empty(n_in, dtype=torch.uint8, pin_memory=True)
        self.h_out = torch.empty(n_out, dtype=torch.uint8, pin_memory=True)
        self.in_np, self.out_np = self.h_in.numpy(), self.h_out.numpy()
        self.cap = (n_in, n_out)


class _Layout:
    """Byte layout of one micro-batch's device buffer for a request signature:
    [batch_exec workspace | models | geometry rows | chi^2 | gradients], the
    workspace size being the library planner's own figure for the call."""

    def __init__(self, ex, sig):
        from . import JOB_PROFILE

        K = len(sig)
        nr = np.array([s[3] for s in sig], dtype=np.int64)
        grad = np.array([s[4] for s in sig], dtype=bool)
        specs = [(ex.datasets[s[0]], JOB_PROFILE, s[1], s[2], s[3], s[4]) for s in sig]
        self.K, self.el = K, ex.el
        self.ws = _al(ex._ws_bytes(specs))
        self.mo = np.concatenate([[0], np.cumsum(nr)]).astype(np.int64)   # model offsets
        n_model = int(self.mo[-1])
        gof = np.concatenate([[0], np.cumsum(np.where(grad, nr, 0))]).astype(np.int64)
        self.n_grad = int(gof[-1])
        self.goff = np.where(grad, gof[:-1], -1)                           # gradient offsets
        self.nr, self.grad = nr, grad
        self.o_model = self.ws
        self.o_geo = self.o_model + _al(self.el * n_model)
        self.o_chi2 = self.o_geo + _al(48 * K)
        self.o_grad = self.o_chi2 + _al(8 * K)
        self.total = self.o_grad + _al(self.el * max(self.n_grad, 1))
        # the gal_job table: everything but the device addresses, filled per launch
        self.jobs = np.zeros(K, dtype=ex._job_dtype)
        self.jobs["ds"] = [ex.datasets[s[0]]._h.value for s in sig]
        self.jobs["kind"] = JOB_PROFILE
        self.jobs["Nxy"] = [s[1] for s in sig]
        self.jobs["dxy"] = [s[2] for s in sig]
        self.jobs["Nr"] = nr
        self.rel_model = self.o_model + self.el * self.mo[:-1]
        self.rel_geo = self.o_geo + 48 * np.arange(K, dtype=np.int64)
        self.rel_grad = np.where(grad, self.o_grad + self.el * np.maximum(self.goff, 0), 0)


class GpuExecutor:
    """HIP executor: datasets resident in HBM, one stream and pinned staging
    per in-flight slot, one gal_batch_exec call per micro-batch (any mix of
    requests, gradients included).

    Device memory: each micro-batch gets one buffer of exactly
    ``footprint(reqs)`` bytes -- the batch_exec workspace that the library's
    planner computes for its job list, then the models, geometry rows, chi^2
    and gradient outputs -- taken on the slot's stream when it is launched and
    released when its results are collected.  The scheduler's count of bytes
    in flight is therefore the device memory the micro-batches hold.

    Host cost per micro-batch: the layout of a request signature (datasets,
    grids, profile lengths, gradient flags) is planned once and cached; a
    launch fills one pinned staging buffer, makes one copy to the device, one
    library call with a job table built from the cached layout, and one copy
    back.  The workspace's status word is not read here (a request whose
    geometry fails the device checks gets a NaN chi^2)."""

    mixed_batches = True

    def __init__(self, device=None, dtype=None, max_batch: int = 16, max_inflight: int = 4,
                 layout_cache: int = 4096):
        import ctypes

        import torch

        from . import Dataset, _lib, _native, exec_workspace_bytes

        self.torch = torch
        self._Dataset, self._ws_bytes = Dataset, exec_workspace_bytes
        self._lib, self._check = _lib, _native.check
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.dtype = torch.float64 if dtype is None else dtype
        self.np_dtype = np.float64 if self.dtype == torch.float64 else np.float32
        self.el = 8 if self.dtype == torch.float64 else 4
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.slots = [_Slot(torch) for _ in range(max_inflight)]
        self.datasets = {}
        self._layouts = collections.OrderedDict()
        self._layout_cap = int(layout_cache)
        G = _native.GalJob
        names = [f[0] for f in G._fields_]
        fmt = {"ds": np.uint64, "model": np.uint64, "geo": np.uint64, "vis": np.uint64,
               "dxy": np.float64}
        self._job_dtype = np.dtype({"names": names,
                                    "formats": [fmt.get(n, np.int32) for n in names],
                                    "offsets": [getattr(G, n).offset for n in names],
                                    "itemsize": ctypes.sizeof(G)})

    def default_budget(self) -> int:
        free, total = self.torch.cuda.mem_get_info(self.device)
        return int(0.8 * free)

    def bind_thread(self):
        self.torch.cuda.set_device(self.device)

    def add_dataset(self, name, u, v, re, im, w):
        t = lambda a: self.torch.as_tensor(np.ascontiguousarray(a), dtype=self.dtype,
                                           device=self.device)
        self.datasets[name] = self._Dataset(t(u), t(v), t(re), t(im), t(w))
        self._layouts.clear()
        return self.datasets[name]

    def layout(self, reqs) -> _Layout:
        """The micro-batch's buffer layout (cached per request signature)."""
        sig = tuple(r.key() for r in reqs)
        L = self._layouts.get(sig)
        if L is None:
            L = _Layout(self, sig)
            self._layouts[sig] = L
            if len(self._layouts) > self._layout_cap:
                self._layouts.popitem(last=False)
        return L

    def footprint(self, reqs) -> int:
        """Device bytes a micro-batch holds while in flight (exact)."""
        return self.layout(reqs).total

    def launch(self, reqs, slot):
        torch = self.torch
        st, S = self.streams[slot], self.slots[slot]
        L = self.layout(reqs)
        n_in, n_out = L.o_chi2 - L.o_model, L.total - L.o_chi2
        S.grow(n_in, n_out)
        hm = S.in_np[: L.el * int(L.mo[-1])].view(self.np_dtype)
        hg = S.in_np[L.o_geo - L.o_model: L.o_geo - L.o_model + 48 * L.K].view(np.float64)
        hg = hg.reshape(L.K, 6)
        models = [r.I.detach().cpu().numpy() if torch.is_tensor(r.I) else r.I for r in reqs]
        np.concatenate(models, out=hm, casting="same_kind")
        hg[:] = [(r.Rmin, r.dR, r.inc, r.PA, r.dRA, r.dDec) for r in reqs]
        with torch.cuda.stream(st):
            buf = torch.empty(L.total, dtype=torch.uint8, device=self.device)
            buf[L.o_model:L.o_chi2].copy_(S.h_in[:n_in], non_blocking=True)
            base = buf.data_ptr()
            jobs = L.jobs.copy()
            jobs["model"] = base + L.rel_model
            jobs["geo"] = base + L.rel_geo
            grads = None
            if L.n_grad:
                grads = np.where(L.grad, base + L.rel_grad, 0).astype(np.uint64)
            self._check(self._lib().gal_batch_exec(
                jobs.ctypes.data, L.K, base + L.o_chi2,
                None if grads is None else grads.ctypes.data, base, L.ws,
                st.cuda_stream), "serve launch")
            S.h_out[:n_out].copy_(buf[L.o_chi2:L.total], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        return [ev, S, L, buf]

    def done(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle):
        ev, S, L = handle[:3]
        ev.synchronize()
        handle[3] = None   # the micro-batch's device buffer goes back to the allocator
        c = S.out_np[: 8 * L.K].view(np.float64)
        g0 = L.o_grad - L.o_chi2
        g = S.out_np[g0: g0 + L.el * max(L.n_grad, 1)].view(self.np_dtype)
        return [(float(c[k]), None if L.goff[k] < 0 else g[L.goff[k]:L.goff[k] + L.nr[k]].copy())
                for k in range(L.K)]
