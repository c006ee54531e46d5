"""Continuous-batching server for characteristic-profile requests.

A request is a hypergraph and its randomized copies (host CSRs); its answer is
their h-motif and 3h-motif counts, the significance (Eq. 1) and the
characteristic profile (Eq. 2), computed by one ``mochy_profile`` call.

The server keeps ``slots`` library contexts, each on its own HIP stream and
driven by its own worker thread (the library calls release the GIL).  A
waiting request is admitted as soon as a slot is free and its device-memory
bound fits in what the running requests leave of the budget, so requests that
arrive while others run start without waiting for them, and their kernels
overlap on the device.  A request's CSRs are uploaded once at admission and
stay resident until its answer is read back.
"""
from __future__ import annotations

import threading
import time
from collections import deque

import numpy as np

from . import _lib


def request_bytes(graphs) -> int:
    """Upper bound of the device memory a request holds while it runs.

    Per graph: incidence and transpose, per-row arrays, and the line graph
    (4-byte column + 16-byte record + 4-byte record mask + 2-byte size word per
    row entry, and the exact counting's neighbour groups, 24 bytes per row
    entry, with |wedges| bounded by sum_v C(deg(v), 2)).
    """
    total = 0
    for ptr, nodes, num_nodes in graphs:
        E = len(ptr) - 1
        nnz = int(ptr[-1]) if E > 0 else 0
        deg = np.bincount(np.asarray(nodes), minlength=int(num_nodes)).astype(np.int64)
        wedges = int((deg * (deg - 1) // 2).sum())
        total += 16 * (E + 1) + 8 * nnz + 9 * (int(num_nodes) + 1) + 40 * E + 2 * wedges * 50
    return total


class Admission:
    """Admission policy (host only).

    Waiting requests are kept in arrival order.  ``take`` scans them in order
    and starts each one whose memory bound fits in the budget left by the
    running requests, while slots remain.  Later requests may start ahead of
    an earlier one that does not fit (backfill) until that one has waited
    ``aging_s`` seconds; from then on nothing passes it.  A large request
    (bound above ``exclusive_frac`` of the budget) runs alone: it starts when
    nothing else runs, and nothing starts beside it, so that its context may
    keep the whole buffer-cache allowance (see CPServer).
    """

    def __init__(self, budget: int, aging_s: float = 1.0, exclusive_frac: float = 0.25):
        self.budget = int(budget)
        self.aging_s = float(aging_s)
        self.exclusive_bytes = float(exclusive_frac) * self.budget
        self.waiting: deque = deque()  # (rid, nbytes, t_enqueued)
        self.in_use = 0
        self.running = 0
        self.exclusive = False  # a large request is running alone

    def is_large(self, nbytes: int) -> bool:
        return nbytes > self.exclusive_bytes

    def add(self, rid, nbytes: int, now: float):
        self.waiting.append((rid, int(nbytes), now))

    def take(self, free_slots: int, now: float) -> list:
        started = []
        kept = deque()
        blocked = False
        while self.waiting:
            rid, nb, t0 = self.waiting.popleft()
            if free_slots == 0 or blocked or self.exclusive:
                kept.append((rid, nb, t0))
                continue
            alone = self.running == 0 and not started
            large = self.is_large(nb)
            fits = alone if large else (self.in_use + nb <= self.budget or alone)
            if fits:
                started.append((rid, nb))
                self.in_use += nb
                self.running += 1
                free_slots -= 1
                self.exclusive = large
            else:
                kept.append((rid, nb, t0))
                if now - t0 >= self.aging_s:
                    blocked = True  # an aged request: no backfill past it
        self.waiting = kept
        return started

    def release(self, nbytes: int):
        self.in_use -= int(nbytes)
        self.running -= 1
        if self.running == 0:
            self.exclusive = False


class Ticket:
    """Handle of a submitted request; ``wait()`` returns its result dict."""

    def __init__(self, rid, arrival: float):
        self.rid = rid
        self.arrival = arrival
        self.start = None
        self.done = None
        self.result = None
        self.error = None
        self._ev = threading.Event()

    def wait(self, timeout=None) -> dict:
        if not self._ev.wait(timeout):
            raise TimeoutError(f"request {self.rid} not finished")
        if self.error is not None:
            raise self.error
        return self.result

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class CPServer:
    """Serves profile requests on one device with ``slots`` concurrent streams."""

    def __init__(self, device: int = 0, slots: int = 4, budget_bytes: int | None = None,
                 eps: float = 1.0, aging_s: float = 1.0, cache_bytes: int | None = None):
        # device memory: budget_bytes for the admitted requests, and each
        # slot's context keeps at most cache_bytes of the buffers its requests
        # freed (by default 80 % and 20 % / slots of what is free now), so
        # that an idle slot's kept buffers never hold what admission hands
        # out.  A large request runs alone (Admission): its context may then
        # keep the whole allowance, slots * cache_bytes, after the idle
        # contexts give theirs back.  Its sub-batches free and allocate
        # buffers of tens of GB, and mapping them again costs: on 40 requests
        # of 1e3 to 2e5 hyperedges, one slot keeping 20 % of the memory served
        # 0.39 requests/s, keeping 5 % 0.23, and four slots 0.24 before large
        # requests took the whole allowance.
        if budget_bytes is None or cache_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info(device)
            if budget_bytes is None:
                budget_bytes = int(0.8 * free)
            if cache_bytes is None:
                cache_bytes = max(0, int(min(0.2 * free, free - budget_bytes) / slots))
        self.eps = float(eps)
        self._cache_small = int(cache_bytes)
        self._cache_large = int(cache_bytes) * slots
        self._ctxs = [_lib.Context(device) for _ in range(slots)]
        for c in self._ctxs:
            c.set_option(_lib.MOCHY_OPT_CACHE_BYTES, cache_bytes)
        self._adm = Admission(budget_bytes, aging_s)
        self._lock = threading.Lock()
        self._pending = {}            # rid -> (ticket, graphs, nbytes)
        self._free = list(range(slots))
        self._work = [None] * slots
        self._cv = [threading.Condition(self._lock) for _ in range(slots)]
        self._stop = False
        self._next = 0
        self._threads = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                         for s in range(slots)]
        for t in self._threads:
            t.start()

    def submit(self, graphs, arrival: float | None = None) -> Ticket:
        """graphs: [(edge_ptr, edge_nodes, num_nodes), ...], graphs[0] the hypergraph."""
        now = time.perf_counter()
        nbytes = request_bytes(graphs)
        with self._lock:
            rid = self._next
            self._next += 1
            t = Ticket(rid, now if arrival is None else arrival)
            self._pending[rid] = (t, list(graphs), nbytes)
            self._adm.add(rid, nbytes, now)
            self._dispatch(now)
        return t

    def _dispatch(self, now):
        # called with the lock held
        for rid, nb in self._adm.take(len(self._free), now):
            s = self._free.pop()
            self._work[s] = rid
            self._cv[s].notify()

    def _worker(self, s):
        ctx = self._ctxs[s]
        while True:
            with self._lock:
                while self._work[s] is None and not self._stop:
                    self._cv[s].wait()
                if self._stop and self._work[s] is None:
                    return
                rid = self._work[s]
                ticket, graphs, nbytes = self._pending.pop(rid)
            ticket.start = time.perf_counter()
            large = self._adm.is_large(nbytes) and len(self._ctxs) > 1
            try:
                if large:  # it runs alone: the idle contexts give their kept buffers back
                    for c in self._ctxs:
                        if c is not ctx:
                            c.set_option(_lib.MOCHY_OPT_CACHE_BYTES, 0)
                            c.set_option(_lib.MOCHY_OPT_CACHE_BYTES, self._cache_small)
                    ctx.set_option(_lib.MOCHY_OPT_CACHE_BYTES, self._cache_large)
                counts, sig26, cp26, sig431, cp431 = _lib.mochy_profile(ctx, graphs, self.eps)
                ticket.result = dict(counts=counts, sig26=sig26, cp26=cp26, sig431=sig431, cp431=cp431)
            except Exception as e:  # reported to the waiter
                ticket.error = e
            finally:
                if large:
                    ctx.set_option(_lib.MOCHY_OPT_CACHE_BYTES, self._cache_small)
            ticket.done = time.perf_counter()
            with self._lock:
                self._work[s] = None
                self._free.append(s)
                self._adm.release(nbytes)
                self._dispatch(time.perf_counter())
            ticket._ev.set()

    def apply_options(self, options: dict):
        """Sets {option: value} (e.g. a tuned launch shape) on every slot's
        context; call before submitting requests."""
        for c in self._ctxs:
            for opt, val in options.items():
                c.set_option(opt, val)

    def tune(self, graphs) -> dict:
        """Tunes the batched pass's launch shape on one representative request
        (``tune.tune_batch`` on the first slot) and applies it to every slot;
        call it before submitting requests (it uses a slot's context from the
        calling thread)."""
        from .tune import tune_batch
        res = tune_batch(self._ctxs[0], graphs)
        self.apply_options({_lib.MOCHY_OPT_BATCH_LAUNCH: res["launch"],
                            _lib.MOCHY_OPT_PAIR_BLOCKS: res["blocks"]})
        return res

    def close(self):
        with self._lock:
            self._stop = True
            for cv in self._cv:
                cv.notify_all()
        for t in self._threads:
            t.join()
        for c in self._ctxs:
            c.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
