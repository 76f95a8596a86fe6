"""Continuous-batching request loop over device-resident models (the serving form).

Requests arrive at any time and are queued in arrival order.  Each call to ``Server.poll``
retires the requests whose device work has finished and admits queued ones (in arrival order
within each kind, so a waiting fit does not hold back assign requests) while

  * the HBM budget allows (every admitted request holds its workspace and outputs,
    counted from the library's ``*_workspace_bytes`` and the output sizes), and
  * a slot is free (``assign_slots`` assign launches in flight, spread over that many HIP
    streams; ``fit_workers`` fits, each on its own stream and host thread, because
    ``kkm_fit`` returns host data and therefore waits for its stream).

A request's rows may still be in production on the submitter's stream when it is submitted: the
backend marks that point of the stream at submission (``mark_ready``), and the server stream that
takes the request waits for the mark before reading the rows, which are also recorded on it so that
their memory is not reused while it reads them.

Small assign requests for the same model that are queued together are coalesced into one
``kkm_assign`` launch (rows concatenated, labels split back): every row's label depends only on
that row and the model, so a request's labels are the same alone and in a batch.  Work admitted
on different streams overlaps on the device.  Models stay resident in HBM between requests; a
fit request can register its result as a new model.

The scheduling logic talks to a backend; ``KkmBackend`` drives the HIP library, and tests may
substitute a host-only backend with the same methods.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

__all__ = ["Request", "Server", "KkmBackend"]


@dataclass(eq=False)
class Request:
    kind: str                      # "assign" | "fit"
    arrival: float                 # host clock (time.perf_counter) at submission
    model: Optional[str] = None    # assign: model name
    X: Any = None                  # device rows (assign: n x d, fit: N x d)
    n: int = 0
    fit_kwargs: Dict[str, Any] = field(default_factory=dict)
    register_as: Optional[str] = None
    admitted: Optional[float] = None
    finished: Optional[float] = None
    result: Any = None
    error: Optional[BaseException] = None
    mem: int = 0
    ready: Any = None              # backend mark of the point where X is complete (or None)

    @property
    def done(self) -> bool:
        return self.finished is not None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class KkmBackend:
    """Backend over the HIP library: assign launches on a pool of streams, fits on worker threads."""

    def __init__(self, n_streams: int, precision: str = "fp32", device: int = 0):
        import torch
        from . import kkm_assign, kkm_assign_workspace_bytes, kkm_fit, kkm_fit_workspace_bytes
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_streams)]
        self.precision = precision
        self._assign, self._assign_ws = kkm_assign, kkm_assign_workspace_bytes
        self._fit, self._fit_ws = kkm_fit, kkm_fit_workspace_bytes

    # ---- memory estimates (bytes held while the request is in flight)
    def assign_bytes(self, model, rows: int, concatenated: bool) -> int:
        ws = self._assign_ws(model, max(1, rows), self.precision)
        concat = rows * model.d * 4 if concatenated else 0
        return ws + 4 * rows + concat

    def fit_bytes(self, X, kw) -> int:
        from . import _kernel, _dtype_code, lib, _params
        import ctypes as ct
        N, d = X.shape
        k = _kernel(kw.get("kernel", "rbf"), kw.get("sigma", 1.0), kw.get("n_atoms", 0))
        keep = []
        p = _params(kw.get("C", 2), kw.get("B", 1), kw.get("s", 1.0), kw.get("max_iter", 20),
                    kw.get("sampling", "stride"), kw.get("init", "kmeans++"), kw.get("precision", self.precision),
                    kw.get("seed", 0), kw.get("landmarks"), kw.get("kmpp_uniforms"), kw.get("init_labels"),
                    kw.get("init_medoids"), keep)
        ws = int(lib().kkm_fit_workspace_bytes(N, d, _dtype_code(X), ct.byref(k), ct.byref(p)))
        C = kw.get("C", 2)
        model = (C + 32) * (d * 4 + 64) + 4096
        return ws + model + 4 * N

    # ---- ordering with the submitter's stream
    def mark_ready(self, X):
        """An event recorded on the submitter's current stream: X is complete once it has fired."""
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(X.device))
        return ev

    def _take(self, s, xs, ready):
        for x, ev in zip(xs, ready or [None] * len(xs)):
            if ev is not None:
                s.wait_event(ev)
            x.record_stream(s)

    # ---- assign
    def launch_assign(self, model, xs: List[Any], slot: int, ready: Optional[List[Any]] = None):
        torch = self.torch
        s = self.streams[slot % len(self.streams)]
        self._take(s, xs, ready)
        with torch.cuda.stream(s):
            X = xs[0] if len(xs) == 1 else torch.cat(xs, 0)
            labels = self._assign(model, X, precision=self.precision, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"ev": ev, "labels": labels, "sizes": [x.shape[0] for x in xs], "X": X}

    def assign_done(self, h) -> bool:
        return h["ev"].query()

    def assign_results(self, h) -> List[Any]:
        out, o = [], 0
        for n in h["sizes"]:
            out.append(h["labels"][o:o + n])
            o += n
        return out

    # ---- fit (its own stream and host thread)
    def start_fit(self, X, kw, slot: int, ready: Optional[List[Any]] = None):
        torch = self.torch
        s = torch.cuda.Stream(device=self.dev)
        self._take(s, [X], ready)
        box: Dict[str, Any] = {}

        def run():
            try:
                with torch.cuda.stream(s):
                    # other streams keep the device busy meanwhile: the kernels whose workgroups wait
                    # for each other are launched cooperatively
                    box["result"] = self._fit(X, stream=s, **{"cooperative": True, **kw})
            except BaseException as e:   # reported on the request
                box["error"] = e

        t = threading.Thread(target=run, daemon=True)
        t.start()
        return {"thread": t, "box": box, "stream": s}

    def fit_done(self, h) -> bool:
        return not h["thread"].is_alive()

    def fit_result(self, h):
        if "error" in h["box"]:
            raise h["box"]["error"]
        return h["box"]["result"]


class Server:
    """Arrival-ordered admission by HBM budget and free slots; retires finished work on ``poll``."""

    def __init__(self, backend, budget_bytes: int, assign_slots: int = 4, fit_workers: int = 2,
                 batch_max_rows: int = 65536, batch_small_rows: int = 4096,
                 clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.assign_slots = assign_slots
        self.fit_workers = fit_workers
        self.batch_max_rows = batch_max_rows
        self.batch_small_rows = batch_small_rows
        self.clock = clock
        self.models: Dict[str, Any] = {}
        self.queue: collections.deque = collections.deque()
        self.running: List[tuple] = []      # (kind, handle, [requests], mem, slot)
        self.in_use = 0
        self.peak_in_use = 0
        self.budget_waits = 0               # admission passes in which the budget held a request back
        self._slot = 0
        self.launches = 0

    # ---- models and submission
    def add_model(self, name: str, model) -> None:
        self.models[name] = model

    def submit_assign(self, model: str, X, arrival: Optional[float] = None) -> Request:
        if model not in self.models:
            raise KeyError(f"unknown model {model!r}")
        r = Request("assign", self.clock() if arrival is None else arrival, model=model, X=X, n=int(X.shape[0]))
        r.ready = self._mark(X)
        self.queue.append(r)
        return r

    def _mark(self, X):
        mark = getattr(self.backend, "mark_ready", None)
        return mark(X) if mark is not None else None

    def submit_fit(self, X, register_as: Optional[str] = None, arrival: Optional[float] = None, **fit_kwargs) -> Request:
        r = Request("fit", self.clock() if arrival is None else arrival, X=X, n=int(X.shape[0]),
                    fit_kwargs=fit_kwargs, register_as=register_as)
        r.ready = self._mark(X)
        self.queue.append(r)
        return r

    # ---- the loop
    def _n_running(self, kind: str) -> int:
        return sum(1 for t in self.running if t[0] == kind)

    def _retire(self) -> int:
        now = None
        keep, done = [], 0
        for kind, h, reqs, mem, slot in self.running:
            fin = self.backend.assign_done(h) if kind == "assign" else self.backend.fit_done(h)
            if not fin:
                keep.append((kind, h, reqs, mem, slot))
                continue
            now = self.clock()
            if kind == "assign":
                for r, lab in zip(reqs, self.backend.assign_results(h)):
                    r.result, r.finished = lab, now
            else:
                r = reqs[0]
                try:
                    r.result = self.backend.fit_result(h)
                    if r.register_as is not None:
                        self.models[r.register_as] = r.result[0]
                except BaseException as e:
                    r.error = e
                r.finished = now
            self.in_use -= mem
            done += len(reqs)
        self.running = keep
        return done

    def _admit(self) -> int:
        """Admit queued requests in arrival order within each kind: a fit waiting for a worker or for
        memory does not hold back the assign requests behind it, and vice versa."""
        admitted = 0
        blocked = set()          # kinds that cannot admit more in this pass
        i = 0
        while i < len(self.queue) and len(blocked) < 2:
            head = self.queue[i]
            if head.kind in blocked:
                i += 1
                continue
            if head.kind == "fit":
                if self._n_running("fit") >= self.fit_workers:
                    blocked.add("fit")
                    continue
                mem = self.backend.fit_bytes(head.X, head.fit_kwargs)
                if mem > self.budget:
                    del self.queue[i]
                    head.error = MemoryError(f"fit needs {mem} B, budget {self.budget} B")
                    head.finished = self.clock()
                    continue
                if self.in_use + mem > self.budget:
                    self.budget_waits += 1
                    blocked.add("fit")
                    continue
                del self.queue[i]
                h = self.backend.start_fit(head.X, head.fit_kwargs, self._slot, ready=[head.ready])
                group = [head]
                kind = "fit"
            else:
                if self._n_running("assign") >= self.assign_slots:
                    blocked.add("assign")
                    continue
                # coalesce small queued requests of the same model, in arrival order, as long as
                # the group stays within the row cap and the whole budget
                model = self.models[head.model]
                mem = self.backend.assign_bytes(model, head.n, False)
                if mem > self.budget:
                    del self.queue[i]
                    head.error = MemoryError(f"assign needs {mem} B, budget {self.budget} B")
                    head.finished = self.clock()
                    continue
                group = [head]
                rows = head.n
                if head.n < self.batch_small_rows:
                    for j in range(i + 1, len(self.queue)):
                        r = self.queue[j]
                        if r.kind != "assign" or r.model != head.model or r.n >= self.batch_small_rows:
                            continue
                        if rows + r.n > self.batch_max_rows:
                            break
                        m2 = self.backend.assign_bytes(model, rows + r.n, True)
                        if m2 > self.budget:
                            break
                        group.append(r)
                        rows += r.n
                        mem = m2
                if self.in_use + mem > self.budget:
                    self.budget_waits += 1
                    blocked.add("assign")
                    continue
                ids = {id(r) for r in group}
                self.queue = collections.deque(r for r in self.queue if id(r) not in ids)
                h = self.backend.launch_assign(model, [r.X for r in group], self._slot,
                                               ready=[r.ready for r in group])
                kind = "assign"
            now = self.clock()
            for r in group:
                r.admitted, r.mem = now, mem
            self.running.append((kind, h, group, mem, self._slot))
            self._slot += 1
            self.in_use += mem
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.launches += 1
            admitted += len(group)
        return admitted

    def poll(self) -> int:
        """Retire finished work, then admit what fits.  Returns the number of requests retired."""
        done = self._retire()
        self._admit()
        return done

    @property
    def idle(self) -> bool:
        return not self.queue and not self.running

    def run_until_idle(self, timeout: float = 600.0) -> None:
        t_end = self.clock() + timeout
        while not self.idle:
            self.poll()
            if self.clock() > t_end:
                raise TimeoutError("serving loop did not drain")
