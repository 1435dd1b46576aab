"""Continuous-batching solve server on one GPU.

Requests (one planted (l, d) instance each) arrive at any time.  A request is
admitted when its device memory (raw rows, bit-plane window table and output
reservation) fits the memory budget; its rows are uploaded once and its
windows built on the device, and it stays resident until it completes.
The server then runs *steps*: each step is one persistent search launch
(``pms_step_launch``) over work items cut from every admitted request's
remaining candidate range, so requests that arrive while others are on the
GPU join the next step and their work overlaps on the device.  Up to two
steps are in flight on the server's stream.

Each admitted request owns a slot in a device-resident instance table and
state table.  Its survivors are appended to its own output buffer at its
slot's running count, so a request's output is contiguous across steps.  When
its last item has completed the codes are copied back and sorted; if the
count exceeded the reservation, the request is re-run once with the exact
capacity.  torch provides device memory, pinned staging and the stream; all
computation runs in the library's kernels.
"""
from __future__ import annotations

import collections
import ctypes
import concurrent.futures as cf
import dataclasses
import math
import threading
import time
from typing import Deque, Dict, List, Optional

import numpy as np

from . import native as nat

MAX_SLOTS = 1024
ITEMS_UNTRACKED = 1 << 31  # serving does not use per-instance completion stamps
EAGER_CODES = 1 << 16      # least codes copied back right after a request's last step


def _estimate(l: int, d: int, n: int, t: int):
    """(expected |M|, expected sequence scans per candidate) under uniform background."""
    ball = sum(math.comb(l, k) * 3 ** k for k in range(d + 1))
    p = ball / 4 ** l
    nw = t - l + 1
    ps = 1.0 - (1.0 - p) ** nw
    ev = sum(ps ** k for k in range(n))
    return 4 ** l * ps ** n + 1.0, ev


@dataclasses.dataclass
class Result:
    motifs: np.ndarray          # sorted uint32 codes
    count: int
    arrival: float              # perf_counter seconds
    admitted: float
    finished: float
    steps: int
    reruns: int
    visits: int
    launched: float = 0.0       # its first step launched
    retired: float = 0.0        # its last step seen complete by the server

    @property
    def latency_s(self) -> float:
        return self.finished - self.arrival


class _Req:
    __slots__ = ("rid", "seqs", "l", "d", "n", "t", "arrival", "future", "slot", "dev_seqs",
                 "dev_win", "dev_out", "cap", "bytes", "total", "cursor", "inflight", "steps",
                 "reruns", "admitted", "cost_per_cand", "stride", "h_out", "failed",
                 "launched", "retired", "est_m")

    def __init__(self, rid, seqs, l, d, arrival, future):
        self.rid = rid
        self.seqs = seqs
        self.l, self.d = l, d
        self.n, self.t = seqs.shape
        self.arrival = arrival
        self.future = future
        self.slot = -1
        self.dev_seqs = self.dev_win = self.dev_out = None
        self.stride = nat.window_stride(self.t, l, nat.LAYOUT_BITSLICED) if l >= 2 else 0
        est_m, ev = _estimate(l, d, self.n, self.t)
        self.est_m = est_m
        self.cap = int(min(4 ** l, 8 * est_m + 4096))
        self.cost_per_cand = (self.t - l + 1) * ev
        self.total = 4 ** l
        self.cursor = 0
        self.inflight = 0
        self.steps = 0
        self.reruns = 0
        self.admitted = 0.0
        self.h_out = None   # pinned copy of the first codes, made right after the last step
        self.failed = False  # its future holds an error; slot kept until its steps retire
        self.launched = 0.0
        self.retired = 0.0
        self.bytes = self._bytes()

    def _bytes(self) -> int:
        return self.n * self.t + self.n * self.stride * 4 + self.cap * 4


class _PinnedRing:
    """Pinned staging slots reused in turn for host-to-device copies on one
    stream: a slot is refilled only after the copy that last read it has run
    (its event), so no request pays for a pinned allocation."""

    def __init__(self, torch, slots: int, slot_bytes: int):
        self.torch = torch
        self.slot_bytes = slot_bytes
        self.buf = torch.zeros(slots * slot_bytes, dtype=torch.uint8).pin_memory()
        self.host = self.buf.numpy()
        self.events = [torch.cuda.Event() for _ in range(slots)]
        self.pending = [False] * slots
        self.next = 0

    def stage(self, data):
        """A pinned uint8 tensor holding `data` (bytes or a uint8 array; None
        if it does not fit a slot)."""
        size = len(data)
        if size > self.slot_bytes:
            return None, None
        k = self.next
        self.next = (k + 1) % len(self.events)
        if self.pending[k]:
            self.events[k].synchronize()
        at = k * self.slot_bytes
        self.host[at:at + size] = np.frombuffer(data, dtype=np.uint8) if isinstance(data, bytes) else data
        return self.buf[at:at + size], k

    def used(self, k, stream):
        """Marks slot k as read by the copies just queued on `stream`."""
        if k is None:
            return
        self.events[k].record(stream)
        self.pending[k] = True


class _PinnedPool:
    """Pinned int32 buffers in power-of-two sizes, handed back once their
    codes have been copied out, so finishing requests allocate no pinned
    memory once the pool holds their sizes."""

    def __init__(self, torch):
        self.torch = torch
        self.free: Dict[int, List] = {}

    def get(self, count: int):
        size = 1 << max(12, (max(count, 1) - 1).bit_length())
        lst = self.free.get(size)
        if lst:
            return lst.pop()
        return self.torch.empty(size, dtype=self.torch.int32, pin_memory=True)

    def put(self, buf):
        if buf is not None:
            self.free.setdefault(buf.numel(), []).append(buf)


_STATE_DTYPE = np.dtype([("count", "<u8"), ("visits", "<u8"), ("t_done", "<u8"),
                         ("items_left", "<u4"), ("reserved", "<u4")])


class _StepBuf:
    """Pinned staging and device copies of one step's tables."""

    def __init__(self, torch, dev, max_items: int):
        self.max_items = max_items
        self.h_work = torch.zeros(max_items * 16, dtype=torch.uint8).pin_memory()
        self.d_work = torch.zeros(max_items * 16, dtype=torch.uint8, device=dev)
        self.d_ctr = torch.zeros(ctypes.sizeof(nat.DevCounters) // 8, dtype=torch.int64, device=dev)
        self.h_ctr = torch.zeros(ctypes.sizeof(nat.DevCounters) // 8, dtype=torch.int64).pin_memory()
        self.h_state = torch.zeros(MAX_SLOTS * 32, dtype=torch.uint8).pin_memory()
        # Recorded again by every launch of this buffer (it is only reused
        # after the step that recorded them has retired).
        self.start = torch.cuda.Event(enable_timing=True)
        self.event = torch.cuda.Event(enable_timing=True)   # end of the search launch
        self.done = torch.cuda.Event()                      # state snapshot copied to the host
        self.launched = 0.0         # host time of the launch (step watchdog)
        self.compares = 0.0         # estimated window compares of the step
        self.budget = 0.0           # the step's budget when it was built
        self.reqs: List[_Req] = []
        self.items_per_req: Dict[int, int] = {}


class StepTimeout(RuntimeError):
    """A step did not complete within the server's step timeout."""


class Server:
    """Continuous-batching server.  ``submit`` returns a Future of ``Result``.

    Failures: a request whose window table cannot be built fails alone; a
    step whose launch fails, or whose kernel reports an error (an instance it
    could not run), fails the requests it held and the server goes on with
    the others.  A step that has not completed ``step_timeout_s`` after it
    was launched fails every pending request with ``StepTimeout`` and stops
    the server: the device queue is then blocked behind that step.
    """

    def __init__(self, mem_budget: int = 256 << 20, step_ms: float = 2.0,
                 max_inflight: int = 2, compares_per_s: float = 2.5e14,
                 device: int = 0, config: Optional[dict] = None, reserve: Optional[int] = None,
                 items_per_step: int = 16384, oldest_share: float = 0.5,
                 min_step_ms: Optional[float] = None, backlog_share: float = 0.25,
                 step_timeout_s: float = 60.0, lookahead_ms: float = 0.25,
                 idle_wait_ms: float = 1.0, tail_split: float = 0.125):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        torch.cuda.set_device(self.dev)
        self.stream = torch.cuda.Stream(self.dev)
        self.mem_budget = int(mem_budget)
        # Steps are sized in estimated window compares; the rate starts at
        # compares_per_s and follows the measured device time of each step.
        # A step holds backlog_share of the admitted work left, between
        # min_step_ms (default step_ms / 2) and step_ms of device time: short
        # steps let new requests in sooner, long ones cost fewer fixed
        # per-step costs when there is a backlog to clear.
        self.step_s = step_ms * 1e-3
        self.min_step_s = (step_ms / 2 if min_step_ms is None else min_step_ms) * 1e-3
        self.backlog_share = float(backlog_share)
        self.rate = float(compares_per_s)
        self.step_compares = self.step_s * self.rate
        self.items_per_step = int(items_per_step)
        # The last tail_split of each request's share of a step goes in items
        # a quarter of the size, so that a step ends on short items (the
        # wavefronts then finish together).
        self.tail_split = float(tail_split)
        self.oldest_share = float(oldest_share)
        self.copy_stream = torch.cuda.Stream(self.dev)
        self.max_inflight = int(max_inflight)
        # A further step is queued behind the ones in flight only once they
        # are expected to end within lookahead_ms (from the estimated device
        # rate): enough to hide the host's turn between steps, short enough
        # that a request arriving meanwhile waits behind about one step, not
        # max_inflight of them.
        self.lookahead_s = lookahead_ms * 1e-3
        self.queue_end = 0.0
        # An idle server thread waits for requests in slices of idle_wait_ms
        # (a submit wakes it at once either way; short slices keep its wake-up
        # from a long idle period quick).
        self.idle_wait_s = idle_wait_ms * 1e-3
        # Steps run a grouped kernel, whose windows are bit-sliced: 64
        # candidates per lane, or 16 when a step holds an l = 2 request.
        self.config = dict(config or {})
        if self.config.get("variant", nat.VARIANT_AUTO) not in (
                nat.VARIANT_AUTO, nat.VARIANT_GROUP, nat.VARIANT_GROUP64):
            raise ValueError("the server's window tables are bit-sliced: variant must be "
                             "AUTO, GROUP or GROUP64")
        self.step_timeout_s = float(step_timeout_s)
        self.reserve = reserve  # fixed first output reservation (tests of the rerun path)
        self.d_insts = torch.zeros(MAX_SLOTS * 40, dtype=torch.uint8, device=self.dev)
        self.d_state = torch.zeros(MAX_SLOTS * 32, dtype=torch.uint8, device=self.dev)
        self.free_slots = list(range(MAX_SLOTS - 1, -1, -1))
        # Pinned staging of uploaded rows and slot records (larger rows are
        # pinned one by one).
        self.ring = _PinnedRing(torch, 64, 64 << 10)
        self.pool = _PinnedPool(torch)
        self.bufs = [_StepBuf(torch, self.dev, 2 * self.items_per_step) for _ in range(max_inflight)]
        self.idle_bufs = list(self.bufs)
        self.inflight: Deque[_StepBuf] = collections.deque()
        self.finishing: Deque[tuple] = collections.deque()   # codes on their way to the host
        self.waiting: Deque[_Req] = collections.deque()
        self.active: List[_Req] = []
        self.mem_used = 0
        self.cv = threading.Condition()
        self.running = True
        self.next_id = 0
        self.error: Optional[BaseException] = None
        self.stats = collections.Counter()
        self.thread = threading.Thread(target=self._loop, name="pms-serve", daemon=True)
        self.thread.start()

    # ------------------------------------------------------------------ API
    def submit(self, seqs, l: int, d: int) -> cf.Future:
        fut: cf.Future = cf.Future()
        m = np.ascontiguousarray(np.asarray(seqs, dtype=np.uint8))
        try:
            self._validate(m, l, d)
        except nat.PmsError as e:
            fut.set_exception(e)
            return fut
        if l == 1:
            # Four candidates: answered directly by the host-level solve.
            t0 = time.perf_counter()
            try:
                codes = nat.solve(m, 1, d)
            except nat.PmsError as e:
                fut.set_exception(e)
                return fut
            t1 = time.perf_counter()
            fut.set_result(Result(codes, int(codes.size), t0, t0, t1, 0, 0, 0))
            return fut
        with self.cv:
            if not self.running:
                raise RuntimeError("server is closed")
            req = _Req(self.next_id, m, int(l), int(d), time.perf_counter(), fut)
            if self.reserve is not None:
                req.cap = int(self.reserve)
                req.bytes = req._bytes()
            self.next_id += 1
            self.waiting.append(req)
            self.cv.notify_all()
        return fut

    def close(self, wait: bool = True):
        with self.cv:
            self.running = False
            self.cv.notify_all()
        if wait:
            self.thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ internals
    @staticmethod
    def _validate(m: np.ndarray, l: int, d: int):
        if m.ndim != 2 or m.shape[0] < 1:
            raise nat.PmsError(nat.PMS_ERR_INVALID, "rows must be an (n, t) byte matrix")
        n, t = m.shape
        if not (1 <= n <= nat.PMS_MAX_N and 1 <= l <= nat.PMS_MAX_L and l <= t <= nat.PMS_MAX_T
                and 0 <= d <= l):
            raise nat.PmsError(nat.PMS_ERR_INVALID, f"size out of range n={n} t={t} l={l} d={d}")
        f = m | 0x20   # fold upper case onto lower
        if not ((f == 97) | (f == 99) | (f == 103) | (f == 116)).all():   # a c g t
            raise nat.PmsError(nat.PMS_ERR_INVALID, "a byte is not A/C/G/T")

    def _admit(self):
        """Moves waiting requests in, oldest first, while memory and slots allow."""
        while self.waiting and self.free_slots:
            req = self.waiting[0]
            if self.mem_used + req.bytes > self.mem_budget and (self.active or self.inflight):
                self.stats["admission_waits"] += 1
                return
            self.waiting.popleft()
            try:
                self._upload(req)
            except nat.PmsError as e:
                # This request alone: its slot was never referenced by a step.
                self.free_slots.append(req.slot)
                req.dev_seqs = req.dev_win = req.dev_out = None
                self.stats["failed_admissions"] += 1
                req.future.set_exception(e)
                continue
            self.active.append(req)
            self.mem_used += req.bytes
            req.admitted = time.perf_counter()

    def _fail(self, reqs, exc: BaseException):
        """Fails these requests: each future gets `exc` now; a request's slot
        and memory are released once no step in flight refers to them."""
        for r in reqs:
            if r.failed:
                continue
            r.failed = True
            if r in self.active:
                self.active.remove(r)
            if not r.future.done():
                r.future.set_exception(exc)
            self.stats["failed"] += 1
            if r.inflight == 0:
                self._release(r)

    def _release(self, r: _Req):
        self.free_slots.append(r.slot)
        self.mem_used -= r.bytes
        r.dev_seqs = r.dev_win = r.dev_out = None
        self.pool.put(r.h_out)
        r.h_out = None

    def _launch_max_n(self, reqs) -> int:
        """The largest n of a step (it sizes the kernel's stage queues)."""
        return max(r.n for r in reqs)

    def _upload(self, req: _Req):
        torch = self.torch
        req.slot = self.free_slots.pop()
        raw = req.seqs.reshape(-1)
        staged, k = self.ring.stage(raw)
        with torch.cuda.stream(self.stream):
            # One device block per request: rows, window table and output,
            # each starting on a 256-byte boundary.
            seq_w = (raw.size + 255) // 256 * 64
            win_w = req.n * req.stride
            out_at = seq_w + (win_w + 63) // 64 * 64
            block = torch.empty(out_at + max(req.cap, 1), dtype=torch.int32, device=self.dev)
            req.dev_seqs = block[:seq_w].view(torch.uint8)[:raw.size]
            req.dev_win = block[seq_w:seq_w + win_w]
            req.dev_out = block[out_at:]
            if staged is None:
                staged = torch.from_numpy(raw).pin_memory()
            req.dev_seqs.copy_(staged, non_blocking=True)
            self.ring.used(k, self.stream)
        nat.build_windows(req.dev_seqs, req.n, req.t, req.l, req.dev_win, None, stream=self.stream,
                          layout=nat.LAYOUT_BITSLICED)
        self._write_slot(req)

    def _write_slot(self, req: _Req):
        """Device instance record and a cleared state for the request's slot."""
        torch = self.torch
        inst = nat.DevInstance(req.dev_win.data_ptr(), req.dev_out.data_ptr(), req.cap, req.n,
                               req.stride, req.l, req.d)
        st = nat.DevState(0, 0, 0, ITEMS_UNTRACKED, 0)
        h, k = self.ring.stage(bytes(inst) + bytes(st))
        with torch.cuda.stream(self.stream):
            self.d_insts[req.slot * 40:(req.slot + 1) * 40].copy_(h[:40], non_blocking=True)
            self.d_state[req.slot * 32:(req.slot + 1) * 32].copy_(h[40:72], non_blocking=True)
            self.ring.used(k, self.stream)

    def _build_step(self, buf: _StepBuf) -> int:
        """Fills one step's work table up to the step budget.

        Shortest remaining work first for requests that fit in one step (it
        minimises the mean latency), then the longer requests in arrival
        order; the oldest admitted request is always given half of the step
        so that a long request is never starved by a stream of short ones.
        Shares are cut into items of about 1 / items_per_step of the step's
        planned window compares each, so every step offers a few items per
        resident wavefront whatever the request sizes are.
        """
        live = [r for r in self.active if r.cursor < r.total]
        if not live:
            return 0
        buf.compares = 0.0
        backlog = sum((r.total - r.cursor) * r.cost_per_cand for r in live)
        budget = min(max(self.backlog_share * backlog, self.min_step_s * self.rate), self.step_compares)
        if len(live) == 1 and not self.waiting:
            # Nothing to share the device with: one step takes all of it.
            budget = max(budget, backlog)
        buf.budget = budget
        oldest = min(live, key=lambda r: r.arrival)
        order = sorted(live, key=lambda r: (r.total - r.cursor) * r.cost_per_cand)
        shares = {oldest.rid: self.oldest_share * budget}
        left = (1.0 - self.oldest_share) * budget
        # Requests that fit in one step, shortest first; what is left goes to
        # the longer ones in arrival order, so that two long requests run one
        # after the other instead of both finishing late.
        longer = []
        for r in order:
            want = (r.total - r.cursor) * r.cost_per_cand - shares.get(r.rid, 0.0)
            if want > budget:
                longer.append(r)
                continue
            give = min(max(want, 0.0), left)
            shares[r.rid] = shares.get(r.rid, 0.0) + give
            left -= give
        for r in sorted(longer, key=lambda r: r.arrival):
            if left <= 0:
                break
            want = (r.total - r.cursor) * r.cost_per_cand - shares.get(r.rid, 0.0)
            give = min(max(want, 0.0), left)
            shares[r.rid] = shares.get(r.rid, 0.0) + give
            left -= give
        if left > 0:
            shares[oldest.rid] += left
        # Items sized from the work the step will hold (a lone short request
        # does not fill the budget): about items_per_step of them in all.
        planned = sum(min(shares.get(r.rid, 0.0), (r.total - r.cursor) * r.cost_per_cand)
                      for r in order)
        item_compares = max(planned, 1.0) / self.items_per_step
        per_req: Dict[int, int] = {}
        used = 0
        table = buf.h_work.data_ptr()
        for r in order:
            # Shares and items in whole blocks of 4096 candidates (64 groups
            # of 64) where the request has them, as the library's own work
            # plan cuts them: every item then starts a block, and a stage-0
            # batch is one block, which the window filter takes alone.
            unit = 4096 if r.total >= 4096 else 64
            cands = int(shares.get(r.rid, 0.0) / r.cost_per_cand)
            cands = max(unit, (cands + unit - 1) // unit * unit)
            cands = min(cands, r.total - r.cursor)
            if cands <= 0:
                continue
            room = buf.max_items - used
            if room <= 0:
                break
            size = int(item_compares / r.cost_per_cand)
            # A small request is still spread over up to ~1024 items, so that
            # it runs on many wavefronts.
            size = min(size, max(unit, cands // 1024))
            size = max(unit, (size + unit - 1) // unit * unit)
            small = max(unit, (size // 4 + unit - 1) // unit * unit)
            tail = 0
            if self.tail_split > 0 and small < size:
                tail = min(cands, (int(cands * self.tail_split) + small - 1) // small * small)
            head = cands - tail
            # Items written straight into the pinned table (pms_work_item records).
            k = nat.fill_work_items(r.cursor, head, size, r.slot, table + 16 * used, room) if head else 0
            if k < 0:
                continue
            covered = min(head, k * size)
            if covered == head and tail and k < room:
                k2 = nat.fill_work_items(r.cursor + head, tail, small, r.slot,
                                         table + 16 * (used + k), room - k)
                if k2 > 0:
                    k += k2
                    covered += min(tail, k2 * small)
            if k <= 0:
                continue
            r.cursor += covered
            buf.compares += float(covered) * r.cost_per_cand
            per_req[r.slot] = k
            used += k
        if used == 0:
            return 0
        buf.reqs = [r for r in live if r.slot in per_req]
        buf.items_per_req = per_req
        return used

    def _launch(self) -> bool:
        if not self.idle_bufs:
            return False
        if self.inflight and time.perf_counter() < self.queue_end - self.lookahead_s:
            return False
        buf = self.idle_bufs[-1]
        n_items = self._build_step(buf)
        if n_items == 0:
            return False
        self.idle_bufs.pop()
        torch = self.torch
        max_n = self._launch_max_n(buf.reqs)
        cfg = dict(self.config)
        # 64 candidates per lane need l >= 3: a step holding an l = 2
        # request runs the 16-candidate kernel (same bit-sliced windows).
        if min(r.l for r in buf.reqs) < 3:
            cfg["variant"] = nat.VARIANT_GROUP
        elif cfg.get("variant", nat.VARIANT_AUTO) == nat.VARIANT_AUTO:
            cfg["variant"] = nat.VARIANT_GROUP64
        with torch.cuda.stream(self.stream):
            buf.d_work[:n_items * 16].copy_(buf.h_work[:n_items * 16], non_blocking=True)
            buf.d_ctr.zero_()
            buf.start.record(self.stream)
        try:
            nat.step_launch(self.d_insts, MAX_SLOTS, max_n, buf.d_work, n_items, self.d_state,
                            buf.d_ctr, config=cfg, stream=self.stream)
        except nat.PmsError as e:
            # Nothing of this step runs: its requests fail, the others go on.
            self.stats["failed_steps"] += 1
            reqs, buf.reqs = buf.reqs, []
            self.idle_bufs.append(buf)
            self._fail(reqs, e)
            return True
        with torch.cuda.stream(self.stream):
            buf.event.record(self.stream)
            buf.h_state.copy_(self.d_state, non_blocking=True)
            buf.h_ctr.copy_(buf.d_ctr, non_blocking=True)
            # Requests whose last candidates are in this step: their first
            # codes come back on this stream, before the next step's kernel
            # takes every compute unit (a copy queued behind it would wait
            # a whole step).  The count is known only at retirement; more
            # codes than were copied take the side-stream path.
            for r in buf.reqs:
                if EAGER_CODES and r.cursor >= r.total:
                    # Twice the expected motif count, at least EAGER_CODES.
                    k = int(min(r.cap, max(EAGER_CODES, 2 * r.est_m)))
                    self.pool.put(r.h_out)
                    r.h_out = self.pool.get(k)
                    r.h_out[:k].copy_(r.dev_out[:k], non_blocking=True)
            buf.done.record(self.stream)
        buf.launched = time.perf_counter()
        self.queue_end = max(buf.launched, self.queue_end) + buf.compares / self.rate
        for r in buf.reqs:
            r.inflight += 1
            r.steps += 1
            if not r.launched:
                r.launched = buf.launched
        self.inflight.append(buf)
        self.stats["steps"] += 1
        self.stats["items"] += n_items
        return True

    def _retire(self, buf: _StepBuf):
        buf.done.synchronize()
        ms = buf.start.elapsed_time(buf.event)
        # Only steps that filled at least half their budget say how fast the
        # device is; a step that held all the work there was is dominated by
        # fixed costs and would drag the estimate (and the steps) down.
        if ms > 0.05 and buf.compares >= 0.5 * buf.budget:
            measured = buf.compares / (ms * 1e-3)
            self.rate = min(max(0.7 * self.rate + 0.3 * measured, 1e11), 1e16)
            self.step_compares = self.step_s * self.rate
        # A view of the pinned snapshot (read below, before the buffer's next use).
        states = buf.h_state.numpy().view(_STATE_DTYPE)
        ctr = nat.DevCounters.from_buffer_copy(buf.h_ctr.numpy().tobytes())
        reqs, buf.reqs = buf.reqs, []
        self.idle_bufs.append(buf)
        if ctr.error:
            # The kernel skipped an instance it could not run (pms_dev_counters.error):
            # every request of the step is in doubt.
            self.stats["failed_steps"] += 1
            for r in reqs:
                r.inflight -= 1
                if r.failed and r.inflight == 0:
                    self._release(r)
            self._fail([r for r in reqs if not r.failed],
                       nat.PmsError(nat.PMS_ERR_DEVICE,
                                    "a search step reported an instance it could not run"))
            return
        for r in reqs:
            r.inflight -= 1
            if r.failed:
                if r.inflight == 0:
                    self._release(r)
                continue
            if r.cursor >= r.total and r.inflight == 0:
                r.retired = time.perf_counter()
                self._finish(r, int(states[r.slot]["count"]), int(states[r.slot]["visits"]),
                             buf.event)

    def _finish(self, r: _Req, count: int, visits: int, done_event):
        torch = self.torch
        if count > r.cap:
            # Reservation too small: run the request again with the exact size.
            self.pool.put(r.h_out)
            r.h_out = None
            self.mem_used -= r.bytes
            r.cap = count
            r.bytes = r._bytes()
            self.mem_used += r.bytes
            r.dev_out = torch.empty(max(r.cap, 1), dtype=torch.int32, device=self.dev)
            r.cursor = 0
            r.reruns += 1
            self.stats["reruns"] += 1
            self._write_slot(r)
            return
        # The request's last step has completed (done_event).  Its codes are
        # copied on a side stream, so the copy does not wait for steps queued
        # after it, into pinned memory, asynchronously: the request completes
        # in _complete once the copy's event has fired, and the loop goes on
        # launching steps meanwhile.  Its slot is free now (no later step
        # refers to it); its buffers stay referenced until the copy is done.
        self.active.remove(r)
        self.free_slots.append(r.slot)
        eager_k = int(min(r.cap, max(EAGER_CODES, 2 * r.est_m)))
        if r.h_out is not None and count <= eager_k:
            # The codes came back with the step (done_event has completed).
            host, r.h_out = r.h_out, None
            self._deliver(r, host, count, visits)
            return
        self.pool.put(r.h_out)
        r.h_out = None
        host = None
        if count:
            host = self.pool.get(count)
            self.copy_stream.wait_event(done_event)
            with torch.cuda.stream(self.copy_stream):
                host[:count].copy_(r.dev_out[:count], non_blocking=True)
        copied = torch.cuda.Event()
        copied.record(self.copy_stream)
        self.finishing.append((r, host, count, visits, copied))

    def _complete(self, block: bool):
        """Completes requests whose codes have reached the host, in order;
        with block, waits for the first one."""
        while self.finishing:
            r, host, count, visits, copied = self.finishing[0]
            if block:
                copied.synchronize()
                block = False
            elif not copied.query():
                return
            self.finishing.popleft()
            self._deliver(r, host, count, visits)

    def _deliver(self, r: _Req, host, count: int, visits: int):
        """Sorts the codes copied to the pinned buffer `host` (handed back to
        the pool) and completes the request."""
        codes = np.zeros(0, dtype=np.uint32)
        if count:
            try:
                codes = nat.sort_codes(host[:count].numpy().view(np.uint32).copy(), r.l)
            except nat.PmsError as e:   # a repeated code: this request's result is wrong
                self.pool.put(host)
                self.mem_used -= r.bytes
                r.dev_seqs = r.dev_win = r.dev_out = None
                self.stats["failed"] += 1
                r.future.set_exception(e)
                return
        self.pool.put(host)
        res = Result(codes, count, r.arrival, r.admitted, time.perf_counter(), r.steps,
                     r.reruns, visits, r.launched, r.retired)
        self.mem_used -= r.bytes
        r.dev_seqs = r.dev_win = r.dev_out = None
        self.stats["completed"] += 1
        r.future.set_result(res)

    def _wait_step(self, buf: _StepBuf) -> bool:
        """Waits for a step to complete, up to the step timeout from its
        launch (polling: an event wait could not be abandoned).  Returns False
        as soon as a request arrives, so that it is admitted and can join the
        next step while this one runs, or when the next step should be
        queued behind this one."""
        deadline = buf.launched + self.step_timeout_s
        while not buf.done.query():
            if time.perf_counter() > deadline:
                self.stats["step_timeouts"] += 1
                raise StepTimeout(f"a search step has not completed {self.step_timeout_s:g} s "
                                  "after its launch")
            if self.waiting and self.free_slots:
                return False
            if (self.idle_bufs and time.perf_counter() >= self.queue_end - self.lookahead_s
                    and any(r.cursor < r.total for r in self.active)):
                return False    # time to queue the next step behind this one
            time.sleep(0)   # yield only: the step's end is seen within microseconds
        return True

    def _fail_all(self, exc: BaseException):
        for r in list(self.active) + list(self.waiting) + [f[0] for f in self.finishing]:
            if not r.future.done():
                r.future.set_exception(exc)
        self.active.clear()
        self.waiting.clear()
        self.finishing.clear()

    def _loop(self):
        try:
            while True:
                with self.cv:
                    busy = self.waiting or self.active or self.inflight or self.finishing
                    if not self.running and not busy:
                        return
                    if not busy:
                        self.cv.wait(timeout=self.idle_wait_s)
                        continue
                    self._admit()
                launched = False
                while len(self.inflight) < self.max_inflight and self._launch():
                    launched = True
                self._complete(block=False)
                if self.inflight:
                    head = self.inflight[0]
                    if head.done.query() or (not launched and self._wait_step(head)):
                        self.inflight.popleft()
                        self._retire(head)
                elif self.finishing and not launched:
                    self._complete(block=True)
        except BaseException as e:  # noqa: BLE001 - every request learns of the failure
            self.error = e
            with self.cv:
                self.running = False
                self._fail_all(e)
