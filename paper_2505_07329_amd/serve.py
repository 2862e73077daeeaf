"""Request loop for encrypted clear-weight products served to many clients.

A request is one projection of one layer, forward (W [x]) or backward (W^T [g]),
for T encrypted tokens: the server-side product of Sec. 4.1 / Eq. (lora) that
a fine-tuning step issues for every linear layer of the frozen model (Sec. 6.3).

The server keeps every weight matrix resident and owns one output arena of a
fixed byte budget in HBM. Admission is first-in first-out: the request at the
head of the queue is admitted when its output fits the arena; nothing overtakes
it. The arena is a ring (outputs are released in the order they were admitted,
because one stream completes launches in order), so admission needs no device
allocation and never synchronizes. The admitted requests of a scheduling round
go out as one grouped launch (`ct_matmul_batch`); up to `max_inflight` launches
are queued on the stream so the device never waits for the host.

Latency runs from a request's arrival to the completion of its device work;
outputs stay on the device (the copy to the client is not part of it).

The loop is independent of the backend: `GpuBackend` drives the HIP library
through the C ABI, the tests drive the same loop with a fake backend and a
simulated clock.
"""

from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

ALIGN = 256


def _align(n: int) -> int:
    return (n + ALIGN - 1) // ALIGN * ALIGN


@dataclasses.dataclass
class Request:
    rid: int
    client: int
    layer: int
    proj: str
    transpose: bool
    tokens: int
    arrival: float              # seconds on the loop's clock
    d_in: int = 0               # contraction length of this product
    d_out: int = 0              # output LWE ciphertexts per token
    out_bytes: int = 0
    out_off: int = -1           # offset in the output arena once admitted
    start: float = math.nan     # launch time
    done: float = math.nan      # completion of its device work
    status: str = "pending"     # pending, queued, running, done, rejected, expired

    @property
    def macs(self) -> int:
        return self.tokens * self.d_in * self.d_out

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def switched_out_bytes(N: int) -> Callable[[int, int], int]:
    """Output bytes of T tokens x d_out LWE ciphertexts switched to 2^32 (u32, N+1 each)."""
    return lambda T, d_out: T * d_out * (N + 1) * 4


def poisson_arrivals(rate: float, n: int, rng, start: float = 0.0) -> List[float]:
    """n arrival times of a Poisson process of the given rate (inf: all at `start`)."""
    if math.isinf(rate):
        return [start] * n
    t = start + rng.exponential(1.0 / rate, size=n).cumsum()
    return [float(x) for x in t]


def make_requests(shapes: Dict[str, Tuple[int, int]], layers: int, clients: int, n: int,
                  rate: float, rng, out_bytes: Callable[[int, int], int],
                  max_tokens: int = 512) -> List[Request]:
    """n requests: Poisson arrivals (the superposition of `clients` Poisson clients of
    rate rate/clients), each uniform over layers x projections x {forward, backward},
    tokens uniform in 1..max_tokens. shapes: name -> (d_in, d_out) of the forward product."""
    names = list(shapes)
    times = poisson_arrivals(rate, n, rng)
    reqs = []
    for i, t in enumerate(times):
        proj = names[int(rng.integers(0, len(names)))]
        tr = bool(rng.integers(0, 2))
        d_in, d_out = shapes[proj]
        if tr:
            d_in, d_out = d_out, d_in
        T = int(rng.integers(1, max_tokens + 1))
        reqs.append(Request(rid=i, client=int(rng.integers(0, clients)),
                            layer=int(rng.integers(0, layers)), proj=proj, transpose=tr,
                            tokens=T, arrival=t, d_in=d_in, d_out=d_out,
                            out_bytes=out_bytes(T, d_out)))
    return reqs


class RingArena:
    """Byte ring over [0, cap). Allocations are released in allocation order.

    Live allocations form one increasing run of offsets, possibly followed (after
    a wrap to 0) by a second run that ends at or below the first live offset.
    """

    def __init__(self, cap: int):
        self.cap = cap // ALIGN * ALIGN
        self.live: collections.deque = collections.deque()  # (offset, end)

    @property
    def used(self) -> int:
        return sum(e - o for o, e in self.live)

    def alloc(self, nbytes: int) -> Optional[int]:
        n = _align(max(nbytes, 1))
        if n > self.cap:
            return None
        if not self.live:
            off = 0
        else:
            first, last_end = self.live[0][0], self.live[-1][1]
            wrapped = self.live[-1][0] < first
            if not wrapped and last_end + n <= self.cap:
                off = last_end
            elif not wrapped and n <= first:
                off = 0
            elif wrapped and last_end + n <= first:
                off = last_end
            else:
                return None
        self.live.append((off, off + n))
        return off

    def release(self, off: int) -> None:
        if not self.live or self.live[0][0] != off:
            raise ValueError("ring arena: release out of allocation order")
        self.live.popleft()


class Scheduler:
    """FIFO admission into a RingArena.

    One round admits at most `max_batch` requests and stops adding requests once the
    round holds `max_round_macs` MACs (a single larger request still goes alone): the
    requests of a round complete together, so a cap keeps small requests from waiting
    for a large one admitted beside them, while small requests still share a launch.
    """

    def __init__(self, arena: RingArena, max_batch: int = 16, queue_timeout: float = math.inf,
                 max_round_macs: float = math.inf):
        self.arena = arena
        self.max_batch = max_batch
        self.max_round_macs = max_round_macs
        self.queue_timeout = queue_timeout
        self.queue: collections.deque = collections.deque()
        self.rejected: List[Request] = []
        self.expired: List[Request] = []

    def submit(self, r: Request) -> None:
        if _align(max(r.out_bytes, 1)) > self.arena.cap:
            r.status = "rejected"  # could never be admitted
            self.rejected.append(r)
            return
        r.status = "queued"
        self.queue.append(r)

    def expire(self, now: float) -> None:
        """Drop queued requests that waited longer than queue_timeout (never launched ones)."""
        if math.isinf(self.queue_timeout):
            return
        keep = collections.deque()
        for r in self.queue:
            if now - r.arrival > self.queue_timeout:
                r.status = "expired"
                self.expired.append(r)
            else:
                keep.append(r)
        self.queue = keep

    def admit(self) -> List[Request]:
        batch = []
        macs = 0
        while self.queue and len(batch) < self.max_batch:
            if batch and macs + self.queue[0].macs > self.max_round_macs:
                break
            off = self.arena.alloc(self.queue[0].out_bytes)
            if off is None:
                break  # the head waits; nothing overtakes it
            r = self.queue.popleft()
            r.out_off = off
            r.status = "running"
            macs += r.macs
            batch.append(r)
        return batch

    def release(self, batch: Sequence[Request]) -> None:
        for r in batch:
            self.arena.release(r.out_off)


def run_loop(reqs: List[Request], sched: Scheduler, backend, clock: Callable[[], float],
             wait: Callable[[float], None], max_inflight: int = 2) -> dict:
    """Serve every request: arrivals -> queue -> admitted batches -> completion.

    backend.launch(batch) enqueues a batch and returns a handle;
    backend.completed(handle) returns None while the work is running, else its
    completion time on the loop's clock (seconds since backend.start()).
    wait(dt) blocks for about dt seconds (a sleep, or advancing a simulated clock).
    """
    pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
    inflight: collections.deque = collections.deque()  # (handle, batch)
    finished: List[Request] = []
    t0 = clock()
    backend.start()
    while pending or sched.queue or inflight:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            sched.submit(pending.popleft())
        sched.expire(now)
        progressed = False
        while inflight:
            tdone = backend.completed(inflight[0][0])
            if tdone is None:
                break
            h, batch = inflight.popleft()
            for r in batch:
                r.done = tdone
                r.status = "done"
            backend.finish(h)
            sched.release(batch)
            finished.extend(batch)
            progressed = True
        if len(inflight) < max_inflight:
            batch = sched.admit()
            if batch:
                tstart = clock() - t0
                for r in batch:
                    r.start = tstart
                inflight.append((backend.launch(batch), batch))
                progressed = True
        if not progressed:
            nxt = pending[0].arrival - now if pending else math.inf
            wait(min(nxt, backend.poll_interval) if inflight or sched.queue else nxt)
    wall = clock() - t0
    return summarize(finished, wall, len(sched.rejected), len(sched.expired))


def percentile(sorted_vals: Sequence[float], p: float) -> float:
    """Nearest-rank percentile of an ascending sequence."""
    if not sorted_vals:
        return math.nan
    k = min(len(sorted_vals) - 1, max(0, int(math.ceil(p / 100.0 * len(sorted_vals))) - 1))
    return sorted_vals[k]


def summarize(done: List[Request], wall: float, rejected: int = 0, expired: int = 0) -> dict:
    lats = sorted(r.latency for r in done)
    macs = sum(r.macs for r in done)
    first = min((r.arrival for r in done), default=0.0)
    last = max((r.done for r in done), default=0.0)
    span = max(last - first, 1e-12)
    return {"requests": len(done), "rejected": rejected, "expired": expired,
            "p50_s": percentile(lats, 50), "p99_s": percentile(lats, 99),
            "mean_s": sum(lats) / len(lats) if lats else math.nan,
            "macs": macs, "macs_per_s": macs / span, "span_s": span, "wall_s": wall}


class GpuBackend:
    """Admitted batches go out as one ct_matmul_batch each on one stream.

    weights: (layer, proj) -> rlwe.Weights loaded forward and transposed.
    pools:   L -> int64 tensor [max_tokens][L][2][P][N] of input ciphertexts; a
             request of T tokens reads the first T (contiguous) entries.
    arena:   uint8 device tensor of the arena's capacity; a request's output is the
             u32 [T][d_out][N+1] view at its arena offset.
    Completion times come from device timestamps (event elapsed time against an
    event recorded at start), not from when the host happens to poll.
    """

    poll_interval = 2e-4

    def __init__(self, ctx, weights: dict, pools: dict, arena_tensor, stream=None,
                 keep_outputs: bool = False):
        import torch
        from . import rlwe
        self.torch, self.rlwe = torch, rlwe
        self.ctx, self.weights, self.pools = ctx, weights, pools
        self.arena = arena_tensor
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.keep_outputs = keep_outputs
        self.outputs: Dict[int, object] = {}
        self.N = ctx.N

    def out_view(self, r: Request):
        n = r.tokens * r.d_out * (self.N + 1)
        return self.arena[r.out_off: r.out_off + 4 * n].view(self.torch.int32).view(
            r.tokens, r.d_out, self.N + 1)

    def start(self) -> None:
        torch = self.torch
        self.stream.synchronize()
        self.t_ev = torch.cuda.Event(enable_timing=True)
        self.t_ev.record(self.stream)
        self.t_ev.synchronize()

    def launch(self, batch: Sequence[Request]):
        torch, rlwe = self.torch, self.rlwe
        items = []
        for r in batch:
            w = self.weights[(r.layer, r.proj)]
            L = (r.d_in + self.N - 1) // self.N
            ct = self.pools[L][: r.tokens]
            items.append((w.handle, r.transpose, ct, r.tokens, self.out_view(r)))
        rlwe.ct_matmul_batch(self.ctx.handle, items, rlwe.RLWE_OUT_SWITCHED, self.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        if self.keep_outputs:
            with torch.cuda.stream(self.stream):  # copies ordered after the batch
                for r in batch:
                    self.outputs[r.rid] = self.out_view(r).clone()
        return ev

    def completed(self, ev) -> Optional[float]:
        if not ev.query():
            return None
        return self.t_ev.elapsed_time(ev) * 1e-3

    def finish(self, ev) -> None:
        pass
