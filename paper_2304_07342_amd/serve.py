"""Continuous-batching serving loop for compress / decompress requests.

Requests arrive over time (each with an arrival time, an operation, a symbol
width and a device-resident input). The server keeps a FIFO of arrived
requests and, whenever a batch slot is free, admits the longest prefix of
the queue whose device memory (input + output + workspace share) fits in the
remaining HBM budget, and launches it as one gpulz_compress_batch plus one
gpulz_decompress_batch on the next of several streams. Batches in flight on
different streams overlap on the device; requests that arrive meanwhile
wait only for a slot and for memory, not for the running batches to finish.
A request's latency is its completion (a device event after its batch)
minus its scheduled arrival.

`Scheduler` is the pure admission logic; `DeviceBackend` runs batches on
the GPU through the batch C ABI, `PlainBackend` runs the same admitted
requests one gpulz_compress / gpulz_decompress call each (the plain path it
is measured against); `serve` drives any of them with a clock.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import sys
import time

import numpy as np

COMPRESS, DECOMPRESS = "compress", "decompress"


@dataclasses.dataclass
class Request:
    rid: int
    op: str
    arrival: float            # seconds from the start of the run
    nbytes: int               # input bytes
    symbol_bytes: int = 1     # width (compress only)
    src: object = None        # backend handle of the input
    out_cap: int = 0          # output bytes to allocate
    need: int = 0             # bytes charged against the budget while in flight
    done: float | None = None
    status: int | None = None
    result: object = None     # output (kept only if the backend is asked to)


class Scheduler:
    """FIFO admission against a byte budget and a number of batch slots."""

    def __init__(self, budget_bytes: int, slots: int, max_batch: int = 512):
        self.budget = budget_bytes
        self.slots = slots
        self.max_batch = max_batch
        self.queue = collections.deque()
        self.in_flight_bytes = 0
        self.in_flight_batches = 0
        self.rejected = []

    def arrive(self, req: Request) -> None:
        if req.need > self.budget:
            self.rejected.append(req)  # can never fit
        else:
            self.queue.append(req)

    def next_batch(self):
        """The requests to launch now (possibly empty)."""
        if self.in_flight_batches >= self.slots or not self.queue:
            return []
        room = self.budget - self.in_flight_bytes
        batch = []
        while self.queue and len(batch) < self.max_batch and self.queue[0].need <= room:
            r = self.queue.popleft()
            room -= r.need
            batch.append(r)
        if batch:
            self.in_flight_bytes += sum(r.need for r in batch)
            self.in_flight_batches += 1
        return batch

    def finish(self, batch) -> None:
        self.in_flight_bytes -= sum(r.need for r in batch)
        self.in_flight_batches -= 1


def serve(trace, backend, budget_bytes: int, slots: int = 3, max_batch: int = 512,
          poll_s: float = 2e-4, progress=None):
    """Run all requests of `trace` (sorted by arrival); returns the scheduler."""
    sched = Scheduler(budget_bytes, slots, max_batch)
    pending = collections.deque(trace)
    running = []  # (handle, batch)
    backend.start()
    last_report = 0.0
    while pending or sched.queue or running:
        now = backend.now()
        while pending and pending[0].arrival <= now:
            sched.arrive(pending.popleft())
        still = []
        for handle, batch in running:
            t = backend.poll(handle)
            if t is None:
                still.append((handle, batch))
            else:
                # one completion time for the batch, or one per request
                for k, r in enumerate(batch):
                    r.done = t[k] if isinstance(t, list) else t
                backend.release(handle, batch)
                sched.finish(batch)
        running = still
        launched = False
        while True:
            batch = sched.next_batch()
            if not batch:
                break
            running.append((backend.launch(batch), batch))
            launched = True
        if progress and now - last_report >= 5.0:
            last_report = now
            progress(now, len(pending), len(sched.queue), len(running), sched.in_flight_bytes)
        if not launched:
            nxt = pending[0].arrival if pending else None
            backend.idle(now, nxt, poll_s, bool(running))
    return sched


# ---- the GPU backend -----------------------------------------------------------

class DeviceBackend:
    """Launches batches with the batch C ABI on a rotating set of streams."""

    def __init__(self, nstreams: int = 3, keep_results: bool = False):
        import torch
        from . import gpulz
        self.torch = torch
        self.gpulz = gpulz
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.k = 0
        self.keep = keep_results
        self.start_event = None

    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.start_event = torch.cuda.Event(enable_timing=True)
        self.start_event.record()
        self.start_event.synchronize()
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def idle(self, now, next_arrival, poll_s, busy):
        wait = poll_s if busy or next_arrival is None else max(0.0, min(next_arrival - now, 0.01))
        if wait > 0:
            time.sleep(wait)

    def _arrays(self, stream, cols):
        """Copy per-request int64 columns to the device on `stream` through
        pinned memory (no host synchronisation)."""
        torch = self.torch
        n = len(cols[0])
        host = torch.empty((len(cols), n), dtype=torch.int64, pin_memory=True)
        for i, c in enumerate(cols):
            host[i] = torch.tensor(c, dtype=torch.int64)
        dev = host.to("cuda", non_blocking=True)
        return host, dev

    def launch(self, batch):
        torch, gpulz = self.torch, self.gpulz
        stream = self.streams[self.k % len(self.streams)]
        self.k += 1
        keep = []
        with torch.cuda.stream(stream):
            for op in (COMPRESS, DECOMPRESS):
                reqs = [r for r in batch if r.op == op]
                if not reqs:
                    continue
                outs = [torch.empty(max(r.out_cap, 1), dtype=torch.uint8, device="cuda") for r in reqs]
                total = max(1, sum(r.nbytes for r in reqs))
                cols = [[r.src.data_ptr() for r in reqs], [r.nbytes for r in reqs],
                        [o.data_ptr() for o in outs], [r.out_cap for r in reqs]]
                host, dev = self._arrays(stream, cols)
                meta = torch.zeros(len(reqs), dtype=torch.int64, device="cuda")
                status = torch.zeros(len(reqs), dtype=torch.int32, device="cuda")
                if op == COMPRESS:
                    widths = torch.tensor([r.symbol_bytes for r in reqs], dtype=torch.uint8
                                          ).pin_memory().to("cuda", non_blocking=True)
                    ws_bytes = gpulz.gpulz_compress_batch_workspace_size(len(reqs), total)
                    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
                    st = gpulz.gpulz_compress_batch(
                        len(reqs), dev[0].data_ptr(), dev[1].data_ptr(), widths.data_ptr(), None,
                        dev[2].data_ptr(), dev[3].data_ptr(), meta.data_ptr(), status.data_ptr(),
                        total, ws.data_ptr(), ws_bytes, stream.cuda_stream)
                    keep.append(widths)
                else:
                    ws_bytes = gpulz.gpulz_decompress_batch_workspace_size(len(reqs), total)
                    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
                    st = gpulz.gpulz_decompress_batch(
                        len(reqs), dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(),
                        dev[3].data_ptr(), meta.data_ptr(), status.data_ptr(), total, ws.data_ptr(),
                        ws_bytes, stream.cuda_stream)
                if st != gpulz.GPULZ_OK:
                    raise gpulz.GpulzError(st, f"{op} batch")
                keep += [host, dev, ws, outs, meta, status, reqs]
        done = torch.cuda.Event(enable_timing=True)
        done.record(stream)
        return (done, keep)

    def poll(self, handle):
        done, _ = handle
        if not done.query():
            return None
        return self.start_event.elapsed_time(done) / 1e3

    def release(self, handle, batch):
        _, keep = handle
        # keep = [..., outs, meta, status, reqs] per operation
        for i in range(0, len(keep)):
            item = keep[i]
            if isinstance(item, list) and item and isinstance(item[0], Request):
                outs, meta, status = keep[i - 3], keep[i - 2], keep[i - 1]
                sizes = meta.cpu().tolist()
                stats = status.cpu().tolist()
                for r, o, n, s in zip(item, outs, sizes, stats):
                    r.status = s
                    if self.keep:
                        r.result = o[:n]


class PlainBackend(DeviceBackend):
    """The plain path under the same admission: each admitted request is one
    gpulz_compress or gpulz_decompress call of its own (with its own
    workspace), issued in arrival order on the batch's stream, and completes
    at its own device event."""

    def launch(self, batch):
        torch, gpulz = self.torch, self.gpulz
        stream = self.streams[self.k % len(self.streams)]
        self.k += 1
        keep = []
        with torch.cuda.stream(stream):
            for r in batch:
                out = torch.empty(max(r.out_cap, 1), dtype=torch.uint8, device="cuda")
                meta = torch.zeros(2, dtype=torch.int64, device="cuda")
                if r.op == COMPRESS:
                    C, W, MIN, _ = gpulz.gpulz_default_params(r.symbol_bytes)
                    ws_bytes = gpulz.gpulz_compress_workspace_size(r.nbytes, r.symbol_bytes, C)
                    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
                    st = gpulz.gpulz_compress(r.src.data_ptr(), r.nbytes, r.symbol_bytes, C, W, MIN,
                                              out.data_ptr(), r.out_cap, meta.data_ptr(),
                                              meta.data_ptr() + 8, ws.data_ptr(), ws_bytes,
                                              stream.cuda_stream)
                else:
                    ws_bytes = gpulz.gpulz_decompress_workspace_size(r.nbytes)
                    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device="cuda")
                    st = gpulz.gpulz_decompress(r.src.data_ptr(), r.nbytes, out.data_ptr(),
                                                r.out_cap, meta.data_ptr(), meta.data_ptr() + 8,
                                                ws.data_ptr(), ws_bytes, stream.cuda_stream)
                if st != gpulz.GPULZ_OK:
                    raise gpulz.GpulzError(st, f"plain {r.op}")
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                keep.append((out, meta, ws, ev))
        return keep

    def poll(self, handle):
        if not handle[-1][3].query():
            return None
        return [self.start_event.elapsed_time(ev) / 1e3 for _, _, _, ev in handle]

    def release(self, handle, batch):
        for r, (out, meta, _, _) in zip(batch, handle):
            n, status = meta.cpu().tolist()
            r.status = status & 0xFFFFFFFF
            if self.keep:
                r.result = out[:n]


# ---- workload -------------------------------------------------------------------

def make_trace(rate: float, duration: float, seed: int, compress_frac: float = 0.7,
               lo: int = 64 << 10, hi: int = 256 << 20):
    """Poisson arrivals at `rate` per second for `duration` seconds: (arrival,
    op, size, width, pick) tuples; `pick` selects a source."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        op = COMPRESS if rng.random() < compress_frac else DECOMPRESS
        size = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        S = int(rng.choice([1, 2, 4, 8]))
        out.append((t, op, size, S, int(rng.integers(0, 1 << 30))))
    return out


def build_requests(trace, pools, streams, budget_ws_factor: float = 1.1):
    """Turn trace tuples into Requests over device pools (compress: a slice of
    the width's pool; decompress: one of the prepared streams)."""
    from . import gpulz, synth
    reqs = []
    for i, (t, op, size, S, pick) in enumerate(trace):
        if op == COMPRESS:
            kinds = synth.WIDTH_KINDS[S]
            pool = pools[kinds[pick % len(kinds)]]
            n = max(S, min(size, pool.numel()) // S * S)
            off = (pick % (pool.numel() - n + 1)) // 16 * 16
            C, W, MIN, _ = gpulz.gpulz_default_params(S)
            cap = gpulz.gpulz_compress_bound(n, S, C, MIN)
            r = Request(i, op, t, n, S, pool[off:off + n], cap)
            r.need = n + cap + int(budget_ws_factor * cap)
        else:
            s, orig = streams[pick % len(streams)]
            r = Request(i, op, t, s.numel(), 0, s, orig)
            r.need = s.numel() + orig
        reqs.append(r)
    return reqs


def summarize(reqs, wall_s, offered_rate, duration):
    lat = np.array([r.done - r.arrival for r in reqs if r.done is not None])
    done_bytes = sum(r.nbytes for r in reqs if r.done is not None)
    ok = sum(1 for r in reqs if r.status == 0)
    q = lambda p: float(np.percentile(lat, p)) * 1e3 if lat.size else None
    return {"requests": len(reqs), "completed": int(lat.size), "ok": ok,
            "offered_req_per_s": offered_rate,
            "offered_GBps": round(sum(r.nbytes for r in reqs) / duration / 1e9, 3),
            "throughput_GBps": round(done_bytes / wall_s / 1e9, 3), "wall_s": round(wall_s, 3),
            "latency_ms": {"p50": q(50), "p99": q(99), "max": q(100)}}


def main_bench(args):
    """bench.py --workload serve: the full-rate run, then a short rate sweep."""
    import torch
    from . import autotune, gpulz, synth
    log = lambda *a: print("[serve]", *a, file=sys.stderr, flush=True)
    pool_bytes = args.pool_mib << 20
    pools = {}
    for i, kind in enumerate(synth.POOL_KINDS):
        log(f"pool {kind}")
        pools[kind] = torch.from_numpy(synth.POOL_KINDS[kind][1](pool_bytes, 100 + i)[:pool_bytes]).cuda()
    autotune.tune({S: pools[k[0]][: 64 << 20] for S, k in synth.WIDTH_KINDS.items()}, log=log)
    # streams for decompress requests: compress a set of log-uniform slices once
    rng = np.random.Generator(np.random.PCG64(44))
    srcs, widths = [], []
    for j in range(args.serve_streams):
        S = int(rng.choice([1, 2, 4, 8]))
        kind = synth.WIDTH_KINDS[S][j % len(synth.WIDTH_KINDS[S])]
        n = int(np.exp(rng.uniform(np.log(64 << 10), np.log(min(256 << 20, pool_bytes)))))
        n = max(S, n // S * S)
        off = int(rng.integers(0, pool_bytes - n + 1)) // 16 * 16
        srcs.append(pools[kind][off:off + n])
        widths.append(S)
    bc = gpulz.BatchCompressor(srcs, widths, None)
    bc.run()
    streams = []
    for (st, s), x in zip(bc.results(), srcs):
        assert st == gpulz.GPULZ_OK
        streams.append((s.clone(), x.numel()))
    del bc
    # every prepared stream must decode back to its source
    bd = gpulz.BatchDecompressor([s for s, _ in streams], [n for _, n in streams])
    bd.run()
    for (st, y), x in zip(bd.results(), srcs):
        if st != gpulz.GPULZ_OK or not torch.equal(y, x):
            raise SystemExit("a prepared decompress stream does not round-trip")
    del bd
    torch.cuda.empty_cache()
    runs = [(args.serve_rate, args.serve_seconds)] + [(r, args.sweep_seconds) for r in args.sweep_rates]
    backends = {"batched": DeviceBackend, "plain": PlainBackend}
    for rate, dur in runs:
        for name in getattr(args, "serve_backends", ["batched", "plain"]):
            trace = make_trace(rate, dur, seed=4)
            reqs = build_requests(trace, pools, streams)
            log(f"{name}: rate {rate}/s for {dur} s: {len(reqs)} requests")
            backend = backends[name](nstreams=args.serve_slots)
            t0 = time.perf_counter()
            sched = serve(reqs, backend, args.budget_gb * 10**9, slots=args.serve_slots,
                          progress=lambda now, p, q, r, b: log(
                              f"t={now:.1f}s pending={p} queued={q} running={r} "
                              f"inflight={b / 1e9:.1f} GB"))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            res = summarize(reqs, wall, rate, dur)
            res.update({"metric": "serving throughput and p50/p99 latency",
                        "workload": f"serve-{name}-{rate}", "backend": name,
                        "budget_GB": args.budget_gb, "slots": args.serve_slots,
                        "rejected": len(sched.rejected), "duration_s": dur})
            print(json.dumps(res), flush=True)
            del reqs, backend, sched
            torch.cuda.empty_cache()
