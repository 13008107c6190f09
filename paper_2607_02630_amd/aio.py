"""asyncio integration of the engine: submit, suspend, resume.

The paper's Python server reroutes its offload with asyncio (Sec. 3, the
event-loop-with-executor row of Table 1; Appendix A, Table 2): instead of
calling the offload on the event loop, a handler submits it, suspends on a
future, and is resumed when the offload completes.  Here the executor is the
engine itself: ``AsyncEngine.crypt`` submits a request, registers a future
under its ticket, and awaits it; the engine's completion file descriptor is
watched by the loop (``add_reader``), whose callback polls the pending
tickets and resolves the futures of those that finished.  No thread is
parked per request.

Running this module (``python -m paper_2607_02630_amd.aio``) reproduces the
shape of Table 2 on one MI355X: a single-event-loop server with N concurrent
clients, each request doing some per-request CPU work plus one AES-CTR
offload of the block size, served synchronously (the offload blocks the
loop) and rerouted (submit / await / resume), in requests per second.
"""
from __future__ import annotations

import argparse
import asyncio
import hashlib
import json
import os
import time

from . import Engine, Request, aes_ctr_crypt, aes_expand_key


class AsyncEngine:
    """Awaitable front end of an Engine on one asyncio loop."""

    def __init__(self, engine: Engine, loop: asyncio.AbstractEventLoop | None = None):
        self.engine = engine
        self.loop = loop or asyncio.get_running_loop()
        self.fd = engine.completion_fd()
        self.pending: dict[int, asyncio.Future] = {}
        self.loop.add_reader(self.fd, self._on_ready)

    def _on_ready(self) -> None:
        try:
            os.read(self.fd, 8)
        except BlockingIOError:
            pass
        for t in list(self.pending):
            try:
                done = self.engine.poll(t)
            except Exception as exc:          # failed request: resume with its error
                self.pending.pop(t).set_exception(exc)
                continue
            if done:
                self.pending.pop(t).set_result(None)

    async def crypt(self, req: Request) -> None:
        ticket = self.engine.submit(req)       # 1. submit
        fut = self.loop.create_future()        # 2. suspend: registered before the loop can
        self.pending[ticket] = fut             #    run the completion callback
        await fut                              # 3. resume on completion

    def close(self) -> None:
        self.loop.remove_reader(self.fd)


def _cpu_work(header: bytes) -> bytes:
    """Stand-in for the server's own per-request processing."""
    return hashlib.sha256(header).digest()


async def _serve(mode: str, size: int, clients: int, seconds: float, torch) -> float:
    """Closed-loop clients against one event loop; returns requests/s."""
    nonce = bytes(12)
    sched = aes_expand_key(bytes(range(16)))
    bufs = [(torch.randint(0, 256, (size,), dtype=torch.uint8, device="cuda"),
             torch.empty(size, dtype=torch.uint8, device="cuda")) for _ in range(clients)]
    torch.cuda.synchronize()        # the engine's streams are not ordered after torch's
    header = os.urandom(4096)
    done = 0
    stop = time.perf_counter() + seconds
    aeng = None
    engine = None
    if mode == "async":
        engine = Engine(budget_bytes=max(4 << 30, 2 * clients * size))
        aeng = AsyncEngine(engine)
    stream = torch.cuda.current_stream()

    async def client(i: int) -> None:
        nonlocal done
        x, y = bufs[i]
        while time.perf_counter() < stop:
            _cpu_work(header)
            if mode == "sync":
                aes_ctr_crypt(sched, nonce, 1, x, y, stream=stream)
                stream.synchronize()          # the offload blocks the loop
            else:
                await aeng.crypt(Request(sched, nonce, 1, x, y))
            done += 1
            await asyncio.sleep(0)            # the loop serves other clients

    t0 = time.perf_counter()
    await asyncio.gather(*(client(i) for i in range(clients)))
    el = time.perf_counter() - t0
    if aeng:
        aeng.close()
        engine.close()
    return done / el


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--clients", type=int, default=50)
    ap.add_argument("--seconds", type=float, default=1.0)
    ap.add_argument("--sizes", default=",".join(str(4096 << i) for i in range(12)))
    args = ap.parse_args(argv)
    import torch
    rows = []
    for size in (int(s) for s in args.sizes.split(",")):
        sync = asyncio.run(_serve("sync", size, args.clients, args.seconds, torch))
        asy = asyncio.run(_serve("async", size, args.clients, args.seconds, torch))
        rows.append({"block_bytes": size, "sync_rps": round(sync, 1), "async_rps": round(asy, 1),
                     "speedup": round(asy / sync, 2)})
        print(json.dumps(rows[-1]), flush=True)


if __name__ == "__main__":
    main()
