"""The asyncio front end (AsyncEngine) on the CPU, against a stand-in engine.

The stand-in has the engine's submit / poll / completion_fd surface: a
helper thread completes tickets after random delays (some of them failed)
and writes to a pipe that plays the completion descriptor.  Every awaiting
coroutine must be resumed exactly once, with the failure of its own ticket
where there is one, also when several completions arrive behind one
wake-up, and no future may stay registered afterwards.
"""
from __future__ import annotations

import asyncio
import os
import random
import threading
import time

import pytest


class StandInEngine:
    def __init__(self, fail_every: int, seed: int):
        self.r, self.w = os.pipe()
        os.set_blocking(self.r, False)
        self.lock = threading.Lock()
        self.next = 0
        self.finished: dict[int, bool] = {}       # ticket -> failed
        self.fail_every = fail_every
        self.rng = random.Random(seed)
        self.timers: list[threading.Timer] = []

    def completion_fd(self) -> int:
        return self.r

    def _complete(self, t: int) -> None:
        with self.lock:
            self.finished[t] = self.fail_every > 0 and t % self.fail_every == 0
        os.write(self.w, (1).to_bytes(8, "little"))

    def submit(self, req) -> int:
        with self.lock:
            t = self.next
            self.next += 1
        tm = threading.Timer(self.rng.uniform(0, 0.004), self._complete, args=(t,))
        self.timers.append(tm)
        tm.start()
        return t

    def poll(self, t: int) -> bool:
        with self.lock:
            if t not in self.finished:
                return False
            failed = self.finished.pop(t)
        if failed:
            raise RuntimeError(f"ticket {t} failed")
        return True

    def close(self) -> None:
        for tm in self.timers:
            tm.join()
        os.close(self.r)
        os.close(self.w)


@pytest.mark.parametrize("fail_every", [0, 7])
def test_every_request_is_resumed_once(fail_every):
    from paper_2607_02630_amd.aio import AsyncEngine
    eng = StandInEngine(fail_every, seed=11 + fail_every)
    n_clients, per_client = 16, 40
    results: dict[tuple[int, int], str] = {}

    async def main():
        aeng = AsyncEngine(eng)

        async def client(c):
            for j in range(per_client):
                try:
                    await aeng.crypt(None)
                    results[(c, j)] = "ok"
                except RuntimeError as e:
                    results[(c, j)] = str(e)
                await asyncio.sleep(0)

        await asyncio.wait_for(asyncio.gather(*(client(c) for c in range(n_clients))), 30)
        assert not aeng.pending
        aeng.close()

    t0 = time.perf_counter()
    asyncio.run(main())
    eng.close()
    assert len(results) == n_clients * per_client
    failed = [v for v in results.values() if v != "ok"]
    n = n_clients * per_client
    assert len(failed) == (0 if fail_every == 0 else (n + fail_every - 1) // fail_every)
    # Each failure carries its own ticket's error, and every ticket failed once.
    assert len(set(failed)) == len(failed)
    assert time.perf_counter() - t0 < 30
