"""GPU test of the asyncio front end: coroutines on one event loop submit
requests of the serving size mix through AsyncEngine, suspend, and are
resumed from the engine's completion descriptor.  Every output equals the
single-request call on the same input and the CPU oracle on sampled blocks
(0 bits of tolerance)."""
from __future__ import annotations

import asyncio

import numpy as np
import pytest

from gpu_util import log, torch_cuda
from test_gpu_engine import check_alone_and_oracle, make_requests

pytestmark = pytest.mark.gpu


def test_async_engine_resumes_every_request():
    torch = torch_cuda()
    import paper_2607_02630_amd as A
    from paper_2607_02630_amd.aio import AsyncEngine
    src, dst, reqs, offs, lens = make_requests(torch, 300, 21)
    log(f"asyncio: {len(reqs)} requests, {sum(lens) / 2**20:.1f} MiB, 8 coroutines")
    done = []

    async def main():
        with A.Engine(budget_bytes=1 << 30, n_streams=2) as eng:
            aeng = AsyncEngine(eng)

            async def client(c):
                for i in range(c, len(reqs), 8):
                    await aeng.crypt(reqs[i][4])
                    done.append(i)

            await asyncio.wait_for(asyncio.gather(*(client(c) for c in range(8))), 60)
            assert not aeng.pending
            aeng.close()

    asyncio.run(main())
    assert sorted(done) == list(range(len(reqs)))
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(22))
