"""Helpers shared by the GPU tests: host <-> device copies and digests."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(a: np.ndarray, pad: int = 0, offset: int = 0):
    """Copy a uint8 array to a fresh device buffer at byte ``offset``;
    returns (buffer tensor, view tensor of len(a) bytes)."""
    torch = torch_cuda()
    buf = torch.empty(len(a) + offset + pad, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + len(a)]
    if len(a):
        view.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return buf, view


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def golden() -> dict:
    with open(os.path.join(HERE, "golden", "ctr_digests.json")) as f:
        return json.load(f)


def log(msg: str) -> None:
    print(msg, flush=True)
