"""Helpers for the GPU tests: host <-> device copies of word arrays."""
import sys

import numpy as np


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def to_dev(x: np.ndarray, word: int = 64):
    import torch
    if word == 64:
        t = torch.from_numpy(np.ascontiguousarray(x.astype(np.uint64)).view(np.int64))
    else:
        t = torch.from_numpy(np.ascontiguousarray(x.astype(np.uint32)).view(np.int32))
    return t.cuda()


def from_dev(t, word: int = 64) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint64) if word == 64 else a.view(np.uint32).astype(np.uint64)
