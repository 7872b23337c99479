"""Capture of a whole optimisation step into one HIP graph.

The step (forward, loss and dL/dobs in PyTorch, backward, parameter update)
is recorded once and replayed.  Every replay must see a fresh random stream,
so the library reads the epoch from a device scalar (`ssa_config.d_epoch`)
that the captured step itself advances.  Nothing in the captured library calls
allocates or clears memory with a memset: counters are cleared by a fill
kernel, so the recorded nodes replay correctly.
"""
from __future__ import annotations

from typing import Callable

import torch


class CapturedStep:
    """step_fn enqueues one step on the current stream using preallocated
    tensors only (its outputs are overwritten in place on every replay)."""

    def __init__(self, step_fn: Callable[[], None], warmup: int = 2):
        self.step_fn = step_fn
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):            # warm-up outside capture (allocator, lazy init)
            for _ in range(warmup):
                step_fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            step_fn()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
