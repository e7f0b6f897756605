"""Batched uneven projection: several cone / helical problems in one persistent forward
launch, and forward + adjoint of the whole batch captured once in a hipGraph and
replayed."""
from __future__ import annotations

import torch

from . import xrt as X


class BatchGraph:
    """Forward then adjoint of every member, captured in a graph on first use.

    The graph reads the image tensors `imgs` and writes `sinos` and `backs` (all owned by
    this object; copy new inputs into `imgs` before `replay()`)."""

    def __init__(self, batch: X.Batch, adjoint_mode: str = "auto"):
        self.batch = batch
        self.mode = adjoint_mode
        dev = f"cuda:{batch.device}"
        self.imgs = [torch.zeros(tuple(p.image_shape), dtype=torch.float32, device=dev) for p in batch.plans]
        self.sinos = [torch.empty(tuple(p.sino_shape), dtype=torch.float32, device=dev) for p in batch.plans]
        self.backs = [torch.empty(tuple(p.image_shape), dtype=torch.float32, device=dev) for p in batch.plans]
        self.graph = None

    def _run(self):
        self.batch.forward(self.imgs, out=self.sinos)
        self.batch.adjoint(self.sinos, mode=self.mode, out=self.backs)

    def capture(self):
        # one eager pass first (library and kernel loading happen outside the capture)
        self._run()
        torch.cuda.synchronize(self.batch.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run()
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
