"""GPU timing by graph replay (shared by the autotuner and the benchmark).

Calls are captured into HIP graphs (torch.cuda.CUDAGraph on the library's
stream) and replayed back to back with a HIP event between replays, so the
GPU never idles waiting for the host: interval k is replay k's GPU time.
"""
import numpy as np


class Graphs:
    def __init__(self, torch):
        self.torch = torch

    def capture(self, fn):
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()  # warm-up outside the capture (sets kernel attributes)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        return g

    def replay_ms(self, graphs, n):
        """Replay graphs[k % len] for k < n; returns the n intervals in ms."""
        torch = self.torch
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        graphs[0].replay()  # prime the queue so the first interval is GPU-bound
        ev[0].record()
        for k in range(n):
            graphs[k % len(graphs)].replay()
            ev[k + 1].record()
        torch.cuda.synchronize()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(n)]


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))
