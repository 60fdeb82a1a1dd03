"""Bootstrap particle filter driver around the resampling library.

The filter of Sec. 1 (initialisation, propagation, weighting, resampling)
for the linear-Gaussian model x_t = A x_{t-1} + N(0, qI), y_t = x_t + N(0, rI),
resampling at every step. Every step runs in the library's kernels: the
propagate+weight kernel, the chosen resampler with the ancestor copy fused
in, and the step's likelihood factor mean_i w_i = exp(lse - log P), read
from the reduction the resampler performs anyway (a separate log-sum-exp
only for the fixed-B Metropolis resampler, which never sums the weights).
The whole run can be captured once into a HIP graph and replayed.
"""
import torch

from . import api


class BootstrapFilter:
    def __init__(self, A, P, q=0.1, r=0.5, seed=0, resampler="stratified", B=64, device=None,
                 eps=0.01):
        """resampler: 'stratified', 'systematic', 'multinomial', 'metropolis'
        (fixed B) or 'metropolis_adaptive' (B from eq. (5) each step, at most
        B, tolerance eps)."""
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.A = torch.as_tensor(A, dtype=torch.float64).contiguous().to(self.device)
        self.D = int(self.A.shape[0])
        self.P, self.q, self.r, self.seed = int(P), float(q), float(r), int(seed)
        self.resampler, self.B, self.eps = resampler, int(B), float(eps)
        dev = self.device
        self.x = torch.empty((self.P, self.D), dtype=torch.float32, device=dev)
        self.xp = torch.empty_like(self.x)
        self.lw = torch.empty(self.P, dtype=torch.float32, device=dev)
        self.anc = torch.empty(self.P, dtype=torch.int32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws = api.workspace(self.P, api.MULTINOMIAL, dev)
        self.B_used = torch.zeros(1, dtype=torch.int32, device=dev)

    def _step(self, t, y_t, lse_t):
        api.filter_propagate_weight(self.x, self.A, y_t, self.q, self.r, self.seed, t,
                                    x_out=self.xp, lw=self.lw)
        if self.resampler == "metropolis":
            api.rs_log_sum_exp(self.lw, out=lse_t, ws=self.ws, status=self.status)
            api.resample_and_copy("metropolis", self.lw, self.xp, self.seed, t, B=self.B,
                                  anc=self.anc, x_out=self.x, status=self.status)
            return
        if self.resampler == "metropolis_adaptive":
            api.resample_metropolis_adaptive(self.lw, self.seed, t, eps=self.eps, B_max=self.B,
                                             anc=self.anc, B_used=self.B_used, ws=self.ws,
                                             status=self.status)
            api.permute_copy(self.anc, self.xp, x_out=self.x, status=self.status)
        else:
            # the resampler's own reduction gives the likelihood factor
            api.resample_and_copy(self.resampler, self.lw, self.xp, self.seed, t, anc=self.anc,
                                  x_out=self.x, ws=self.ws, status=self.status)
        api.rs_workspace_log_sum_exp(self.ws, self.P, out=lse_t)

    def _run(self, y, lse):
        api.filter_init(self.x, self.seed)
        for t in range(1, y.shape[0] + 1):
            self._step(t, y[t - 1], lse[t - 1:t])

    def run(self, y, graph=False):
        """Log-likelihood estimate for observations y[T, D]; one host sync."""
        y = torch.as_tensor(y, dtype=torch.float32).contiguous().to(self.device)
        lse = torch.empty(y.shape[0], dtype=torch.float64, device=self.device)
        if graph:
            g = self.capture(y, lse)
            g.replay()
        else:
            self._run(y, lse)
        return self.loglik(lse)

    def capture(self, y, lse):
        """HIP graph of a whole run on (y, lse); replay() re-runs it."""
        s = torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self._run(y, lse)  # warm-up outside the capture
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._run(y, lse)
        return g

    def loglik(self, lse):
        """sum_t (lse_t - log P), summed on the device by the library."""
        flags = int(self.status.item())
        if flags:
            raise RuntimeError(f"resampling flagged the weights (status {flags})")
        return float(api.filter_loglik(lse, self.P).item())
