"""Algorithm 1 (Steepest Gaussian Splatting) as a training loop on the device.

Every iteration either takes a gradient step -- forward with the fused L1
loss, backward with the splitting matrices accumulated into S, Adam (which
also accumulates the position gradient G and, for the ADC-style gate, its
norm) -- or, on densification
iterations, runs Steepest Density Control with S and G averaged over the
steps since the last one (s_scale = g_scale = 1 / steps), remaps the Adam
moments onto the new layout (offspring start from zero) and restarts the
accumulation.  The schedule follows the 3DGS pipeline the paper keeps
(Sec. 5.1): densify every 100 steps from step 500 up to step 15,000.

All arithmetic runs in the HIP library; this module sequences calls and owns
buffers (torch device memory).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _lib as L
from .pipeline import CameraBatch, Rasterizer, densify

# 3DGS defaults: position, log-scale, quaternion, opacity logit, SH degree 0, SH degrees >= 1
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3, 2.5e-3 / 20)


@dataclass
class Schedule:
    densify_from: int = 500
    densify_every: int = 100
    densify_until: int = 15_000

    def is_densify(self, t: int) -> bool:
        """t counts iterations from 1."""
        return self.densify_from <= t <= self.densify_until and t % self.densify_every == 0

    def accumulate_from(self) -> int:
        """first step whose S and G feed the first densification"""
        return max(1, self.densify_from - self.densify_every + 1)


@dataclass
class SplitEvent:
    step: int
    n_before: int
    n_split: int
    accumulated_steps: int


@dataclass
class SteepGSTrainer:
    params: torch.Tensor            # [F, n] float32, device
    sh_degree: int
    cams: CameraBatch
    target: torch.Tensor            # packed [3 * total_pixels]
    eps: float = 1e-3               # offspring displacement (Algorithm 1's stepsize)
    eps_split: float = -1e-6        # Sec. 5.1
    eps_grad: float = 0.0           # compactest gate (off when 0)
    adc_tau: float = 0.0            # ADC-style gate on the mean gradient norm (off when 0)
    budget: int = 0                 # increment budget (off when 0)
    lr: tuple = DEFAULT_LR
    schedule: Schedule = field(default_factory=Schedule)
    history: list = field(default_factory=list)

    def __post_init__(self):
        dev = self.params.device
        self.params = self.params.contiguous().clone()
        self.opts = L.make_adam_opts(self.lr)
        self.step_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.ras = Rasterizer(self.cams, self.sh_degree)
        self.t = 0
        self._alloc_state(self.params.shape[1])
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)

    def _alloc_state(self, n):
        dev = self.params.device
        self.grads = torch.zeros((self.params.shape[0], n), dtype=torch.float32, device=dev)
        self.S = torch.zeros((6, n), dtype=torch.float32, device=dev)
        self.G = torch.zeros((3, n), dtype=torch.float32, device=dev)
        self.Gabs = torch.zeros(n, dtype=torch.float32, device=dev)
        self.acc_steps = 0

    @property
    def n(self) -> int:
        return self.params.shape[1]

    def gradient_step(self):
        r = self.ras
        r.forward(self.params, self.target)
        self.grads.zero_()
        r.backward(self.params, self.grads, self.S, target=self.target)
        L.steepgs_adam_step(self.params, self.grads, self.m, self.v, self.n, self.sh_degree, self.opts, self.step_dev,
                            G=self.G, Gabs=self.Gabs if self.adc_tau > 0 else None)
        self.acc_steps += 1

    def window_scale(self) -> float:
        """1 / (accumulated steps x views): a step's loss sums the V per-view
        means, each view one image of Algorithm 1's gradient steps, so S, G and
        the gradient-norm sum average over images as the algorithm's interval
        average does, and eps_split applies per image."""
        return 1.0 / (max(self.acc_steps, 1) * self.cams.V)

    def densify_step(self):
        n = self.n
        sc = self.window_scale()
        out = densify(self.params, self.sh_degree, self.S, sc, self.eps, self.eps_split,
                      G=self.G if self.eps_grad > 0 else None, g_scale=sc, eps_grad=self.eps_grad,
                      budget=self.budget, Gabs=self.Gabs if self.adc_tau > 0 else None, adc_tau=self.adc_tau)
        if out["status"] != L.OK:
            raise RuntimeError("densification output capacity exceeded")
        n_out = out["n_out"]
        split = out["split"]
        ws = torch.empty(L.steepgs_workspace_size(L.STAGE_DENSIFY, n, 1) // 4 + 64, dtype=torch.int32,
                         device=self.params.device)
        F = self.params.shape[0]
        moments = []
        for state in (self.m, self.v):
            dst = torch.empty((F, n_out), dtype=torch.float32, device=self.params.device)
            L.steepgs_split_remap(state, F, n, split, dst, n_out, ws)
            moments.append(dst)
        self.m, self.v = moments
        self.params = out["params"].contiguous().clone()
        self.history.append(SplitEvent(self.t, n, n_out - n, self.acc_steps))
        self._alloc_state(n_out)
        return out

    def iterate(self):
        """One iteration of Algorithm 1."""
        self.t += 1
        if self.t == self.schedule.accumulate_from():
            self.S.zero_()
            self.G.zero_()
            self.Gabs.zero_()
            self.acc_steps = 0
        if self.schedule.is_densify(self.t):
            return self.densify_step()
        self.gradient_step()
        return None

    def loss(self) -> float:
        return float(self.ras.loss.sum())
