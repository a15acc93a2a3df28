"""Learned demapper: training on exact-demapper LLR targets and per-SNR
evaluation with fallback to the exact path.

Host-side orchestration only: every step runs in libmdgmi's kernels (device
sample generation, exact LLR targets, MLP forward/backward, Adam, learned
and exact GMI). The host picks SNR points, the learning rate, and the
per-SNR route.

Route rule: on the same held-out samples, an SNR point uses the learned
demapper when GMI_exact - GMI_learned <= max_loss (0.01 bit/symbol), else
the exact demapper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import mdgmi

LOG2E = 1.0 / math.log(2.0)


def sigma2_of(snr_db, dim):
    """Per-real-dimension noise variance of a unit-energy format."""
    return 1.0 / (dim * 10.0 ** (np.asarray(snr_db, dtype=np.float64) / 10.0))


@dataclass
class TrainConfig:
    hidden: tuple = (256, 256, 256)
    batch: int = 16384            # samples per step
    slices: int = 16              # SNR points per step (batch / slices samples each)
    snr_lo: float = 2.0
    snr_hi: float = 17.0
    snr_step: float = 0.25        # training SNRs are drawn from this grid
    lr: float = 1e-3
    lr_min: float = 1e-5          # cosine decay to this
    steps: int = 2000
    seed: int = 1234
    path: str = "mfma"            # exact demapper producing the targets
    log_every: int = 100


@dataclass
class TrainResult:
    steps: int
    samples: int
    losses: list = field(default_factory=list)   # (step, loss in nats per sample)


class Trainer:
    """Trains a network [dim + 1, hidden..., m] on one format."""

    def __init__(self, gf: mdgmi.Format, cfg: TrainConfig, net: mdgmi.MLP | None = None):
        import torch
        self.gf, self.cfg = gf, cfg
        self.net = net or mdgmi.MLP([gf.dim + 1, *cfg.hidden, gf.m], seed=cfg.seed)
        B = cfg.batch
        assert B % cfg.slices == 0
        self.per = B // cfg.slices
        self.y = torch.empty((B, gf.dim), dtype=torch.float32, device="cuda")
        self.tx = torch.empty((B,), dtype=torch.int32, device="cuda")
        self.lam = torch.empty((B, gf.m), dtype=torch.float32, device="cuda")
        self.x = torch.empty((B, gf.dim + 1), dtype=torch.float32, device="cuda")
        self.loss = torch.empty(1, dtype=torch.float64, device="cuda")
        self.grid = np.arange(cfg.snr_lo, cfg.snr_hi + 1e-9, cfg.snr_step)
        self.rng = np.random.default_rng(cfg.seed)
        self.llr_ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, self.per, cfg.path))
        self.step_no = 0

    def lr_at(self, k):
        c = self.cfg
        return c.lr_min + 0.5 * (c.lr - c.lr_min) * (1.0 + math.cos(math.pi * min(k, c.steps) / c.steps))

    def step(self):
        c, gf, per = self.cfg, self.gf, self.per
        snrs = self.rng.choice(self.grid, size=c.slices)
        for q, snr in enumerate(snrs):
            sl = slice(q * per, (q + 1) * per)
            s2 = float(sigma2_of(snr, gf.dim))
            slot = 1_000_000 + self.step_no * c.slices + q          # fresh counters every slice
            mdgmi.mdgmi_generate(gf, c.seed, [s2], per, snr_slot0=slot, y=self.y[sl].view(1, per, gf.dim),
                                 tx_idx=self.tx[sl].view(1, per))
            mdgmi.mdgmi_llr(gf, self.y[sl], s2, path=c.path, llr=self.lam[sl], ws=self.llr_ws)
            mdgmi.mdgmi_mlp_features(self.y[sl], float(snr), x=self.x[sl])
        self.net.loss_grad(self.x, self.lam, loss=self.loss)
        self.net.adam_step(self.lr_at(self.step_no))
        self.step_no += 1

    def train(self, steps=None, log=None):
        steps = steps or self.cfg.steps
        res = TrainResult(0, 0)
        for _ in range(steps):
            self.step()
            if self.step_no % self.cfg.log_every == 0 or self.step_no == 1:
                v = float(self.loss.item())
                res.losses.append((self.step_no, v))
                if log:
                    log(f"step {self.step_no} loss {v:.5f} nats ({v * LOG2E:.5f} bits)")
        res.steps = self.step_no
        res.samples = self.step_no * self.cfg.batch
        return res


@dataclass
class Evaluation:
    snr_db: list
    gmi_exact: list
    gmi_learned: list
    loss: list                   # GMI_exact - GMI_learned, paired
    route: list                  # "learned" or "exact" per SNR
    gmi: list                    # the routed estimate
    s_opt: list = field(default_factory=list)         # s maximising GMI(s) of the learned LLRs
    gmi_learned_sopt: list = field(default_factory=list)  # GMI(s*) of the learned LLRs


def evaluate(net: mdgmi.MLP, gf: mdgmi.Format, snr_db, n: int, seed: int = 99, max_loss: float = 0.01,
             path: str = "mfma", snr_slot0: int = 5_000_000, sopt: bool = False):
    """Paired learned vs exact GMI on the same held-out device samples, and
    the per-SNR route."""
    import torch
    snr = np.asarray(snr_db, dtype=np.float64)
    s2 = sigma2_of(snr, gf.dim)
    y, tx = mdgmi.mdgmi_generate(gf, seed, s2, n, snr_slot0=snr_slot0, dtype=torch.float32)
    ex = mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path).cpu().numpy()
    le = mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr).cpu().numpy()
    loss = ex[:, 0] - le[:, 0]
    ok = np.isfinite(le[:, 0]) & (loss <= max_loss)
    route = ["learned" if v else "exact" for v in ok]
    gmi = np.where(ok, le[:, 0], ex[:, 0])
    ev = Evaluation(list(snr), list(ex[:, 0]), list(le[:, 0]), list(loss), route, list(gmi))
    if sopt:
        ev.s_opt, ev.gmi_learned_sopt = sopt_of_learned(net, gf, y, tx, snr)
    return ev, y, tx


def sopt_of_learned(net: mdgmi.MLP, gf: mdgmi.Format, y, tx, snr_db, chunk: int = 1 << 20):
    """Per SNR point, the s-optimised GMI of the network's LLRs (a decoder
    that scales them by s): the learned LLRs of every sample are formed in
    chunks, then mdgmi_gmi_sopt finds s*."""
    import torch
    s_opt, g_opt = [], []
    n = y.shape[1]
    lam = torch.empty((n, gf.m), dtype=torch.float32, device="cuda")
    x = torch.empty((min(chunk, n), gf.dim + 1), dtype=torch.float32, device="cuda")
    for q, v in enumerate(snr_db):
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            xs = x[: c1 - c0]
            mdgmi.mdgmi_mlp_features(y[q, c0:c1].contiguous(), float(v), x=xs)
            net.forward(xs, out=lam[c0:c1])
        o = mdgmi.mdgmi_gmi_sopt(gf, lam, tx[q]).cpu().numpy()
        s_opt.append(float(o[mdgmi.FIELDS_S.index("s_opt")]))
        g_opt.append(float(o[mdgmi.FIELDS_S.index("gmi_sopt")]))
    return s_opt, g_opt
