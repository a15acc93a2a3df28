"""Learned demapper: training on exact-demapper LLR targets and per-SNR
evaluation with fallback to the exact path.

Host-side orchestration only: every step runs in libmdgmi's kernels (device
sample generation, exact LLR targets, the MLP's forward/backward/Adam in
mdgmi_mlp_train_step, learned and exact GMI); the per-SNR route is decided
inside the library by mdgmi_learned_calibrate. The host picks SNR points
and the learning rate.

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
    batch: int = 4096             # samples per Adam step
    slices: int = 16              # SNR points per step (batch / slices samples each)
    chunk: int = 32               # steps whose samples and targets are generated together
    snr_lo: float = 2.0
    snr_hi: float = 17.0
    snr_step: float = 0.25        # training SNRs are drawn from this grid
    lr: float = 4e-3
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
    curve: list = field(default_factory=list)    # (samples seen, paired GMI loss per held-out SNR point)


class HeldOut:
    """Fixed held-out samples at a few SNR points with their exact GMI: the
    paired GMI loss GMI_exact - GMI_learned of a network on them, per SNR
    point (a training curve that does not mix SNR points)."""

    def __init__(self, gf: mdgmi.Format, snr_db=(2.0, 5.0, 8.0, 11.0, 14.0, 17.0), n: int = 65536,
                 seed: int = 999, snr_slot0: int = 7_000_000, path: str = "mfma"):
        import torch
        self.gf = gf
        self.snr = np.asarray(snr_db, dtype=np.float64)
        s2 = sigma2_of(self.snr, gf.dim)
        self.y, self.tx = mdgmi.mdgmi_generate(gf, seed, s2, n, snr_slot0=snr_slot0)
        self.exact = mdgmi.mdgmi_gmi(gf, self.y, self.tx, s2, path=path).cpu().numpy()[:, 0]
        self.out = torch.empty((self.snr.size, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
        self.ws = None

    def loss(self, net: mdgmi.MLP):
        if self.ws is None:
            self.ws = mdgmi.workspace(mdgmi.mdgmi_mlp_gmi_workspace_size(net, self.y.shape[1]))
        mdgmi.mdgmi_mlp_gmi(net, self.gf, self.y, self.tx, self.snr, out=self.out, ws=self.ws)
        return self.exact - self.out.cpu().numpy()[:, 0]


class Trainer:
    """Trains a network [dim + 1, hidden..., m] on one format. Every `chunk`
    steps, slices x chunk x (batch / slices) samples are generated on the
    device at `slices` SNR points drawn from the grid, with their exact LLRs;
    step c of the chunk takes the c-th block of every slice."""

    def __init__(self, gf: mdgmi.Format, cfg: TrainConfig, net: mdgmi.MLP | None = None):
        import torch
        self.gf, self.cfg = gf, cfg
        self.net = net or mdgmi.MLP([gf.dim + 1, *cfg.hidden, gf.m], seed=cfg.seed)
        B, S, C = cfg.batch, cfg.slices, cfg.chunk
        assert B % S == 0
        self.per = B // S
        n = C * self.per
        self.y = torch.empty((S, n, gf.dim), dtype=torch.float32, device="cuda")
        self.tx = torch.empty((S, n), dtype=torch.int32, device="cuda")
        self.lam = torch.empty((S, n, gf.m), dtype=torch.float32, device="cuda")
        # the chunk regrouped by step: step k's batch (block k of every
        # slice) is yb[k], contiguous, so a step copies nothing
        self.yb = torch.empty((C, B, gf.dim), dtype=torch.float32, device="cuda")
        self.lb = torch.empty((C, B, gf.m), dtype=torch.float32, device="cuda")
        self.snr = torch.empty(B, dtype=torch.float32, device="cuda")
        self.loss = torch.empty(1, dtype=torch.float64, device="cuda")
        self.grid = np.arange(cfg.snr_lo, cfg.snr_hi + 1e-9, cfg.snr_step)
        self.rng = np.random.default_rng(cfg.seed)
        self.llr_ws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, n, cfg.path))
        self.train_ws = mdgmi.workspace(self.net.train_workspace_size(B))
        self.step_no = 0

    def lr_at(self, k):
        c = self.cfg
        return c.lr_min + 0.5 * (c.lr - c.lr_min) * (1.0 + math.cos(math.pi * min(k, c.steps) / c.steps))

    def _chunk(self):
        import torch
        c, gf = self.cfg, self.gf
        snrs = self.rng.choice(self.grid, size=c.slices)
        s2 = sigma2_of(snrs, gf.dim)
        slot = 1_000_000 + self.step_no * c.slices             # fresh counters every chunk
        mdgmi.mdgmi_generate(gf, c.seed, s2, c.chunk * self.per, snr_slot0=slot, y=self.y, tx_idx=self.tx)
        for q in range(c.slices):
            mdgmi.mdgmi_llr(gf, self.y[q], float(s2[q]), path=c.path, llr=self.lam[q], ws=self.llr_ws)
        S, per = c.slices, self.per
        self.yb.view(c.chunk, S, per, gf.dim).copy_(self.y.view(S, c.chunk, per, gf.dim).transpose(0, 1))
        self.lb.view(c.chunk, S, per, gf.m).copy_(self.lam.view(S, c.chunk, per, gf.m).transpose(0, 1))
        self.snr.copy_(torch.from_numpy(np.repeat(snrs, self.per).astype(np.float32)))

    def step(self):
        c = self.cfg
        k = self.step_no % c.chunk
        if k == 0:
            self._chunk()
        self.net.train_step(self.yb[k], self.snr, self.lb[k], self.lr_at(self.step_no), loss=self.loss,
                            ws=self.train_ws)
        self.step_no += 1

    def train(self, steps=None, log=None, held_out: HeldOut | None = None, curve_points: int = 8):
        """Runs `steps` Adam steps; with held_out, the paired GMI loss per
        held-out SNR point is recorded curve_points times along the way."""
        steps = steps or self.cfg.steps
        res = TrainResult(0, 0)
        marks = {max(1, round(steps * (q + 1) / curve_points)) for q in range(curve_points)} if held_out else set()
        for k in range(1, steps + 1):
            self.step()
            if self.step_no % self.cfg.log_every == 0 or self.step_no == 1:
                v = float(self.loss.item())
                res.losses.append((self.step_no, v))
                if log:
                    log(f"step {self.step_no} loss {v:.5f} nats ({v * LOG2E:.5f} bits)")
            if k in marks:
                lv = held_out.loss(self.net)
                res.curve.append((self.step_no * self.cfg.batch, [float(v) for v in lv]))
                if log:
                    log(f"{self.step_no * self.cfg.batch:.3g} samples: held-out GMI loss " +
                        " ".join(f"{a:g}dB:{b:.4f}" for a, b in zip(held_out.snr, lv)))
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
    """Paired learned vs exact GMI on the same held-out device samples; the
    per-SNR route is decided by the library (mdgmi_learned_calibrate), which
    attaches the network to gf for MDGMI_PATH_LEARNED_BF16."""
    import torch
    snr = np.asarray(snr_db, dtype=np.float64)
    s2 = sigma2_of(snr, gf.dim)
    y, tx = mdgmi.mdgmi_generate(gf, seed, s2, n, snr_slot0=snr_slot0, dtype=torch.float32)
    res = mdgmi.mdgmi_learned_calibrate(gf, net, y, tx, s2, exact_path=path, max_loss=max_loss)
    ok = res[:, 3] == 1
    route = ["learned" if v else "exact" for v in ok]
    gmi = np.where(ok, res[:, 1], res[:, 0])
    ev = Evaluation(list(snr), list(res[:, 0]), list(res[:, 1]), list(res[:, 2]), route, list(gmi))
    if sopt:
        ev.s_opt, ev.gmi_learned_sopt = sopt_of_learned(net, gf, y, tx, snr)
    return ev, y, tx


def sopt_of_learned(net: mdgmi.MLP, gf: mdgmi.Format, y, tx, snr_db):
    """Per SNR point, the s-optimised GMI of the network's LLRs (a decoder
    that scales them by s): mdgmi_mlp_llr forms the LLRs of every sample,
    then mdgmi_gmi_sopt finds s*."""
    import torch
    s_opt, g_opt = [], []
    n = y.shape[1]
    lam = torch.empty((n, gf.m), dtype=torch.float32, device="cuda")
    snr = torch.empty(n, dtype=torch.float32, device="cuda")
    for q, v in enumerate(snr_db):
        snr.fill_(float(v))
        net.llr(y[q], snr, out=lam)
        o = mdgmi.mdgmi_gmi_sopt(gf, lam, tx[q]).cpu().numpy()
        s_opt.append(float(o[mdgmi.FIELDS_S.index("s_opt")]))
        g_opt.append(float(o[mdgmi.FIELDS_S.index("gmi_sopt")]))
    return s_opt, g_opt
