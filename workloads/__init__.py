"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds only input generation: constellation geometries with their
bit labels, the SNR -> noise-variance convention, and a counter-based random
number generator that draws transmitted symbol indices and Gaussian noise.
It contains none of the demapping arithmetic (no distances to the
constellation, no LLRs, no GMI or MI), so both sides of every parity test can
consume the very same arrays.

Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), a counter-based generator, so any single
sample can be regenerated on its own from (seed, SNR slot, sample index).
Gaussian deviates come from the Box-Muller transform (Box & Muller 1958).
The HIP library carries its own implementation of the same published
definition for large on-device workloads; the two are compared in the tests.

Channel (standard AWGN model, the one behind the AWGN/SNR glossary entries):
y = x_i + z, i uniform on the M points, z ~ N(0, sigma2 * I_N), with the
constellation normalised to unit average energy per N-dimensional symbol and
SNR = E||x||^2 / E||z||^2, i.e. sigma2 = 1 / (N * 10^(SNR_dB/10)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Philox-4x32-10 (Salmon et al., SC'11): 10 rounds of a 4-word S-P network
# driven by two 32x32->64 multiplications, with a Weyl-sequence key schedule.
# ---------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

# Counter word 3 selects the purpose of a draw for one sample.
CALL_INDEX = 0          # word 0 -> transmitted symbol index
CALL_NORMAL0 = 1        # calls 1, 2 -> four Gaussian deviates each
# Counter word 2 for format-generation draws (kept apart from SNR slots).
FORMAT_TAG = 0x464D5400  # "FMT\0"


def philox4x32_10(ctr, key):
    """Philox-4x32-10 on arrays.

    ctr: uint32 array of shape (..., 4); key: uint32 array of shape (..., 2)
    (broadcastable against ctr[..., :2]). Returns uint32 (..., 4).
    """
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def _key(seed: int) -> np.ndarray:
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)


def _counters(idx: np.ndarray, word2: int, call: int) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = np.empty(idx.shape + (4,), dtype=np.uint32)
    ctr[..., 0] = (idx & _MASK32).astype(np.uint32)
    ctr[..., 1] = (idx >> np.uint64(32)).astype(np.uint32)
    ctr[..., 2] = np.uint32(word2 & 0xFFFFFFFF)
    ctr[..., 3] = np.uint32(call)
    return ctr


def uniform_open01(w: np.ndarray) -> np.ndarray:
    """32-bit word -> float64 in (0, 1): (w + 1/2) * 2^-32 (exact in FP64)."""
    return (w.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


TWO_PI = 6.283185307179586


def box_muller(w_a: np.ndarray, w_b: np.ndarray):
    """Two uniform words -> two independent N(0,1) deviates (FP64)."""
    u1 = uniform_open01(w_a)
    u2 = uniform_open01(w_b)
    r = np.sqrt(-2.0 * np.log(u1))
    ang = TWO_PI * u2
    return r * np.cos(ang), r * np.sin(ang)


def normals(seed: int, word2: int, idx: np.ndarray, dim: int) -> np.ndarray:
    """dim Gaussian deviates for every counter index in idx -> (len(idx), dim)."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = _key(seed)
    out = np.empty((idx.shape[0], dim), dtype=np.float64)
    ncalls = (dim + 3) // 4
    for c in range(ncalls):
        w = philox4x32_10(_counters(idx, word2, CALL_NORMAL0 + c), key)
        z0, z1 = box_muller(w[:, 0], w[:, 1])
        z2, z3 = box_muller(w[:, 2], w[:, 3])
        for q, z in enumerate((z0, z1, z2, z3)):
            d = 4 * c + q
            if d < dim:
                out[:, d] = z
    return out


def symbol_indices(seed: int, snr_slot: int, idx: np.ndarray, m: int) -> np.ndarray:
    """Uniform transmitted indices in [0, 2^m): top m bits of Philox word 0."""
    idx = np.asarray(idx, dtype=np.uint64)
    if m == 0:
        return np.zeros(idx.shape[0], dtype=np.uint32)
    w = philox4x32_10(_counters(idx, snr_slot, CALL_INDEX), _key(seed))
    return (w[:, 0] >> np.uint32(32 - m)).astype(np.uint32)


# ---------------------------------------------------------------------------
# Constellations (formats). X is (M, N) float64, labels[j] is the m-bit label
# of row j; bit k of the label is LLR column k (LSB first).
# ---------------------------------------------------------------------------
@dataclass
class Format:
    name: str
    X: np.ndarray                 # (M, N) float64, unit average energy
    labels: np.ndarray            # (M,) uint32, a permutation of [0, M)
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.X.shape[0])

    @property
    def dim(self) -> int:
        return int(self.X.shape[1])

    @property
    def m(self) -> int:
        return int(round(math.log2(self.M)))


def gray(i):
    return i ^ (i >> 1)


def normalize(X: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    return X / math.sqrt(float(np.mean(np.sum(X * X, axis=1))))


def check_labels(labels: np.ndarray, M: int) -> bool:
    labels = np.asarray(labels)
    return labels.shape == (M,) and np.array_equal(np.sort(labels.astype(np.int64)),
                                                  np.arange(M, dtype=np.int64))


def pam(m: int) -> Format:
    """Gray-labelled 2^m-PAM on one real axis (levels ascending)."""
    L = 1 << m
    a = np.arange(L)
    X = (2.0 * a - (L - 1)).reshape(L, 1)
    return Format(f"{L}-PAM", normalize(X), gray(a).astype(np.uint32), {"kind": "pam"})


def qam(m_i: int, m_q: int) -> Format:
    """Gray-labelled (rectangular when m_i != m_q) QAM: label = g(aI)<<m_q | g(aQ)."""
    LI, LQ = 1 << m_i, 1 << m_q
    aI, aQ = np.meshgrid(np.arange(LI), np.arange(LQ), indexing="ij")
    aI, aQ = aI.ravel(), aQ.ravel()
    X = np.stack([2.0 * aI - (LI - 1), 2.0 * aQ - (LQ - 1)], axis=1)
    labels = ((gray(aI) << m_q) | gray(aQ)).astype(np.uint32)
    return Format(f"{LI * LQ}-QAM", normalize(X), labels, {"kind": "qam"})


def square_qam(m: int) -> Format:
    assert m % 2 == 0
    return qam(m // 2, m // 2)


def psk(m: int, offset: float = 0.0) -> Format:
    """Gray-labelled 2^m-PSK, point k at angle offset + 2*pi*k/M."""
    M = 1 << m
    k = np.arange(M)
    ang = offset + 2.0 * math.pi * k / M
    X = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return Format(f"{M}-PSK", normalize(X), gray(k).astype(np.uint32), {"kind": "psk"})


def two_ring_8(ratio: float = 1.8) -> Format:
    """8 points: inner/outer rings (radius 1 and `ratio`), phases pi/4 + k*pi/2
    on both rings, label = ring<<2 | gray(k)."""
    k = np.arange(4)
    ang = math.pi / 4 + k * math.pi / 2
    pts, labs = [], []
    for ring, r in enumerate((1.0, ratio)):
        for kk in k:
            pts.append([r * math.cos(ang[kk]), r * math.sin(ang[kk])])
            labs.append((ring << 2) | int(gray(kk)))
    return Format(f"2ring8-{ratio}", normalize(np.array(pts)), np.array(labs, dtype=np.uint32),
                  {"kind": "ring"})


def product(fa: Format, fb: Format, name: str | None = None) -> Format:
    """Cartesian product: point (a, b) = [x_a, x_b], label = l_a << m_b | l_b."""
    Ma, Mb = fa.M, fb.M
    ia, ib = np.meshgrid(np.arange(Ma), np.arange(Mb), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()
    X = np.concatenate([fa.X[ia], fb.X[ib]], axis=1)
    labels = ((fa.labels[ia].astype(np.uint64) << np.uint64(fb.m)) | fb.labels[ib]).astype(np.uint32)
    return Format(name or f"{fa.name}x{fb.name}", normalize(X), labels, {"kind": "product"})


def single_point(dim: int = 2) -> Format:
    return Format("point", np.zeros((1, dim)), np.zeros(1, dtype=np.uint32), {"kind": "point"})


def random_shells(dim: int, M: int, seed: int, radii=(1.0, 1.6)) -> Format:
    """Seeded random format: g_j ~ N(0, I_dim) (Philox/Box-Muller), projected to
    radius radii[0] for j < M/2 and radii[1] otherwise, normalised to unit
    average energy; label_j = j."""
    g = normals(seed, FORMAT_TAG + dim, np.arange(M, dtype=np.uint64), dim)
    r = np.where(np.arange(M) < M // 2, radii[0], radii[1])
    X = g / np.linalg.norm(g, axis=1, keepdims=True) * r[:, None]
    return Format(f"shells{dim}D-{M}", normalize(X), np.arange(M, dtype=np.uint32),
                  {"kind": "shells", "seed": seed})


def qam_product(dim: int, m: int) -> Format:
    """dim/2 Gray-QAM components sharing m bits as evenly as possible
    (square QAM for an even share, rectangular for odd, BPSK for one bit,
    a single point at the origin for none)."""
    ncomp = dim // 2
    shares = [m // ncomp + (1 if c < m % ncomp else 0) for c in range(ncomp)]
    comps = []
    for b in shares:
        if b == 0:
            comps.append(single_point(2))
        else:
            comps.append(qam((b + 1) // 2, b // 2))
    f = comps[0]
    for c in comps[1:]:
        f = product(f, c)
    f.name = f"qamprod{dim}D-{1 << m}"
    f.meta = {"kind": "qamprod", "shares": shares}
    return f


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def sigma2_from_snr_db(snr_db, dim: int):
    """Per-real-dimension noise variance for unit-energy formats."""
    return 1.0 / (dim * 10.0 ** (np.asarray(snr_db, dtype=np.float64) / 10.0))


def format_16qam() -> Format:
    return square_qam(4)


def format_4d64() -> Format:
    f = product(two_ring_8(1.8), two_ring_8(1.8), name="4D-64-2ring")
    return f


FORMAT_8D_SEED = 2048


def format_8d2048() -> Format:
    f = random_shells(8, 2048, FORMAT_8D_SEED, radii=(1.0, 1.6))
    f.name = "8D-2048-2shell"
    return f


@dataclass
class Workload:
    name: str
    fmt: Format
    snr_db: np.ndarray
    n: int            # samples per SNR
    seed: int
    dtype: str        # "f64" or "f32"

    @property
    def sigma2(self) -> np.ndarray:
        return sigma2_from_snr_db(self.snr_db, self.fmt.dim)


def paper_formats() -> list:
    """The modulation formats the paper transmits: Gray PAM-2/4/8/16 on one
    real axis (IM/DD chain) and Gray square QAM-4/16/64 (Kramers-Kronig
    chain), unit average energy."""
    return [pam(1), pam(2), pam(3), pam(4), square_qam(2), square_qam(4), square_qam(6)]


def workload_qam16(n: int = 100_000, seed: int = 0) -> Workload:
    return Workload("2D 16-QAM Gray, 11 SNR x 1e5", format_16qam(),
                    np.arange(0.0, 20.0 + 1e-9, 2.0), n, seed, "f64")


def workload_4d64(n: int = 10_000_000, seed: int = 1) -> Workload:
    return Workload("4D M=64 two-ring product, 21 SNR x 1e7", format_4d64(),
                    np.arange(-2.0, 18.0 + 1e-9, 1.0), n, seed, "f32")


def workload_8d2048(n: int = 10_000_000, seed: int = 2) -> Workload:
    return Workload("8D M=2048 two-shell, 16 SNR x 1e7", format_8d2048(),
                    np.arange(2.0, 17.0 + 1e-9, 1.0), n, seed, "f32")


def ragged_formats(seed: int = 3) -> list:
    """48 formats: 16 per dimension in {2,4,8}; M cycles over 4..4096; the kind
    alternates between seeded random shells and Gray-QAM products."""
    fmts = []
    ms = list(range(2, 13))
    for di, dim in enumerate((2, 4, 8)):
        for q in range(16):
            m = ms[(q + 5 * di) % len(ms)]
            M = 1 << m
            if q % 2 == 0:
                f = random_shells(dim, M, seed * 1000 + di * 16 + q)
            else:
                f = qam_product(dim, m)
            fmts.append(f)
    return fmts


def ragged_counts(n_formats: int, n_snr: int, seed: int = 3, lo: float = 4.0, hi: float = 7.0):
    """Symbol counts per (format, SNR), log-uniform in [10^lo, 10^hi]."""
    w = philox4x32_10(_counters(np.arange(n_formats * n_snr, dtype=np.uint64), 0x52414744, 0),
                      _key(seed))
    u = uniform_open01(w[:, 0])
    return np.round(10.0 ** (lo + (hi - lo) * u)).astype(np.int64).reshape(n_formats, n_snr)


RAGGED_SNR_DB = np.arange(-5.0, 25.0 + 1e-9, 1.0)


# ---------------------------------------------------------------------------
# Channel samples on the host (the device generator produces the same values)
# ---------------------------------------------------------------------------
def channel_samples(fmt: Format, sigma2: float, seed: int, snr_slot: int, idx=None, n: int | None = None):
    """Returns (y float64 (len, N), tx_idx uint32) for sample indices idx (or
    0..n-1) in SNR slot snr_slot: y = x_i + sqrt(sigma2) * z."""
    if idx is None:
        idx = np.arange(n, dtype=np.uint64)
    idx = np.asarray(idx, dtype=np.uint64)
    tx = symbol_indices(seed, snr_slot, idx, fmt.m)
    z = normals(seed, snr_slot, idx, fmt.dim)
    y = fmt.X[tx] + math.sqrt(float(sigma2)) * z
    return y, tx


def workload_samples(wl: Workload, n: int | None = None, dtype=None):
    """All SNR slots of a workload: y (n_snr, n, N), tx (n_snr, n)."""
    n = wl.n if n is None else n
    ys, txs = [], []
    for s, s2 in enumerate(wl.sigma2):
        y, tx = channel_samples(wl.fmt, s2, wl.seed, s, n=n)
        ys.append(y)
        txs.append(tx)
    y = np.stack(ys)
    if dtype is not None:
        y = y.astype(dtype)
    return y, np.stack(txs)
