"""Penalty-scan harness: the experiment shape of Sec. III (Figs. 3-7) on
synthetic instances.

For every instance and every penalty strength lambda, the embeddings (ME on
Chimera as in the paper, optionally the clique-chain ME, and LHZ; Sec. II A /
II B) are annealed with SQA, every replica's readout slice is decoded, and the
success probability p_s is the fraction of replicas whose decoded logical
state is a ground state of Eq. (1).  The optimal penalty of an
instance and scheme is the lambda with the largest p_s (Fig. 5).

Units.  The paper's couplings are J_ij in {+-0.1, ..., +-1} (Sec. III).  The
library works in integers, so every coefficient is multiplied by 10
(J' in {+-1..+-10}, penalty coefficient -10 lambda) and the temperature and
transverse field are rescaled so that the Trotter action is unchanged:
beta' = beta / 10 and Gamma' = 10 Gamma (beta' Gamma' = beta Gamma,
beta' J' = beta J).

Schedule (the paper shows it only in a figure): Gamma linear from
`gamma_start` to `gamma_end` (paper units) with B = 1, and the inverse
temperature chosen so that the final effective temperature is the one the
caption of Fig. 2 states (about 0.05 in units of J): beta_eff = 20.

Everything runs through the C ABI: one persistent batched launch per scan
(all instances x penalties x embeddings), device decoders, device exhaustive
ground states.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence

import numpy as np

from . import sqa
from .workloads import LHZ, ME, MEC, sk_instance

KINDS = {"mec": MEC, "me": ME, "lhz": LHZ}

SCALE = 10
PAPER_VALUES = tuple(v for v in range(-SCALE, SCALE + 1) if v != 0)   # J * 10, J in {+-0.1..+-1}


def paper_instance(n: int, seed: int) -> np.ndarray:
    """SK-like instance with J_ij uniform in {+-0.1, ..., +-1}, returned times 10."""
    return sk_instance(n, seed, values=PAPER_VALUES)


def penalty_coefficient(lam: float) -> int:
    """Signed integer coefficient of a penalty strength lambda (paper units)."""
    c = int(round(SCALE * lam))
    if abs(SCALE * lam - c) > 1e-9:
        raise ValueError("penalty strengths are multiples of 0.1")
    return -c


@dataclasses.dataclass
class ScanConfig:
    """SQA parameters of the paper's main results: L = 64 (Appendix B), 10^4 sweeps and
    1000 reads per instance and penalty (Sec. III, Appendix D), Wolff moves."""
    sweeps: int = 10_000
    reads: int = 1000
    slices: int = 64
    beta_eff: float = 20.0           # 1 / (final effective temperature 0.05), paper units
    gamma_start: float = 3.0         # paper units
    gamma_end: float = 0.01
    move: int = sqa.SQA_MOVE_WOLFF
    schemes: Sequence[str] = ("mec", "lhz")    # ME on Chimera, LHZ; "me" adds the clique-chain ME
    lhz_decoders: Sequence[str] = ("mvd", "mwd", "bp")
    trees: int = 3                   # majority-vote trees (3 for K8, 5 for K16 in Fig. 2)
    seed: int = 0x5EED


@dataclasses.dataclass
class ScanResult:
    penalties: List[float]
    ground_energy: List[int]                       # per instance, J' units
    p_s: Dict[str, np.ndarray]                     # scheme -> [instance][penalty]
    seconds_anneal: float = 0.0
    site_slices: float = 0.0

    def optimal(self, scheme: str):
        """(optimal penalty, p_s there) per instance."""
        ps = self.p_s[scheme]
        idx = np.argmax(ps, axis=1)
        return [self.penalties[i] for i in idx], ps[np.arange(ps.shape[0]), idx]


def penalty_scan(instances: Sequence[np.ndarray], penalties: Sequence[float], cfg: ScanConfig | None = None,
                 stream=None) -> ScanResult:
    """Runs the scan; instances are integer J matrices in the times-10 units."""
    import time
    cfg = cfg or ScanConfig()
    beta = cfg.beta_eff / SCALE
    g0, g1 = SCALE * cfg.gamma_start, SCALE * cfg.gamma_end
    handles, keys = [], []
    kinds = [KINDS[x] for x in cfg.schemes]
    for i, J in enumerate(instances):
        for k, lam in enumerate(penalties):
            pen = penalty_coefficient(lam)
            for kind in kinds:
                seed = cfg.seed + 1000 * i + 10 * k + kind
                handles.append(sqa.SQA(kind, J, pen, beta, cfg.slices, cfg.sweeps, cfg.reads, g0, g1, seed,
                                       move=cfg.move))
                keys.append((i, k, kind))
    e0 = [sqa.sqa_ground_state(J)[0] for J in instances]
    batch = sqa.Batch(handles)
    t0 = time.perf_counter()
    batch.run(stream)
    handles[0].sync()
    dt = time.perf_counter() - t0
    batch.close()
    nI, nP = len(instances), len(penalties)
    out = {}
    for x in cfg.schemes:
        if x == "lhz":
            for d in cfg.lhz_decoders:
                out["lhz_" + d] = np.zeros((nI, nP))
        else:
            out[x] = np.zeros((nI, nP))
    site_slices = 0.0
    for h, (i, k, kind) in zip(handles, keys):
        site_slices += float(h.sites) * h.slices * h.replicas * h.sweeps
        N = instances[i].shape[0]
        if kind != LHZ:
            _, E = h.decode(sqa.SQA_DEC_ME_MAJORITY, 0)
            out["mec" if kind == MEC else "me"][i, k] = float(np.mean(E == e0[i]))
            continue
        trees = sqa.sqa_random_trees(cfg.seed + i, N, cfg.trees)
        for d in cfg.lhz_decoders:
            if d == "mvd":
                _, E = h.decode(sqa.SQA_DEC_LHZ_TREES, 0, trees=trees)
            elif d == "mwd":
                _, E = h.decode(sqa.SQA_DEC_LHZ_MWD, 0)
            elif d == "bp":
                _, E = h.decode(sqa.SQA_DEC_LHZ_BP, 0, trees=trees[:1], error_rate=0.2, iterations=10)
            elif d == "mld":
                _, E = h.decode(sqa.SQA_DEC_LHZ_MLD, 0, error_rate=0.2)
            else:
                raise ValueError(f"unknown decoder {d}")
            out["lhz_" + d][i, k] = float(np.mean(E == e0[i]))
    for h in handles:
        h.close()
    return ScanResult(list(penalties), e0, out, dt, site_slices)


# ------------------------------------------------------------- PT penalty scan
@dataclasses.dataclass
class PTScanConfig:
    """PT parameters of Appendix B: 64 temperatures with beta geometric from 20 down to
    0.1 (paper units, Eq. (B2)), 10 sweeps per swap.  The paper runs 10^5 swaps; the
    default here is 10^4.  Every (instance, penalty, scheme) runs `runs` independent
    ladders; the final state of each ladder's slot at a temperature is one sample of
    that temperature (reading: the paper does not say how it sampled p_s)."""
    temps: int = 64
    beta_max: float = 20.0           # paper units
    beta_min: float = 0.1
    sweeps_per_swap: int = 10
    swaps: int = 10_000
    runs: int = 32
    schemes: Sequence[str] = ("mec", "lhz")
    lhz_decoder: str = "mvd"          # majority vote over spanning trees (Eq. (5)), as for Fig. 7; or "mwd"
    trees: int = 3
    seed: int = 0x97

    @property
    def sweeps(self) -> int:
        return self.swaps * self.sweeps_per_swap


@dataclasses.dataclass
class PTScanResult:
    penalties: List[float]
    betas: np.ndarray                              # ladder, paper units, slot 0 coldest
    ground_energy: List[int]
    p_s: Dict[str, np.ndarray]                     # scheme -> [instance][penalty][slot]
    seconds_pt: float = 0.0
    attempts: float = 0.0

    def critical(self, scheme: str, slot: int = 0) -> List[float]:
        """Per instance, the penalty at which p_s at `slot` (slot 0: beta = 20) first
        reaches 0.5 (Fig. 7), linearly interpolated between the two scan points around
        the crossing; the first penalty if p_s is already >= 0.5 there, NaN if it never
        gets there."""
        out = []
        for ps in self.p_s[scheme][:, :, slot]:
            lam = float("nan")
            for k, p in enumerate(ps):
                if p >= 0.5:
                    if k == 0:
                        lam = self.penalties[0]
                    else:
                        l0, l1, p0 = self.penalties[k - 1], self.penalties[k], ps[k - 1]
                        lam = l0 + (0.5 - p0) * (l1 - l0) / (p - p0)
                    break
            out.append(lam)
        return out


def pt_seed(cfg: PTScanConfig, i: int, k: int, kind: int, run: int) -> int:
    return cfg.seed + (((i * 64 + k) * 4 + kind) << 16) + run


def pt_penalty_scan(instances: Sequence[np.ndarray], penalties: Sequence[float], cfg: PTScanConfig | None = None,
                    stream=None) -> PTScanResult:
    """Runs every ladder of the scan in one batched PT launch, then decodes each
    ladder's final states on the device (ME: majority vote of the chains, Eq. (4);
    LHZ: spanning-tree majority vote, Eq. (5), or minimum-weight decoding) and
    scores them against the exhaustive ground state."""
    import time
    cfg = cfg or PTScanConfig()
    bmin, bmax = cfg.beta_min / SCALE, cfg.beta_max / SCALE
    kinds = [KINDS[x] for x in cfg.schemes]
    ladders, keys = [], []
    for i, J in enumerate(instances):
        for k, lam in enumerate(penalties):
            pen = penalty_coefficient(lam)
            for kind in kinds:
                for run in range(cfg.runs):
                    ladders.append(sqa.PT(kind, J, pen, bmin, bmax, cfg.temps, cfg.sweeps, cfg.sweeps_per_swap,
                                          pt_seed(cfg, i, k, kind, run)))
                keys.append((i, k, kind))
    e0 = [sqa.sqa_ground_state(J)[0] for J in instances]
    t0 = time.perf_counter()
    sqa.pt_run_batch(ladders, stream)
    dt = time.perf_counter() - t0
    attempts = float(sum(h.sites * h.temps for h in ladders)) * cfg.sweeps
    nI, nP, T = len(instances), len(penalties), cfg.temps
    out = {x: np.zeros((nI, nP, T)) for x in cfg.schemes}
    names = {v: k for k, v in KINDS.items()}
    for q, (i, k, kind) in enumerate(keys):
        J = instances[i]
        N = J.shape[0]
        group = ladders[q * cfg.runs:(q + 1) * cfg.runs]
        states = np.stack([h.read()[0] for h in group])          # [run][slot][site]
        # the samples as the replicas of a one-slice handle of the same embedding, decoded on the device
        dec = sqa.SQA(kind, J, penalty_coefficient(penalties[k]), 1.0, 1, 1, cfg.runs * T, 1.0, 1.0, 0)
        dec.write_spins(states.reshape(cfg.runs * T, 1, -1))
        if kind != LHZ:
            _, E = dec.decode(sqa.SQA_DEC_ME_MAJORITY, 0)
        elif cfg.lhz_decoder == "mwd":
            _, E = dec.decode(sqa.SQA_DEC_LHZ_MWD, 0)
        else:
            _, E = dec.decode(sqa.SQA_DEC_LHZ_TREES, 0, trees=sqa.sqa_random_trees(cfg.seed + i, N, cfg.trees))
        dec.close()
        out[names[kind]][i, k] = np.mean((E == e0[i]).reshape(cfg.runs, T), axis=0)
    for h in ladders:
        h.close()
    betas = bmax * np.power(bmin / bmax, np.arange(T) / max(T - 1, 1)) * SCALE
    return PTScanResult(list(penalties), betas, e0, out, dt, attempts)
