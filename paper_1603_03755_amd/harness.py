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
