"""Named synthetic workloads (sizes follow the paper's 4-electron
beryllium runs: 2 alpha + 2 beta electrons, CISD / CISDT / CISDTQ).

Each workload fixes norb, box length, number of auxiliary points, the
excitation level and the screening threshold; the integrals come from
recipe A with the given seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    norb: int
    nalpha: int = 2
    nbeta: int = 2
    level: int = 2          # max excitation level: 2 CISD, 3 CISDT, 4 CISDTQ
    tau: float = 1e-14
    nvec: int = 1
    nroots: int = 1
    box: float | None = None
    naux: int | None = None
    seed: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def gas_boundary(self) -> int:
        """Two-space GAS boundary orbital (0: the excitation hierarchy)."""
        return int(self.extra.get("gas_boundary", 0))

    @property
    def box_len(self) -> float:
        return float(self.norb) if self.box is None else float(self.box)

    @property
    def n_aux(self) -> int:
        return int(round(2 * self.box_len)) if self.naux is None else int(self.naux)

    def integrals(self, recipe: str = "A"):
        from .recipes import recipe_a, recipe_b
        f = {"A": recipe_a, "B": recipe_b}[recipe]
        return f(self.norb, self.box_len, self.n_aux, self.seed)


WORKLOADS = {
    # plain CISD, 20 orbitals in a 20 bohr box, 40 aux points
    "cisd_n20": Workload("cisd_n20", norb=20, level=2, tau=1e-14, nvec=1),
    # plain CISDT, 60 orbitals, 120 aux points (tau sweep 0 / 1e-14 / 1e-10)
    "cisdt_n60": Workload("cisdt_n60", norb=60, level=3, tau=1e-14, nvec=8),
    "cisdt_n30": Workload("cisdt_n30", norb=30, level=3, tau=1e-14, nvec=1),
    "cisdt_n120": Workload("cisdt_n120", norb=120, level=3, tau=1e-14, nvec=1),
    # served-size CISDT, 160 orbitals, tau 1e-12, 4 vectors (one-body classes
    # in the spectator form dominate)
    "cisdt_n160": Workload("cisdt_n160", norb=160, level=3, tau=1e-12, nvec=4),
    # CISDTQ = FCI for 4 electrons, 48 orbitals, 8 simultaneous vectors
    "fci_n48": Workload("fci_n48", norb=48, level=4, tau=1e-14, nvec=8),
    # two-space GAS: full CI in the 16 lowest orbitals, at most one electron
    # in the 184 above them (the single-continuum-electron restriction),
    # 200 orbitals in a 200 bohr box, tau 1e-12, 8 vectors
    "gas1_n200": Workload("gas1_n200", norb=200, level=1, tau=1e-12, nvec=8,
                          extra={"gas_boundary": 16}),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_instances(count: int = 64, seed: int = 7, nmin: int = 20,
                      nmax: int = 80, tau: float = 1e-12):
    """Uneven instances for the batched pattern: norb ~ U{nmin..nmax},
    level ~ {CISD, CISDT}, roots ~ U{1..4}, per-instance seeds."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        norb = int(rng.integers(nmin, nmax + 1))
        level = int(rng.choice([2, 3]))
        nroots = int(rng.integers(1, 5))
        out.append(Workload(f"batch{i}", norb=norb, level=level, tau=tau,
                            nroots=nroots, seed=1000 + i))
    return out


def served_requests(count: int = 2000, rate: float = 50.0, seed: int = 11,
                    nmin: int = 40, nmax: int = 200, tau: float = 1e-12,
                    fci_dim_limit: int = 5_000_000):
    """Poisson arrivals (exponential gaps, mean 1/rate seconds); norb
    log-uniform in [nmin, nmax]; level in {CISD, CISDT, CISDTQ if its
    dimension is below fci_dim_limit}; 1..3 roots."""
    from math import comb
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        norb = int(round(float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))))
        levels = [2, 3]
        if comb(norb, 2) ** 2 < fci_dim_limit:
            levels.append(4)
        level = int(rng.choice(levels))
        nroots = int(rng.integers(1, 4))
        out.append((t, Workload(f"req{i}", norb=norb, level=level, tau=tau,
                                nroots=nroots, seed=5000 + i)))
    return out
