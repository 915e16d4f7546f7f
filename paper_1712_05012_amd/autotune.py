"""Autotuner for a batch of chains: cell edge, force-kernel launch shape and
iterations per graph.

Three settings change the speed of an iteration but not its results beyond
rounding order: the edge of the cells of the grid (``kcm_params.cell_size``;
0 picks half the reach), the launch shape of the force kernel
(``kcm_set_force_variant``: candidates per lane per trip, the block of
neighbours step 1 reads before its saturation check and the atoms' order
over the XCDs; identical results) and
how many iterations one replayed HIP graph holds (``kcm_set_graphs``).
``tune`` builds trial copies of the chains for every candidate edge, times a
few iterations at every shape and depth on the device, and returns the
fastest setting together with the whole table it measured.  The trial chains
are freed; the caller builds its own with the chosen parameters.

The timing runs through the C ABI only (``kcm_step`` on the given stream),
with one device synchronisation before and after each timed run.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field


@dataclass
class TuneResult:
    cell_size: float                 # 0.0: automatic (half the reach)
    graph_depth: int                 # iterations per replayed graph
    atom_steps_per_s: float
    force_variant: int = 0           # launch shape of the force kernel
    table: list = field(default_factory=list)  # (cell_size, variant, depth, grid cell edge, atom-steps/s)

    def as_dict(self):
        return {"cell_size": self.cell_size, "force_variant": self.force_variant, "graph_depth": self.graph_depth,
                "atom_steps_per_s": self.atom_steps_per_s,
                "table": [{"cell_size": c, "force_variant": v, "graph_depth": d, "grid_cell": g,
                           "atom_steps_per_s": r} for c, v, d, g, r in self.table]}


def tune(residue_types, items, precision, cell_sizes=(0.0, 4.4, 3.6), variants=(0, 1, 2, 3), depths=(1, 4, 8),
         iters: int = 8, warmup: int = 2, stream=None) -> TuneResult:
    """items: [(res_type, theta0)] of the batch; returns the fastest setting.
    Leaves the force variant at the fastest one and graphs at depth 1."""
    import torch

    from . import kcm

    if not items:
        raise ValueError("nothing to tune")
    table = []
    try:
        for cs in cell_sizes:
            p = kcm.kcm_default_params(precision=precision, cell_size=cs)
            chains = [kcm.Chain(seq, residue_types, p, theta0=th, stream=stream) for seq, th in items]
            atoms = sum(c.n_atoms for c in chains)
            try:
                for v in variants:
                    kcm.kcm_set_force_variant(v)
                    for d in depths:
                        kcm.kcm_set_graphs(d)
                        kcm.kcm_step(chains, warmup + d, stream, report=False)  # captures the graphs
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        kcm.kcm_step(chains, iters * d, stream, report=False)
                        torch.cuda.synchronize()
                        rate = atoms * iters * d / (time.perf_counter() - t0)
                        table.append((float(cs), int(v), int(d), float(chains[0].cells(stream)["cell"]), rate))
            finally:
                for c in chains:
                    c.free()
    finally:
        kcm.kcm_set_graphs(1)
    cs, v, d, _, rate = max(table, key=lambda row: row[4])
    kcm.kcm_set_force_variant(v)
    return TuneResult(cell_size=cs, graph_depth=d, atom_steps_per_s=rate, force_variant=v, table=table)
