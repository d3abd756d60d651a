"""Step driver: the sequence of library calls that makes one PIC step.

    pic_yee_step(half=1)                  E^n, B^n, J^n   -> E^{n+1/2}, B^{n+1/2}
    J = 0
    pic_gather_push_deposit(species ...)  particles n -> n+1, J^{n+1}
    pic_yee_step(half=2)                  -> E^{n+1}, B^{n+1}
    pic_sort of each species every `sort_every` steps (FP32 layout; a slow
    species, such as the ions, may take a longer interval of its own)

Orchestration only (Sec. II.F of the paper gives the order); every step runs
in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import torch

from . import _lib as L
from .workloads import RawParticles, Workload, fields_for, to_fp32, to_fp64


class Simulation:
    def __init__(self, cfg: L.Config, species: List[L.Species], particles: List[L.Particles],
                 fields: L.Fields, sort_every: int = 8, device="cuda",
                 sort_every_species: Optional[List[int]] = None):
        self.cfg = cfg
        self.ctx = L.pic_init(cfg)
        self.species = species
        self.particles = particles
        self.fields = fields
        self.sort_every = max(1, int(sort_every))
        # steps between the sorts of each species (default: sort_every for all)
        self.sort_every_species = ([max(1, int(v)) for v in sort_every_species] if sort_every_species
                                   else [self.sort_every] * len(particles))
        if len(self.sort_every_species) != len(particles):
            raise ValueError("sort_every_species needs one interval per species")
        self.device = device
        self.fp32 = cfg.precision == L.PIC_FP32_MIXED
        self.bits, self.tile, self.ntiles = L.pic_get_layout(self.ctx)
        self.spare: List[Optional[L.Particles]] = []
        if self.fp32:
            for p in particles:
                if p.tile_start is None:
                    p.tile_start = torch.zeros(self.ntiles + 1, dtype=torch.int64, device=device)
                self.spare.append(p.empty_like())
        self.diag = torch.zeros(4, dtype=torch.float64, device=device)
        # scratch for the largest species up front: no call grows it later
        L.pic_reserve(self.ctx, max([p.capacity or p.n for p in particles] + [0]))
        self.step_index = 0
        self.sorted_at = [-1] * len(particles)  # step of each species' last sort (-1: never)

    @staticmethod
    def from_workload(wl: Workload, precision=L.PIC_FP32_MIXED, device="cuda", sort_every=8,
                      from_fp32=False, with_chi=False, drift=2, tile=None, heavy_sort_factor=1):
        """heavy_sort_factor: species of mass >= 100 m_e (the ions) are sorted
        every heavy_sort_factor * sort_every steps."""
        cfg = L.Config(**{**wl.cfg.__dict__})
        cfg.precision = precision
        cfg.drift = drift
        if tile is not None:
            cfg.tile = tile
        ctx_probe = L.pic_init(cfg)
        bits, _, _ = L.pic_get_layout(ctx_probe)
        L.pic_destroy(ctx_probe)
        dtype = torch.float32 if precision == L.PIC_FP32_MIXED else torch.float64
        fields = fields_for(cfg, wl, device, dtype)
        sps, parts = [], []
        for q, m, raw in wl.species:
            raw = RawParticles([c.to(device) for c in raw.cell], [o.to(device) for o in raw.off],
                               [v.to(device) for v in raw.u], raw.w.to(device))
            sps.append(L.Species(q, m, 1.0))
            if precision == L.PIC_FP32_MIXED:
                parts.append(to_fp32(raw, bits, with_chi=with_chi))
            else:
                parts.append(to_fp64(raw, cfg, from_fp32=from_fp32, with_chi=with_chi))
        every = [sort_every * (max(1, int(heavy_sort_factor)) if m >= 100.0 else 1) for _, m, _ in wl.species]
        sim = Simulation(cfg, sps, parts, fields, sort_every=sort_every, device=device, sort_every_species=every)
        for b in wl.beams:  # self-fields of relativistic bunches (Sec. III(c))
            L.pic_beam_fields(sim.ctx, b, sim.fields)
        return sim

    def sort(self, which=None):
        """Sort the species `which` (indices; default every species)."""
        for k in range(len(self.particles)) if which is None else which:
            p, dst = self.particles[k], self.spare[k]
            # the arrays' tile offsets from their last sort let pic_sort move
            # only the particles that changed tiles; before the first sort
            # there are none to give
            src = p if self.sorted_at[k] >= 0 else dataclasses.replace(p, tile_start=None)
            L.pic_sort(self.ctx, src, dst)
            self.particles[k], self.spare[k] = dst, p
            self.sorted_at[k] = self.step_index

    def sort_due(self):
        """Indices of the species whose sort interval has run out (FP32)."""
        if not self.fp32:
            return []
        return [k for k, at in enumerate(self.sorted_at)
                if at < 0 or self.step_index - at >= self.sort_every_species[k]]

    def restart_sort_cycles(self):
        """Make the next step sort every species (a timed window that starts
        with whole sort cycles)."""
        self.sorted_at = [self.step_index - e for e in self.sort_every_species]

    def step(self, with_diag: bool = False, events=None, gauss=None):
        """One step; `events` = (start, end) torch events recorded on the
        current stream around the gather-push-deposit launches; `gauss` =
        (rho, residual) FP64 planes that receive the charge density at the
        half step and div E - rho after the first half field update (the
        residual's maximum goes to diag[3] when with_diag)."""
        due = self.sort_due()
        if due:
            self.sort(due)
        diag = self.diag if with_diag else None
        L.pic_yee_step(self.ctx, 1, self.fields)
        if gauss is not None:
            rho, res = gauss
            rho.zero_()
            for sp, p in zip(self.species, self.particles):
                L.pic_deposit_rho(self.ctx, sp, p, rho, at_half=True)
            L.pic_gauss_residual(self.ctx, self.fields, rho, res, diag)
        for j in self.fields.J:
            j.zero_()
        if events is not None:
            events[0].record()
        if self.fp32 and 1 < len(self.species) <= L.PIC_MAX_SPECIES:
            # one pass over the tiles for every species
            L.pic_gather_push_deposit_multi(self.ctx, self.species, self.particles, self.fields, diag)
        else:
            for sp, p in zip(self.species, self.particles):
                L.pic_gather_push_deposit(self.ctx, sp, p, self.fields, diag)
        if events is not None:
            events[1].record()
        L.pic_yee_step(self.ctx, 2, self.fields, diag)
        self.step_index += 1

    def check(self):
        return L.pic_check(self.ctx)

    def energy(self):
        """Run-time diagnostics accumulated since the last reset: kinetic,
        charge, field energy (FP64, from the last step with_diag)."""
        return self.diag.cpu().tolist()

    def positions64(self, k=0):
        """Absolute FP64 positions of species k (for comparisons)."""
        p = self.particles[k]
        if not self.fp32:
            return [x.clone() for x in p.x]
        out = []
        mask = [(1 << b) - 1 for b in self.bits]
        cell = p.cell.to(torch.int64)
        shift = 0
        for a in range(self.cfg.dim):
            c = (cell >> shift) & mask[a]
            shift += self.bits[a]
            out.append((c.to(torch.float64) + p.off[a].to(torch.float64)) * self.cfg.d[a])
        return out


def autotune_tiles(wl: Workload, candidates, steps: int = 8, warmup: int = 1, device="cuda"):
    """Tile shape and drift allowance of the FP32 push, chosen by timing.

    For each (tile, drift) of `candidates` whose LDS window fits, builds the
    workload's simulation, sorts once and times `steps` whole steps (the
    sort at their start included, so shapes that shed more stragglers pay
    for the sorts they need).  Returns ((tile, drift) of the fastest,
    {label: ms per step or the reason it was skipped})."""
    timings = {}
    best, best_ms = None, float("inf")
    for tile, drift in candidates:
        label = "x".join(str(t) for t in tile) + f" drift {drift}"
        try:
            sim = Simulation.from_workload(wl, precision=L.PIC_FP32_MIXED, device=device, sort_every=steps,
                                           tile=tuple(tile), drift=drift)
        except L.PicError as e:  # window beyond the LDS, tile not dividing the grid, ...
            timings[label] = str(e)
            continue
        for _ in range(warmup):
            sim.step()
        sim.restart_sort_cycles()  # the timed window starts with a sort
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            sim.step()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        timings[label] = ms
        if ms < best_ms:
            best, best_ms = (tuple(tile), drift), ms
        del sim
        torch.cuda.empty_cache()
    if best is None:
        raise L.PicError(L.PIC_E_UNSUPPORTED, f"no candidate tile fits: {timings}")
    return best, timings
