"""Seeded synthetic inputs shaped like the paper's cases.

Input generation only: cell occupancy, random in-cell positions, momenta,
weights and initial fields.  Nothing here performs a step of the method; the
same arrays feed the HIP library and the oracle.  All randomness comes from a
``torch.Generator`` seeded explicitly, on the device the arrays are made on.

Units are those of Eq. 8 of the paper.  With the laser frequency as the
reference (w_r = w_L) the wavelength is 2 pi and the critical density is 1;
with w_r = w_p the plasma density is 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import torch

from ._lib import PIC_FP32_MIXED, PIC_FP64_PLAIN, Beam, Config, Fields, Particles

LAMBDA = 2.0 * math.pi  # laser wavelength in c / w_L


def courant_dt(d, frac=0.95):
    """frac times the Courant limit 1/sqrt(sum 1/d^2)."""
    return frac / math.sqrt(sum(1.0 / v ** 2 for v in d))


@dataclass
class RawParticles:
    """Particles as generated: integer cells (int64), FP64 in-cell offsets in
    [0,1), FP64 momenta and weights."""
    cell: list          # per axis, int64
    off: list           # per axis, float64
    u: list             # 3 x float64
    w: torch.Tensor     # float64

    @property
    def n(self):
        return self.u[0].numel()

    def subset(self, idx):
        return RawParticles([c[idx] for c in self.cell], [o[idx] for o in self.off],
                            [v[idx] for v in self.u], self.w[idx])


def plasma(cfg: Config, ppc: int, density: Callable, gen: torch.Generator, device,
           uth: float = 0.0, ux_fn: Optional[Callable] = None) -> RawParticles:
    """`ppc` particles in every cell whose density (a function of the cell's
    x index, vectorised) is positive, uniform random positions in the cell,
    Gaussian momenta of spread `uth` per component plus ux_fn(x) along x,
    weight density/ppc (density in n_r)."""
    dim = cfg.dim
    n = list(cfg.n) + [1] * (3 - len(cfg.n))
    ix = torch.arange(n[0], device=device)
    dens_x = density(ix.to(torch.float64))
    occupied = torch.nonzero(dens_x > 0).flatten()
    nx_occ = occupied.numel()
    ncell = nx_occ * n[1] * n[2]
    N = ncell * ppc
    # cells enumerated x-fastest over the occupied x range
    lin = torch.arange(N, device=device, dtype=torch.int64) // ppc
    cx = occupied[lin % nx_occ]
    rest = lin // nx_occ
    cy = rest % n[1]
    cz = rest // n[1]
    cells = [cx, cy, cz][:dim]
    off = [torch.rand(N, generator=gen, device=device, dtype=torch.float64) for _ in range(dim)]
    u = [torch.randn(N, generator=gen, device=device, dtype=torch.float64) * uth for _ in range(3)]
    if ux_fn is not None:
        u[0] = u[0] + ux_fn((cx.to(torch.float64) + off[0]) * cfg.d[0])
    w = dens_x[cx] / ppc
    return RawParticles(cells, off, u, w)


def concat(parts):
    return RawParticles([torch.cat([p.cell[a] for p in parts]) for a in range(len(parts[0].cell))],
                        [torch.cat([p.off[a] for p in parts]) for a in range(len(parts[0].off))],
                        [torch.cat([p.u[a] for p in parts]) for a in range(3)],
                        torch.cat([p.w for p in parts]))


def packed_cells(cells, bits):
    c = cells[0].to(torch.int64)
    if len(cells) > 1:
        c = c | (cells[1].to(torch.int64) << bits[0])
    if len(cells) > 2:
        c = c | (cells[2].to(torch.int64) << (bits[0] + bits[1]))
    return c.to(torch.int32)


def to_fp32(raw: RawParticles, bits, with_w=True, with_chi=False) -> Particles:
    """FP32 layout: packed int32 cell, float32 offsets (an offset that rounds
    up to 1.0 is clamped to the largest float below 1), float32 u and w."""
    off = []
    one_minus = torch.tensor(1.0, dtype=torch.float32).nextafter(torch.tensor(0.0)).item()
    for o in raw.off:
        o32 = o.to(torch.float32)
        off.append(torch.clamp(o32, max=one_minus).contiguous())
    return Particles(
        n=raw.n, u=[v.to(torch.float32).contiguous() for v in raw.u],
        cell=packed_cells(raw.cell, bits).contiguous(), off=off,
        w=raw.w.to(torch.float32).contiguous() if with_w else None,
        chi=torch.zeros(raw.n, dtype=torch.float32, device=raw.w.device) if with_chi else None)


def to_fp64(raw: RawParticles, cfg: Config, from_fp32: bool = False, with_w=True,
            with_chi=False) -> Particles:
    """FP64 layout: absolute x = (cell + offset) d.  With from_fp32 the offsets
    and momenta are first rounded as in to_fp32, so both paths start from the
    same physical state."""
    xs, us = [], []
    one_minus = torch.tensor(1.0, dtype=torch.float32).nextafter(torch.tensor(0.0)).item()
    for a in range(cfg.dim):
        o = raw.off[a]
        if from_fp32:
            o = torch.clamp(o.to(torch.float32), max=one_minus).to(torch.float64)
        xs.append(((raw.cell[a].to(torch.float64) + o) * cfg.d[a]).contiguous())
    for v in raw.u:
        us.append((v.to(torch.float32).to(torch.float64) if from_fp32 else v).contiguous())
    w = raw.w
    if from_fp32:
        w = w.to(torch.float32).to(torch.float64)
    return Particles(n=raw.n, u=us, x=xs, w=w.contiguous() if with_w else None,
                     chi=torch.zeros(raw.n, dtype=torch.float32, device=w.device) if with_chi else None)


# --------------------------------------------------------------- the configs

@dataclass
class Workload:
    name: str
    cfg: Config
    species: list          # (q, m, RawParticles)
    E0: Optional[list] = None   # initial E planes (float64) or None = zero
    B0: Optional[list] = None
    steps: int = 0
    beams: list = field(default_factory=list)  # Beam bunches whose self-fields are added at start


def langmuir_2d(seed=643, n=(64, 64), ppc=16, device="cpu", order=1, precision=PIC_FP64_PLAIN) -> Workload:
    """2D3V periodic box, dx = dy = 0.05 c/w_p, 16 electrons per cell at
    uniform random positions, Maxwellian thermal spread 0.01 c per component
    plus a 0.001 c sinusoidal drift (Langmuir mode k = 2 pi / L_x), immobile
    neutralizing ions (not represented), linear (CIC) weights, dt = 0.95 of the
    Courant limit, 200 steps, FP64."""
    d = (0.05, 0.05)
    cfg = Config(dim=2, n=n, d=d, dt=courant_dt(d), order=order, precision=precision, seed=seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    L = n[0] * d[0]
    raw = plasma(cfg, ppc, lambda x: torch.ones_like(x), gen, device, uth=0.01,
                 ux_fn=lambda x: 0.001 * torch.sin(2 * math.pi * x / L))
    return Workload("langmuir_2d_64x64_cic", cfg, [(-1.0, 1.0, raw)], steps=200)


def laser_fields(cfg: Config, device, a0: float, waist: float, x_start: float, n_cycles: int,
                 circular: bool = False, backward: bool = False):
    """A laser pulse already inside the box, moving along +x (or -x with
    `backward`): transverse E and the matching B (E_y = B_z, E_z = -B_y;
    B reversed for -x), Gaussian transverse profile of waist `waist`, sin^2
    field envelope over `n_cycles` periods starting at x_start.  Linear
    polarisation along y with amplitude a0; circular with a0 on each
    transverse component.  Sampled at each component's Yee location.
    Returns (E, B) as float64 planes."""
    dim = cfg.dim
    n = list(cfg.n) + [1] * (3 - len(cfg.n))
    shape = (n[2], n[1], n[0])
    k_i = torch.arange(n[2], device=device, dtype=torch.float64).view(-1, 1, 1)
    j_i = torch.arange(n[1], device=device, dtype=torch.float64).view(1, -1, 1)
    i_i = torch.arange(n[0], device=device, dtype=torch.float64).view(1, 1, -1)
    length = n_cycles * LAMBDA
    yc = n[1] * cfg.d[1] / 2
    zc = n[2] * cfg.d[2] / 2 if dim == 3 else 0.0

    def profile(sx, sy, sz, phase_shift):
        x = (i_i + sx) * cfg.d[0]
        y = (j_i + sy) * cfg.d[1]
        r2 = (y - yc) ** 2
        if dim == 3:
            z = (k_i + sz) * cfg.d[2]
            r2 = r2 + (z - zc) ** 2
        xi = (x - x_start) / length
        env = torch.where((xi >= 0) & (xi <= 1), torch.sin(math.pi * xi) ** 2, torch.zeros_like(xi))
        return (a0 * env * torch.exp(-r2 / waist ** 2) * torch.sin(x + phase_shift)).expand(shape)

    zero = lambda: torch.zeros(shape, device=device, dtype=torch.float64)  # noqa: E731
    E = [zero(), profile(0, 0.5, 0, 0.0).contiguous(), zero()]
    B = [zero(), zero(), profile(0.5, 0.5, 0, 0.0).contiguous()]
    if circular:
        E[2] = profile(0, 0, 0.5, math.pi / 2).contiguous()
        B[1] = (-profile(0.5, 0, 0.5, math.pi / 2)).contiguous()
    if backward:
        B = [-b for b in B]
    return E, B


ME_KEV = 510.99895  # electron rest energy


def laser_plasma_2d(seed=644, scale=1, device="cuda", ppc=32, order=2, t_kev=1.0,
                    x_pulse=12.0) -> Workload:
    """2D3V laser-plasma case: 4096 x 2048 cells at 20 cells per laser
    wavelength, linearly polarized Gaussian pulse a0 = 2 (waist 5 lambda,
    10-cycle sin^2 envelope) moving into an underdense electron plasma of
    density 0.01 n_c behind a 2-lambda linear ramp, 32 particles per cell,
    quadratic weights, dt = 0.95 of the Courant limit.  Periodic faces unless
    the caller sets cfg.bc_x (the benchmark absorbs at the x faces);
    the ramp spans [12, 14] lambda and the pulse starts at x_pulse (default
    [12, 22] lambda: already inside the plasma, the state in which a
    1000-step run spends almost all of its steps; 1 lambda puts it in the
    vacuum gap).  Electrons start with a Maxwellian spread of temperature
    t_kev (1 keV as in the paper's 2D benchmark), so every particle carries
    current from the first step.  `scale` divides both cell counts."""
    n = (4096 // scale, 2048 // scale)
    d = (LAMBDA / 20, LAMBDA / 20)
    cfg = Config(dim=2, n=n, d=d, dt=courant_dt(d), order=order, seed=seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    x0, x1 = 12 * LAMBDA, 14 * LAMBDA
    if scale > 1:  # keep a plasma region on small boxes
        x0, x1 = 0.3 * n[0] * d[0], 0.4 * n[0] * d[0]

    def density(ix):
        x = (ix + 0.5) * d[0]
        return 0.01 * torch.clamp((x - x0) / (x1 - x0), 0.0, 1.0)

    raw = plasma(cfg, ppc, density, gen, device, uth=math.sqrt(t_kev / ME_KEV))
    xs = x_pulse * LAMBDA if scale == 1 else 0.02 * n[0] * d[0]
    ncyc = 10 if scale == 1 else max(2, int(0.25 * n[0] * d[0] / LAMBDA))
    E, B = laser_fields(cfg, device, a0=2.0, waist=5 * LAMBDA if scale == 1 else 0.2 * n[1] * d[1],
                        x_start=xs, n_cycles=ncyc)
    shape = {1: "linear", 2: "quadratic", 4: "quartic"}[order]
    return Workload(f"laser_plasma_2d_{n[0]}x{n[1]}_ppc{ppc}_{shape}", cfg, [(-1.0, 1.0, raw)], E, B,
                    steps=1000)


def laser_plasma_3d(seed=645, scale=1, device="cuda", ppc=8, order=2, tile=(8, 8, 4),
                    t_kev=1.0) -> Workload:
    """3D3V laser-plasma case: 512 x 256 x 256 cells at 20 cells per
    wavelength, electrons and protons (mass 1836) with 8 particles per cell
    each at 0.05 n_c behind a 2-lambda ramp, circularly polarized pulse
    a0 = 5 (waist 3 lambda, 10-cycle sin^2), quadratic weights, electrons and
    ions at t_kev.  Periodic box; the pulse starts at x = 0 and overlaps the
    ramp.  `scale` divides the cell counts."""
    n = (512 // scale, 256 // scale, 256 // scale)
    d = (LAMBDA / 20,) * 3
    cfg = Config(dim=3, n=n, d=d, dt=courant_dt(d), order=order, seed=seed, tile=tile)
    gen = torch.Generator(device=device).manual_seed(seed)
    x0, x1 = 2 * LAMBDA, 4 * LAMBDA
    if scale > 1:
        x0, x1 = 0.1 * n[0] * d[0], 0.2 * n[0] * d[0]

    def density(ix):
        x = (ix + 0.5) * d[0]
        return 0.05 * torch.clamp((x - x0) / (x1 - x0), 0.0, 1.0)

    el = plasma(cfg, ppc, density, gen, device, uth=math.sqrt(t_kev / ME_KEV))
    ion = plasma(cfg, ppc, density, gen, device, uth=math.sqrt(t_kev / ME_KEV / 1836.0))
    E, B = laser_fields(cfg, device, a0=5.0, waist=3 * LAMBDA if scale == 1 else 0.2 * n[1] * d[1],
                        x_start=0.0, n_cycles=10 if scale == 1 else 2, circular=True)
    shape = {1: "linear", 2: "quadratic", 4: "quartic"}[order]
    return Workload(f"laser_plasma_3d_{n[0]}x{n[1]}x{n[2]}_ppc{ppc}x2_{shape}", cfg,
                    [(-1.0, 1.0, el), (1.0, 1836.0, ion)], E, B, steps=500)


def beam_wakefield_3d(seed=648, scale=1, device="cuda", ppc=8, beam_ppc=4, order=2, tile=(8, 8, 4),
                      gamma_b=1957.0, nb=4.0, sigma=0.5, x_beam=3.0, uth=1e-3) -> Workload:
    """3D3V beam-driven wakefield case (Sec. III(c)), plasma units (w_r = w_p,
    so n_p = 1 and lambda_p = 2 pi): a 4 lambda_p x 2 lambda_p x 2 lambda_p box
    of 512 x 192 x 192 cells, electrons and protons (mass 1836) at 8 per cell
    each, and a 1-GeV drive electron beam (gamma 1957) with a bi-Gaussian
    density of peak nb = 4 n_p and k_p sigma_x = k_p sigma_r = 0.5, sampled by
    4 particles per cell within 4 sigma of its centre (x = x_beam lambda_p,
    on the axis).  The beam's self-fields (the rest-frame Poisson solution
    boosted to the lab, Sec. III(c)) are not in E0/B0: the workload lists the
    bunch in `beams` and the simulation adds its fields with pic_beam_fields.
    Periodic faces unless the caller sets cfg.bc_x; `scale` divides the cell
    counts."""
    lam_p = 2.0 * math.pi
    n = (512 // scale, 192 // scale, 192 // scale)
    d = (4 * lam_p / 512, 2 * lam_p / 192, 2 * lam_p / 192)
    cfg = Config(dim=3, n=n, d=d, dt=courant_dt(d), order=order, seed=seed, tile=tile,
                 drift=0 if order == 4 else 1)
    gen = torch.Generator(device=device).manual_seed(seed)
    el = plasma(cfg, ppc, lambda ix: torch.ones_like(ix), gen, device, uth=uth)
    ion = plasma(cfg, ppc, lambda ix: torch.ones_like(ix), gen, device, uth=uth / math.sqrt(1836.0))
    # beam cells: within 4 sigma of the centre
    xb = x_beam * lam_p if scale == 1 else 0.75 * n[0] * d[0]
    yc, zc = 0.5 * n[1] * d[1], 0.5 * n[2] * d[2]
    reach = 4 * sigma
    ix = torch.arange(n[0], device=device)
    iy = torch.arange(n[1], device=device)
    iz = torch.arange(n[2], device=device)
    cx = ix[((ix + 0.5) * d[0] - xb).abs() <= reach]
    cy, cz = torch.meshgrid(iy, iz, indexing="ij")
    r2 = ((cy + 0.5) * d[1] - yc) ** 2 + ((cz + 0.5) * d[2] - zc) ** 2
    sel = r2 <= reach ** 2
    cy, cz, r2 = cy[sel], cz[sel], r2[sel]
    nt = cy.numel()
    lin = torch.arange(cx.numel() * nt * beam_ppc, device=device) // beam_ppc
    bx, tr = cx[lin // nt], lin % nt
    by, bz = cy[tr], cz[tr]
    N = lin.numel()
    off = [torch.rand(N, generator=gen, device=device, dtype=torch.float64) for _ in range(3)]
    dens = nb * torch.exp(-(((bx + 0.5) * d[0] - xb) ** 2) / (2 * sigma ** 2) - r2[tr].to(torch.float64) / (2 * sigma ** 2))
    ub = math.sqrt(gamma_b ** 2 - 1.0)
    u = [torch.full((N,), ub, device=device, dtype=torch.float64), torch.zeros(N, device=device, dtype=torch.float64),
         torch.zeros(N, device=device, dtype=torch.float64)]
    beam = RawParticles([bx.to(torch.int64), by.to(torch.int64), bz.to(torch.int64)], off, u,
                        (dens / beam_ppc).to(torch.float64))
    bunch = Beam(charge=-1.0, density=nb, center=(xb, yc, zc), sigma=(sigma, sigma, sigma), gamma=gamma_b)
    shape_name = {1: "linear", 2: "quadratic", 4: "quartic"}[order]
    return Workload(f"beam_wakefield_3d_{n[0]}x{n[1]}x{n[2]}_ppc{ppc}x2+{beam_ppc}_{shape_name}", cfg,
                    [(-1.0, 1.0, el), (1.0, 1836.0, ion), (-1.0, 1.0, beam)], steps=0, beams=[bunch])


QED_HBAR_OMEGA = 2.4263e-6  # hbar w_L / (m_e c^2) at lambda = 1 um


def qed_foil_2d(seed=646, scale=1, device="cuda", ppc=16, order=2, a0=500.0, n_foil=100.0,
                x_pulse=8.0, t_kev=1.0) -> Workload:
    """2D3V strong-field QED case: 2048 x 1024 cells at 64 cells per
    wavelength (the 100 n_c foil's skin depth, lambda / 63, spans a cell), a
    linearly polarized Gaussian pulse a0 = 500 (waist 3 lambda, 10-cycle
    sin^2) on a 2-lambda electron foil at 100 n_c over [16, 18] lambda with 16
    particles per cell and immobile ions; positrons and photons come from the
    QED step (lambda = 1 um for chi).  The pulse spans [x_pulse, x_pulse + 10]
    lambda: with the default its front already sits in the foil.  Periodic
    box; `scale` divides the cell counts."""
    n = (2048 // scale, 1024 // scale)
    d = (LAMBDA / 64, LAMBDA / 64)
    cfg = Config(dim=2, n=n, d=d, dt=courant_dt(d), order=order, seed=seed, hbar_omega_mc2=QED_HBAR_OMEGA)
    gen = torch.Generator(device=device).manual_seed(seed)
    x0, x1 = 16 * LAMBDA, 18 * LAMBDA
    if scale > 1:
        x0, x1 = 0.5 * n[0] * d[0], 0.56 * n[0] * d[0]

    def density(ix):
        x = (ix + 0.5) * d[0]
        return torch.where((x >= x0) & (x < x1), torch.full_like(x, n_foil), torch.zeros_like(x))

    raw = plasma(cfg, ppc, density, gen, device, uth=math.sqrt(t_kev / ME_KEV))
    xs = x_pulse * LAMBDA if scale == 1 else 0.25 * n[0] * d[0]
    E, B = laser_fields(cfg, device, a0=a0, waist=3 * LAMBDA if scale == 1 else 0.2 * n[1] * d[1],
                        x_start=xs, n_cycles=10 if scale == 1 else 2)
    shape = {1: "linear", 2: "quadratic", 4: "quartic"}[order]
    return Workload(f"qed_foil_2d_{n[0]}x{n[1]}_ppc{ppc}_{shape}", cfg, [(-1.0, 1.0, raw)], E, B, steps=0)


def plasma_fp32(cfg: Config, bits, ppc: int, density: Callable, gen: torch.Generator, device,
                uth: float = 0.0, capacity: Optional[int] = None, chunk: int = 1 << 26) -> Particles:
    """The FP32 layout generated directly, chunk by chunk, for particle counts
    whose FP64 form would not fit next to it: `ppc` particles in every cell
    of positive density (cells x-fastest), float32 offsets uniform in [0, 1),
    Gaussian momenta of spread `uth`, weight density/ppc, chi 0, and the QED
    columns: tau 0, tau_thr = -ln r, identifiers 1..N.  Arrays hold
    `capacity` (default N) entries."""
    n = list(cfg.n) + [1] * (3 - len(cfg.n))
    dens_x = density(torch.arange(n[0], device=device, dtype=torch.float64))
    occupied = torch.nonzero(dens_x > 0).flatten()
    nx_occ = occupied.numel()
    N = nx_occ * n[1] * n[2] * ppc
    cap = N if capacity is None else max(int(capacity), N)
    f32 = dict(device=device, dtype=torch.float32)
    cell = torch.zeros(cap, device=device, dtype=torch.int32)
    off = [torch.zeros(cap, **f32) for _ in range(cfg.dim)]
    u = [torch.zeros(cap, **f32) for _ in range(3)]
    w = torch.zeros(cap, **f32)
    tau_thr = torch.zeros(cap, **f32)
    one_minus = torch.tensor(1.0, dtype=torch.float32).nextafter(torch.tensor(0.0)).item()
    for s0 in range(0, N, chunk):
        s1 = min(N, s0 + chunk)
        lin = torch.arange(s0, s1, device=device, dtype=torch.int64) // ppc
        cx = occupied[lin % nx_occ]
        rest = lin // nx_occ
        cy, cz = rest % n[1], rest // n[1]
        c = cx | (cy << bits[0])
        if cfg.dim == 3:
            c = c | (cz << (bits[0] + bits[1]))
        cell[s0:s1] = c.to(torch.int32)
        for a in range(cfg.dim):
            off[a][s0:s1] = torch.rand(s1 - s0, generator=gen, **f32).clamp_(max=one_minus)
        for a in range(3):
            u[a][s0:s1] = torch.randn(s1 - s0, generator=gen, **f32) * uth
        w[s0:s1] = (dens_x[cx] / ppc).to(torch.float32)
        tau_thr[s0:s1] = -torch.log(torch.rand(s1 - s0, generator=gen, **f32).clamp_(min=1e-30))
    ids = torch.arange(1, cap + 1, device=device, dtype=torch.int64)
    return Particles(N, u, cell=cell, off=off, w=w, chi=torch.zeros(cap, **f32),
                     tau=torch.zeros(cap, device=device, dtype=torch.float64), tau_thr=tau_thr, id=ids,
                     capacity=cap, n_dev=torch.tensor([N], device=device, dtype=torch.int64))


def qed_3d_full(seed=647, scale=1, device="cuda", ppc=4, order=2, a0=300.0, n_e=50.0, tile=(8, 8, 4),
                t_kev=1.0, capacity=None):
    """3D3V QED case at full HBM: 1024 x 512 x 512 cells at 20 cells per
    wavelength, 4 electrons per cell in every cell (1.07e9) at 50 n_c (the
    slab fills the periodic box; ions immobile), and two circularly polarized
    pulses a0 = 300 (waist 3 lambda, 6-cycle sin^2) that start 1 lambda on
    either side of the box centre and move toward it.  Returns
    (cfg, electrons in the FP32 layout with the QED columns, E, B as float32
    planes); `scale` divides the cell counts."""
    n = (1024 // scale, 512 // scale, 512 // scale)
    d = (LAMBDA / 20,) * 3
    cfg = Config(dim=3, n=n, d=d, dt=courant_dt(d), order=order, seed=seed, tile=tile,
                 drift=0 if order == 4 else 1, hbar_omega_mc2=QED_HBAR_OMEGA)
    from ._lib import pic_destroy, pic_get_layout, pic_init
    ctx = pic_init(cfg)
    bits, _, _ = pic_get_layout(ctx)
    pic_destroy(ctx)
    gen = torch.Generator(device=device).manual_seed(seed)
    el = plasma_fp32(cfg, bits, ppc, lambda ix: torch.full_like(ix, n_e), gen, device,
                     uth=math.sqrt(t_kev / ME_KEV), capacity=capacity)
    xc = 0.5 * n[0] * d[0]
    ncyc = 6 if scale == 1 else 2
    waist = 3 * LAMBDA if scale == 1 else 0.2 * n[1] * d[1]
    gap = LAMBDA if scale == 1 else 0.02 * n[0] * d[0]
    E1, B1 = laser_fields(cfg, device, a0, waist, xc - gap - ncyc * LAMBDA, ncyc, circular=True)
    E = [e.to(torch.float32) for e in E1]
    B = [b.to(torch.float32) for b in B1]
    del E1, B1
    E2, B2 = laser_fields(cfg, device, a0, waist, xc + gap, ncyc, circular=True, backward=True)
    for a in range(3):
        E[a] += E2[a].to(torch.float32)
        B[a] += B2[a].to(torch.float32)
    del E2, B2
    return cfg, el, E, B


def fields_for(cfg: Config, wl: Workload, device, dtype) -> Fields:
    f = Fields.zeros(cfg, device, dtype)
    if wl.E0 is not None:
        for a in range(3):
            f.E[a].copy_(wl.E0[a].to(device=device, dtype=dtype))
            f.B[a].copy_(wl.B0[a].to(device=device, dtype=dtype))
    return f
