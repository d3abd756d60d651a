"""Parity at the full sizes of the paper-shaped cases, in the launch
configuration the benchmark times (tiles, drift allowance, sort), on outputs
the oracle can compute one particle at a time, and on properties that hold
at any size.

For each case a random sample of particles is pushed by the oracle from the
same FP32 state and the same half-step fields as the GPU, which pushes the
whole population; the QED cases also compare chi, the optical depth and the
recoil/photon pairs of the sampled leptons.  Sort: tile order and tile
offsets of the whole population.  Current: sum of J_x over the grid against
sum q w v_x over the particles (charge-conserving deposit)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import qed_step as Q
from paper_2104_00642_amd import _lib as L
from paper_2104_00642_amd import workloads as W
from paper_2104_00642_amd.sim import Simulation

from _helpers import (DEV, host_fields, np64, oracle_grid, oracle_sample, positions_fp32, push_errors, rel_l2,
                      sampled_push)

pytestmark = pytest.mark.gpu

U_TOL = 2e-6      # FP32 path: relative momentum error of one step
X_TOL = 2e-6      # position error in cells
J_TOL = 1e-6      # sum J_x against sum q w v_x


def check_sorted(p: L.Particles, bits, tile, ntiles, cfg, chunk=1 << 27):
    """Tile ids non-decreasing and the tile offsets equal to the counts'
    exclusive scan, over the whole population (in chunks)."""
    nta = [cfg.n[a] // tile[a] for a in range(cfg.dim)]
    counts = torch.zeros(ntiles, dtype=torch.int64, device=p.cell.device)
    last = -1
    for s0 in range(0, p.n, chunk):
        cell = p.cell[s0:min(p.n, s0 + chunk)].to(torch.int64)
        t = torch.zeros_like(cell)
        stride, shift = 1, 0
        for a in range(cfg.dim):
            c = (cell >> shift) & ((1 << bits[a]) - 1)
            shift += bits[a]
            t += (c // tile[a]) * stride
            stride *= nta[a]
        assert int(t[0]) >= last and bool((t[1:] >= t[:-1]).all())
        last = int(t[-1])
        counts += torch.bincount(t, minlength=ntiles)
    start = torch.zeros(ntiles + 1, dtype=torch.int64, device=counts.device)
    start[1:] = torch.cumsum(counts, 0)
    assert torch.equal(p.tile_start.to(torch.int64), start)


def current_consistency(fields: L.Fields, sp: L.Species, p: L.Particles, cfg):
    """|sum J_x - sum q w v_x| / sum |q w v_x| after one push from J = 0
    (J is per unit cell volume here: the grid sum times dV is the total)."""
    jx = float(fields.J[0].double().sum().item())
    u = [t[: p.n].double() for t in p.u]
    gam = torch.sqrt(1 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    w = p.w[: p.n].double() if p.w is not None else sp.w0
    qwv = sp.q * w * u[0] / gam
    return abs(jx - float(qwv.sum().item())) / max(float(qwv.abs().sum().item()), 1e-300)


def window_snapshot(sim, lo, size, margin=4):
    """Every particle whose deposit can reach the cells [lo, lo + size) (a
    particle in cell c deposits on nodes [c - 2, c + 3]; the margin covers
    that with room), periodic, per species: FP64 positions, momenta and
    weights before the push."""
    out = []
    for p in sim.particles:
        cell = p.cell[: p.n].to(torch.int64)
        keep = torch.ones(p.n, dtype=torch.bool, device=cell.device)
        shift = 0
        for a in range(sim.cfg.dim):
            c = (cell >> shift) & ((1 << sim.bits[a]) - 1)
            shift += sim.bits[a]
            keep &= torch.remainder(c - (lo[a] - margin), sim.cfg.n[a]) < size[a] + 2 * margin
        del cell
        idx = torch.nonzero(keep).flatten()
        out.append(dict(idx=idx, x0=positions_fp32(p, sim.bits, sim.cfg, idx), u0=[np64(t[idx]) for t in p.u],
                        w0=np64(p.w[idx])))
    return out


def window_current(sim, snaps, F, lo, size):
    """The oracle's current of the snapshot particles (same FP32 state and
    fields), on the window cells; with the GPU's."""
    g = oracle_grid(sim.cfg)
    J = [np.zeros(F[0].shape) for _ in range(3)]
    for sp, snap in zip(sim.species, snaps):
        osp = O.Species(sp.q, sp.m, [a.copy() for a in snap["x0"]], [a.copy() for a in snap["u0"]],
                        snap["w0"].copy(), sp.w0)
        O.push(g, osp, F, J)
    dim = sim.cfg.dim
    ix = [np.arange(lo[a], lo[a] + size[a]) % sim.cfg.n[a] for a in range(dim)]
    sel = np.ix_(*([ix[2]] if dim == 3 else [[0]]), ix[1], ix[0])
    got = [np64(j)[sel] for j in sim.fields.J]
    return [Jc[sel] for Jc in J], got


def check_windows(sim, windows, snaps, F):
    """Element-wise current on each window: relative L2 within 1e-5 (the
    per-step field bar) and every node within 1e-5 of the window's largest
    |J| component."""
    for (lo, size), snap in zip(windows, snaps):
        ref, got = window_current(sim, snap, F, lo, size)
        rel = [rel_l2(g, r) for g, r in zip(got, ref)]
        jmax = max(float(np.abs(r).max()) for r in ref)
        mabs = max(float(np.abs(g - r).max()) for g, r in zip(got, ref)) / max(jmax, 1e-300)
        npart = sum(len(s["w0"]) for s in snap)
        print(f"  J window at {lo} size {size}: {npart} particles, rel L2 {max(rel):.2e}, "
              f"max |dJ| / max |J| {mabs:.2e} (max |J| {jmax:.3e})", flush=True)
        assert jmax > 0.0
        assert max(rel) < 1e-5 and mabs < 1e-5


def laser_case(wl, tile, drift, nsample=2000, windows=()):
    sim = Simulation.from_workload(wl, precision=L.PIC_FP32_MIXED, device=DEV, sort_every=1 << 30,
                                   tile=tile, drift=drift)
    sim.sort()
    torch.cuda.synchronize()
    for p in sim.particles:
        check_sorted(p, sim.bits, sim.tile, sim.ntiles, sim.cfg)
    L.pic_yee_step(sim.ctx, 1, sim.fields)
    for j in sim.fields.J:
        j.zero_()
    torch.cuda.synchronize()
    F = host_fields(sim.fields)
    snaps = [window_snapshot(sim, lo, size) for lo, size in windows]
    worst = []
    for k, (sp, p) in enumerate(zip(sim.species, sim.particles)):
        jx_before = float(sim.fields.J[0].double().sum().item())
        snap = sampled_push(sim.ctx, sim.cfg, sp, p, sim.fields, sim.bits, nsample, seed=7 + k)
        osp, _, _ = oracle_sample(sim.cfg, sp, snap, F)
        du, dx = push_errors(sim.cfg, snap, osp)
        st, flags, _ = sim.check()
        assert st == L.PIC_OK, flags
        # the current of this species alone
        jx = float(sim.fields.J[0].double().sum().item()) - jx_before
        u = [t[: p.n].double() for t in p.u]
        gam = torch.sqrt(1 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
        qwv = sp.q * p.w[: p.n].double() * u[0] / gam
        jrel = abs(jx - float(qwv.sum().item())) / float(qwv.abs().sum().item())
        print(f"  species {k}: {p.n} particles, sample {nsample}: du {du:.2e}, dx {dx:.2e} cells, "
              f"sum J_x vs sum q w v_x {jrel:.2e}", flush=True)
        worst.append((du, dx, jrel))
    check_windows(sim, windows, snaps, F)
    return sim, worst


def test_laser_2d_full_size():
    """4096 x 2048 cells, 32 electrons per cell (2.53e8), quadratic, tile
    16 x 16, drift 2: the benchmark's case and launch configuration."""
    print("full size: 2D laser-plasma 4096x2048, 32 ppc, FP32", flush=True)
    wl = W.laser_plasma_2d(device=DEV)
    # element-wise current on two 64 x 64 windows in the pulse: one on the
    # axis, one across the periodic y seam; both span several tile windows
    sim, worst = laser_case(wl, (16, 16), 2, windows=[((300, 992), (64, 64)), ((300, 2016), (64, 64))])
    for du, dx, jrel in worst:
        assert du < U_TOL and dx < X_TOL and jrel < J_TOL
    del sim
    torch.cuda.empty_cache()
    # the plain FP64 path on the same workload: same sample, round-off bar
    print("full size: 2D laser-plasma 4096x2048, 32 ppc, FP64 plain", flush=True)
    sim = Simulation.from_workload(wl, precision=L.PIC_FP64_PLAIN, device=DEV)
    L.pic_yee_step(sim.ctx, 1, sim.fields)
    for j in sim.fields.J:
        j.zero_()
    torch.cuda.synchronize()
    F = host_fields(sim.fields)
    p, sp = sim.particles[0], sim.species[0]
    gen = torch.Generator().manual_seed(9)
    idx = torch.randint(0, p.n, (2000,), generator=gen).to(DEV)
    x0, u0, w0 = [np64(t[idx]) for t in p.x], [np64(t[idx]) for t in p.u], np64(p.w[idx])
    L.pic_gather_push_deposit(sim.ctx, sp, p, sim.fields)
    torch.cuda.synchronize()
    osp = O.Species(sp.q, sp.m, [a.copy() for a in x0], [a.copy() for a in u0], w0.copy(), sp.w0)
    O.push(oracle_grid(sim.cfg), osp, F, [np.zeros(F[0].shape) for _ in range(3)])
    for a in range(3):
        assert np.allclose(np64(p.u[a][idx]), osp.u[a], rtol=1e-12, atol=1e-12)
    for a in range(2):
        Lx = sim.cfg.n[a] * sim.cfg.d[a]
        dxa = np64(p.x[a][idx]) - osp.x[a]
        assert np.abs(dxa - Lx * np.round(dxa / Lx)).max() < 1e-12 * Lx
    assert current_consistency(sim.fields, sp, p, sim.cfg) < 1e-12


def test_laser_3d_full_size():
    """512 x 256 x 256 cells, electrons and protons at 8 per cell each
    (4.95e8), quadratic, tile 8 x 8 x 4, drift 1."""
    print("full size: 3D laser-plasma 512x256x256, 8+8 ppc, FP32", flush=True)
    wl = W.laser_plasma_3d(device=DEV, tile=(8, 8, 4))
    # element-wise current on two 32^3 windows in the pulse: one on the
    # axis, one across the periodic y and z seams
    sim, worst = laser_case(wl, (8, 8, 4), 1, windows=[((60, 112, 112), (32, 32, 32)),
                                                      ((60, 240, 240), (32, 32, 32))])
    for du, dx, jrel in worst:
        assert du < U_TOL and dx < X_TOL and jrel < J_TOL


def test_laser_3d_full_size_species_in_one_pass():
    """The same case in the benchmark's timed launch: tile 8 x 8 x 8 with
    drift 0 (its choice by timing) and both species in one pass over the
    tiles (pic_gather_push_deposit_multi, as Simulation.step pushes them):
    sampled particles of each species against the oracle, the charge-
    conserving sum over both species, and the element-wise current on two
    32^3 windows (one across the periodic y and z seams)."""
    print("full size: 3D laser-plasma 512x256x256, 8+8 ppc, FP32, species in one pass", flush=True)
    wl = W.laser_plasma_3d(device=DEV, tile=(8, 8, 8))
    sim = Simulation.from_workload(wl, precision=L.PIC_FP32_MIXED, device=DEV, sort_every=1 << 30,
                                   tile=(8, 8, 8), drift=0)
    sim.sort()
    torch.cuda.synchronize()
    for p in sim.particles:
        check_sorted(p, sim.bits, sim.tile, sim.ntiles, sim.cfg)
    L.pic_yee_step(sim.ctx, 1, sim.fields)
    for j in sim.fields.J:
        j.zero_()
    torch.cuda.synchronize()
    F = host_fields(sim.fields)
    windows = [((60, 112, 112), (32, 32, 32)), ((60, 240, 240), (32, 32, 32))]
    snaps = [window_snapshot(sim, lo, size) for lo, size in windows]
    samples = []
    for k, (sp, p) in enumerate(zip(sim.species, sim.particles)):
        gen = torch.Generator().manual_seed(17 + k)
        idx = torch.randint(0, p.n, (2000,), generator=gen).to(DEV)
        samples.append(dict(idx=idx, x0=positions_fp32(p, sim.bits, sim.cfg, idx), u0=[np64(t[idx]) for t in p.u],
                            w0=np64(p.w[idx])))
    L.pic_gather_push_deposit_multi(sim.ctx, sim.species, sim.particles, sim.fields)
    torch.cuda.synchronize()
    st, flags, nstray = sim.check()
    assert st == L.PIC_OK, flags
    jx = float(sim.fields.J[0].double().sum().item())
    qwv_sum, qwv_abs = 0.0, 0.0
    for k, (sp, p, snap) in enumerate(zip(sim.species, sim.particles, samples)):
        idx = snap["idx"]
        snap.update(x1=positions_fp32(p, sim.bits, sim.cfg, idx), u1=[np64(t[idx]) for t in p.u])
        osp, _, _ = oracle_sample(sim.cfg, sp, snap, F)
        du, dx = push_errors(sim.cfg, snap, osp)
        print(f"  species {k}: {p.n} particles, sample 2000: du {du:.2e}, dx {dx:.2e} cells", flush=True)
        assert du < U_TOL and dx < X_TOL
        u = [t[: p.n].double() for t in p.u]
        qwv = sp.q * p.w[: p.n].double() * u[0] / torch.sqrt(1 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
        qwv_sum += float(qwv.sum().item())
        qwv_abs += float(qwv.abs().sum().item())
        del u, qwv
    jrel = abs(jx - qwv_sum) / qwv_abs
    print(f"  {nstray} stragglers; sum J_x vs sum q w v_x over both species {jrel:.2e}", flush=True)
    assert jrel < J_TOL
    check_windows(sim, windows, snaps, F)


# the trained surrogate's rate error over its chi range (its training test
# bounds the maximum at 1e-3); outside the range the tables answer
NET_RATE_REL = 1e-3


def network(ctx):
    from test_gpu_qed import trained_network
    net, loss, secs = trained_network(ctx)
    print(f"  network trained in {secs:.1f} s (loss {loss:.2e})", flush=True)
    return net


def test_beam_wakefield_3d_full_size():
    """512 x 192 x 192 cells, electrons and protons at 8 per cell each and a
    1-GeV electron beam at 4 per cell (3.03e8 particles in all), with the
    beam's self-fields; tile 8 x 8 x 4, drift 0 (the benchmark's launch
    configuration for this case)."""
    print("full size: 3D beam-driven wakefield 512x192x192, 8+8+4 ppc, FP32", flush=True)
    wl = W.beam_wakefield_3d(device=DEV, tile=(8, 8, 4))
    sim, worst = laser_case(wl, (8, 8, 4), 0)
    for du, dx, jrel in worst:
        assert du < U_TOL and dx < X_TOL and jrel < J_TOL


def qed_species(n, capacity, dim, device=DEV):
    f32 = dict(device=device, dtype=torch.float32)
    return L.Particles(n, [torch.zeros(capacity, **f32) for _ in range(3)],
                       cell=torch.zeros(capacity, device=device, dtype=torch.int32),
                       off=[torch.zeros(capacity, **f32) for _ in range(dim)], w=torch.zeros(capacity, **f32),
                       chi=torch.zeros(capacity, **f32),
                       tau=torch.zeros(capacity, device=device, dtype=torch.float64),
                       tau_thr=torch.zeros(capacity, **f32),
                       id=torch.zeros(capacity, device=device, dtype=torch.int64), capacity=capacity,
                       n_dev=torch.tensor([n], device=device, dtype=torch.int64))


def qed_checks(cfg, ctx, sp, el, fields, bits, photons, step, nsample=2000, seed=5, mode=L.PIC_QED_TABLE,
               net=None, rate_rel=0.0):
    """Push the leptons (chi on), run one QED step (tables, or the network
    with its rate error `rate_rel` allowed), and check a sample: push vs the
    oracle, chi vs the oracle's chi, tau vs W dt from the oracle's F_rad (or
    an event where tau crossed its threshold), and for every sampled event
    the photon the GPU appended: its identifier and k = u_before - u_after
    (collinear recoil)."""
    L.pic_yee_step(ctx, 1, fields)
    for j in fields.J:
        j.zero_()
    torch.cuda.synchronize()
    F = host_fields(fields)
    snap = sampled_push(ctx, cfg, sp, el, fields, bits, nsample, seed)
    idx = snap["idx"]
    tau0 = np64(el.tau[idx])
    thr = np64(el.tau_thr[idx])
    ids = [int(v) for v in el.id[idx].cpu().numpy()]
    L.pic_qed_step(ctx, fields, electrons=el, photons=photons, mode=mode, step=step, photon_min_energy=0.0,
                   mlp=net)
    torch.cuda.synchronize()
    st, flags, _ = L.pic_check(ctx)
    assert st == L.PIC_OK, flags
    tau1 = np64(el.tau[idx])
    thr1 = np64(el.tau_thr[idx])
    u2 = [np64(t[idx]) for t in el.u]
    osp, chi_o, chi_scale = oracle_sample(cfg, sp, snap, F)
    du, dx = push_errors(cfg, snap, osp)
    # chi in FP32 cancels terms of size chi_scale (a lepton riding a plane
    # wave cancels gamma E against u x B): allow a few FP32 rounding units of
    # those terms, and 1e-4 of chi
    chi_g = snap["chi1"]
    chi_tol = 1e-5 * chi_scale + 1e-4 * chi_o + 1e-9
    chi_err = np.max(np.abs(chi_g - chi_o) / chi_tol)
    # tau: W dt with the oracle's own F_rad at its own chi and gamma^{n+1}.
    # dF/dchi is at most its classical-limit value 5 pi / 2, so chi's
    # allowance moves W dt by at most that much; plus 1e-4 of tau
    rates = {}
    fired_o = np.zeros(nsample, dtype=bool)
    near = np.zeros(nsample, dtype=bool)
    tau_err = 0.0
    worst_tau = None
    dt32 = float(np.float32(cfg.dt))
    for k in range(nsample):
        c = float(chi_o[k])
        if c not in rates:
            rates[c] = O.frad(c) if c > 0 else 0.0
        g1 = math.sqrt(1.0 + sum(osp.u[a][k] ** 2 for a in range(3)))
        t = tau0[k] + Q.A_CONST / cfg.hbar_omega_mc2 * rates[c] / g1 * dt32
        allow = (1e-4 * t + rate_rel * (t - tau0[k]) +
                 Q.A_CONST / cfg.hbar_omega_mc2 * 2.5 * math.pi * chi_tol[k] / g1 * dt32 + 1e-12)
        fired_o[k] = t >= thr[k] and c > 0
        near[k] = abs(t - thr[k]) <= 2 * allow
        if not fired_o[k] and not near[k] and abs(tau1[k] - t) / allow > tau_err:
            tau_err = abs(tau1[k] - t) / allow
            worst_tau = (c, float(chi_g[k]), t, float(tau1[k]), g1)
    fired_g = (tau1 == 0.0) & (thr1 != thr)  # an event restarts tau and draws a new threshold
    assert np.array_equal(fired_g[~near], fired_o[~near])
    # photons of the sampled events: identifier, k = u^{n+1} - u_after
    nph = int(photons.n_dev.item())
    pid = photons.id[:nph]
    checked = 0
    for k in np.nonzero(fired_g & ~near)[0]:
        cid = Q.child_id(cfg.seed, ids[k], step, 1)
        cid_s = cid - (1 << 64) if cid >= (1 << 63) else cid
        hit = torch.nonzero(pid == cid_s).flatten()
        kvec = np.array([snap["u1"][a][k] - u2[a][k] for a in range(3)])
        assert hit.numel() == 1  # every photon is kept (no energy threshold here)
        j = int(hit[0])
        kg = np.array([float(photons.u[a][j]) for a in range(3)])
        # u - u f in FP32 loses the bits of u that k does not carry
        umag = math.sqrt(sum(snap["u1"][a][k] ** 2 for a in range(3)))
        assert np.allclose(kg, kvec, rtol=1e-4, atol=1e-6 * (1 + umag))
        checked += 1
    print(f"  sample {nsample}: du {du:.2e}, dx {dx:.2e} cells, chi and tau at {chi_err:.2f} and "
          f"{tau_err:.2f} of their allowance, "
          f"{int(fired_o.sum())} events ({int(near.sum())} near the threshold), {checked} photons checked; "
          f"{nph} photons in all; worst tau (chi_o, chi_g, tau_o, tau_g, gamma): {worst_tau}", flush=True)
    assert du < U_TOL and dx < X_TOL
    assert chi_err <= 1.0 and tau_err <= 1.0
    return fired_o.sum(), checked


def test_qed_foil_2d_full_size():
    """2048 x 1024 cells, a0 = 500 on a 2-lambda foil at 100 n_c with 16
    electrons per cell, QED with tables: push, chi, optical depth, events
    and the photons of a sample against the oracle."""
    print("full size: 2D QED foil 2048x1024, 16 ppc, a0 500", flush=True)
    wl = W.qed_foil_2d(device=DEV)
    cfg = wl.cfg
    sim = Simulation.from_workload(wl, precision=L.PIC_FP32_MIXED, device=DEV, sort_every=1 << 30,
                                   with_chi=True)
    q, m, raw = wl.species[0]
    el = sim.particles[0]
    n = el.n
    gen = torch.Generator(device=DEV).manual_seed(31)
    el.tau = torch.zeros(n, device=DEV, dtype=torch.float64)
    el.tau_thr = -torch.log(torch.rand(n, generator=gen, device=DEV).clamp_min(1e-30))
    el.id = torch.arange(1, n + 1, device=DEV, dtype=torch.int64)
    el.capacity = n
    el.n_dev = torch.tensor([n], device=DEV, dtype=torch.int64)
    sim.spare = [el.empty_like()]
    sim.sort()
    el = sim.particles[0]
    el.n_dev = torch.tensor([n], device=DEV, dtype=torch.int64)
    check_sorted(el, sim.bits, sim.tile, sim.ntiles, cfg)
    photons = qed_species(0, n, 2)
    # two steps with the tables (the first lets the pulse accelerate the foil
    # electrons), then one with the trained network
    for step in (1, 2):
        events, checked = qed_checks(cfg, sim.ctx, sim.species[0], el, sim.fields, sim.bits, photons, step)
        L.pic_yee_step(sim.ctx, 2, sim.fields)
    assert events > 0 and checked > 0
    net = network(sim.ctx)
    events, checked = qed_checks(cfg, sim.ctx, sim.species[0], el, sim.fields, sim.bits, photons, 3,
                                 mode=L.PIC_QED_MLP, net=net, rate_rel=NET_RATE_REL)


def test_qed_3d_full_hbm():
    """1024 x 512 x 512 cells with 4 electrons in every cell (1.07e9) at
    50 n_c and two colliding a0 = 300 pulses: the FP32 state with the QED
    columns held in HBM (sorted copy included), one push and one QED step;
    the sample against the oracle as in the 2D case."""
    print("full size: 3D QED 1024x512x512, 4 ppc (1.07e9 electrons)", flush=True)
    cfg, el, E, B = W.qed_3d_full(device=DEV)
    ctx = L.pic_init(cfg)
    bits, tile, ntiles = L.pic_get_layout(ctx)
    n = el.n
    assert n == 1024 * 512 * 512 * 4
    el.tile_start = torch.zeros(ntiles + 1, dtype=torch.int64, device=DEV)
    dst = el.empty_like()
    L.pic_sort(ctx, el, dst)
    del el
    dst.n_dev = torch.tensor([n], device=DEV, dtype=torch.int64)
    torch.cuda.synchronize()
    check_sorted(dst, bits, tile, ntiles, cfg)
    fields = L.Fields(E, B, [torch.zeros_like(E[0]) for _ in range(3)])
    photons = qed_species(0, 1 << 24, 3)
    sp = L.Species(-1.0, 1.0, 1.0)
    events, checked = qed_checks(cfg, ctx, sp, dst, fields, bits, photons, step=1)
    L.pic_yee_step(ctx, 2, fields)
    net = network(ctx)
    events, checked = qed_checks(cfg, ctx, sp, dst, fields, bits, photons, step=2, mode=L.PIC_QED_MLP,
                                 net=net, rate_rel=NET_RATE_REL)
    print(f"  HBM in use: {torch.cuda.max_memory_allocated() / 2**30:.1f} GiB", flush=True)
