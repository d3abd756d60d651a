"""Bunch self-fields on the GPU (pic_beam_fields, Sec. III(c)) against the
oracle's Coulomb-law fields, the line-charge limit and Gauss's law.  Calls go
through the C ABI (ctypes)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import beam as BM
from paper_2104_00642_amd import _lib as L
from paper_2104_00642_amd.workloads import courant_dt

from _helpers import DEV, np64

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")]

# Yee position of each component, in cells: E_x, E_y, E_z, B_x, B_y, B_z
STAGGER = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def beam_case(dim, precision, gamma, n=None, d=None, center=None, sigma=None, density=3.0):
    n = n or ((40, 24, 20) if dim == 3 else (48, 32))
    d = d or ((0.1, 0.09, 0.11) if dim == 3 else (0.1, 0.08))
    cfg = L.Config(dim=dim, n=n, d=d, dt=courant_dt(d), order=2, precision=precision, drift=1)
    center = center or tuple(0.47 * n[a] * d[a] for a in range(dim))
    sigma = sigma or ((0.4, 0.3, 0.35) if dim == 3 else (0.4, 0.3))
    beam = L.Beam(charge=-1.0, density=density, center=center, sigma=sigma, gamma=gamma)
    ctx = L.pic_init(cfg)
    dt = torch.float64 if precision == L.PIC_FP64_PLAIN else torch.float32
    f = L.Fields.zeros(cfg, DEV, dt)
    L.pic_beam_fields(ctx, beam, f)
    torch.cuda.synchronize()
    ob = BM.Bunch(beam.charge, beam.density, center, sigma, gamma, dim=dim)
    return cfg, f, ob


def node_value(f, comp, idx):
    plane = (f.E + f.B)[comp]
    return float(plane[idx].double().item())


@pytest.mark.parametrize("dim,precision,gamma,nodes", [
    (3, L.PIC_FP64_PLAIN, 3.0, 4), (3, L.PIC_FP32_MIXED, 20.0, 2),
    (2, L.PIC_FP64_PLAIN, 1.0, 8), (2, L.PIC_FP64_PLAIN, 5.0, 8), (2, L.PIC_FP32_MIXED, 3.0, 6)])
def test_beam_fields_match_oracle(dim, precision, gamma, nodes):
    """Every component at seeded nodes (near the bunch, at the box's edge and
    at its corner) equals the oracle's line-of-sight Coulomb integral at that
    component's Yee position: 1e-9 of the sampled maximum in FP64, FP32
    rounding in FP32."""
    print(f"beam fields dim={dim} prec={precision} gamma={gamma}", flush=True)
    cfg, f, ob = beam_case(dim, precision, gamma)
    n = cfg.n[:dim]
    rng = np.random.default_rng(int(gamma * 10) + dim)
    pts = [tuple(int(v) for v in rng.integers(0, n)) for _ in range(nodes - 2)]
    pts += [tuple(v - 1 for v in n), tuple(0 for _ in n)]
    comps = [0, 1, 5] if dim == 2 else [0, 1, 2, 4, 5]
    got, want = [], []
    for p in pts:
        idx = tuple(reversed(p)) if dim == 3 else (0, p[1], p[0])
        for c in comps:
            pos = [(p[a] + STAGGER[c][a]) * cfg.d[a] for a in range(dim)]
            want.append(BM.lab_field(ob, c, *pos))
            got.append(node_value(f, c, idx))
    got, want = np.array(got), np.array(want)
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    print(f"  {len(got)} values, max |E| {scale:.3e}, max error {err:.2e} of it")
    assert err < (1e-9 if precision == L.PIC_FP64_PLAIN else 3e-7)
    # components the bunch leaves alone stay zero
    for c in ([2, 3, 4] if dim == 2 else [3]):
        assert float((f.E + f.B)[c].abs().max().item()) == 0.0


def test_beam_fields_of_the_wakefield_bunch_are_the_line_charge_field():
    """The wakefield case's 1-GeV bunch (gamma 1957, sigma 0.5, n_b = 4) on a
    128 x 48 x 48 box: within 1e-5 of the ultrarelativistic closed form
    E_r = Lambda(x) (1 - exp(-r^2 / (2 sigma^2))) / (2 pi r) at every node
    (the departure, of order ln(gamma)/gamma^2, is about 2e-6 here), E_x at
    most 1e-5 of E_perp, B = beta x^ x E."""
    print("beam fields: wakefield bunch, line-charge limit", flush=True)
    lam_p = 2 * math.pi
    n = (128, 48, 48)
    d = (4 * lam_p / 512, 2 * lam_p / 192, 2 * lam_p / 192)
    center = (0.75 * n[0] * d[0], 0.5 * n[1] * d[1], 0.5 * n[2] * d[2])
    gamma, sigma, nb = 1957.0, 0.5, 4.0
    cfg, f, _ = beam_case(3, L.PIC_FP64_PLAIN, gamma, n=n, d=d, center=center, sigma=(sigma,) * 3, density=nb)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")

    def closed(sx, sy, sz):
        x = (i + sx) * d[0] - center[0]
        y = (j + sy) * d[1] - center[1]
        z = (k + sz) * d[2] - center[2]
        r2 = y * y + z * z
        lam = -nb * np.exp(-x * x / (2 * sigma ** 2)) * 2 * math.pi * sigma ** 2
        er_r = lam * (1 - np.exp(-r2 / (2 * sigma ** 2))) / (2 * math.pi * r2)
        return er_r * y, er_r * z
    ey, _ = closed(0, 0.5, 0)
    _, ez = closed(0, 0, 0.5)
    E = [np64(t) for t in f.E]
    B = [np64(t) for t in f.B]
    for got, want in ((E[1], ey), (E[2], ez)):
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        print(f"  rel L2 against the closed form {err:.2e}, max {np.abs(got - want).max() / np.abs(want).max():.2e}")
        assert err < 1e-5
    assert np.abs(E[0]).max() < 1e-5 * np.abs(E[1]).max()
    beta = math.sqrt(1 - 1 / gamma ** 2)
    _, ez_by = closed(0.5, 0, 0.5)
    ey_bz, _ = closed(0.5, 0.5, 0)
    assert np.linalg.norm(B[1] + beta * ez_by) < 1e-5 * np.linalg.norm(ez_by)
    assert np.linalg.norm(B[2] - beta * ey_bz) < 1e-5 * np.linalg.norm(ey_bz)


@pytest.mark.parametrize("dim", [2, 3])
def test_beam_fields_satisfy_gauss_law(dim):
    """The discrete divergence of the GPU's E equals the bunch's lab charge
    density on the nodes near it, up to the Yee divergence's second-order
    error, (d/sigma)^2/12 per axis; fields add to what the planes hold."""
    print(f"beam fields: Gauss's law dim={dim}", flush=True)
    cfg, f, ob = beam_case(dim, L.PIC_FP64_PLAIN, 2.5)
    g = O.Grid(dim, tuple(cfg.n[:dim]), tuple(cfg.d[:dim]), cfg.dt, 2)
    E = [np64(t) for t in f.E]
    dv = O.div(g, E)
    n, d = cfg.n, cfg.d
    if dim == 3:
        z, y, x = np.meshgrid(np.arange(n[2]) * d[2], np.arange(n[1]) * d[1], np.arange(n[0]) * d[0],
                              indexing="ij")
        q2 = [((x - ob.center[0]) / ob.sigma[0]) ** 2, ((y - ob.center[1]) / ob.sigma[1]) ** 2,
              ((z - ob.center[2]) / ob.sigma[2]) ** 2]
    else:
        y, x = np.meshgrid(np.arange(n[1]) * d[1], np.arange(n[0]) * d[0], indexing="ij")
        y, x = y[None], x[None]
        q2 = [((x - ob.center[0]) / ob.sigma[0]) ** 2, ((y - ob.center[1]) / ob.sigma[1]) ** 2]
    rho = ob.q * ob.n_b * np.exp(-0.5 * sum(q2))
    # within 3 sigma, and off the first node of each axis, where the
    # divergence's backward difference wraps across the (non-periodic) field
    near = sum(q2) < 9.0
    if dim == 3:
        near[0, :, :] = False
    near[:, 0, :] = False
    near[:, :, 0] = False
    err = np.linalg.norm((dv - rho)[near]) / np.linalg.norm(rho[near])
    bound = sum((d[a] / ob.sigma[a]) ** 2 / 12 for a in range(dim))
    print(f"  relative L2 {err:.2e} (bound {bound:.2e})")
    assert err < bound
    # adding a second call doubles the fields
    before = np64(f.E[1]).copy()
    ctx = L.pic_init(cfg)
    L.pic_beam_fields(ctx, L.Beam(ob.q, ob.n_b, ob.center, ob.sigma, ob.gamma), f)
    torch.cuda.synchronize()
    assert np.allclose(np64(f.E[1]), 2 * before, rtol=1e-14, atol=0)


def test_beam_fields_reject_bad_arguments():
    cfg = L.Config(dim=3, n=(16, 16, 16), d=(0.1,) * 3, dt=0.05, precision=L.PIC_FP64_PLAIN)
    ctx = L.pic_init(cfg)
    f = L.Fields.zeros(cfg, DEV, torch.float64)
    for bad in (dict(gamma=0.5), dict(sigma=(0.1, 0.0, 0.1)), dict(density=float("nan"))):
        kw = dict(charge=-1.0, density=1.0, center=(0.8, 0.8, 0.8), sigma=(0.2, 0.2, 0.2), gamma=2.0)
        kw.update(bad)
        with pytest.raises(L.PicError):
            L.pic_beam_fields(ctx, L.Beam(**kw), f)
