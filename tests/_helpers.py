"""Shared helpers of the GPU parity tests: seeded inputs and comparisons.
No arithmetic of the method lives here."""
import math

import numpy as np
import torch

import oracle as O
from paper_2104_00642_amd import _lib as L
from paper_2104_00642_amd.workloads import RawParticles, courant_dt, to_fp32, to_fp64

DEV = "cuda"


def random_raw(cfg: L.Config, n: int, seed: int, uth: float = 0.8, cells=None) -> RawParticles:
    g = torch.Generator().manual_seed(seed)
    dim = cfg.dim
    if cells is None:
        cells = [torch.randint(0, cfg.n[a], (n,), generator=g) for a in range(dim)]
    off = [torch.rand(n, generator=g, dtype=torch.float64) for _ in range(dim)]
    u = [torch.randn(n, generator=g, dtype=torch.float64) * uth for _ in range(3)]
    w = 0.5 + torch.rand(n, generator=g, dtype=torch.float64)
    return RawParticles([c.to(torch.int64) for c in cells], off, u, w)


def random_fields(cfg: L.Config, seed: int, amp: float = 0.4):
    g = torch.Generator().manual_seed(seed + 1000)
    shp = cfg.plane_shape
    E = [torch.randn(shp, generator=g, dtype=torch.float64) * amp for _ in range(3)]
    B = [torch.randn(shp, generator=g, dtype=torch.float64) * amp for _ in range(3)]
    return E, B


def oracle_grid(cfg: L.Config) -> O.Grid:
    return O.Grid(cfg.dim, tuple(cfg.n[: cfg.dim]), tuple(cfg.d[: cfg.dim]), cfg.dt, cfg.order,
                  pusher=cfg.pusher)


def oracle_species(cfg, raw: RawParticles, q, m, from_fp32: bool):
    p = to_fp64(raw, cfg, from_fp32=from_fp32)
    return O.Species(q=q, m=m, x=[x.numpy().copy() for x in p.x],
                     u=[u.numpy().copy() for u in p.u], w=p.w.numpy().copy(), w0=1.0)


def np64(t):
    return t.detach().to("cpu", torch.float64).numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def periodic_dx(a, b, L):
    d = np.asarray(a) - np.asarray(b)
    return d - L * np.round(d / L)
