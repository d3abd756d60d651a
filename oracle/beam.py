"""Self-fields of a relativistic bi-Gaussian bunch, FP64 reference (test
infrastructure only).

Sec. III(c) initializes an ultrarelativistic beam by solving Poisson's
equation in the beam's rest frame and Lorentz-transforming the fields to the
laboratory frame.  This module does exactly that for a Gaussian bunch in free
space, straight from Coulomb's law, with no Green's-function identity:

  rest frame:  E'(p) = Int rho'(r) (p - r) / (4 pi |p - r|^3) d^3r
               (div E = rho in the units of Eq. 8; in 2D the kernel is
               (p - r) / (2 pi |p - r|^2), the bunch uniform along z).
  Centred on p with r = p - l n (n a unit vector, l >= 0) the volume element
  l^2 dl dOmega cancels the 1/l^2, so
               E'(p) = 1/(4 pi) Int dOmega n Int_0^inf rho'(p - l n) dl
  (2D: 1/(2 pi) Int dtheta n Int_0^inf rho'(p - l n) dl).  For a Gaussian
  rho' the inner integral is a Gaussian integral over a half line, in closed
  form with erfc; the outer one is taken by adaptive quadrature.

  lab frame (bunch moving along +x with Lorentz factor gamma): the rest-frame
  bunch is gamma times longer along x and its density 1/gamma of the lab's
  (same total charge Q = q n_b (2 pi)^{D/2} prod sigma_lab); a lab point
  (x, y, z) at the lab time of the initialization sits at
  x' = gamma (x - x_c); E_x = E'_x, E_perp = gamma E'_perp, B = beta x^ x E
  (B' = 0 in the rest frame).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, special


@dataclass
class Bunch:
    """Charge q per particle, peak density n_b of the bunch's particles in
    the lab, centre, lab rms sizes (sigma_z unused in 2D), Lorentz factor of
    the motion along +x, dimension of the box (2 or 3)."""
    q: float
    n_b: float
    center: tuple
    sigma: tuple
    gamma: float
    dim: int = 3

    @property
    def charge(self) -> float:
        s = self.sigma[: self.dim]
        return self.q * self.n_b * (2 * math.pi) ** (self.dim / 2) * float(np.prod(s))

    @property
    def rest_sigma(self):
        return (self.gamma * self.sigma[0],) + tuple(self.sigma[1: self.dim])


def _half_line(q, n, sig) -> float:
    """Int_0^inf exp(-1/2 sum_b (q_b - l n_b)^2 / sig_b^2) dl, written as
    exp(-(A l^2 - 2 B l + C) / 2) and integrated in closed form."""
    A = sum(nb * nb / (s * s) for nb, s in zip(n, sig))
    B = sum(qb * nb / (s * s) for qb, nb, s in zip(q, n, sig))
    C = sum(qb * qb / (s * s) for qb, s in zip(q, sig))
    x = -B / math.sqrt(2 * A)
    if x <= 0.0:
        v = math.exp(-0.5 * (C - B * B / A)) * special.erfc(x)
    else:  # erfc(x) = erfcx(x) exp(-x^2): keeps the two exponentials from overflowing
        v = math.exp(-0.5 * C) * special.erfcx(x)
    return v * math.sqrt(math.pi / (2 * A))


def rest_frame_field(Q: float, sig, p, epsrel: float = 1e-11, comps=None):
    """E' at p (relative to the bunch centre) of a Gaussian bunch of total
    charge Q and rms sizes `sig` (2 or 3 of them) at rest, from Coulomb's
    law along lines of sight; `comps` limits the components computed (the
    others are returned as None)."""
    dim = len(sig)
    norm = Q / ((2 * math.pi) ** (dim / 2) * float(np.prod(sig)))
    p = [float(v) for v in p[:dim]]
    comps = range(dim) if comps is None else comps
    if dim == 2:
        out = [None, None]
        for a in comps:
            def f(th, a=a):
                n = (math.cos(th), math.sin(th))
                return n[a] * _half_line(p, n, sig)
            # the line through the centre and its opposite are the sharp features
            th0 = math.atan2(-p[1], -p[0])
            pts = sorted({(th0 + k * math.pi / 2) % (2 * math.pi) for k in range(4)})
            v, _ = integrate.quad(f, 0.0, 2 * math.pi, points=pts, epsabs=0.0, epsrel=epsrel, limit=400)
            out[a] = norm * v / (2 * math.pi)
        return out
    out = [None, None, None]
    for a in comps:
        # n = (mu, sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi), dOmega = dmu dphi
        def inner(mu, a=a):
            st = math.sqrt(max(0.0, 1.0 - mu * mu))

            def g(ph):
                n = (mu, st * math.cos(ph), st * math.sin(ph))
                return n[a] * _half_line(p, n, sig)
            v, _ = integrate.quad(g, 0.0, 2 * math.pi, epsabs=0.0, epsrel=epsrel, limit=400)
            return v
        # the bunch's long axis is x: the integrand peaks at mu = +-1
        v, _ = integrate.quad(inner, -1.0, 1.0, points=[-0.999, -0.99, -0.9, 0.9, 0.99, 0.999], epsabs=0.0,
                              epsrel=epsrel, limit=400)
        out[a] = norm * v / (4 * math.pi)
    return out


def lab_field(b: Bunch, comp: int, x, y, z=0.0, epsrel: float = 1e-11) -> float:
    """Component `comp` (0-2: E_x..E_z, 3-5: B_x..B_z) of the moving
    bunch's field at the lab point (x, y, z)."""
    g = b.gamma
    beta = math.sqrt(max(0.0, 1.0 - 1.0 / (g * g)))
    q = [g * (x - b.center[0]), y - b.center[1]] + ([z - b.center[2]] if b.dim == 3 else [])
    if comp == 3 or (b.dim == 2 and comp == 2):
        return 0.0
    # rest-frame component and the factor of the transformation
    rc, fac = {0: (0, 1.0), 1: (1, g), 2: (2, g), 4: (2, -beta * g), 5: (1, beta * g)}[comp]
    if b.dim == 2 and rc == 2:
        return 0.0
    return fac * rest_frame_field(b.charge, b.rest_sigma, q, epsrel, comps=[rc])[rc]


def lab_fields(b: Bunch, x, y, z=0.0, epsrel: float = 1e-11):
    """(E_x, E_y, E_z, B_x, B_y, B_z) at one lab point."""
    return tuple(lab_field(b, c, x, y, z, epsrel) for c in range(6))


def lab_density(b: Bunch, x, y, z=0.0) -> float:
    """q n_b exp(-sum (x_a - c_a)^2 / (2 sigma_a^2)): the lab charge density."""
    r = [x - b.center[0], y - b.center[1]] + ([z - b.center[2]] if b.dim == 3 else [])
    return b.q * b.n_b * math.exp(-0.5 * sum((v / s) ** 2 for v, s in zip(r, b.sigma)))
