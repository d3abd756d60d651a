"""FP64 reference of one Monte-Carlo QED step (test infrastructure only).

Sec. IV of the paper, Method I written in optical-depth form: a particle
accumulates tau += W dt with W the total rate of Eq. 23 (photon emission) or
Eq. 24 (pair creation); when tau reaches its threshold tau_thr = -ln r' the
event happens, the energy fraction is the inverse of the cumulative spectrum
at a uniform r, tau restarts from 0 and a fresh threshold is drawn.  The
uniforms of particle `id` at `step` are Philox4x32-10 at counter
(id_lo, id_hi, step, 0) with key = seed; created particles get the identifier
Philox(parent_lo, parent_hi, step, 0x80000000 | tag) (tag 1 photon,
2 positron, 3 electron) and their first threshold from counter
(id_lo, id_hi, step, 1).  Recoil is collinear: u <- u (1 - eps_gamma/|u|),
clamped at 0.  Plain Python loops: meant for small particle counts.

Method II of Sec. IV (rejection) is here too: each step a lepton draws
(r1, r2), proposes the photon energy fraction u0 = r1^3 and emits when
3 r1^2 (d^2W/du dt)(u0) dt > r2; the paper leaves dt out of the printed
condition, a probability per step needs it.  For pair creation the
proposal is x0 = r1 (the spectrum of Eq. 24 has no endpoint singularity to
remove) and the test (d^2W/dx dt)(x0) dt > r2.  (r1, r2) are the same
counter-(id, step, 0) uniforms Method I uses; tau is not involved.
"""
from __future__ import annotations

import math

from . import chi as chi_of
from . import (compton_bracket, compton_inverse, fpair, frad, gather, pair_bracket, pair_inverse,
               philox4x32_10, qed_uniforms)

ALPHA = 1.0 / 137.035999084
A_CONST = ALPHA / (math.sqrt(3.0) * math.pi)


def child_id(seed: int, parent: int, step: int, tag: int) -> int:
    out = philox4x32_10([parent & 0xFFFFFFFF, (parent >> 32) & 0xFFFFFFFF, step & 0xFFFFFFFF,
                         0x80000000 | tag], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return (out[1] << 32) | out[0]


def first_threshold(seed: int, pid: int, step: int) -> float:
    a, _ = qed_uniforms(seed, pid, step, 1)
    return -math.log(a)


class Rates:
    """F_rad / F_pair and their inverse spectra from the oracle quadrature,
    memoised per chi (tests reuse a few chi values).  With nodes > 0 the
    inverse spectrum is the monotone linear interpolation of the exact
    cumulative integral at `nodes` points (in s = u^(1/3) for emission, in x
    for pairs) instead of a bisection over full quadratures: statistical tests
    draw thousands of events."""

    def __init__(self, nodes: int = 0):
        self._fr, self._fp = {}, {}
        self.nodes = nodes
        self._cum = {}

    def frad(self, chi):
        if chi not in self._fr:
            self._fr[chi] = frad(chi) if chi > 0 else 0.0
        return self._fr[chi]

    def fpair(self, chi):
        if chi not in self._fp:
            self._fp[chi] = fpair(chi) if chi > 0 else 0.0
        return self._fp[chi]

    def _table(self, proc, chi):
        key = (proc, chi)
        if key not in self._cum:
            from . import compton_cum, pair_cum
            xs = [i / self.nodes for i in range(self.nodes + 1)]
            if proc == 0:
                cum = [compton_cum(chi, s ** 3) for s in xs]
            else:
                cum = [pair_cum(chi, x) for x in xs]
            self._cum[key] = (xs, cum)
        return self._cum[key]

    def inverse(self, proc, chi, r):
        if self.nodes <= 0:
            return compton_inverse(chi, r) if proc == 0 else pair_inverse(chi, r)
        xs, cum = self._table(proc, chi)
        target = r * cum[-1]
        lo, hi = 0, len(xs) - 1
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if cum[mid] < target:
                lo = mid
            else:
                hi = mid
        f = (target - cum[lo]) / (cum[hi] - cum[lo]) if cum[hi] > cum[lo] else 0.0
        v = xs[lo] + f * (xs[hi] - xs[lo])
        return v ** 3 if proc == 0 else v


def lepton_step(leptons: dict, seed: int, step: int, dt: float, hbar_w: float, emin: float,
                rates: Rates, photons_out: list | None):
    """leptons: dict of lists u (3 x n), chi, tau, tau_thr, id, w, pos (opaque
    position token copied to created photons).  Updated in place; created
    photons are appended to photons_out as dicts."""
    R = 1.0 / hbar_w
    n = len(leptons["chi"])
    for p in range(n):
        w = leptons["w"][p]
        if w == 0.0:
            continue
        u = [leptons["u"][a][p] for a in range(3)]
        chi = leptons["chi"][p]
        pu2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        gam = math.sqrt(1.0 + pu2)
        W = A_CONST * R * rates.frad(chi) / gam
        tau = leptons["tau"][p] + W * dt
        if tau >= leptons["tau_thr"][p] and chi > 0.0:
            pid = leptons["id"][p]
            ru, rt = qed_uniforms(seed, pid, step, 0)
            uf = rates.inverse(0, chi, ru)
            eps = uf * gam
            pm = math.sqrt(pu2)
            if pm > 0:
                k = [eps * c / pm for c in u]
                if photons_out is not None and eps >= emin:
                    cid = child_id(seed, pid, step, 1)
                    photons_out.append(dict(k=k, w=w, pos=leptons["pos"][p], id=cid,
                                            tau_thr=first_threshold(seed, cid, step)))
                f = max(0.0, 1.0 - eps / pm)
                for a in range(3):
                    leptons["u"][a][p] = u[a] * f
            tau = 0.0
            leptons["tau_thr"][p] = -math.log(rt)
        leptons["tau"][p] = tau


def photon_move_chi(grid, F, photons: dict, dt: float, hbar_w: float):
    """The photon part of a step before pair creation (Sec. IV): a photon of
    momentum k (energy eps = |k|, m c^2 units) moves at the speed of light,
    x <- x + dt k / eps, and its chi_gamma is taken at the new position,
    (hbar w_r / m c^2) sqrt((eps E + k x B)^2 - (k . E)^2), with E and B
    gathered there as for any particle (Eq. 19).  photons: dict of lists
    x (dim x n, absolute positions), k (3 x n), w; writes chi.  Periodic
    wrap; with absorbing x faces (grid.absorb_x) a photon whose new position
    leaves [0, (n_x - 1) d_x] is absorbed (w = 0, chi = 0), like a lepton."""
    n = len(photons["w"])
    photons.setdefault("chi", [0.0] * n)
    L = [grid.n[a] * grid.d[a] for a in range(grid.dim)]
    for p in range(n):
        if photons["w"][p] == 0.0:
            continue
        k = [photons["k"][a][p] for a in range(3)]
        eps = math.sqrt(sum(c * c for c in k))
        if not eps > 0.0:
            continue
        xn = [photons["x"][a][p] + dt * k[a] / eps for a in range(grid.dim)]
        if grid.absorb_x and (xn[0] < 0.0 or xn[0] >= (grid.n[0] - 1) * grid.d[0]):
            photons["w"][p] = 0.0
            photons["chi"][p] = 0.0
        for a in range(grid.dim):
            photons["x"][a][p] = xn[a] % L[a]
        if photons["w"][p] == 0.0:
            continue
        EB = gather(grid, F, [photons["x"][a][p] for a in range(grid.dim)] + [0.0] * (3 - grid.dim))
        photons["chi"][p] = chi_of(hbar_w, eps, k, EB[:3], EB[3:])


def photon_decay(photons: dict, seed: int, step: int, dt: float, hbar_w: float, rates: Rates,
                 positrons_out: list, electrons_out: list):
    """photons: dict of lists k (3 x n), chi (chi_gamma, already at the photon),
    tau, tau_thr, id, w, pos.  Pair creation above 2 m c^2."""
    R = 1.0 / hbar_w
    n = len(photons["chi"])
    for p in range(n):
        w = photons["w"][p]
        if w == 0.0:
            continue
        k = [photons["k"][a][p] for a in range(3)]
        eps = math.sqrt(sum(c * c for c in k))
        chi = photons["chi"][p]
        W = A_CONST * R * rates.fpair(chi) / eps
        tau = photons["tau"][p] + W * dt
        if tau >= photons["tau_thr"][p] and eps > 2.0 and chi > 0.0:
            pid = photons["id"][p]
            rx, _ = qed_uniforms(seed, pid, step, 0)
            x = rates.inverse(1, chi, rx)
            ep, em = x * eps, (1.0 - x) * eps
            npl = math.sqrt(max(ep * ep - 1.0, 0.0)) / eps
            nmi = math.sqrt(max(em * em - 1.0, 0.0)) / eps
            for out, nn, tag in ((positrons_out, npl, 2), (electrons_out, nmi, 3)):
                cid = child_id(seed, pid, step, tag)
                out.append(dict(u=[nn * c for c in k], w=w, pos=photons["pos"][p], id=cid,
                                tau_thr=first_threshold(seed, cid, step)))
            photons["w"][p] = 0.0
            tau = 0.0
        photons["tau"][p] = tau


# ------------------------------------------------------------- Method II

def emission_acceptance(chi: float, gamma: float, r1: float, dt: float, hbar_w: float) -> float:
    """3 r1^2 (d^2W_rad/du dt)(r1^3) dt in the units of Eq. 8: Eq. 23's
    prefactor alpha m c^2 / (sqrt3 pi hbar w_r gamma) times its bracket, with
    the Jacobian du/dr1 = 3 r1^2 of the proposal u0 = r1^3."""
    return A_CONST / hbar_w / gamma * 3.0 * r1 * r1 * compton_bracket(r1 ** 3, chi) * dt


def pair_acceptance(chi: float, eps: float, x0: float, dt: float, hbar_w: float) -> float:
    """(d^2W_pair/dx dt)(x0) dt with x = eps_+/eps_gamma: Eq. 24 times
    d eps_+/dx = eps_gamma, i.e. alpha m c^2 / (sqrt3 pi hbar w_r eps_gamma)
    times its bracket."""
    return A_CONST / hbar_w / eps * pair_bracket(x0, chi) * dt


def lepton_step_method2(leptons: dict, seed: int, step: int, dt: float, hbar_w: float, emin: float,
                        photons_out: list | None) -> bool:
    """Method II photon emission for one step; same containers as lepton_step
    (tau and tau_thr untouched).  Returns True when some acceptance exceeded 1
    (the step is too long for the rate: the emission probability saturates)."""
    saturated = False
    n = len(leptons["chi"])
    for p in range(n):
        w = leptons["w"][p]
        chi = leptons["chi"][p]
        if w == 0.0 or not chi > 0.0:
            continue
        u = [leptons["u"][a][p] for a in range(3)]
        pu2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        gam = math.sqrt(1.0 + pu2)
        pid = leptons["id"][p]
        r1, r2 = qed_uniforms(seed, pid, step, 0)
        acc = emission_acceptance(chi, gam, r1, dt, hbar_w)
        saturated |= acc > 1.0
        if acc <= r2:
            continue
        eps = r1 ** 3 * gam
        pm = math.sqrt(pu2)
        if pm > 0:
            k = [eps * c / pm for c in u]
            if photons_out is not None and eps >= emin:
                cid = child_id(seed, pid, step, 1)
                photons_out.append(dict(k=k, w=w, pos=leptons["pos"][p], id=cid,
                                        tau_thr=first_threshold(seed, cid, step)))
            f = max(0.0, 1.0 - eps / pm)
            for a in range(3):
                leptons["u"][a][p] = u[a] * f
    return saturated


def photon_decay_method2(photons: dict, seed: int, step: int, dt: float, hbar_w: float,
                         positrons_out: list, electrons_out: list) -> bool:
    """Method II pair creation for one step (photons above 2 m c^2); same
    containers as photon_decay.  Returns the saturation flag."""
    saturated = False
    n = len(photons["chi"])
    for p in range(n):
        w = photons["w"][p]
        chi = photons["chi"][p]
        if w == 0.0:
            continue
        k = [photons["k"][a][p] for a in range(3)]
        eps = math.sqrt(sum(c * c for c in k))
        if not (eps > 2.0 and chi > 0.0):
            continue
        pid = photons["id"][p]
        r1, r2 = qed_uniforms(seed, pid, step, 0)
        acc = pair_acceptance(chi, eps, r1, dt, hbar_w)
        saturated |= acc > 1.0
        if acc <= r2:
            continue
        ep, em = r1 * eps, (1.0 - r1) * eps
        npl = math.sqrt(max(ep * ep - 1.0, 0.0)) / eps
        nmi = math.sqrt(max(em * em - 1.0, 0.0)) / eps
        for out, nn, tag in ((positrons_out, npl, 2), (electrons_out, nmi, 3)):
            cid = child_id(seed, pid, step, tag)
            out.append(dict(u=[nn * c for c in k], w=w, pos=photons["pos"][p], id=cid,
                            tau_thr=first_threshold(seed, cid, step)))
        photons["w"][p] = 0.0
    return saturated


# ------------------------------------------------ cascade in a uniform field

def cascade_uniform_b(b0: float, gamma0: float, n_el: int, steps: int, dt: float, hbar_w: float, seed: int,
                      ids=None, emin: float = 0.0, first_step: int = 0):
    """Electron-positron cascade of the Fig. 9 setup (Sec. IV): electrons of
    Lorentz factor gamma0 moving along x across a uniform magnetic field
    B = b0 z^ (E = 0), photon emission and pair creation by Method II only,
    with the field left external (no current feedback: the test particles of
    the setup).  Each step, in the order of the library's step: every lepton
    that exists at the start of the step is pushed by Boris (Eqs. 13-16) and
    takes chi_e at u^{n+1/2} = (u^n + u^{n+1})/2; the photons that exist at
    the start of the step take chi_gamma and may decay into a pair (Eq. 24);
    then the leptons of the start of the step may emit (Eq. 23), the photon
    going along u with recoil.  Particles created in a step act from the next
    step on.  Positions do not enter (the field is uniform).  Returns the
    containers: electrons and positrons (dicts of u, chi, w, id, pos, q) and
    photons (k, chi, w, id, pos), and the saturation flag of Method II."""
    from . import boris
    u0 = math.sqrt(gamma0 * gamma0 - 1.0)
    ids = list(range(1, n_el + 1)) if ids is None else list(ids)
    el = dict(u=[[u0] * n_el, [0.0] * n_el, [0.0] * n_el], chi=[0.0] * n_el, tau=[0.0] * n_el, tau_thr=[0.0] * n_el,
              id=ids, w=[1.0] * n_el, pos=list(range(n_el)), q=-1.0)
    po = dict(u=[[], [], []], chi=[], tau=[], tau_thr=[], id=[], w=[], pos=[], q=1.0)
    ph = dict(k=[[], [], []], chi=[], tau=[], tau_thr=[], id=[], w=[], pos=[])
    E0 = [0.0, 0.0, 0.0]
    B0 = [0.0, 0.0, b0]
    saturated = False

    def append_lepton(L, p):
        for a in range(3):
            L["u"][a].append(p["u"][a])
        L["chi"].append(0.0)
        L["tau"].append(0.0)
        L["tau_thr"].append(p["tau_thr"])
        L["id"].append(p["id"])
        L["w"].append(p["w"])
        L["pos"].append(p["pos"])

    for s in range(first_step, first_step + steps):
        for L in (el, po):
            for p in range(len(L["w"])):
                u = [L["u"][a][p] for a in range(3)]
                un = boris(L["q"], dt, E0, B0, u)
                uh = [0.5 * (u[a] + un[a]) for a in range(3)]
                gh = math.sqrt(1.0 + sum(c * c for c in uh))
                L["chi"][p] = chi_of(hbar_w, gh, uh, E0, B0)
                for a in range(3):
                    L["u"][a][p] = float(un[a])
        nph = len(ph["w"])
        for p in range(nph):
            k = [ph["k"][a][p] for a in range(3)]
            eps = math.sqrt(sum(c * c for c in k))
            ph["chi"][p] = chi_of(hbar_w, eps, k, E0, B0) if eps > 0 else 0.0
        view = {key: (val[:nph] if key != "k" else [v[:nph] for v in val]) for key, val in ph.items()}
        pos_out, ele_out = [], []
        saturated |= photon_decay_method2(view, seed, s, dt, hbar_w, pos_out, ele_out)
        ph["w"][:nph] = view["w"]
        n0 = (len(el["w"]), len(po["w"]))
        ph_out = []
        for L, n in zip((el, po), n0):
            sub = {key: (val[:n] if key not in ("u", "q") else ([v[:n] for v in val] if key == "u" else val))
                   for key, val in L.items()}
            saturated |= lepton_step_method2(sub, seed, s, dt, hbar_w, emin, ph_out)
            for a in range(3):
                L["u"][a][:n] = sub["u"][a]
        for p in pos_out:
            append_lepton(po, p)
        for p in ele_out:
            append_lepton(el, p)
        for p in ph_out:
            for a in range(3):
                ph["k"][a].append(p["k"][a])
            ph["chi"].append(0.0)
            ph["tau"].append(0.0)
            ph["tau_thr"].append(p["tau_thr"])
            ph["id"].append(p["id"])
            ph["w"].append(p["w"])
            ph["pos"].append(p["pos"])
    return el, po, ph, saturated
