"""FP64 CPU oracle for the particle-in-cell hot path (test infrastructure only).

This package is a plain, slow, obviously correct implementation of the method
of Song, Wang & Li, "YUNIC: A Multi-Dimensional Particle-In-Cell Code for
Laser-Plasma Interaction" (arXiv:2104.00642): shape-function field
interpolation (Sec. II.D, Eqs. 17-19), the Boris pusher (Sec. II.C,
Eqs. 11-16) and the Vay pusher Sec. II.C names as its alternative, Esirkepov's charge-conserving current deposit (Sec. II.E,
Eqs. 20-22), the Yee FDTD field update split in half steps (Sec. II.B Eqs. 9-10,
arranged as in Sec. II.F) and the Monte-Carlo QED rates (Sec. IV, Eqs. 23-24).

Only the test-suite, the smoke entry and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library (``paper_2104_00642_amd``)
and never imports it.  The C sources are in ``pic_oracle.c`` and
``qed_oracle.c``; this module is the ctypes marshalling plus the composition of
the half steps into a full step.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("order", C.c_int32), ("n", C.c_int64 * 3),
                ("d", C.c_double * 3), ("dt", C.c_double), ("pusher", C.c_int32),
                ("absorb_x", C.c_int32), ("laser", C.c_double * 4), ("laser_circular", C.c_int32)]


@dataclass
class Grid:
    """Grid and step: dim (2 or 3), shape order (1 CIC, 2 quadratic, 4 quartic), cells per
    axis, cell sizes and time step, all in the units of Eq. 8."""
    dim: int
    n: tuple
    d: tuple
    dt: float
    order: int = 2
    pusher: int = 0  # 0 Boris, 1 Vay
    absorb_x: int = 0  # absorbing x faces: 1 first-order, 2 second-order Mur rule for the fields
    laser: tuple = (0.0, 0.0, 0.0, 0.0)  # a0, waist, duration, t0 of the pulse injected at x = 0
    laser_circular: int = 0

    def c(self) -> _Grid:
        g = _Grid()
        g.dim = self.dim
        g.order = self.order
        g.pusher = self.pusher
        g.absorb_x = self.absorb_x
        for a in range(4):
            g.laser[a] = float(self.laser[a])
        g.laser_circular = self.laser_circular
        n = list(self.n) + [1] * (3 - len(self.n))
        d = list(self.d) + [1.0] * (3 - len(self.d))
        for a in range(3):
            g.n[a] = int(n[a])
            g.d[a] = float(d[a])
        g.dt = float(self.dt)
        return g

    @property
    def shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0])  # numpy planes indexed [k, j, i]

    @property
    def ncell(self):
        return int(np.prod(self.shape))

    @property
    def dV(self):
        return float(np.prod(self.d[: self.dim]))


_D = C.POINTER(C.c_double)
_PP = C.POINTER(C.POINTER(C.c_double))
_GP = C.POINTER(_Grid)


def _declare(L):
    L.orc_shape.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_int64), _D]
    L.orc_shape.restype = C.c_int
    L.orc_gather.argtypes = [_GP, _PP, _D, _D]
    L.orc_boris.argtypes = [C.c_double, C.c_double, _D, _D, _D]
    L.orc_vay.argtypes = [C.c_double, C.c_double, _D, _D, _D]
    L.orc_deposit.argtypes = [_GP, C.c_double, _D, _D, C.c_double, _PP]
    L.orc_push.argtypes = [_GP, C.c_double, C.c_double, C.c_int64, _PP, _PP, _D, C.c_double,
                           _PP, _PP, _D]
    L.orc_half_e.argtypes = [_GP, _PP, _PP, _PP, C.c_double, _D, C.POINTER(C.c_int32)]
    L.orc_half_b.argtypes = [_GP, _PP, _PP]
    L.orc_field_energy.argtypes = [_GP, _PP]
    L.orc_field_energy.restype = C.c_double
    L.orc_rho.argtypes = [_GP, C.c_double, C.c_int64, _PP, _D, C.c_double, _D]
    L.orc_div.argtypes = [_GP, _PP, _D]
    L.orc_curl_e.argtypes = [_GP, _PP, _PP]
    L.orc_sort.argtypes = [_GP, C.POINTER(C.c_int64), C.c_int64,
                           C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.c_int64),
                           C.POINTER(C.c_int64)]
    L.orc_sort.restype = C.c_int
    for name in ("orc_bessel_k",):
        getattr(L, name).argtypes = [C.c_double, C.c_double]
        getattr(L, name).restype = C.c_double
    for name in ("orc_int_k13", "orc_frad", "orc_fpair"):
        getattr(L, name).argtypes = [C.c_double]
        getattr(L, name).restype = C.c_double
    for name in ("orc_compton_bracket", "orc_pair_bracket", "orc_compton_cum", "orc_pair_cum",
                 "orc_compton_inverse", "orc_pair_inverse"):
        getattr(L, name).argtypes = [C.c_double, C.c_double]
        getattr(L, name).restype = C.c_double
    L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_uint32)]
    L.orc_u01.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_qed_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, _D, _D]
    L.orc_chi.argtypes = [C.c_double, C.c_double, _D, _D, _D]
    L.orc_chi.restype = C.c_double


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_D)


def _pp(arrs):
    ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dp(a) for a in arrs])
    return ptrs


# ------------------------------------------------------------------ pieces

def shape(order: int, xi: float):
    """(first node, weights) of the cell-integrated shape at position xi (cell units)."""
    i0 = C.c_int64()
    w = np.zeros(5)
    nw = lib().orc_shape(order, float(xi), C.byref(i0), _dp(w))
    return i0.value, w[:nw].copy()


def gather(grid: Grid, F, x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))
    out = np.zeros(6)
    lib().orc_gather(C.byref(grid.c()), _pp(F), _dp(x), _dp(out))
    return out


def boris(qm: float, dt: float, E, B, u):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().orc_boris(qm, dt, _dp(E), _dp(B), _dp(u))
    return u


def vay(qm: float, dt: float, E, B, u):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().orc_vay(qm, dt, _dp(E), _dp(B), _dp(u))
    return u


def deposit(grid: Grid, qw: float, xh, xe, vz: float, J):
    xh = np.ascontiguousarray(np.asarray(xh, dtype=np.float64).reshape(3))
    xe = np.ascontiguousarray(np.asarray(xe, dtype=np.float64).reshape(3))
    lib().orc_deposit(C.byref(grid.c()), qw, _dp(xh), _dp(xe), vz, _pp(J))


class MurHistory:
    """Face values of E_y, E_z (x nodes 0, 1, n-2, n-1) on entry to the last
    E half update: the earlier time level of the second-order Mur rule."""

    def __init__(self, grid: "Grid"):
        n = list(grid.n) + [1] * (3 - len(grid.n))
        self.values = np.zeros(8 * n[1] * n[2])
        self.valid = C.c_int32(0)


def half_e(grid: Grid, E, B, J, t: float = 0.0, mur: "MurHistory" = None):
    """E half step; t is the time of E on entry (used by the injected pulse).
    With second-order absorbing faces (absorb_x = 2) `mur` carries the face
    history from call to call (without it, or on its first use, the
    first-order rule runs)."""
    if mur is None:
        lib().orc_half_e(C.byref(grid.c()), _pp(E), _pp(B), _pp(J), float(t), None, None)
    else:
        lib().orc_half_e(C.byref(grid.c()), _pp(E), _pp(B), _pp(J), float(t), _dp(mur.values),
                         C.byref(mur.valid))


def half_b(grid: Grid, E, B):
    lib().orc_half_b(C.byref(grid.c()), _pp(E), _pp(B))


def field_energy(grid: Grid, E, B) -> float:
    return lib().orc_field_energy(C.byref(grid.c()), _pp(list(E) + list(B)))


def rho(grid: Grid, q: float, x, w=None, w0: float = 1.0):
    out = np.zeros(grid.shape)
    xs = [np.ascontiguousarray(a, dtype=np.float64) for a in x]
    while len(xs) < 3:
        xs.append(np.zeros_like(xs[0]))
    wp = _dp(np.ascontiguousarray(w, dtype=np.float64)) if w is not None else None
    lib().orc_rho(C.byref(grid.c()), q, len(xs[0]), _pp(xs), wp, w0, _dp(out))
    return out


def div(grid: Grid, V):
    out = np.zeros(grid.shape)
    lib().orc_div(C.byref(grid.c()), _pp(V), _dp(out))
    return out


def curl_e(grid: Grid, E):
    out = [np.zeros(grid.shape) for _ in range(3)]
    lib().orc_curl_e(C.byref(grid.c()), _pp(E), _pp(out))
    return out


def sort(grid: Grid, tile, cells):
    """Tile binning order (tile, rank-in-cell, cell-in-tile); returns (perm, tile_start)."""
    cs = [np.ascontiguousarray(c, dtype=np.int32) for c in cells]
    while len(cs) < 3:
        cs.append(np.zeros_like(cs[0]))
    np_ = len(cs[0])
    t = list(tile) + [1] * (3 - len(tile))
    ntiles = 1
    n = list(grid.n) + [1] * (3 - len(grid.n))
    for a in range(grid.dim):
        ntiles *= n[a] // t[a]
    perm = np.zeros(max(np_, 1), dtype=np.int64)
    start = np.zeros(ntiles + 1, dtype=np.int64)
    tarr = (C.c_int64 * 3)(*t)
    cp = (C.POINTER(C.c_int32) * 3)(*[c.ctypes.data_as(C.POINTER(C.c_int32)) for c in cs])
    rc = lib().orc_sort(C.byref(grid.c()), tarr, np_, cp,
                        perm.ctypes.data_as(C.POINTER(C.c_int64)),
                        start.ctypes.data_as(C.POINTER(C.c_int64)))
    assert rc == 0
    return perm[:np_], start


# ------------------------------------------------------------ composition

@dataclass
class Species:
    """One particle species: charge q (units of e), mass m (units of m_e),
    absolute FP64 positions x[dim] and momenta u[3] = p/m, per-particle
    weights w (density in n_r) or the constant w0."""
    q: float
    m: float
    x: list
    u: list
    w: np.ndarray | None = None
    w0: float = 1.0

    @property
    def n(self):
        return len(self.u[0])


@dataclass
class State:
    grid: Grid
    E: list
    B: list
    J: list
    species: list = field(default_factory=list)
    t: float = 0.0
    mur: "MurHistory" = None  # second-order absorbing faces: made by the first step

    @staticmethod
    def zeros(grid: Grid):
        z = lambda: [np.zeros(grid.shape) for _ in range(3)]  # noqa: E731
        return State(grid, z(), z(), z(), [])


def push(grid: Grid, sp: Species, F, J, diag=None):
    """Gather + Boris + move + Esirkepov deposit for every particle of `sp`
    (fields F at n+1/2); positions and momenta updated in place, J accumulated."""
    xs = list(sp.x)
    if grid.dim == 2:
        xs = xs[:2] + [np.zeros(sp.n)]
    wp = _dp(sp.w) if sp.w is not None else None
    dg = _dp(diag) if diag is not None else None
    lib().orc_push(C.byref(grid.c()), sp.q, sp.m, sp.n, _pp(xs), _pp(sp.u), wp, sp.w0, _pp(F),
                   _pp(J), dg)


_omp = None


def push_parallel(grid: Grid, sp: Species, F, J) -> int:
    """`push` on every host thread (the benchmark's CPU baseline): one chunk
    of particles per thread, thread-private current planes summed into J.
    Returns the number of threads that ran."""
    global _omp
    if _omp is None:
        if not os.path.exists(_build.OMP_LIB):
            _build.build_omp()
        _omp = C.CDLL(_build.OMP_LIB)
        _omp.orc_push_omp.argtypes = [_GP, C.c_double, C.c_double, C.c_int64, _PP, _PP, _D, C.c_double, _PP, _PP,
                                      C.POINTER(C.c_int)]
        _omp.orc_push_omp.restype = C.c_int
    xs = list(sp.x)
    if grid.dim == 2:
        xs = xs[:2] + [np.zeros(sp.n)]
    wp = _dp(sp.w) if sp.w is not None else None
    used = C.c_int(0)
    rc = _omp.orc_push_omp(C.byref(grid.c()), sp.q, sp.m, sp.n, _pp(xs), _pp(sp.u), wp, sp.w0, _pp(F), _pp(J),
                           C.byref(used))
    assert rc == 0, "cannot allocate the per-thread current planes"
    return used.value


def step(st: State, diag=None):
    """One full step in the half-step arrangement of Sec. II.F:
    E += dt/2 (curl B - J^n); B -= dt/2 curl E; particles (J^{n+1} from zero);
    B -= dt/2 curl E; E += dt/2 (curl B - J^{n+1}).  J^n is the current left
    in st.J by the previous step (zero at start)."""
    g = st.grid
    if g.absorb_x == 2 and st.mur is None:
        st.mur = MurHistory(g)
    half_e(g, st.E, st.B, st.J, st.t, st.mur)
    half_b(g, st.E, st.B)
    for a in range(3):
        st.J[a][...] = 0.0
    F = list(st.E) + list(st.B)
    for sp in st.species:
        push(g, sp, F, st.J, diag)
    half_b(g, st.E, st.B)
    half_e(g, st.E, st.B, st.J, st.t + 0.5 * g.dt, st.mur)
    st.t += g.dt


def kinetic_energy(grid: Grid, sp: Species) -> float:
    u = sp.u
    gam = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    w = sp.w if sp.w is not None else sp.w0
    return float(np.sum(w * sp.m * (gam - 1.0)) * grid.dV)


def total_energy(st: State) -> float:
    return field_energy(st.grid, st.E, st.B) + sum(kinetic_energy(st.grid, s) for s in st.species)


# --------------------------------------------------------------------- QED

def bessel_k(nu: float, y: float) -> float:
    return lib().orc_bessel_k(nu, y)


def int_k13(y: float) -> float:
    return lib().orc_int_k13(y)


def frad(chi: float) -> float:
    return lib().orc_frad(chi)


def fpair(chi: float) -> float:
    return lib().orc_fpair(chi)


def compton_bracket(u: float, chi: float) -> float:
    return lib().orc_compton_bracket(u, chi)


def pair_bracket(x: float, chi: float) -> float:
    return lib().orc_pair_bracket(x, chi)


def compton_cum(chi: float, u0: float) -> float:
    return lib().orc_compton_cum(chi, u0)


def pair_cum(chi: float, x0: float) -> float:
    return lib().orc_pair_cum(chi, x0)


def compton_inverse(chi: float, r: float) -> float:
    return lib().orc_compton_inverse(chi, r)


def pair_inverse(chi: float, r: float) -> float:
    return lib().orc_pair_inverse(chi, r)


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def u01(hi: int, lo: int) -> float:
    return lib().orc_u01(hi, lo)


def qed_uniforms(seed: int, pid: int, step: int, stream: int):
    a, b = C.c_double(), C.c_double()
    lib().orc_qed_uniforms(seed, pid, step, stream, C.byref(a), C.byref(b))
    return a.value, b.value


def chi(hbar_w_mc2: float, g: float, u, E, B) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    return lib().orc_chi(hbar_w_mc2, g, _dp(u), _dp(E), _dp(B))
