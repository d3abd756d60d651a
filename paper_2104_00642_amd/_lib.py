"""ctypes binding of libpic (include/pic.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and takes
torch tensors (device memory) for the arrays; it converts them to raw
pointers, passes the current HIP stream, and raises ``PicError`` on a
non-OK status.  All computation happens in the HIP kernels of the library.
Loading fails loudly when ``libpic.so`` is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_E_ARG, PIC_E_CFL, PIC_E_UNSUPPORTED, PIC_E_NOMEM, PIC_E_HIP, PIC_E_CAPACITY, PIC_E_STATE = range(8)
STATUS_NAMES = ["PIC_OK", "PIC_E_ARG", "PIC_E_CFL", "PIC_E_UNSUPPORTED", "PIC_E_NOMEM", "PIC_E_HIP",
                "PIC_E_CAPACITY", "PIC_E_STATE"]
PIC_FP32_MIXED, PIC_FP64_PLAIN = 0, 1
PIC_BC_PERIODIC = 0
PIC_F_NONFINITE, PIC_F_OFFSET, PIC_F_STRAGGLER, PIC_F_CAPACITY, PIC_F_QED_SATURATED = 1, 2, 4, 8, 16

PIC_QED_TABLE, PIC_QED_MLP, PIC_QED_METHOD2 = 0, 1, 2
PIC_PUSH_BORIS, PIC_PUSH_VAY = 0, 1
PIC_BC_ABSORB = 1
PIC_BC_ABSORB2 = 2
PIC_MAX_SPECIES = 4
PIC_MLP_NPARAM = 4610
PIC_MLP_BYTES = 18440
PIC_MLP_STATE_FLOATS = 4 * PIC_MLP_NPARAM + 1

EXPORTED = ["pic_init", "pic_destroy", "pic_last_error", "pic_get_layout", "pic_gather_push_deposit",
            "pic_yee_step", "pic_sort", "pic_check", "pic_qed_step", "pic_mlp_forward", "pic_mlp_grad",
            "pic_mlp_train", "pic_qed_training_data", "pic_qed_table_lookup", "pic_set_laser", "pic_reserve",
            "pic_deposit_rho", "pic_gauss_residual", "pic_beam_fields", "pic_gather_push_deposit_noalloc",
            "pic_gather_push_deposit_multi"]


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


class pic_config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("order", C.c_int32), ("precision", C.c_int32),
                ("drift", C.c_int32), ("n", C.c_int64 * 3), ("d", C.c_double * 3),
                ("dt", C.c_double), ("bc", C.c_int32 * 3), ("tile", C.c_int32 * 3),
                ("seed", C.c_uint64), ("hbar_omega_mc2", C.c_double), ("pusher", C.c_int32)]


class pic_laser(C.Structure):
    _fields_ = [("a0", C.c_double), ("waist", C.c_double), ("duration", C.c_double), ("t0", C.c_double),
                ("circular", C.c_int32)]


class pic_beam(C.Structure):
    _fields_ = [("charge", C.c_double), ("density", C.c_double), ("center", C.c_double * 3),
                ("sigma", C.c_double * 3), ("gamma", C.c_double)]


class pic_species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w0", C.c_double)]


class pic_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("cell", C.c_void_p), ("off", C.c_void_p * 3),
                ("x", C.c_void_p * 3), ("u", C.c_void_p * 3), ("w", C.c_void_p),
                ("chi", C.c_void_p), ("tile_start", C.c_void_p),
                ("tau", C.c_void_p), ("tau_thr", C.c_void_p), ("id", C.c_void_p),
                ("capacity", C.c_int64), ("n_dev", C.c_void_p)]


class pic_fields(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3)]


class pic_qed_args(C.Structure):
    _fields_ = [("electrons", C.POINTER(pic_particles)), ("positrons", C.POINTER(pic_particles)),
                ("photons", C.POINTER(pic_particles)), ("fields", C.POINTER(pic_fields)),
                ("mode", C.c_int32), ("step", C.c_uint32), ("photon_min_energy", C.c_double),
                ("mlp", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_00642_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.pic_init.argtypes = [C.POINTER(pic_config), C.POINTER(C.c_void_p)]
        L.pic_init.restype = C.c_int
        L.pic_destroy.argtypes = [C.c_void_p]
        L.pic_destroy.restype = None
        L.pic_last_error.argtypes = [C.c_void_p]
        L.pic_last_error.restype = C.c_char_p
        L.pic_get_layout.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64)]
        L.pic_get_layout.restype = C.c_int
        L.pic_gather_push_deposit.argtypes = [C.c_void_p, C.POINTER(pic_species), C.POINTER(pic_particles),
                                              C.POINTER(pic_fields), C.c_void_p, C.c_void_p]
        L.pic_gather_push_deposit.restype = C.c_int
        L.pic_yee_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(pic_fields), C.c_void_p, C.c_void_p]
        L.pic_set_laser.argtypes = [C.c_void_p, C.POINTER(pic_laser), C.c_double]
        L.pic_set_laser.restype = C.c_int
        L.pic_yee_step.restype = C.c_int
        L.pic_sort.argtypes = [C.c_void_p, C.POINTER(pic_particles), C.POINTER(pic_particles), C.c_void_p]
        L.pic_sort.restype = C.c_int
        L.pic_check.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]
        L.pic_check.restype = C.c_int
        L.pic_qed_step.argtypes = [C.c_void_p, C.POINTER(pic_qed_args), C.c_void_p]
        L.pic_qed_step.restype = C.c_int
        L.pic_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.pic_mlp_forward.restype = C.c_int
        L.pic_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p]
        L.pic_mlp_grad.restype = C.c_int
        L.pic_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_int32, C.c_int32, C.c_float, C.c_void_p, C.c_void_p]
        L.pic_mlp_train.restype = C.c_int
        L.pic_qed_training_data.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p, C.c_void_p,
                                            C.c_void_p]
        L.pic_qed_training_data.restype = C.c_int
        L.pic_qed_table_lookup.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_int64, C.c_void_p, C.c_void_p]
        L.pic_qed_table_lookup.restype = C.c_int
        L.pic_gather_push_deposit_noalloc.argtypes = [C.c_void_p, C.POINTER(pic_species),
                                                      C.POINTER(pic_particles), C.POINTER(pic_fields), C.c_void_p,
                                                      C.c_void_p]
        L.pic_gather_push_deposit_noalloc.restype = C.c_int
        L.pic_gather_push_deposit_multi.argtypes = [C.c_void_p, C.c_int32, C.POINTER(pic_species),
                                                    C.POINTER(C.POINTER(pic_particles)), C.POINTER(pic_fields),
                                                    C.c_void_p, C.c_void_p]
        L.pic_gather_push_deposit_multi.restype = C.c_int
        L.pic_reserve.argtypes = [C.c_void_p, C.c_int64]
        L.pic_reserve.restype = C.c_int
        L.pic_deposit_rho.argtypes = [C.c_void_p, C.POINTER(pic_species), C.POINTER(pic_particles), C.c_int32,
                                      C.c_void_p, C.c_void_p]
        L.pic_deposit_rho.restype = C.c_int
        L.pic_gauss_residual.argtypes = [C.c_void_p, C.POINTER(pic_fields), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        L.pic_gauss_residual.restype = C.c_int
        L.pic_beam_fields.argtypes = [C.c_void_p, C.POINTER(pic_beam), C.POINTER(pic_fields), C.c_void_p]
        L.pic_beam_fields.restype = C.c_int
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_contiguous(), "arrays must be contiguous"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return None
    return C.c_void_p(int(stream))


# ----------------------------------------------------------------- containers

@dataclass
class Config:
    """Mirror of pic_config (units of Eq. 8 of the paper)."""
    dim: int
    n: tuple
    d: tuple
    dt: float
    order: int = 2
    precision: int = PIC_FP32_MIXED
    drift: int = 2
    tile: tuple = (0, 0, 0)
    seed: int = 0
    hbar_omega_mc2: float = 0.0
    pusher: int = PIC_PUSH_BORIS
    bc_x: int = PIC_BC_PERIODIC  # or PIC_BC_ABSORB / PIC_BC_ABSORB2 (first- / second-order field rule)

    def c(self) -> pic_config:
        cfg = pic_config()
        cfg.dim, cfg.order, cfg.precision, cfg.drift = self.dim, self.order, self.precision, self.drift
        n = list(self.n) + [1] * (3 - len(self.n))
        d = list(self.d) + [1.0] * (3 - len(self.d))
        t = list(self.tile) + [0] * (3 - len(self.tile))
        for a in range(3):
            cfg.n[a], cfg.d[a], cfg.tile[a] = int(n[a]), float(d[a]), int(t[a])
            cfg.bc[a] = int(self.bc_x) if a == 0 else PIC_BC_PERIODIC
        cfg.dt = float(self.dt)
        cfg.seed = int(self.seed)
        cfg.hbar_omega_mc2 = float(self.hbar_omega_mc2)
        cfg.pusher = int(self.pusher)
        return cfg

    @property
    def ncell(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return n[0] * n[1] * n[2]

    @property
    def plane_shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0])


@dataclass
class Species:
    q: float
    m: float
    w0: float = 1.0

    def c(self) -> pic_species:
        return pic_species(self.q, self.m, self.w0)


@dataclass
class Particles:
    """Structure of arrays of one species (torch tensors on the device).
    FP32 path: cell (int32 packed), off[dim] (float32), u[3] (float32), w, chi,
    tile_start (int64, ntiles+1).  FP64 path: x[dim] (float64), u[3], w, chi."""
    n: int
    u: list
    cell: Optional[torch.Tensor] = None
    off: list = field(default_factory=list)
    x: list = field(default_factory=list)
    w: Optional[torch.Tensor] = None
    chi: Optional[torch.Tensor] = None
    tile_start: Optional[torch.Tensor] = None
    tau: Optional[torch.Tensor] = None       # float64
    tau_thr: Optional[torch.Tensor] = None   # float32
    id: Optional[torch.Tensor] = None        # int64 (bits of the uint64 identifiers)
    capacity: int = 0
    n_dev: Optional[torch.Tensor] = None     # int64[1]

    def c(self) -> pic_particles:
        p = pic_particles()
        p.n = int(self.n)
        p.cell = _ptr(self.cell)
        for a, t in enumerate(self.off):
            p.off[a] = _ptr(t)
        for a, t in enumerate(self.x):
            p.x[a] = _ptr(t)
        for a, t in enumerate(self.u):
            p.u[a] = _ptr(t)
        p.w = _ptr(self.w)
        p.chi = _ptr(self.chi)
        p.tile_start = _ptr(self.tile_start)
        p.tau = _ptr(self.tau)
        p.tau_thr = _ptr(self.tau_thr)
        p.id = _ptr(self.id)
        p.capacity = int(self.capacity if self.capacity else self.n)
        p.n_dev = _ptr(self.n_dev)
        return p

    def empty_like(self) -> "Particles":
        e = lambda t: None if t is None else torch.empty_like(t)  # noqa: E731
        return Particles(self.n, [e(t) for t in self.u], e(self.cell), [e(t) for t in self.off],
                         [e(t) for t in self.x], e(self.w), e(self.chi), e(self.tile_start),
                         e(self.tau), e(self.tau_thr), e(self.id), self.capacity, e(self.n_dev))


@dataclass
class Fields:
    E: list
    B: list
    J: list

    def c(self) -> pic_fields:
        f = pic_fields()
        for a in range(3):
            f.E[a], f.B[a], f.J[a] = _ptr(self.E[a]), _ptr(self.B[a]), _ptr(self.J[a])
        return f

    @staticmethod
    def zeros(cfg: Config, device, dtype):
        z = lambda: [torch.zeros(cfg.plane_shape, device=device, dtype=dtype) for _ in range(3)]  # noqa: E731
        return Fields(z(), z(), z())


# -------------------------------------------------------------- entry points

class Context:
    def __init__(self, handle: int, cfg: Config):
        self.handle = handle
        self.cfg = cfg

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().pic_destroy(C.c_void_p(self.handle))
            except Exception:
                pass
            self.handle = None


def _check(status: int, ctx_handle):
    if status != PIC_OK:
        msg = lib().pic_last_error(ctx_handle)
        raise PicError(status, msg.decode() if msg else "")


def pic_init(cfg: Config) -> Context:
    h = C.c_void_p()
    c = cfg.c()
    st = lib().pic_init(C.byref(c), C.byref(h))
    _check(st, None)
    return Context(h.value, cfg)


def pic_destroy(ctx: Context):
    if ctx.handle:
        lib().pic_destroy(C.c_void_p(ctx.handle))
        ctx.handle = None


def pic_last_error(ctx: Optional[Context]) -> str:
    r = lib().pic_last_error(C.c_void_p(ctx.handle) if ctx else None)
    return r.decode() if r else ""


def pic_get_layout(ctx: Context):
    bits = (C.c_int32 * 3)()
    tile = (C.c_int32 * 3)()
    nt = C.c_int64()
    _check(lib().pic_get_layout(C.c_void_p(ctx.handle), bits, tile, C.byref(nt)), C.c_void_p(ctx.handle))
    return list(bits), list(tile), nt.value


def pic_gather_push_deposit(ctx: Context, sp: Species, p: Particles, f: Fields,
                            diag: Optional[torch.Tensor] = None, stream=None):
    sc, pc, fc = sp.c(), p.c(), f.c()
    st = lib().pic_gather_push_deposit(C.c_void_p(ctx.handle), C.byref(sc), C.byref(pc), C.byref(fc),
                                       _ptr(diag), _stream(stream))
    _check(st, C.c_void_p(ctx.handle))


def pic_gather_push_deposit_multi(ctx: Context, species: List[Species], parts: List[Particles], f: Fields,
                                  diag: Optional[torch.Tensor] = None, stream=None):
    """Several species in one call: species[k] with parts[k]."""
    if len(species) != len(parts):
        raise ValueError("one Particles per Species")
    sa = (pic_species * max(1, len(species)))(*[sp.c() for sp in species])
    pcs = [p.c() for p in parts]
    pa = (C.POINTER(pic_particles) * max(1, len(pcs)))(*[C.pointer(pc) for pc in pcs])
    fc = f.c()
    st = lib().pic_gather_push_deposit_multi(C.c_void_p(ctx.handle), len(species), sa, pa, C.byref(fc),
                                             _ptr(diag), _stream(stream))
    _check(st, C.c_void_p(ctx.handle))


def pic_gather_push_deposit_noalloc(ctx: Context, sp: Species, p: Particles, f: Fields,
                                    diag: Optional[torch.Tensor] = None, stream=None):
    sc, pc, fc = sp.c(), p.c(), f.c()
    st = lib().pic_gather_push_deposit_noalloc(C.c_void_p(ctx.handle), C.byref(sc), C.byref(pc), C.byref(fc),
                                               _ptr(diag), _stream(stream))
    _check(st, C.c_void_p(ctx.handle))


def pic_yee_step(ctx: Context, half: int, f: Fields, diag: Optional[torch.Tensor] = None, stream=None):
    fc = f.c()
    st = lib().pic_yee_step(C.c_void_p(ctx.handle), int(half), C.byref(fc), _ptr(diag), _stream(stream))
    _check(st, C.c_void_p(ctx.handle))


def pic_set_laser(ctx: Context, a0: float, waist: float, duration: float, t0: float, circular: bool = False,
                  t: float = 0.0):
    las = pic_laser(float(a0), float(waist), float(duration), float(t0), int(bool(circular)))
    _check(lib().pic_set_laser(C.c_void_p(ctx.handle), C.byref(las), float(t)), C.c_void_p(ctx.handle))


def pic_sort(ctx: Context, src: Particles, dst: Particles, stream=None):
    s, d = src.c(), dst.c()
    st = lib().pic_sort(C.c_void_p(ctx.handle), C.byref(s), C.byref(d), _stream(stream))
    _check(st, C.c_void_p(ctx.handle))


def pic_check(ctx: Context, stream=None):
    """Returns (status, flags, stragglers) without raising on data conditions."""
    fl = C.c_uint32()
    ns = C.c_uint64()
    st = lib().pic_check(C.c_void_p(ctx.handle), _stream(stream), C.byref(fl), C.byref(ns))
    if st not in (PIC_OK, PIC_E_STATE, PIC_E_CAPACITY):
        _check(st, C.c_void_p(ctx.handle))
    return st, fl.value, ns.value


def pic_qed_step(ctx: Context, fields: Fields, electrons: Optional[Particles] = None,
                 positrons: Optional[Particles] = None, photons: Optional[Particles] = None,
                 mode: int = PIC_QED_TABLE, step: int = 0, photon_min_energy: float = 2.0,
                 mlp: Optional[torch.Tensor] = None, stream=None):
    keep = []

    def ref(p):
        if p is None:
            return None
        c = p.c()
        keep.append(c)
        return C.pointer(c)
    fc = fields.c()
    a = pic_qed_args(ref(electrons), ref(positrons), ref(photons), C.pointer(fc), int(mode), int(step) & 0xFFFFFFFF,
                     float(photon_min_energy), _ptr(mlp))
    _check(lib().pic_qed_step(C.c_void_p(ctx.handle), C.byref(a), _stream(stream)), C.c_void_p(ctx.handle))


def pic_mlp_forward(ctx: Context, mlp: torch.Tensor, x: torch.Tensor, y: torch.Tensor, stream=None):
    _check(lib().pic_mlp_forward(C.c_void_p(ctx.handle), _ptr(mlp), _ptr(x), x.shape[0], _ptr(y),
                                 _stream(stream)), C.c_void_p(ctx.handle))


def pic_mlp_grad(ctx: Context, mlp, x, t, grad, loss=None, stream=None):
    _check(lib().pic_mlp_grad(C.c_void_p(ctx.handle), _ptr(mlp), _ptr(x), _ptr(t), x.shape[0], _ptr(grad),
                              _ptr(loss), _stream(stream)), C.c_void_p(ctx.handle))


def pic_mlp_train(ctx: Context, state, mlp, x, t, batch: int, iters: int, lr: float, loss=None, stream=None):
    _check(lib().pic_mlp_train(C.c_void_p(ctx.handle), _ptr(state), _ptr(mlp), _ptr(x), _ptr(t), x.shape[0],
                               int(batch), int(iters), float(lr), _ptr(loss), _stream(stream)),
           C.c_void_p(ctx.handle))


def pic_qed_training_data(ctx: Context, n: int, seed: int, x, t, stream=None):
    _check(lib().pic_qed_training_data(C.c_void_p(ctx.handle), int(n), int(seed), _ptr(x), _ptr(t),
                                       _stream(stream)), C.c_void_p(ctx.handle))


def pic_qed_table_lookup(ctx: Context, proc: int, what: int, chi, r, out, stream=None):
    _check(lib().pic_qed_table_lookup(C.c_void_p(ctx.handle), int(proc), int(what), _ptr(chi), _ptr(r),
                                      chi.shape[0], _ptr(out), _stream(stream)), C.c_void_p(ctx.handle))


def pic_reserve(ctx: Context, particles: int):
    _check(lib().pic_reserve(C.c_void_p(ctx.handle), int(particles)), C.c_void_p(ctx.handle))


def pic_deposit_rho(ctx: Context, sp: Species, p: Particles, rho: torch.Tensor, at_half: bool = True,
                    stream=None):
    assert rho.dtype == torch.float64
    sc, pc = sp.c(), p.c()
    _check(lib().pic_deposit_rho(C.c_void_p(ctx.handle), C.byref(sc), C.byref(pc), int(bool(at_half)), _ptr(rho),
                                 _stream(stream)), C.c_void_p(ctx.handle))


def pic_gauss_residual(ctx: Context, f: Fields, rho: torch.Tensor, residual: Optional[torch.Tensor] = None,
                       diag: Optional[torch.Tensor] = None, stream=None):
    assert rho.dtype == torch.float64 and (residual is None or residual.dtype == torch.float64)
    fc = f.c()
    _check(lib().pic_gauss_residual(C.c_void_p(ctx.handle), C.byref(fc), _ptr(rho), _ptr(residual), _ptr(diag),
                                    _stream(stream)), C.c_void_p(ctx.handle))


@dataclass
class Beam:
    """A bi-Gaussian bunch moving along +x: particle charge, peak lab
    density, centre, lab rms sizes and Lorentz factor (pic_beam)."""
    charge: float
    density: float
    center: tuple
    sigma: tuple
    gamma: float

    def c(self) -> pic_beam:
        b = pic_beam()
        b.charge = float(self.charge)
        b.density = float(self.density)
        for a in range(3):
            b.center[a] = float(self.center[a]) if a < len(self.center) else 0.0
            b.sigma[a] = float(self.sigma[a]) if a < len(self.sigma) else 1.0
        b.gamma = float(self.gamma)
        return b


def pic_beam_fields(ctx: Context, beam: Beam, f: Fields, stream=None):
    bc = beam.c()
    fc = f.c()
    _check(lib().pic_beam_fields(C.c_void_p(ctx.handle), C.byref(bc), C.byref(fc), _stream(stream)),
           C.c_void_p(ctx.handle))
