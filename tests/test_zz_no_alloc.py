"""pic_gather_push_deposit_noalloc (the push for callers that cannot
allocate) through the C ABI against pic_gather_push_deposit on the same
inputs: two calls in a row, the second with fewer particles, FP32 tiled and
FP64 plain layouts; and the size limit of its static scratch."""
import numpy as np
import pytest
import torch

from paper_2104_00642_amd import _lib as L
from paper_2104_00642_amd.workloads import courant_dt, to_fp32, to_fp64

from _helpers import DEV, np64, random_fields, random_raw, rel_l2

pytestmark = pytest.mark.gpu


def cfg_of(precision):
    d = (0.3, 0.25)
    return L.Config(dim=2, n=(48, 40), d=d, dt=courant_dt(d, 0.9), order=2, precision=precision, tile=(16, 8),
                    drift=2)


def state(cfg, ctx, n, seed):
    bits, _, ntiles = L.pic_get_layout(ctx)
    raw = random_raw(cfg, n, seed=seed, uth=0.5)
    if cfg.precision == L.PIC_FP32_MIXED:
        p = to_fp32(raw, bits)
        p = L.Particles(n, [t.to(DEV) for t in p.u], cell=p.cell.to(DEV), off=[t.to(DEV) for t in p.off],
                        w=p.w.to(DEV), tile_start=torch.zeros(ntiles + 1, dtype=torch.int64, device=DEV))
        dst = p.empty_like()
        L.pic_sort(ctx, p, dst)
        return dst
    p = to_fp64(raw, cfg)
    return L.Particles(n, [t.to(DEV) for t in p.u], x=[t.to(DEV) for t in p.x], w=p.w.to(DEV))


def clone(p):
    c = lambda t: None if t is None else t.clone()  # noqa: E731
    return L.Particles(p.n, [c(t) for t in p.u], c(p.cell), [c(t) for t in p.off], [c(t) for t in p.x], c(p.w),
                       c(p.chi), c(p.tile_start))


@pytest.mark.parametrize("precision", [L.PIC_FP32_MIXED, L.PIC_FP64_PLAIN])
def test_noalloc_push_equals_the_push(precision):
    cfg = cfg_of(precision)
    ctx = L.pic_init(cfg)
    dtype = torch.float32 if precision == L.PIC_FP32_MIXED else torch.float64
    E, B = random_fields(cfg, seed=5, amp=0.3)
    sp = L.Species(-1.0, 1.0, 1.0)
    for call, n in enumerate((20011, 3001)):
        print(f"noalloc prec={precision} call {call} n={n}", flush=True)
        p0 = state(cfg, ctx, n, seed=31 + call)
        p1 = clone(p0)
        out = []
        for fn, p in ((L.pic_gather_push_deposit, p0), (L.pic_gather_push_deposit_noalloc, p1)):
            f = L.Fields([e.to(DEV, dtype) for e in E], [b.to(DEV, dtype) for b in B],
                         [torch.zeros(cfg.plane_shape, device=DEV, dtype=dtype) for _ in range(3)])
            diag = torch.zeros(4, dtype=torch.float64, device=DEV)
            fn(ctx, sp, p, f, diag)
            torch.cuda.synchronize()
            st, flags, _ = L.pic_check(ctx)
            assert st == L.PIC_OK, flags
            out.append((p, f, diag))
        (pa, fa, da), (pb, fb, db) = out
        # same kernels, same inputs: particles bit for bit; the diagnostics
        # are fixed-order sums; J differs only by the order of the global
        # float atomics of the flush
        cols_a = list(pa.u) + ([pa.cell] + list(pa.off) if precision == L.PIC_FP32_MIXED else list(pa.x))
        cols_b = list(pb.u) + ([pb.cell] + list(pb.off) if precision == L.PIC_FP32_MIXED else list(pb.x))
        for a, b in zip(cols_a, cols_b):
            assert torch.equal(a, b)
        assert torch.equal(da, db)
        for a in range(3):
            err = rel_l2(np64(fb.J[a]), np64(fa.J[a]))
            assert err < (1e-6 if precision == L.PIC_FP32_MIXED else 1e-14), err


def test_noalloc_rejects_a_push_beyond_its_scratch():
    cfg = cfg_of(L.PIC_FP32_MIXED)
    ctx = L.pic_init(cfg)
    bits, _, ntiles = L.pic_get_layout(ctx)
    n = 6_000_000  # 12 B per particle: 72 MB of lists, beyond 64 MiB
    f32 = dict(device=DEV, dtype=torch.float32)
    p = L.Particles(n, [torch.zeros(n, **f32) for _ in range(3)], cell=torch.zeros(n, dtype=torch.int32, device=DEV),
                    off=[torch.full((n,), 0.5, **f32) for _ in range(2)], w=torch.ones(n, **f32),
                    tile_start=torch.zeros(ntiles + 1, dtype=torch.int64, device=DEV))
    f = L.Fields.zeros(cfg, DEV, torch.float32)
    with pytest.raises(L.PicError) as e:
        L.pic_gather_push_deposit_noalloc(ctx, L.Species(-1.0, 1.0, 1.0), p, f)
    assert e.value.status == L.PIC_E_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(p.off[0] == 0.5)  # nothing ran
