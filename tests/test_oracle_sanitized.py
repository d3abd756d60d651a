"""The oracle's C sources built with AddressSanitizer and
UndefinedBehaviorSanitizer, exercised in a child process on the CPU: every
entry point the tests use, on small 2D and 3D grids (every shape order,
both pushers, absorbing faces of both orders with injection, the sort, rho
and div, the QED
integrals and Philox).  Any out-of-bounds access, leak-free use after free
or undefined behaviour aborts the child."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle as O
from oracle import qed_step as Q
rng = np.random.default_rng(3)
for dim, n, d in ((2, (16, 12), (0.3, 0.25)), (3, (8, 6, 6), (0.3, 0.25, 0.2))):
    for order in (1, 2, 4):
        for pusher in (0, 1):
            for absorb in (0, 1, 2):
                g = O.Grid(dim, n, d, 0.1, order, pusher=pusher, absorb_x=absorb,
                           laser=(1.0, 1.0, 3.0, 0.0) if absorb else (0.0, 0.0, 0.0, 0.0))
                st = O.State.zeros(g)
                for c in st.E + st.B:
                    c[...] = rng.normal(0, 0.2, c.shape)
                m = 300
                x = [rng.uniform(0, n[a] * d[a], m) for a in range(dim)]
                u = [rng.normal(0, 0.8, m) for _ in range(3)]
                st.species.append(O.Species(-1.0, 1.0, x, u, rng.uniform(0.5, 1.5, m)))
                diag = np.zeros(2)
                for _ in range(3):
                    O.step(st, diag)
                O.rho(g, -1.0, st.species[0].x, st.species[0].w)
                O.div(g, st.E)
                O.curl_e(g, st.E)
                O.field_energy(g, st.E, st.B)
                cells = [np.floor(xx / d[a]).astype(np.int32) for a, xx in enumerate(st.species[0].x)]
                cells[0][:5] = -1
                O.sort(g, [4] * dim, cells)
for chi in (1e-3, 0.49, 4.9, 49.0):
    O.frad(chi); O.fpair(chi); O.compton_inverse(chi, 0.3); O.pair_inverse(chi, 0.7)
    O.compton_cum(chi, 0.2); O.pair_cum(chi, 0.4)
O.philox4x32_10([1, 2, 3, 4], [5, 6])
O.qed_uniforms(7, 9, 11, 0)
print("sanitized oracle ok")
'''


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if out and os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed for the sanitized build")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    ubsan = _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc has no sanitizer runtimes here")
    # a copy of the oracle package whose library is the sanitized build
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp"))
    lib = pkg / "liboracle.so"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
           str(pkg / "pic_oracle.c"), str(pkg / "qed_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = f"{asan}:{ubsan}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = str(tmp_path)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
