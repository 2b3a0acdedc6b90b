"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host-side mesh and stencil setup (csrc/setup.cpp) is built with
tests/host_setup_check.cpp into a program of its own and run over 1-D, 2-D
(bounded and doubly periodic) and 3-D meshes with every flux, order, refit
and characteristic option; the oracle's C core is built instrumented and run
through its Python harness in a child process with the sanitizer runtime
preloaded.  Any sanitizer report fails the test (reports abort the process:
-fno-sanitize-recover=all)."""

import os
import struct
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from conftest import ROOT
from workloads import jittered_cube, jittered_square, jittered_square_periodic, periodic_line

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
CSRC = os.path.join(ROOT, "paper_1602_02694_amd", "csrc")


def _runtime(name):
    path = subprocess.check_output(["gcc", "-print-file-name=" + name]).decode().strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def _write_mesh(path, mesh, flags):
    v = np.ascontiguousarray(mesh.verts, dtype=np.float64).reshape(-1, mesh.dim)
    c = np.ascontiguousarray(mesh.cells, dtype=np.int32).reshape(-1, mesh.dim + 1)
    with open(path, "wb") as f:
        f.write(struct.pack("<iqqI", mesh.dim, v.shape[0], c.shape[0], flags))
        f.write(v.tobytes())
        f.write(c.tobytes())


def test_host_setup_under_sanitizers(tmp_path):
    _runtime("libasan.so")
    exe = str(tmp_path / "host_setup_check")
    subprocess.check_call(["g++", "-std=c++17", "-ffp-contract=off", "-I" + CSRC] + SAN +
                          [os.path.join(ROOT, "tests", "host_setup_check.cpp"), os.path.join(CSRC, "setup.cpp"),
                           "-o", exe])
    # p,n_lo,n_hi,flux,balance,characteristic,bc
    cases = [
        (periodic_line(40, 0.1, 11), 1, ["2,3,3,0,0,0,0", "3,5,5,0,0,0,0", "5,7,7,1,0,0,0"]),
        (jittered_square(12, 0.3, 12), 0, ["2,6,12,0,0,0,0", "3,12,20,1,0,0,0", "3,12,20,0,1,0,1", "4,20,36,2,0,0,0",
                                           "4,20,36,2,0,1,3", "5,24,30,0,0,0,2", "3,12,20,2,0,0,0",
                                           "9,12,20,0,0,0,0", "3,20,12,0,0,0,0", "3,12,20,0,1,1,0"]),
        (jittered_square_periodic(10, 0.3, 13), 2, ["3,12,20,1,0,0,0", "5,24,30,2,0,1,0"]),
        (jittered_cube(4, 0.15, 14), 0, ["2,8,16,0,0,0,0", "3,30,50,1,1,0,0", "3,30,50,0,0,0,1"]),
    ]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for k, (mesh, flags, prms) in enumerate(cases):
        mf = str(tmp_path / f"mesh{k}.bin")
        _write_mesh(mf, mesh, flags)
        r = subprocess.run([exe, mf] + prms, capture_output=True, text=True, env=env, timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
        assert out.count("stencil rows") + out.count("refused") == len(prms), out


def test_oracle_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared"] + SAN +
                          ["-o", lib, os.path.join(ROOT, "oracle", "wlseno_oracle.c"), "-lm"])
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, "tests")!r})
        import numpy as np
        import oracle, oracle.core as core
        core.build = lambda force=False, extended=False, tangent=False: {lib!r}
        from workloads import jittered_square, jittered_square_periodic, jittered_cube, periodic_line, fields
        m = periodic_line(40, 0.1, 21)
        o = oracle.Oracle(1, m.verts, m.cells, True, p=3, n_lo=5, n_hi=5, flux="burgers")
        u = np.sin(2 * np.pi * np.arange(m.n_cell) / m.n_cell)
        o.rhs(u); o.step(u, 1e-3, 2)
        m = jittered_square(8, 0.3, 22)
        ub = fields.cell_averages(m, fields.gaussian_bump_with_step_2d)
        for kw in (dict(p=3, n_lo=12, n_hi=20, flux="burgers"), dict(p=3, n_lo=12, n_hi=20, flux="advection", balance=True),
                   dict(p=2, n_lo=6, n_hi=12, flux="advection", bc=1)):
            o = oracle.Oracle(2, m.verts, m.cells, **kw)
            o.rhs(ub); o.step(ub, 1e-4, 2); o.reconstruct(ub)
        ue = fields.cell_averages(m, fields.euler_quadrants(23))
        for ch in (False, True):
            o = oracle.Oracle(2, m.verts, m.cells, p=3, n_lo=12, n_hi=20, flux="euler", characteristic=ch)
            o.rhs(ue); o.step(ue, 1e-4, 1)
        m = jittered_square_periodic(8, 0.3, 24)
        o = oracle.Oracle(2, m.verts, m.cells, True, p=3, n_lo=12, n_hi=20, flux="burgers")
        o.rhs(fields.cell_averages(m, fields.gaussian_bump_with_step_2d))
        m = jittered_cube(3, 0.15, 25)
        uc = fields.cell_averages(m, fields.sine_with_sphere_3d)
        o = oracle.Oracle(3, m.verts, m.cells, p=2, n_lo=8, n_hi=16, flux="burgers")
        o.rhs(uc); o.step(uc, 1e-4, 1)
        print("oracle under sanitizers: ok")
    """)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "oracle under sanitizers: ok" in out and "runtime error" not in out, out[-4000:]
