"""CPU checks of bench.py's bookkeeping: the algorithmic operation and byte
counts behind its roofline fractions, its parity statistics, and the refusal
of more than one GPU."""

import os
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_update_bytes_2d_p3():
    # 4F sibling ids + 8F d normals + 8 (1/|tau|) + 8FQ own values + 8*4/3 stage inputs + 8 output
    assert bench.update_bytes(1, 2, 3, 2) == pytest.approx(12 + 48 + 8 + 48 + 32 / 3 + 8)
    assert bench.update_bytes(10, 2, 3, 2, V=4) == pytest.approx(10 * (12 + 48 + 8 + 4 * (48 + 32 / 3 + 8)))


def test_recon_flops_by_hand():
    """n = 3 rows, m = 2 coefficients, 1-D, 2 facets of 1 point, counted term
    by term: rows 3(1 + 2), weights 12, W A and W u 9, scaling 18 + 4,
    QR (6*3*2 + 3 + 6) + (6*2*1 + 2 + 6), back substitution 6, evaluation 12."""
    expect = 9 + 12 + 9 + 22 + (36 + 3 + 6) + (12 + 2 + 6) + 6 + 12
    assert bench.recon_flops(3, 2, 1, 2, 1) == pytest.approx(expect)
    # linear in n, so the mean over cells is the count at the mean stencil size
    n = np.array([12, 13, 14, 20])
    assert np.mean(bench.recon_flops(n, 6, 2, 3, 2)) == pytest.approx(bench.recon_flops(n.mean(), 6, 2, 3, 2))


def test_parity_stats():
    o = np.linspace(-1.0, 1.0, 1001)
    s = bench.parity_stats(o * (1 + 1e-13), o)
    assert s["pass"] and s["count_above_tolerance"] == 0 and s["max_rel_err_vs_oracle"] <= 1.01e-13
    g = o.copy()
    g[500] += 1e-10          # o[500] = 0: measured against 1% of the largest |o|
    s = bench.parity_stats(g, o)
    assert not s["pass"] and s["count_above_tolerance"] == 1
    assert s["max_rel_err_vs_oracle"] == pytest.approx(1e-8)
    s = bench.parity_stats(g, o, scale=np.full_like(o, 1.0))
    assert s["max_rel_err_vs_oracle"] == pytest.approx(1e-10)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
