"""Host logic of bench.py: the oracle leg and the site check reproduce the
oracle's full-lattice apply, and the multi-GPU request is refused."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import dirac  # noqa: E402
from paper_1611_01034_amd import synth  # noqa: E402

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def small():
    dims = (8, 4, 4, 6)
    U = synth.gauge_field(dims, 0.3, 5001)
    b0 = synth.spinor(dims, 5101)
    x0 = synth.spinor(dims, 5102)
    op = dirac.WilsonClover(U, bench.KAPPA, bench.CSW, bench.MU)
    return dims, U, b0, x0, op.apply(b0), op.apply(x0)


def test_oracle_leg_slices_equal_full_apply(small):
    dims, U, b0, _, yb, _ = small
    leg = bench.OracleLeg(torch.from_numpy(U), torch.from_numpy(b0), 2)
    assert leg.ts == [0, 1, 5]
    cpu, check = leg.result({t: yb[t] for t in range(dims[0])})
    assert check["dirac_slices_max_abs_diff_over_max"] == 0.0
    assert check["dirac_sites_checked"] == 3 * 4 * 4 * 6
    assert cpu["cores"] == 2 and cpu["value"] > 0 and cpu["kind"] == "oracle"
    # a planted difference in the library's values is seen
    bad = {t: yb[t].copy() for t in range(dims[0])}
    bad[5][1, 2, 3] += 1e-3
    leg = bench.OracleLeg(torch.from_numpy(U), torch.from_numpy(b0), 2)
    _, check = leg.result(bad)
    assert check["dirac_slices_max_abs_diff_over_max"] > 1e-6


def test_oracle_sites(small):
    _, U, b0, x0, _, yx = small
    Ut, xt, yt = torch.from_numpy(U), torch.from_numpy(x0), torch.from_numpy(yx)
    # b = D x: zero residual at every site, library and oracle agree exactly
    r = bench.oracle_sites(Ut, xt, yt, yt, 16)
    assert r["oracle_residual_at_sites"] == 0.0 and r["dirac_x0_max_rel_diff_at_sites"] == 0.0
    # an unrelated b: residual of order one
    r = bench.oracle_sites(Ut, xt, torch.from_numpy(b0), yt, 16)
    assert r["oracle_residual_at_sites"] > 0.1


def test_multi_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
