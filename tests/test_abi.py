"""The C interface loads and exports every function include/ddamg.h declares;
host-side argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ddamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ddamg_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    from paper_1611_01034_amd import ddamg
    lib = ctypes.CDLL(ddamg.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(ddamg.exported_symbols()) == names


def test_default_params_follow_listing_1_names():
    from paper_1611_01034_amd import ddamg
    p = ddamg.default_params()
    gold = dict(l.split() for l in open(os.path.join(ROOT, "tests", "golden", "listing1_params.txt"))
                if l.strip() and not l.startswith("#"))
    # block sizes of the first aggregation and the coarser ones of Sec. 2 (4^4, then 2^4)
    assert [p.block[0][d] for d in range(4)] == [int(gold["MGBlockT"]), int(gold["MGBlockZ"]),
                                                 int(gold["MGBlockY"]), int(gold["MGBlockX"])]
    assert [p.block[1][d] for d in range(4)] == [2, 2, 2, 2]
    assert p.nvec[0] == int(gold["MGNumberOfVectors"])
    q = ddamg.default_params(levels=int(gold["MGNumberOfLevels"]), setup_iters=int(gold["MGSetupIter"]),
                             coarse_setup_iters=int(gold["MGCoarseSetupIter"]),
                             coarse_mu_factor=float(gold["MGCoarseMuFactor"]))
    assert (q.levels, q.setup_iters, q.coarse_setup_iters, q.coarse_mu_factor) == (3, 5, 3, 5.0)
    # the setup frees its test vectors unless asked to keep them for an update
    assert p.keep_test_vectors == 0
    # the tail of the struct, as the library fills it (a layout mismatch shifts these)
    assert (p.precision, p.batch, p.rhs_batch) == (ddamg.FP64, 16, 1)


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 6), (2, 2, 2, 2)),   # odd number of blocks in X
                                        ((4, 4, 4, 4), (2, 2, 2, 3)),   # odd block extent
                                        ((4, 4, 4, 4), (4, 4, 4, 4)),   # one block per direction
                                        ((8, 8, 8, 8), (8, 8, 2, 2))])  # block larger than 256 sites
def test_create_rejects_bad_shapes_before_any_device_call(dims, block):
    from paper_1611_01034_amd import ddamg
    with pytest.raises(ddamg.DDAMGError) as e:
        ddamg.DDAMG(dims, block, 0.13729, 1.57551, 0.0009)
    assert e.value.status == ddamg.INVALID_ARG


def test_null_context_calls_fail_cleanly():
    from paper_1611_01034_amd import ddamg
    lib = ddamg._lib
    assert lib.ddamg_set_gauge(None, None, 0) == ddamg.INVALID_ARG
    assert lib.ddamg_solve(None, None, None, 1, 1e-10, None, 0) == ddamg.INVALID_ARG
    assert lib.ddamg_update_gauge(None, None, 0, None) == ddamg.INVALID_ARG
    assert lib.ddamg_set_boundary_phases(None, None) == ddamg.INVALID_ARG
    assert lib.ddamg_solve_odd_shifted(None, None, None, 0.0, 1e-10, None, 0) == ddamg.INVALID_ARG
    assert lib.ddamg_last_error(None) == b"null context"
