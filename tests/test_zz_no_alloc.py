"""sdp_diagnostics_noalloc: the allocation-free diagnostics entry point (scratch
in the library's static device array) against sdp_diagnostics on the same
handle state, through the C ABI.  Two calls in a row, the second on a smaller
handle, so the second reuses scratch the first left behind; and the size
limit is rejected before anything is launched."""
import numpy as np
import pytest

import sdpgen

pytestmark = pytest.mark.gpu

KEYS = ("eps_p", "eps_d", "eps_g", "eps_alpha", "objective", "iters", "status")


def log(msg):
    print(msg, flush=True)


def check_same(a, b):
    for k in KEYS:
        x, y = a[k], b[k]
        assert np.isfinite(x) and np.isfinite(y), k
        # same kernels, same arithmetic: only the scratch address differs
        assert x == y or abs(x - y) <= 1e-14 * max(abs(x), abs(y)), (k, x, y)


def run_pair(sdp, insts, n_iter, precision):
    with sdp.Solver(insts, tol=1e-4, precision=precision) as S:
        S.step(n_iter)
        na = S.diagnostics(noalloc=True)
        ref = S.diagnostics()
        na2 = S.diagnostics(noalloc=True)
    for a, b, c in zip(na, ref, na2):
        check_same(a, b)
        check_same(c, b)
        assert b["eps_alpha"] >= 0.0 and b["eps_d"] > 0.0
    return ref


def test_noalloc_diagnostics_two_calls_second_smaller(sdp, gpu):
    big = [sdpgen.banded_instance(600, 9, 120, seed=1), sdpgen.block_arrow_instance(5, 8, 3, 30, seed=2)]
    log("no-alloc diagnostics: banded n=600 w=9 m=120 + block-arrow (5,8,3) m=30, fp64, 25 iterations")
    run_pair(sdp, big, 25, "fp64")
    small = [sdpgen.block_arrow_instance(3, 4, 2, 9, seed=3)]
    log("no-alloc diagnostics: block-arrow (3,4,2) m=9, fp32, 7 iterations")
    run_pair(sdp, small, 7, "fp32")


def test_noalloc_diagnostics_sparse_a(sdp, gpu):
    inst = sdpgen.block_arrow_instance(6, 10, 4, 40, seed=5, density=0.05)
    log("no-alloc diagnostics: sparse block-arrow (6,10,4) m=40, fp64, 12 iterations")
    run_pair(sdp, [inst], 12, "fp64")


def test_noalloc_diagnostics_rejects_handles_beyond_the_limit(sdp, gpu):
    # 3 * 2^18-odd coordinate slots exceed the 2^21-double scratch
    inst = sdpgen.banded_instance(50000, 15, 4, seed=0)
    log("no-alloc diagnostics: banded n=50000 w=15 m=4 (beyond the scratch limit)")
    with sdp.Solver([inst], tol=1e-4, precision="fp64") as S:
        S.step(2)
        with pytest.raises(sdp.SdpError) as e:
            S.diagnostics(noalloc=True)
        assert e.value.code == sdp._native.ERR_UNSUPPORTED
        ok = S.diagnostics()[0]
        assert np.isfinite(ok["eps_d"])
