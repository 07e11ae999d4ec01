"""cg_spmv_static (scratch in the library's static device array, no
allocation) against cg_spmv on the same handle: bit-identical products on two
calls in a row, the second with a smaller system, for every format and plan
(CSR slices, symmetric CSR in compact blocks and in coloured line ranges, CSC
panels), each also within 1e-13 of the oracle's product; and the size limit
is refused with an error before any launch."""
import numpy as np
import pytest

from paper_1010_4639_amd import cgmi
from paper_1010_4639_amd import workload as W
from tests.gpu_util import check_spmv, say, to_dev

pytestmark = pytest.mark.gpu


def _arrays(fmt, s):
    if fmt == cgmi.CG_FMT_SYM_CSR:
        return W.upper_triangle(s.rowptr, s.col, s.val)
    return s.rowptr, s.col, s.val


@pytest.mark.parametrize("fmt,plan", [(cgmi.CG_FMT_CSR, "default"), (cgmi.CG_FMT_SYM_CSR, "default"),
                                      (cgmi.CG_FMT_SYM_CSR, "colour"), (cgmi.CG_FMT_CSC, "default")])
def test_static_matches_spmv_two_calls(fmt, plan, monkeypatch):
    if plan == "colour":
        monkeypatch.setenv("CGMI_SYM_PLAN", "colour")
    for dims in ((40, 36, 33), (17, 15, 13)):   # the second call: a smaller system
        s = W.fem_p1_system(*dims, seed=31, with_rhs=False)
        arrs = _arrays(fmt, s)
        x = W.uniform_vector(s.n, seed=32)
        say(f"static product fmt={fmt} plan={plan} n={s.n}")
        with cgmi.Solver(fmt, *arrs) as S:
            st = S.stats()
            assert (st["compact"] == 1) == (fmt == cgmi.CG_FMT_SYM_CSR and plan == "default")
            xd = to_dev(x)
            y_ref = S.spmv(xd).cpu().numpy()
            y_static = S.spmv_static(xd).cpu().numpy()
            y_static2 = S.spmv_static(xd).cpu().numpy()
        assert np.array_equal(y_static, y_ref), float(np.max(np.abs(y_static - y_ref)))
        assert np.array_equal(y_static2, y_ref)
        check_spmv(fmt, *arrs, x, label=f"static n={s.n}")   # the handle's product vs the oracle


def test_static_refuses_oversized_scratch():
    # CSC parks one sum per row: 4.5M rows need 36 MB > the 32 MiB array
    n = 4_500_000
    ptr = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    ptr[-1] = 2 * n - 1
    idx = np.empty(2 * n - 1, np.int32)
    idx[0::2] = np.arange(n)
    idx[1::2] = np.arange(1, n)
    val = np.ones(idx.size)
    with cgmi.Solver(cgmi.CG_FMT_CSC, ptr, idx, val) as S:
        x = to_dev(np.ones(n))
        with pytest.raises(cgmi.CgError) as e:
            S.spmv_static(x)
        assert e.value.status == cgmi.CG_ERR_ARG and "scratch" in str(e.value)
        y = S.spmv(x).cpu().numpy()                  # the handle's own product still works
        assert y[0] == 1.0 and np.all(y[1:] == 2.0)
