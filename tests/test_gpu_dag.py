"""The dataflow (algorithm-by-blocks) factorization, LUPP_OPT_LOOKAHEAD >= 2,
through the C ABI.

Each task computes what the same step of the blocked loop computes, in the
same order per entry, so factors, pivots and info must equal those of the
in-order single-stream factorization (lookahead 0) bit for bit, for every
depth, shape, block size and update format; on top of that the oracle bars
(separated-prefix pivots, scaled residual < 10) and the Pi*D closed form at a
size the oracle cannot run."""
import numpy as np
import pytest

import synth
from oracle import checks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - GPU machine only
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_05782_amd as lupp  # noqa: E402
from gpu_util import announce, to_dev, to_host  # noqa: E402


def _factor(A0, depth, nb=None, prec=None, timing=0):
    h = lupp.Handle()
    h.set_option(4, depth)
    if nb:
        h.set_option(1, nb)
    if prec is not None:
        h.set_option(5, prec)
    if timing:
        h.set_option(3, 1)
    A = torch.empty_like(A0.t()).t()
    A.copy_(A0)
    m, n = A0.shape
    ipiv = torch.empty(max(1, min(m, n)), dtype=torch.int32, device="cuda")
    info = torch.full((1,), -5, dtype=torch.int32, device="cuda")
    (lupp.lupp_dgetrf if A0.dtype == torch.float64 else lupp.lupp_sgetrf)(A, ipiv, info, handle=h)
    h.sync()
    panels = h.timing_summary("panel")[0] if timing else None
    h.close()
    return A, ipiv[:min(m, n)], int(info.item()), panels


def _rand(m, n, dtype, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    A0 = torch.empty((n, m), dtype=dtype, device="cuda").t()
    return A0.uniform_(-1.0, 1.0, generator=g)


@pytest.mark.parametrize("shape,nb,dtype", [
    ((4133, 4133), 512, torch.float64),
    ((4133, 4133), 256, torch.float32),
    ((8192, 8192), 512, torch.float64),
    ((6000, 2500), 256, torch.float64),   # tall
    ((2500, 6000), 512, torch.float64),   # wide: the last blocks have no rows below
    ((40000, 1536), 512, torch.float64),  # column blocks on the 64-CU stream pair
])
def test_dataflow_bit_identical(shape, nb, dtype):
    m, n = shape
    A0 = _rand(m, n, dtype, 50 + m % 97)
    ref = _factor(A0, 0, nb)
    for depth in (2, 3, 5):
        announce("dataflow %dx%d nb=%d %s depth %d" % (m, n, nb, dtype, depth))
        A, p, info, _ = _factor(A0, depth, nb)
        assert info == ref[2] == 0
        assert torch.equal(p, ref[1]), depth
        assert torch.equal(A, ref[0]), depth


def test_dataflow_low_precision_update_bit_identical():
    """sgetrf with BF16 trailing updates: the same bits with and without the
    dataflow runtime (each update task scales its own operand blocks exactly
    as the corresponding launch of the loop does)."""
    n = 6144
    announce("dataflow bf16 updates n=%d" % n)
    A0 = _rand(n, n, torch.float32, 61)
    ref = _factor(A0, 0, 512, lupp.PREC["bf16"])
    A, p, info, _ = _factor(A0, 3, 512, lupp.PREC["bf16"])
    assert info == ref[2] == 0
    assert torch.equal(p, ref[1]) and torch.equal(A, ref[0])


def test_dataflow_matches_oracle():
    n = 1536
    announce("dataflow vs oracle n=%d" % n)
    import oracle
    A = synth.uniform(20210901, 0, n, n)
    h = lupp.Handle()
    h.set_option(4, 4)
    h.set_option(1, 256)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    LU, ip = to_host(dA), ipiv.cpu().numpy()
    h.close()
    _, po, info_o, gap = oracle.getrf(A, with_gap=True, nthreads=8)
    assert int(info.item()) == info_o == 0
    ok, cmp, first = checks.pivot_prefix_match(ip, po, gap, 1e-9)
    assert ok and cmp == n, (first, cmp)
    L, U = checks.unpack(LU)
    assert np.abs(L).max() <= 1.0
    assert checks.scaled_residual(A, LU, ip) < 10


def test_dataflow_pi_d_closed_form():
    n = 8192
    announce("dataflow Pi*D n=%d" % n)
    A, perm = synth.pi_times_coldom(23, 4, n)
    h = lupp.Handle()
    h.set_option(4, 3)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    h.close()
    assert int(info.item()) == 0
    assert np.array_equal(ipiv.cpu().numpy(), checks.closed_form_ipiv(perm))


def test_dataflow_zero_column_info():
    n = 2048
    A = synth.uniform(77, 0, n, n)
    A[:, 700] = 0.0
    dA0 = to_dev(A)
    ref = _factor(dA0, 0, 256)
    out = _factor(dA0, 2, 256)
    assert ref[2] == out[2] == 701
    assert torch.equal(ref[0], out[0]) and torch.equal(ref[1], out[1])


def test_dataflow_mixed_solve():
    """The mixed-precision solve on a handle in dataflow mode converges."""
    n = 4096
    announce("dataflow mixed solve n=%d" % n)
    A = synth.uniform(20210902, 0, n, n) * 0.5
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1)
    b = synth.uniform(20210902, 1, n, 1)[:, 0]
    h = lupp.Handle()
    h.set_option(4, 3)
    x, rep = lupp.gesv_mixed(to_dev(A), torch.from_numpy(b).cuda(), handle=h, solver="classical",
                             factor_prec="bf16")
    h.close()
    assert rep["status_name"] == "converged" and rep["backward_error"] <= 1e-14
    assert checks.backward_error(A, x.cpu().numpy(), b) <= 1e-14
