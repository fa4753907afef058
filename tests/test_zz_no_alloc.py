"""The allocation-free batched entry point (lupp_dgesv_batched_noalloc),
through the C ABI, against lupp_dgesv_batched on the same inputs: factors,
pivots, info and solutions bit for bit (both run the same kernels, so no
rounding difference is allowed), on two calls in a row with the second
smaller, on a handle that never made an allocating batched call.  The
allocating entry point's results are themselves checked against the CPU
oracle by the batched parity tests; a sample is re-checked here."""
import numpy as np
import pytest

import synth
from oracle import checks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - GPU machine only
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_05782_amd as lupp  # noqa: E402
from gpu_util import announce  # noqa: E402


def _batch(count, seed):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(8, 129, size=count).astype(np.int32)
    sizes[:4] = (1, 32, 64, 128)  # an edge of every size class
    a_off = np.zeros(count, np.int64)
    b_off = np.zeros(count, np.int64)
    a_off[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    b_off[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    A = synth.uniform(seed, 0, int((sizes.astype(np.int64) ** 2).sum()) + 1, 1)[:, 0]
    B = synth.uniform(seed, 1, int(sizes.sum()) + 1, 1)[:, 0]
    return sizes, a_off, b_off, A, B


def _call(fn, sizes, a_off, b_off, A, B, handle):
    dn = torch.from_numpy(sizes).cuda()
    dA = torch.from_numpy(A.copy()).cuda()
    dB = torch.from_numpy(B.copy()).cuda()
    dao = torch.from_numpy(a_off).cuda()
    dbo = torch.from_numpy(b_off).cuda()
    p_off = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    p_off[1:] = torch.cumsum(dn.to(torch.int64), 0)[:-1]
    ipiv = torch.zeros(int(sizes.sum()) + 1, dtype=torch.int32, device="cuda")
    info = torch.full((len(sizes),), 7, dtype=torch.int32, device="cuda")
    fn(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), ipiv.cpu().numpy(), info.cpu().numpy(), dB.cpu().numpy(), p_off.cpu().numpy()


def test_noalloc_matches_allocating_entry_point():
    h_ref = lupp.Handle()
    h = lupp.Handle()
    for call, (count, seed) in enumerate(((3000, 20210601), (700, 20210602))):
        announce("noalloc batched call %d: %d systems, seed %d" % (call, count, seed))
        sizes, a_off, b_off, A, B = _batch(count, seed)
        ref = _call(lupp.lupp_xgesv_batched, sizes, a_off, b_off, A, B, h_ref)
        got = _call(lupp.lupp_dgesv_batched_noalloc, sizes, a_off, b_off, A, B, h)
        for name, r, g in zip(("LU", "ipiv", "info", "x"), ref[:4], got[:4]):
            assert np.array_equal(r.view(np.uint8), g.view(np.uint8)), "call %d: %s differs" % (call, name)
        assert (got[2] == 0).all()
        # a sample against the oracle's acceptance measures
        import oracle
        LU, ipiv, _, X, p_off = got
        for i in range(0, count, max(1, count // 25)):
            n = int(sizes[i])
            Ai = np.asfortranarray(A[a_off[i]:a_off[i] + n * n].reshape(n, n, order="F"))
            LUi = np.asfortranarray(LU[a_off[i]:a_off[i] + n * n].reshape(n, n, order="F"))
            pi = ipiv[p_off[i]:p_off[i] + n]
            _, po, _, gap = oracle.getrf(Ai, with_gap=True)
            ok, _, first = checks.pivot_prefix_match(pi, po, gap, 1e-9)
            assert ok, (call, i, first)
            assert checks.scaled_residual(Ai, LUi, pi) < 10
            assert checks.backward_error(Ai, X[b_off[i]:b_off[i] + n], B[b_off[i]:b_off[i] + n]) \
                <= 8 * n * checks.U64
    h.close()
    h_ref.close()


def test_noalloc_rejects_batch_above_limit():
    """A batch above the scratch capacity is refused on the host (nothing is
    launched, so the device pointers are never read)."""
    h = lupp.Handle()
    one = torch.ones(1, dtype=torch.int32, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = lupp._binding._lib.lupp_dgesv_batched_noalloc(
        h.ptr, lupp.NOALLOC_MAX_BATCH + 1, one.data_ptr(), off.data_ptr(), x.data_ptr(), off.data_ptr(),
        one.data_ptr(), off.data_ptr(), x.data_ptr(), one.data_ptr())
    assert rc == lupp._binding.ERR_UNSUPPORTED
    h.close()
