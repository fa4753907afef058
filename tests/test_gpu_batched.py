"""GPU parity of the batched factorization and solve (lupp_xgesv_batched,
lupp_xgetrf_batched) against the CPU oracle, through the C ABI.

Per system: ipiv identical to the oracle's on the separated prefix (relative
column gap >= tau, as for the large path), scaled residual < 10, backward
error of x <= 8 n u; closed forms bit-exact (dyadic exactly factorable
systems: ipiv, L, U bit for bit; Pi*D: pivots); edge sizes of every size
class; rejected sizes; singular systems leave b untouched; replays of a
captured HIP graph match the eager call bit for bit.
"""
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


def _pack(mats, rhs=None, dtype=np.float64):
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    a_off = np.zeros(len(mats), dtype=np.int64)
    b_off = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        a_off[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
        b_off[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    A = np.concatenate([np.asarray(m, dtype=dtype).ravel(order="F") for m in mats] + [np.zeros(1, dtype)])
    B = None
    if rhs is not None:
        B = np.concatenate([np.asarray(b, dtype=dtype) for b in rhs] + [np.zeros(1, dtype)])
    return sizes, A, a_off, B, b_off


def _run(sizes, A, a_off, B, b_off, solve=True):
    dn = torch.from_numpy(np.ascontiguousarray(sizes)).cuda()
    dA = torch.from_numpy(A.copy()).cuda()
    dao = torch.from_numpy(a_off).cuda()
    dB = torch.from_numpy(B.copy()).cuda() if (solve and B is not None) else None
    dbo = torch.from_numpy(b_off).cuda() if dB is not None else None
    ipiv, p_off, info = lupp.gesv_batched(dn, dA, dao, dB, dbo)
    torch.cuda.synchronize()
    return (dA.cpu().numpy(), ipiv.cpu().numpy(), p_off.cpu().numpy(), info.cpu().numpy(),
            dB.cpu().numpy() if dB is not None else None)


def _system(Ap, off, n):
    return np.asfortranarray(Ap[off:off + n * n].reshape(n, n, order="F"))


def _check_batch(sizes, A, a_off, B, b_off, dtype, tau, sample=None):
    LU, ipiv, p_off, info, X = _run(sizes, A, a_off, B, b_off)
    import oracle
    u = checks.U64 if dtype == np.float64 else checks.U32
    idx = range(len(sizes)) if sample is None else sample
    for i in idx:
        n = int(sizes[i])
        Ai = _system(A, a_off[i], n)
        LUi = _system(LU, a_off[i], n)
        pi = ipiv[p_off[i]:p_off[i] + n]
        _, po, info_o, gap = oracle.getrf(Ai, with_gap=True)
        assert info[i] == info_o == 0, (i, info[i], info_o)
        ok, cmp, first = checks.pivot_prefix_match(pi, po, gap, tau)
        assert ok, "system %d (n=%d): pivot mismatch at step %d" % (i, n, first)
        L, U = checks.unpack(LUi)
        assert np.abs(L).max(initial=0.0) <= 1.0
        assert checks.scaled_residual(Ai.astype(np.float64), LUi, pi, u) < 10
        bi = B[b_off[i]:b_off[i] + n]
        xi = X[b_off[i]:b_off[i] + n]
        assert checks.backward_error(Ai.astype(np.float64), xi.astype(np.float64), bi.astype(np.float64)) \
            <= 8 * n * u
    return LU, ipiv, p_off, info, X


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_random_vs_oracle(dtype):
    """600 systems, n ~ U{8..128}, A and b iid U(-1,1)."""
    announce("batched random 600 %s" % np.dtype(dtype).name)
    sizes = synth.batch_sizes(41, 600)
    A, a_off, B, b_off = synth.batch_uniform(41, sizes, dtype)
    tau = 1e-9 if dtype == np.float64 else 1e-4
    _, _, _, _, X = _check_batch(sizes, A, a_off, B, b_off, dtype, tau)
    # solutions against the oracle's batched solve (FP64): within the conditioning bound
    if dtype == np.float64:
        import oracle
        _, _, _, Xo, info_o = oracle.gesv_batched(sizes, A, a_off, B, b_off, nthreads=8)
        for i in range(0, 600, 7):
            n = int(sizes[i])
            Ai = _system(A, a_off[i], n)
            k = np.linalg.cond(Ai, 1)
            x, xo = X[b_off[i]:b_off[i] + n], Xo[b_off[i]:b_off[i] + n]
            assert np.abs(x - xo).max() / np.abs(xo).max() <= 16 * n * k * checks.U64


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_class_edges(dtype):
    """Orders at and around every size-class boundary, in shuffled order."""
    ns = [1, 2, 3, 8, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 128, 1, 77]
    announce("batched class edges %s" % np.dtype(dtype).name)
    mats = [synth.uniform(42, 10 + i, n, n) for i, n in enumerate(ns)]
    rhs = [synth.uniform(42, 100 + i, n, 1)[:, 0] for i, n in enumerate(ns)]
    sizes, A, a_off, B, b_off = _pack(mats, rhs, dtype)
    _check_batch(sizes, A, a_off, B, b_off, dtype, 1e-9 if dtype == np.float64 else 1e-4)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_exact_factorable(dtype):
    """Dyadic exactly factorable systems: ipiv, L and U bit for bit."""
    ns = [8, 17, 50, 64, 100, 128]
    announce("batched exact-factorable %s" % np.dtype(dtype).name)
    items = [synth.exact_lu_product(43, 20 + 3 * i, n) for i, n in enumerate(ns)]
    mats = [it[0] for it in items]
    rhs = [np.ones(n) for n in ns]
    sizes, A, a_off, B, b_off = _pack(mats, rhs, dtype)
    for solve in (True, False):
        LU, ipiv, p_off, info, _ = _run(sizes, A, a_off, B, b_off, solve)
        for i, (Am, L, U, perm) in enumerate(items):
            n = ns[i]
            assert info[i] == 0
            assert np.array_equal(ipiv[p_off[i]:p_off[i] + n], checks.closed_form_ipiv(perm))
            Lg, Ug = checks.unpack(_system(LU, a_off[i], n))
            assert np.array_equal(Lg, L) and np.array_equal(Ug, U)


def test_batch_pi_d_closed_form():
    ns = [9, 40, 70, 128]
    announce("batched Pi*D")
    items = [synth.pi_times_coldom(44, 30 + 2 * i, n) for i, n in enumerate(ns)]
    sizes, A, a_off, B, b_off = _pack([it[0] for it in items], [np.ones(n) for n in ns])
    LU, ipiv, p_off, info, X = _run(sizes, A, a_off, B, b_off)
    for i, (Am, perm) in enumerate(items):
        n = ns[i]
        assert info[i] == 0
        assert np.array_equal(ipiv[p_off[i]:p_off[i] + n], checks.closed_form_ipiv(perm))


def test_batch_getrf_equals_gesv_factors():
    """The right-hand side does not influence the factors: getrf_batched and
    gesv_batched return identical L\\U and ipiv."""
    announce("batched getrf vs gesv")
    sizes = synth.batch_sizes(45, 120)
    A, a_off, B, b_off = synth.batch_uniform(45, sizes)
    LU1, ip1, _, inf1, _ = _run(sizes, A, a_off, B, b_off, True)
    LU2, ip2, _, inf2, _ = _run(sizes, A, a_off, B, b_off, False)
    assert np.array_equal(LU1.view(np.int64), LU2.view(np.int64))
    assert np.array_equal(ip1, ip2) and np.array_equal(inf1, inf2)


def test_batch_singular_and_rejected():
    """A zero column gives info = its index + 1 and leaves b unchanged;
    orders outside [0, 128] give info = -1 and leave the system untouched;
    n = 0 gives info = 0."""
    announce("batched singular / rejected")
    m0 = synth.uniform(46, 1, 50, 50)
    m0[:, 20] = 0.0
    m1 = synth.uniform(46, 2, 30, 30)
    mats = [m0, m1, np.zeros((0, 0))]
    rhs = [synth.uniform(46, 3, 50, 1)[:, 0], synth.uniform(46, 4, 30, 1)[:, 0], np.zeros(0)]
    sizes, A, a_off, B, b_off = _pack(mats, rhs)
    LU, ipiv, p_off, info, X = _run(sizes, A, a_off, B, b_off)
    assert list(info[:3]) == [21, 0, 0]
    assert np.array_equal(X[:50], B[:50])  # not solved
    assert checks.backward_error(m1, X[50:80], B[50:80]) <= 8 * 30 * checks.U64
    # rejected orders
    bad = torch.tensor([129, -3, 5], dtype=torch.int32, device="cuda")
    dA = torch.from_numpy(np.arange(25 + 2, dtype=np.float64)).cuda()
    aoff = torch.tensor([0, 0, 0], dtype=torch.int64, device="cuda")
    before = dA.clone()
    ipiv, p_off, info = lupp.gesv_batched(bad[:2], dA, aoff[:2])
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [-1, -1]
    assert torch.equal(dA, before)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batch_nonfinite_inputs_isolated(dtype):
    """NaN and +-Inf entries are outside the contract (results unspecified),
    but the call completes, no system is abandoned (info -1000), every pivot
    index stays in range, and the finite systems of the same batch come out
    bit for bit as in a batch without the bad ones."""
    announce("batched non-finite inputs %s" % np.dtype(dtype).name)
    ns = [5, 40, 70, 100, 128, 17, 64, 96]
    good = [synth.uniform(48, 10 + i, n, n) for i, n in enumerate(ns)]
    grhs = [synth.uniform(48, 100 + i, n, 1)[:, 0] for i, n in enumerate(ns)]
    bad = []
    for i, n in enumerate(ns):
        m = synth.uniform(48, 200 + i, n, n)
        m[(3 * i) % n, (5 * i + 1) % n] = np.nan
        m[(7 * i + 2) % n, (2 * i) % n] = np.inf if i % 2 else -np.inf
        bad.append(m)
    brhs = [synth.uniform(48, 300 + i, n, 1)[:, 0] for i, n in enumerate(ns)]
    # interleaved: good, bad, good, bad, ...
    mats = [m for pair in zip(good, bad) for m in pair]
    rhs = [b for pair in zip(grhs, brhs) for b in pair]
    sizes, A, a_off, B, b_off = _pack(mats, rhs, dtype)
    LU, ipiv, p_off, info, X = _run(sizes, A, a_off, B, b_off)
    assert not np.any(info == -1000), info
    for i, n in enumerate(sizes):
        pi = ipiv[p_off[i]:p_off[i] + n]
        assert np.all(pi >= np.arange(1, n + 1)) and np.all(pi <= n), (i, pi)
    sg, Ag, ag, Bg, bg = _pack(good, grhs, dtype)
    LUg, ipg, pg, infg, Xg = _run(sg, Ag, ag, Bg, bg)
    for j, n in enumerate(ns):
        i = 2 * j
        assert info[i] == infg[j] == 0
        assert np.array_equal(LU[a_off[i]:a_off[i] + n * n].view(np.uint8),
                              LUg[ag[j]:ag[j] + n * n].view(np.uint8)), j
        assert np.array_equal(ipiv[p_off[i]:p_off[i] + n], ipg[pg[j]:pg[j] + n])
        assert np.array_equal(X[b_off[i]:b_off[i] + n].view(np.uint8), Xg[bg[j]:bg[j] + n].view(np.uint8))


def test_batch_host_errors():
    announce("batched host errors")
    dn = torch.ones(2, dtype=torch.int32, device="cuda")
    h = lupp.default_handle()
    h.set_stream()
    rc = lupp._binding._lib.lupp_dgesv_batched(h.ptr, -1, dn.data_ptr(), 0, 0, 0, 0, 0, 0, 0)
    assert rc == -2
    rc = lupp._binding._lib.lupp_dgesv_batched(h.ptr, 2, None, 0, 0, 0, 0, 0, 0, 0)
    assert rc == -3
    rc = lupp._binding._lib.lupp_dgesv_batched(h.ptr, 0, None, None, None, None, None, None, None, None)
    assert rc == 0


def test_batch_graph_replay():
    """Captured once, replayed three times with eager work and synchronization
    in between: every replay equals the eager result bit for bit."""
    announce("batched graph replay")
    sizes = synth.batch_sizes(47, 400)
    A, a_off, B, b_off = synth.batch_uniform(47, sizes)
    dn = torch.from_numpy(sizes).cuda()
    dao = torch.from_numpy(a_off).cuda()
    dbo = torch.from_numpy(b_off).cuda()
    A0 = torch.from_numpy(A).cuda()
    B0 = torch.from_numpy(B).cuda()
    dA, dB = A0.clone(), B0.clone()
    n64 = dn.to(torch.int64)
    p_off = torch.zeros_like(n64)
    p_off[1:] = torch.cumsum(n64, 0)[:-1]
    ipiv = torch.zeros(int(n64.sum()), dtype=torch.int32, device="cuda")
    info = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")
    h = lupp.Handle()
    lupp.lupp_xgesv_batched(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle=h)  # eager; creates the workspace
    torch.cuda.synchronize()
    ref = (dA.clone(), dB.clone(), ipiv.clone(), info.clone())
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        dA.copy_(A0)
        dB.copy_(B0)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        lupp.lupp_xgesv_batched(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle=h)
    for rep in range(3):
        dA.copy_(A0)
        dB.copy_(B0)
        ipiv.zero_()
        info.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dA.view(torch.int64), ref[0].view(torch.int64)), rep
        assert torch.equal(dB.view(torch.int64), ref[1].view(torch.int64)), rep
        assert torch.equal(ipiv, ref[2]) and torch.equal(info, ref[3]), rep
        x = dA.sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(x)
    h.close()


def test_batch_full_workload_sampled():
    """20000 systems, n ~ U{8..128} (the benchmark's workload): every system's
    backward error, and oracle pivots on a sample of 200 systems."""
    announce("batched 20000 sampled")
    sizes = synth.batch_sizes(20210513, 20000)
    A, a_off, B, b_off = synth.batch_uniform(20210513, sizes)
    LU, ipiv, p_off, info, X = _run(sizes, A, a_off, B, b_off)
    assert np.all(info == 0)
    worst = 0.0
    for i in range(len(sizes)):
        n = int(sizes[i])
        Ai = _system(A, a_off[i], n)
        eta = checks.backward_error(Ai, X[b_off[i]:b_off[i] + n], B[b_off[i]:b_off[i] + n])
        worst = max(worst, eta / (n * checks.U64))
    assert worst <= 8, worst
    import oracle
    rng = np.random.default_rng(3)
    for i in rng.choice(len(sizes), 200, replace=False):
        n = int(sizes[i])
        Ai = _system(A, a_off[i], n)
        _, po, _, gap = oracle.getrf(Ai, with_gap=True)
        ok, cmp, first = checks.pivot_prefix_match(ipiv[p_off[i]:p_off[i] + n], po, gap, 1e-9)
        assert ok, (i, n, first)
