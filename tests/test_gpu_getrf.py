"""GPU parity of the HIP LU path against the CPU oracle (through the C ABI).

Bars (floating point decides integers here, so pivots are compared where the
oracle's pivot column is separated by a relative gap >= tau, on every step up
to the first non-separated one):
  * ipiv identical to the oracle's on the separated prefix;
  * scaled residual ||PA - LU||_1 / (n eps ||A||_1) < 10 for the GPU factors
    (eps = 2^-53 FP64, 2^-24 FP32), |L| <= 1;
  * closed forms bit-exact at any size (Pi*D pivots; exactly factorable
    dyadic matrices: ipiv, L and U bit for bit);
  * solve: normwise backward error <= 8 n u.
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
from gpu_util import announce, to_dev, to_host  # noqa: E402

TAU = 1e-9


def _oracle():
    import oracle
    return oracle


def _gpu_factor(A, nb=None, leaf=None):
    h = lupp.Handle()
    if nb:
        h.set_option(1, nb)
    if leaf:
        h.set_option(2, leaf)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    torch.cuda.synchronize()
    out = to_host(dA), ipiv.cpu().numpy(), int(info.item())
    h.close()
    return out


def _check_against_oracle(A, LU, ipiv, info, eps, tau=TAU, nthreads=8):
    o = _oracle()
    LUo, ipo, info_o, gap = o.getrf(A, with_gap=True, nthreads=nthreads)
    assert info == info_o
    ok, cmp, first = checks.pivot_prefix_match(ipiv, ipo, gap, tau)
    assert ok, "pivot mismatch at step %d (compared %d, min gap %.3g)" % (first, cmp, float(np.min(gap, initial=1)))
    L, U = checks.unpack(LU)
    assert np.abs(L).max(initial=0.0) <= 1.0
    res = checks.scaled_residual(A, LU, ipiv, eps)
    assert res < 10, res
    return cmp


def test_config1_n512_fp64():
    """n = 512, A and b iid U(-1,1): pivots bit-exact, residual, solve."""
    n = 512
    announce("config1 n=512 fp64")
    A = synth.uniform(synth.DEFAULT_SEED, 0, n, n)
    b = synth.uniform(synth.DEFAULT_SEED, 1, n, 1)[:, 0]
    LU, ipiv, info = _gpu_factor(A)
    cmp = _check_against_oracle(A, LU, ipiv, info, checks.U64)
    assert cmp == n
    dLU = to_dev(LU)
    dip = torch.from_numpy(ipiv).cuda()
    db = torch.from_numpy(b.copy()).cuda()
    lupp.getrs(dLU, dip, db)
    x = db.cpu().numpy()
    assert checks.backward_error(A, x, b) <= 8 * n * checks.U64
    LUo, ipo, _ = _oracle().getrf(A)
    xo, _ = _oracle().getrs(LUo, ipo, b)
    kappa = np.linalg.cond(A, 1)
    assert np.abs(x - xo).max() / np.abs(xo).max() <= 16 * n * kappa * checks.U64


SHAPES = [(1, 1), (2, 2), (3, 7), (7, 3), (33, 33), (64, 64), (100, 100), (257, 257), (300, 200), (200, 300),
          (1000, 1000), (1025, 1025), (1500, 700), (700, 1500)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_ragged_shapes(shape, dtype):
    m, n = shape
    announce("ragged %dx%d %s" % (m, n, dtype))
    A = synth.uniform(7, 3, m, n)
    if dtype == "f32":
        A = A.astype(np.float32)
    for nb, leaf in ((None, None), (64, 16), (96, 48), (100, None)):
        LU, ipiv, info = _gpu_factor(A, nb, leaf)
        _check_against_oracle(A, LU, ipiv, info, checks.U64 if dtype == "f64" else checks.U32,
                              tau=TAU if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("n", [2048, 4096])
def test_multi_group_panels(n):
    """r > 1024 rows: the column-block kernel runs with several cooperating workgroups."""
    announce("multi-group n=%d" % n)
    A = synth.uniform(11, 0, n, n)
    LU, ipiv, info = _gpu_factor(A)
    cmp = _check_against_oracle(A, LU, ipiv, info, checks.U64, nthreads=16)
    assert cmp >= n - 4


def test_empty():
    announce("empty")
    for (m, n) in ((0, 0), (0, 5), (5, 0)):
        dA = torch.zeros((max(n, 1), max(m, 1)), dtype=torch.float64, device="cuda").t()[:m, :n]
        ipiv = torch.zeros(1, dtype=torch.int32, device="cuda")
        info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        lupp.lupp_dgetrf(dA, ipiv, info)
        torch.cuda.synchronize()
        assert int(info.item()) == 0


def test_zero_column_info():
    announce("zero column")
    A = synth.uniform(4, 1, 300, 300)
    A[:, 77] = 0.0
    A[:, 200] = 0.0
    LU, ipiv, info = _gpu_factor(A)
    assert info == 78
    LUo, ipo, info_o = _oracle().getrf(A)
    assert info_o == 78


def test_zero_matrix():
    announce("zero matrix")
    LU, ipiv, info = _gpu_factor(np.zeros((70, 70)))
    assert info == 1 and np.array_equal(ipiv, np.arange(1, 71)) and not np.any(LU)


@pytest.mark.parametrize("n", [100, 1000, 3000])
def test_exact_factorable_bit_exact(n):
    """A = Pi^T L U with dyadic factors: every value is exact, so the GPU must
    return the constructed ipiv, L and U bit for bit (FP64 and FP32)."""
    announce("exact-factorable n=%d" % n)
    A, L, U, perm = synth.exact_lu_product(8, 30, n)
    for dt in (np.float64, np.float32):
        LU, ipiv, info = _gpu_factor(A.astype(dt))
        assert info == 0
        assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))
        Lg, Ug = checks.unpack(LU)
        assert np.array_equal(Lg, L) and np.array_equal(Ug, U)


@pytest.mark.parametrize("n", [500, 4096])
def test_pi_d_closed_form(n):
    announce("Pi*D n=%d" % n)
    A, perm = synth.pi_times_coldom(21, 4, n)
    LU, ipiv, info = _gpu_factor(A)
    assert info == 0
    assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))
    assert checks.scaled_residual(A, LU, ipiv) < 10


def test_deterministic():
    announce("determinism n=1500")
    A = synth.uniform(3, 3, 1500, 1500)
    a1, p1, _ = _gpu_factor(A)
    a2, p2, _ = _gpu_factor(A)
    assert np.array_equal(p1, p2) and np.array_equal(a1.view(np.int64), a2.view(np.int64))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_getrs_multi_rhs(dtype):
    n, nrhs = 777, 5
    announce("getrs n=%d nrhs=%d %s" % (n, nrhs, dtype))
    npdt = np.float64 if dtype == "f64" else np.float32
    A = synth.uniform(5, 0, n, n).astype(npdt)
    B = synth.uniform(5, 1, n, nrhs).astype(npdt)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA)
    dB = to_dev(B)
    lupp.getrs(dA, ipiv, dB)
    torch.cuda.synchronize()
    X = to_host(dB)
    u = checks.U64 if dtype == "f64" else checks.U32
    for j in range(nrhs):
        assert checks.backward_error(A.astype(np.float64), X[:, j].astype(np.float64),
                                     B[:, j].astype(np.float64)) <= 8 * n * u


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [8192 + 77, 8192 + 40])
def test_getrs_wide_blocks_ragged(dtype, n):
    """From order 8192 on the triangular solves use 128-row blocks: ragged
    orders above that threshold -- a last block whose second 64-row half is
    partly filled (77 rows past the boundary) or empty (40 rows) -- solved to
    the backward-error bound."""
    announce("getrs n=%d %s (128-row solve blocks)" % (n, dtype))
    npdt = np.float64 if dtype == "f64" else np.float32
    A = synth.uniform(6, 0, n, n).astype(npdt)
    b = synth.uniform(6, 1, n, 1).astype(npdt)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA)
    assert info == 0
    db = to_dev(b)
    lupp.getrs(dA, ipiv, db)
    torch.cuda.synchronize()
    x = to_host(db)[:, 0].astype(np.float64)
    u = checks.U64 if dtype == "f64" else checks.U32
    assert np.all(np.isfinite(x))
    assert checks.backward_error(A.astype(np.float64), x, b[:, 0].astype(np.float64)) <= 8 * n * u


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1000, 3000])
def test_nonfinite_inputs_complete(n, dtype):
    """NaN and +-Inf entries are outside the contract (results unspecified),
    but getrf and getrs complete without a library error (no expired wait),
    every pivot index stays in range and info is not negative."""
    announce("non-finite n=%d %s" % (n, dtype))
    npdt = np.float64 if dtype == "f64" else np.float32
    A = synth.uniform(49, 0, n, n).astype(npdt)
    A[n // 3, 5] = np.nan
    A[7, n // 2] = np.inf
    A[n - 2, n - 9] = -np.inf
    h = lupp.Handle()
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    torch.cuda.synchronize()
    ip = ipiv.cpu().numpy()
    assert np.all(ip >= np.arange(1, n + 1)) and np.all(ip <= n)
    assert int(info.item()) >= 0
    dB = to_dev(synth.uniform(49, 1, n, 1).astype(npdt))
    lupp.getrs(dA, ipiv, dB, handle=h)
    h.sync()
    torch.cuda.synchronize()
    h.close()


def _factor_opts(A, **opts):
    h = lupp.Handle()
    for k, v in opts.items():
        h.set_option({"nb": 1, "leaf": 2, "lookahead": 4, "defer": lupp._binding.OPT_DEFER_SWAPS}[k], v)
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    torch.cuda.synchronize()
    out = to_host(dA), ipiv.cpu().numpy(), int(info.item())
    h.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape,nb", [((1500, 1500), None), ((2000, 700), 64), ((700, 2000), 96),
                                      ((3000, 1000), 128), ((1031, 1031), 100)])
def test_deferred_interchanges_bit_identical(shape, nb, dtype):
    """The finished columns' interchanges applied once at the end (composed per
    column block) give exactly the factors of the per-step application."""
    m, n = shape
    announce("defer vs per-step %dx%d nb=%s %s" % (m, n, nb, dtype))
    A = synth.uniform(9, 1, m, n)
    if dtype == "f32":
        A = A.astype(np.float32)
    kw = {"nb": nb} if nb else {}
    LU1, p1, i1 = _factor_opts(A, defer=1, **kw)
    LU0, p0, i0 = _factor_opts(A, defer=0, **kw)
    assert i1 == i0 and np.array_equal(p1, p0)
    assert np.array_equal(LU1, LU0)
    _check_against_oracle(A, LU1, p1, i1, checks.U64 if dtype == "f64" else checks.U32,
                          tau=TAU if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype,m", [("f64", 33300), ("f32", 33300)])
def test_tall_deferral_limits(dtype, m):
    """m - nb above the in-register column length of the deferred gather
    (FP64: per-step interchanges instead) and the widest FP32 gather."""
    n = 520
    announce("tall %dx%d %s" % (m, n, dtype))
    A = synth.uniform(10, 2, m, n)
    if dtype == "f32":
        A = A.astype(np.float32)
    LU, ipiv, info = _factor_opts(A)
    _check_against_oracle(A, LU, ipiv, info, checks.U64 if dtype == "f64" else checks.U32,
                          tau=TAU if dtype == "f64" else 1e-4, nthreads=16)


def test_wide_block_uncomposed_interchanges():
    """nb above the composed-run limit (512): the per-column interchange path."""
    n = 1400
    announce("nb=600 n=%d" % n)
    A = synth.uniform(10, 3, n, n)
    LU, ipiv, info = _factor_opts(A, nb=600)
    _check_against_oracle(A, LU, ipiv, info, checks.U64)


def _replay(ipiv, B):
    """Interchanges applied one by one, in order (the definition of row
    interchange with a 1-based pivot vector)."""
    X = B.copy()
    for i, p in enumerate(ipiv):
        p -= 1
        if p != i:
            X[[i, p]] = X[[p, i]]
    return X


@pytest.mark.parametrize("nrhs", [1, 3])
def test_composed_interchanges_bit_exact(nrhs):
    """getrs with L = U = I returns P*B: the composed runs of up to 512
    interchanges must equal the sequential replay bit for bit, for pivot
    vectors with long chains, repeated targets and rows inside the run."""
    n = 1500
    announce("composed interchanges n=%d nrhs=%d" % (n, nrhs))
    rng = np.random.default_rng(77)
    cases = {
        "random": np.array([rng.integers(i, n) for i in range(n)]),
        "last_row": np.full(n, n - 1),
        "next_row": np.minimum(np.arange(n) + 1, n - 1),
        "identity": np.arange(n),
        "block_end": np.array([min(((i // 512) + 1) * 512 - 1, n - 1) for i in range(n)]),
        "few_targets": np.array([max(i, [600, 601, 1499][i % 3]) for i in range(n)]),
    }
    I = np.eye(n)
    dI = to_dev(I)
    for name, piv0 in cases.items():
        ipiv = (piv0 + 1).astype(np.int32)
        B = rng.standard_normal((n, nrhs))
        dB = to_dev(B)
        lupp.getrs(dI, torch.from_numpy(ipiv).cuda(), dB)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(dB), _replay(ipiv, B)), name


def _probe_residual(A0, LU, ipiv, nprobe=4, seed=3):
    """max over probes of ||P A x - L (U x)||_inf / (n ||A||_inf ||x||_inf) on the GPU (FP64)."""
    n = A0.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    L = torch.tril(LU, -1) + torch.eye(n, dtype=LU.dtype, device="cuda")
    U = torch.triu(LU)
    perm = torch.arange(n, device="cuda")
    piv = ipiv.long() - 1
    p_host = perm.cpu().numpy()
    for i, p in enumerate(piv.cpu().numpy()):
        p_host[i], p_host[p] = p_host[p], p_host[i]
    P = torch.from_numpy(p_host).cuda()
    anorm = A0.abs().sum(dim=1).max()
    worst = 0.0
    for _ in range(nprobe):
        x = torch.rand(n, 1, generator=g, dtype=A0.dtype, device="cuda") * 2 - 1
        r = (A0 @ x)[P] - L @ (U @ x)
        worst = max(worst, float(r.abs().max() / (n * anorm * x.abs().max())))
    return worst


def _factor_dev(A0, **opts):
    h = lupp.Handle()
    for k, v in opts.items():
        h.set_option({"nb": 1, "timing": 3, "split": lupp._binding.OPT_SPLIT_UPDATE,
                      "prec": lupp._binding.OPT_UPDATE_PREC, "packed": 8, "lookahead": 4}[k], v)
    A = torch.empty_like(A0.t()).t()
    A.copy_(A0)
    ipiv = torch.empty(A0.shape[0], dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    (lupp.lupp_dgetrf if A0.dtype == torch.float64 else lupp.lupp_sgetrf)(A, ipiv, info, handle=h)
    h.sync()
    updates = h.timing_summary("update")[0] if opts.get("timing") else None
    h.close()
    return A, ipiv, int(info.item()), updates


def test_split_update_bit_identical():
    """n = 16384: the remaining-columns update shared with the panel's CUs
    gives the same factors bit for bit, and the split does happen."""
    n = 16384
    announce("split update n=%d fp64" % n)
    g = torch.Generator(device="cuda").manual_seed(41)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    A1, p1, i1, u1 = _factor_dev(A0, split=1, timing=1)
    A2, p2, i2, u2 = _factor_dev(A0, split=0, timing=1)
    assert i1 == i2 == 0
    assert u1 > u2, (u1, u2)  # extra launches on the panel's CUs
    assert torch.equal(p1, p2)
    assert torch.equal(A1, A2)
    assert _probe_residual(A0, A1, p1) < 10 * checks.U64


def test_timing_level_updates_only():
    """LUPP_OPT_TIMING = 2 brackets the trailing updates only: the same update
    intervals and flops as level 1, no column-block intervals, and the same
    factors as an uninstrumented call."""
    n = 4096
    announce("timing levels n=%d fp64" % n)
    g = torch.Generator(device="cuda").manual_seed(43)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    runs = []
    for level in (0, 1, 2):
        h = lupp.Handle()
        h.set_option(3, level)
        A = torch.empty_like(A0.t()).t()
        A.copy_(A0)
        ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
        info = torch.empty(1, dtype=torch.int32, device="cuda")
        lupp.lupp_dgetrf(A, ipiv, info, handle=h)
        h.sync()
        counts = {ph: h.timing_summary(ph) for ph in ("panel", "panel_leaf", "laswp", "update", "update_big")}
        h.close()
        runs.append((A, ipiv, int(info.item()), counts))
    (A0f, p0, i0, c0), (A1, p1, i1, c1), (A2, p2, i2, c2) = runs
    assert i0 == i1 == i2 == 0
    assert torch.equal(p0, p1) and torch.equal(p0, p2)
    assert torch.equal(A0f, A1) and torch.equal(A0f, A2)
    assert all(c[0] == 0 for c in c0.values())
    assert c1["panel"][0] > 0 and c1["panel_leaf"][0] > 0 and c1["laswp"][0] > 0
    assert c2["panel"][0] == 0 and c2["panel_leaf"][0] == 0 and c2["laswp"][0] == 0
    for ph in ("update", "update_big"):
        assert c2[ph][0] == c1[ph][0] > 0
        assert c2[ph][2] == c1[ph][2] > 0


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("shape", [(4133, 4133), (5000, 3700), (2900, 4500)])
def test_low_precision_packed_operands_bit_identical(fmt, shape):
    """The update's operands rounded once into the packed workspace give the
    same factors and pivots, bit for bit, as rounding them in every tile
    (ragged row, column and k edges; FP16/FP8 with block scales)."""
    m, n = shape
    announce("packed vs staged %s updates %dx%d" % (fmt, m, n))
    g = torch.Generator(device="cuda").manual_seed(44 + m + n)
    A0 = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    A1, p1, i1, _ = _factor_dev(A0, prec=lupp.PREC[fmt], packed=1)
    A2, p2, i2, _ = _factor_dev(A0, prec=lupp.PREC[fmt], packed=0)
    k = min(m, n)  # the pivot buffer holds m entries; the first min(m, n) are written
    assert i1 == i2 == 0
    assert torch.equal(p1[:k], p2[:k])
    assert torch.equal(A1, A2)


def test_dataflow_scaled_low_precision_bit_identical():
    """Dataflow runtime with FP16 updates (per-block scales): each stream has
    its own scale and packing slot, so overlapping update tasks give the
    loop's bits exactly."""
    n = 8192
    announce("dataflow fp16 updates n=%d" % n)
    g = torch.Generator(device="cuda").manual_seed(45)
    A0 = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    ref = _factor_dev(A0, prec=lupp.PREC["fp16"])
    out = _factor_dev(A0, prec=lupp.PREC["fp16"], lookahead=4)
    assert ref[2] == out[2] == 0
    assert torch.equal(ref[1], out[1]) and torch.equal(ref[0], out[0])


def test_option_ranges():
    """lupp_set_option accepts each option's documented range and rejects the
    rest with -3 (value) or -2 (unknown option), leaving the handle usable."""
    b = lupp._binding
    h = lupp.Handle()
    lib = b._lib
    cases = {b.OPT_NB: ([1, 512, 1024], [0, 1025]),
             b.OPT_PANEL_LEAF: ([16, 64, 256], [0, 8, 24, 272]),
             b.OPT_TIMING: ([0, 1, 2], [-1, 3]),
             b.OPT_LOOKAHEAD: ([0, 1, 2, 16], [-1, 17]),
             b.OPT_UPDATE_PREC: ([0, 1, 2, 3], [-1, 4]),
             b.OPT_DEFER_SWAPS: ([0, 1], [2]),
             b.OPT_SPLIT_UPDATE: ([0, 1], [-1, 2]),
             b.OPT_LP_PACKED: ([0, 1], [2])}
    for opt, (good, bad) in cases.items():
        for v in good:
            assert lib.lupp_set_option(h.ptr, opt, v) == 0, (opt, v)
        for v in bad:
            assert lib.lupp_set_option(h.ptr, opt, v) == -3, (opt, v)
    for opt in (0, 9, 100):
        assert lib.lupp_set_option(h.ptr, opt, 1) == -2, opt
    # restore the defaults and factor once
    for opt, v in ((b.OPT_NB, 512), (b.OPT_PANEL_LEAF, 64), (b.OPT_TIMING, 0), (b.OPT_LOOKAHEAD, 1),
                   (b.OPT_UPDATE_PREC, 0), (b.OPT_DEFER_SWAPS, 1), (b.OPT_SPLIT_UPDATE, 1), (b.OPT_LP_PACKED, 1)):
        h.set_option(opt, v)
    n = 1000
    g = torch.Generator(device="cuda").manual_seed(46)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    A = torch.empty_like(A0.t()).t()
    A.copy_(A0)
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    lupp.lupp_dgetrf(A, ipiv, info, handle=h)
    h.sync()
    h.close()
    assert int(info.item()) == 0
    assert _probe_residual(A0, A, ipiv) < 10 * checks.U64


def test_split_update_low_precision():
    """The same split with BF16 updates (each share scales its own blocks):
    a valid factorization within the update format's residual bound."""
    n = 16384
    announce("split update n=%d bf16 updates" % n)
    g = torch.Generator(device="cuda").manual_seed(42)
    A0 = torch.empty((n, n), dtype=torch.float32, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    A1, p1, i1, _ = _factor_dev(A0, split=1, prec=lupp.PREC["bf16"])
    assert i1 == 0
    assert float(torch.tril(A1, -1).abs().max()) <= 1.0
    assert _probe_residual(A0.double(), A1.double(), p1) < 10 * 2.0 ** -8


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lookahead_wide_panel_pair_bit_identical(dtype):
    """m = 40000: the next block's factorization needs 40 workgroups, so it
    runs beside the update on the 64-CU stream pair; the factors equal those
    of the in-order single-stream run bit for bit."""
    m, n = 40000, 1280
    announce("wide panel pair %dx%d %s" % (m, n, dtype))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(43)
    A0 = torch.empty((n, m), dtype=tdt, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    outs = []
    for la in (1, 0):
        h = lupp.Handle()
        h.set_option(4, la)
        A = torch.empty_like(A0.t()).t()
        A.copy_(A0)
        ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
        info = torch.empty(1, dtype=torch.int32, device="cuda")
        (lupp.lupp_dgetrf if dtype == "f64" else lupp.lupp_sgetrf)(A, ipiv, info, handle=h)
        h.sync()
        h.close()
        outs.append((A, ipiv, int(info.item())))
    (A1, p1, i1), (A2, p2, i2) = outs
    assert i1 == i2 == 0
    assert torch.equal(p1, p2) and torch.equal(A1, A2)
    # L U reproduces the interchanged rows (probe vectors, FP64)
    L = torch.tril(A1.double(), -1)
    L[:n, :n] += torch.eye(n, dtype=torch.float64, device="cuda")
    U = torch.triu(A1.double()[:n, :n])
    perm = np.arange(m)
    for i, p in enumerate(p1.cpu().numpy() - 1):
        perm[i], perm[p] = perm[p], perm[i]
    P = torch.from_numpy(perm).cuda()
    x = torch.rand(n, 1, generator=g, dtype=tdt, device="cuda").double() * 2 - 1
    r = (A0.double() @ x)[P] - L @ (U @ x)
    u = checks.U64 if dtype == "f64" else checks.U32
    assert float(r.abs().max() / (m * A0.double().abs().sum(dim=1).max() * x.abs().max())) < 10 * u


# ---------------------------------------------------------------- device-side status through lupp_sync
def _solve_setup(n, seed, zero_col=None):
    A = synth.uniform(seed, 0, n, n)
    if zero_col is not None:
        A[:, zero_col] = 0.0
    b = synth.uniform(seed, 1, n, 1)[:, 0]
    h = lupp.Handle()
    dA = to_dev(A)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    return A, b, h, dA, ipiv, int(info.item())


@pytest.mark.gpu
def test_getrs_reports_zero_diagonal():
    """A zero column gives info > 0; a solve with those factors is reported
    as LUPP_ERR_SINGULAR by the next sync, once."""
    n = 300
    announce("getrs singular n=%d" % n)
    A, b, h, dA, ipiv, info = _solve_setup(n, 61, zero_col=200)
    assert info == 201
    db = to_dev(b)
    lupp.getrs(dA, ipiv, db, handle=h)
    with pytest.raises(lupp.LuppError) as ex:
        h.sync()
    assert ex.value.rc == lupp._binding.ERR_SINGULAR
    h.sync()  # reported once
    h.close()


@pytest.mark.gpu
def test_sync_reports_solve_error_flag():
    """The triangular solve's device error flag (set from the host by the
    test hook, as an expired wait sets it) is reported by lupp_sync once."""
    n = 257
    announce("sync trsv error flag n=%d" % n)
    A, b, h, dA, ipiv, info = _solve_setup(n, 62)
    h.inject_fault(1)
    with pytest.raises(lupp.LuppError) as ex:
        h.sync()
    assert ex.value.rc == lupp._binding.ERR_INTERNAL
    db = to_dev(b)
    lupp.getrs(dA, ipiv, db, handle=h)
    h.sync()
    assert checks.backward_error(A, to_host(db), b) <= 8 * n * checks.U64
    h.close()


@pytest.mark.gpu
@pytest.mark.parametrize("n", [700, 8192 + 40])
def test_ticket_mismatch_reported_and_recovered(n):
    """Host and device ticket counts out of step (forced by the test hook, so
    that every workgroup finds its ticket out of range and exits): the solve
    is reported as LUPP_ERR_INTERNAL, and the next solve is correct again."""
    announce("ticket mismatch n=%d" % n)
    A, b, h, dA, ipiv, info = _solve_setup(n, 63)
    assert info == 0
    h.inject_fault(2)
    db = to_dev(b)
    lupp.getrs(dA, ipiv, db, handle=h)
    with pytest.raises(lupp.LuppError) as ex:
        h.sync()
    assert ex.value.rc == lupp._binding.ERR_INTERNAL
    db = to_dev(b)
    lupp.getrs(dA, ipiv, db, handle=h)
    h.sync()
    assert checks.backward_error(A, to_host(db), b) <= 8 * n * checks.U64
    h.close()


@pytest.mark.gpu
def test_workspace_bytes():
    """lupp_workspace_bytes: the documented components, growing with the shape."""
    h = lupp.Handle()
    base = h.workspace_bytes("dgetrs", 0, 1)
    assert h.workspace_bytes("dgetrs", 0, 100) == base
    assert h.workspace_bytes("dgetrs", 0, 64 * 4096) == base + (4096 - 1024) * 4
    assert h.workspace_bytes("batched", 20000) == 20000 * 4 + 256
    assert h.workspace_bytes("batched", 10) == 1024 * 4 + 256
    small = h.workspace_bytes("dgetrf", 400, 400)   # one block: no deferred interchanges
    big = h.workspace_bytes("dgetrf", 4096, 4096)
    assert big > small > 0
    h.set_option(6, 0)  # no deferral: the factorization's base workspace only
    assert h.workspace_bytes("dgetrf", 4096, 4096) == small
    mixed = h.workspace_bytes("dgesv_mixed", 0, 2000, 30)
    assert mixed > 2000 * 2000 * 4 + 31 * 2000 * 8
    assert h.workspace_bytes("dgesv_mixed", 0, 2000, 1) < mixed
    for bad in ((99, 1, 1, 0), (1, -1, 1, 0), (1, 1, -1, 0), (5, 0, 10, 61)):
        rc = lupp._binding._lib.lupp_workspace_bytes(h.ptr, bad[0], bad[1], bad[2], bad[3], None)
        assert rc < 0
    h.close()
