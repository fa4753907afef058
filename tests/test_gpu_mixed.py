"""GPU tests of the low-precision trailing update and of the mixed-precision
solve with FP64 refinement (through the C ABI).

The low-precision factors have no exact reference (their values depend on
rounding in the update format), so they are checked through properties that
hold for any correct partial-pivoting factorization with that update format:
|L| <= 1, valid interchanges, closed-form pivots for Pi*D inputs (the column
dominance margin is far above the update's rounding error), and a residual
scaled by the format's unit roundoff.  The refined solutions are checked by
their backward error recomputed on the host in extended precision, and against
the CPU oracle's FP64 solution within the conditioning bound.
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

# unit roundoff of the update formats
U_LOW = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp8": 2.0 ** -4}
PRECS = ["bf16", "fp16", "fp8"]


def _lp_factor(A32, prec, nb=None):
    h = lupp.Handle()
    h.set_option(lupp._binding.OPT_UPDATE_PREC, lupp.PREC[prec])
    if nb:
        h.set_option(lupp._binding.OPT_NB, nb)
    dA = to_dev(A32)
    ipiv, info = lupp.getrf(dA, handle=h)
    h.sync()
    out = to_host(dA), ipiv.cpu().numpy(), int(info.item())
    h.close()
    return out


def eta_host(A, x, b):
    """Backward error with the residual formed in extended precision."""
    Al = A.astype(np.longdouble)
    r = b.astype(np.longdouble) - Al @ x.astype(np.longdouble)
    num = np.abs(r).max()
    den = np.abs(Al).sum(axis=1).max() * np.abs(x.astype(np.longdouble)).max() + np.abs(b).max()
    return float(num / den)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape,nb", [((300, 300), None), ((1000, 1000), 128), ((1100, 700), None),
                                      ((700, 1100), 96), ((2500, 2500), None)])
def test_lp_update_factorization(prec, shape, nb):
    m, n = shape
    announce("lp sgetrf %s %dx%d nb=%s" % (prec, m, n, nb))
    A = synth.uniform(31, 0, m, n).astype(np.float32)
    LU, ipiv, info = _lp_factor(A, prec, nb)
    assert info == 0
    p = min(m, n)
    assert np.all(ipiv >= np.arange(1, p + 1)) and np.all(ipiv <= m)
    L, U = checks.unpack(LU)
    assert np.abs(L).max() <= 1.0
    res = checks.scaled_residual(A.astype(np.float64), LU, ipiv, U_LOW[prec])
    assert res < 10, res


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [600, 3000])
def test_lp_update_pi_d_closed_form(prec, n):
    """Pi*D with column dominance margin: partial pivoting must pick Pi's rows
    whatever the update format."""
    announce("lp Pi*D %s n=%d" % (prec, n))
    A, perm = synth.pi_times_coldom(21, 4, n)
    LU, ipiv, info = _lp_factor(A.astype(np.float32), prec)
    assert info == 0
    assert np.array_equal(ipiv, checks.closed_form_ipiv(perm))


def _mixed(A, b, solver, prec, **kw):
    dA = to_dev(A)
    db = to_dev(b.reshape(-1, 1))
    dX = torch.empty(1, A.shape[0], dtype=torch.float64, device="cuda").t()
    rep = lupp.lupp_dgesv_mixed(dA, db, dX, lupp.ir_opts(solver, factor_prec=prec, **kw))
    torch.cuda.synchronize()
    return dX[:, 0].cpu().numpy(), rep


@pytest.mark.parametrize("solver", ["classical", "gmres"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp8"])
def test_mixed_diag_dominant(solver, prec):
    """Diagonally dominant (a_ii = row abs-sum), b iid U(-1,1): converges to
    eta <= 1e-14; the solution agrees with the oracle's FP64 solve."""
    n = 2000
    announce("mixed diag-dominant n=%d %s %s" % (n, prec, solver))
    A = synth.diag_dominant(12, 0, n)
    b = synth.uniform(12, 1, n, 1)[:, 0]
    x, rep = _mixed(A, b, solver, prec)
    assert rep["status_name"] == "converged", rep
    assert rep["backward_error"] <= 1e-14
    assert eta_host(A, x, b) <= 1.5e-14
    import oracle
    LUo, ipo, info = oracle.getrf(A, nthreads=8)
    xo, st = oracle.getrs(LUo, ipo, b)
    kappa = np.linalg.cond(A, np.inf)
    fwd = np.abs(x - xo).max() / np.abs(xo).max()
    assert fwd <= 4 * kappa * (1e-14 + n * checks.U64), (fwd, kappa)


@pytest.mark.parametrize("solver", ["classical", "gmres"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_mixed_kappa(solver, prec, kappa):
    """A = U diag(sigma) V^T with condition number kappa: either converged
    (eta <= 1e-14, confirmed on the host) or an honest non-convergence status
    whose reported eta is that of the returned iterate."""
    n = 1024
    announce("mixed kappa=%g n=%d %s %s" % (kappa, n, prec, solver))
    A = synth.kappa_matrix(13, n, kappa)
    b = synth.uniform(13, 1, n, 1)[:, 0]
    x, rep = _mixed(A, b, solver, prec)
    eh = eta_host(A, x, b)
    print("kappa=%g %s %s: %s iters=%d inner=%d eta=%.3g host=%.3g" % (
        kappa, prec, solver, rep["status_name"], rep["iters"], rep["inner_iters"], rep["backward_error"], eh))
    assert rep["status_name"] in ("converged", "stagnated", "diverged", "maxiter")
    # the device eta uses an FP64 residual: agreement up to its rounding
    assert abs(eh - rep["backward_error"]) <= 0.05 * rep["backward_error"] + 5e-15
    if rep["status_name"] == "converged":
        assert eh <= 1.5e-14
    # convergence is required where the theory of the two schemes promises it:
    # the low-precision factors are a useful preconditioner while u_low*kappa
    # stays moderate (GMRES-IR), and classical refinement contracts while it is
    # well below one
    if solver == "gmres" and U_LOW[prec] * kappa <= 5:
        assert rep["status_name"] == "converged"
    if solver == "classical" and U_LOW[prec] * kappa <= 0.1:
        assert rep["status_name"] == "converged"


def test_mixed_multi_rhs_and_ld():
    """Several right-hand sides with padded leading dimensions."""
    n, nrhs = 900, 3
    announce("mixed multi-rhs n=%d nrhs=%d" % (n, nrhs))
    A = synth.diag_dominant(14, 0, n)
    B = synth.uniform(14, 1, n, nrhs)
    big = torch.zeros(n, n + 5, dtype=torch.float64, device="cuda").t()  # ld = n + 5
    dA = big[:n, :n]
    dA.copy_(torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t())
    bigB = torch.zeros(nrhs, n + 3, dtype=torch.float64, device="cuda").t()
    dB = bigB[:n]
    dB.copy_(torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t())
    bigX = torch.zeros(nrhs, n + 7, dtype=torch.float64, device="cuda").t()
    dX = bigX[:n]
    rep = lupp.lupp_dgesv_mixed(dA, dB, dX, lupp.ir_opts("gmres", factor_prec="bf16"))
    torch.cuda.synchronize()
    X = to_host(dX)
    assert rep["status_name"] == "converged"
    for j in range(nrhs):
        assert eta_host(A, X[:, j], B[:, j]) <= 1.5e-14
    assert torch.all(bigX[n:] == 0)  # padding rows untouched


def test_mixed_singular():
    """An exactly zero column: the FP32 factorization reports it (info) and
    the status is singular; X is zero."""
    n = 400
    announce("mixed singular n=%d" % n)
    A = synth.uniform(15, 0, n, n)
    A[:, 123] = 0.0
    b = synth.uniform(15, 1, n, 1)[:, 0]
    x, rep = _mixed(A, b, "classical", "fp16")
    assert rep["status_name"] == "singular" and rep["info"] == 124
    assert not np.any(x)


@pytest.mark.parametrize("solver", ["classical", "gmres"])
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_mixed_nonfinite_input(solver, prec):
    """A NaN and an Inf in A are outside the contract, but the call returns
    normally with a status that does not claim convergence."""
    n = 600
    announce("mixed non-finite n=%d %s %s" % (n, prec, solver))
    A = synth.uniform(17, 0, n, n)
    A[10, 20] = np.nan
    A[300, 5] = np.inf
    b = synth.uniform(17, 1, n, 1)[:, 0]
    _, rep = _mixed(A, b, solver, prec)
    assert rep["status_name"] in ("diverged", "stagnated", "maxiter", "singular"), rep


def test_mixed_fallback_fp64():
    """One FP8 classical iteration cannot reach 1e-14: MAXITER, then the FP64
    fallback solves the system."""
    n = 700
    announce("mixed fallback n=%d" % n)
    A = synth.uniform(16, 0, n, n)
    b = synth.uniform(16, 1, n, 1)[:, 0]
    x, rep = _mixed(A, b, "classical", "fp8", max_iter=1, fallback_fp64=1)
    assert rep["fallback_used"] == 1 and rep["status_name"] in ("maxiter", "diverged")
    assert eta_host(A, x, b) <= 8 * n * checks.U64


def test_mixed_bad_options():
    n = 64
    announce("mixed bad options")
    A = synth.diag_dominant(17, 0, n)
    b = synth.uniform(17, 1, n, 1)[:, 0]
    for kw in ({"gmres_restart": 0}, {"gmres_restart": 61}, {"tol": 0.0}, {"max_iter": 0}, {"factor_prec": 9},
               {"inner_tol": 1.0}):
        prec = kw.pop("factor_prec", "bf16")
        with pytest.raises(lupp.LuppError) as ei:
            _mixed(A, b, "gmres", prec, **kw)
        assert ei.value.rc == -10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,nrhs", [(1500, 1), (1500, 2), (64, 1), (65, 2), (3000, 1)])
def test_getrs_wavefront(dtype, n, nrhs):
    """One or two right-hand sides take the one-launch triangular solve and
    the interchanges in runs of 512."""
    announce("getrs wavefront n=%d nrhs=%d %s" % (n, nrhs, dtype))
    npdt = np.float64 if dtype == "f64" else np.float32
    A = synth.uniform(18, 0, n, n).astype(npdt)
    B = synth.uniform(18, 1, n, nrhs).astype(npdt)
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
