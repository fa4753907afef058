"""GPU parity of the Householder QR (lupp_dgeqrf) against the CPU oracle
(oracle/qr.py, pinned to LAPACK's dgeqrf), through the C ABI.

Bars: R, the Householder vectors and tau agree with the oracle's within a
bound from the arithmetic (both are backward stable; the entries differ by
rounding in the reductions, amplified at most by the conditioning of the
leading columns: 1e3 * max(m, n) * u, relative to the column norms, on
random matrices whose leading blocks are well conditioned); the GPU's own
factors reproduce A (||A - Q R|| <= 30 max(m,n) u ||A||) with orthonormal columns
(||Q^T Q - I|| <= 30 m u for the first min(m, n) columns of Q, formed on the
host in FP64 from the GPU's vectors); closed forms bit for bit (triangular inputs: tau = 0, R = A);
repeated calls bit-identical."""
import numpy as np
import pytest

import synth
from oracle import qr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - GPU machine only
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_05782_amd as lupp  # noqa: E402
from gpu_util import announce, to_dev, to_host  # noqa: E402

U = 2.0 ** -53


def _gpu_qr(A, handle=None):
    dA = to_dev(A)
    h = handle or lupp.Handle()
    tau = lupp.geqrf(dA, h)
    h.sync()
    out = to_host(dA), tau.cpu().numpy()
    if handle is None:
        h.close()
    return out


def _check(A, F, t):
    m, n = A.shape
    k = min(m, n)
    Fo, to = qr.geqr2(A)
    colnorm = np.linalg.norm(A, axis=0).max()
    tol = 1e3 * max(m, n) * U
    assert np.abs(np.triu(F) - np.triu(Fo)).max() <= tol * colnorm, "R"
    assert np.abs(np.tril(F, -1) - np.tril(Fo, -1)).max() <= tol * max(1.0, np.abs(np.tril(Fo, -1)).max()), "V"
    assert np.abs(t - to).max() <= tol, "tau"
    Q = qr.form_q(F, t, k)  # the first k columns of Q
    R = np.triu(F)[:k, :]
    assert np.abs(Q @ R - A).max() <= 30 * max(m, n) * U * np.abs(A).sum(axis=0).max()
    assert np.abs(Q.T @ Q - np.eye(k)).max() <= 30 * m * U


@pytest.mark.parametrize("shape", [(64, 64), (500, 500), (1024, 333), (333, 1024), (1200, 1200), (3000, 400),
                                   (1, 1), (40, 1), (1, 40), (31, 31), (33, 65)])
def test_geqrf_matches_oracle(shape):
    m, n = shape
    announce("geqrf %dx%d" % shape)
    A = synth.uniform(20211001 + m, 0, m, n)
    F, t = _gpu_qr(A)
    _check(A, F, t)


def test_geqrf_many_workgroups():
    """m = 20000: the column-block kernel runs 40 cooperating workgroups."""
    m, n = 20000, 96
    announce("geqrf %dx%d" % (m, n))
    A = synth.uniform(20211002, 0, m, n)
    F, t = _gpu_qr(A)
    _check(A, F, t)


def test_geqrf_closed_forms_bit_exact():
    rng = np.random.default_rng(5)
    for A in (np.triu(rng.uniform(-1, 1, (100, 100))), np.diag(rng.uniform(0.5, 2, 70)),
              np.vstack([np.triu(rng.uniform(-1, 1, (40, 40))), np.zeros((30, 40))])):
        F, t = _gpu_qr(np.asfortranarray(A))
        assert np.array_equal(t, np.zeros_like(t))
        assert np.array_equal(F, A)


def test_geqrf_deterministic_and_empty():
    A = synth.uniform(20211003, 0, 3000, 800)
    h = lupp.Handle()
    F1, t1 = _gpu_qr(A, h)
    F2, t2 = _gpu_qr(A, h)
    h.close()
    assert np.array_equal(F1, F2) and np.array_equal(t1, t2)
    h = lupp.Handle()
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert lupp._binding._lib.lupp_dgeqrf(h.ptr, 0, 5, x.data_ptr(), 1, x.data_ptr()) == 0  # empty: nothing to do
    assert lupp._binding._lib.lupp_dgeqrf(h.ptr, 5, 0, x.data_ptr(), 5, x.data_ptr()) == 0
    h.sync()
    h.close()


@pytest.mark.parametrize("shape", [(9000, 9000), (12288, 6000), (6000, 12288), (20000, 4000), (33000, 2300),
                                   (2600, 1000)])
def test_geqrf_lookahead_bit_identical(shape):
    """Lookahead (the next outer block factored on the panel's CUs while the
    rest of the update runs on the others, for steps whose rest has at least
    2^26 rows x columns) gives the in-order factors and tau bit for bit: every
    product splits its rows as the whole update would.  m = 20000 uses the
    64-CU partition; m = 33000 exceeds both partitions for its first blocks,
    which then run in order; 2600 x 1000 never reaches the overlap size."""
    m, n = shape
    announce("geqrf lookahead %dx%d" % shape)
    g = torch.Generator(device="cuda").manual_seed(m + 7 * n)
    A0 = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    out = []
    for depth in (1, 0):
        h = lupp.Handle()
        h.set_option(4, depth)
        A = torch.empty_like(A0.t()).t()
        A.copy_(A0)
        tau = lupp.geqrf(A, h)
        h.sync()
        h.close()
        out.append((A, tau))
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][0], out[1][0])


def test_geqrf_argument_errors():
    h = lupp.Handle()
    A = to_dev(np.eye(4))
    tau = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = lupp._binding._lib
    assert lib.lupp_dgeqrf(h.ptr, -1, 4, A.data_ptr(), 4, tau.data_ptr()) == -2
    assert lib.lupp_dgeqrf(h.ptr, 4, -1, A.data_ptr(), 4, tau.data_ptr()) == -3
    assert lib.lupp_dgeqrf(h.ptr, 4, 4, A.data_ptr(), 3, tau.data_ptr()) == -5
    assert lib.lupp_dgeqrf(h.ptr, 4, 4, A.data_ptr(), 4, None) == -6
    assert lib.lupp_dgeqrf(h.ptr, 200000, 4, A.data_ptr(), 200000, tau.data_ptr()) == lupp._binding.ERR_UNSUPPORTED
    h.close()
