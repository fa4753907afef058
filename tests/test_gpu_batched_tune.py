"""Batched schedules and the autotuner, through the C ABI.

Every compiled kernel shape must give the factors, pivots, info and
solutions of the initial schedule bit for bit (the elimination order of each
entry does not depend on how columns are dealt to wavefronts); the
autotuner's choice is a valid schedule, no slower than the initial one on its
own sweep, and gives the same results bit for bit; invalid schedules are
refused.  The initial schedule's results are checked against the CPU oracle
by the batched parity tests."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - GPU machine only
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_05782_amd as lupp  # noqa: E402
from gpu_util import announce  # noqa: E402


def _batch(count, seed, dtype, nmin=1, nmax=128):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count).astype(np.int32)
    a_off = np.zeros(count, np.int64)
    b_off = np.zeros(count, np.int64)
    a_off[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    b_off[1:] = np.cumsum(sizes.astype(np.int64))[:-1]
    A = synth.uniform(seed, 0, int((sizes.astype(np.int64) ** 2).sum()) + 1, 1)[:, 0].astype(dtype)
    B = synth.uniform(seed, 1, int(sizes.sum()) + 1, 1)[:, 0].astype(dtype)
    return sizes, a_off, b_off, A, B


def _solve(handle, sizes, a_off, b_off, A, B):
    dn = torch.from_numpy(sizes).cuda()
    dA = torch.from_numpy(A.copy()).cuda()
    dB = torch.from_numpy(B.copy()).cuda()
    ipiv, p_off, info = lupp.gesv_batched(dn, dA, torch.from_numpy(a_off).cuda(), dB,
                                          torch.from_numpy(b_off).cuda(), handle)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (dA, ipiv, info, dB)]


def _same(r, g):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(r, g))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_every_shape_bit_identical(dtype):
    dt = "f64" if dtype == np.float64 else "f32"
    shapes = lupp.batched_shapes()
    h = lupp.Handle(tuned=False)
    data = _batch(1500, 20210701, dtype)
    ref = _solve(h, *data)
    assert (ref[2] == 0).all()
    last = max(range(len(shapes)), key=lambda v: (shapes[v]["nmax"], -v))  # a shape holding 128
    for v, sh in enumerate(shapes):
        announce("batched shape %d %s (%s)" % (v, sh, dt))
        if sh["nmax"] >= 128:
            sched = {"nclass": 1, "nmax": [128], "shape": [v], "grid_pct": [100]}
        else:
            sched = {"nclass": 2, "nmax": [sh["nmax"], 128], "shape": [v, last], "grid_pct": [60, 100]}
        h.set_batched_schedule(dt, sched)
        assert h.batched_schedule(dt) == sched
        assert _same(ref, _solve(h, *data)), "shape %d differs" % v
    h.set_batched_schedule(dt, None)
    h.close()


def test_schedule_validation():
    h = lupp.Handle(tuned=False)
    init = h.batched_schedule("f64")
    assert init["nmax"][-1] == 128
    shapes = lupp.batched_shapes()
    small = min(range(len(shapes)), key=lambda v: shapes[v]["nmax"])
    bad = [
        {"nclass": 1, "nmax": [96], "shape": [init["shape"][-1]], "grid_pct": [100]},           # does not end at 128
        {"nclass": 2, "nmax": [64, 64], "shape": [init["shape"][-1]] * 2, "grid_pct": [100, 100]},  # not increasing
        {"nclass": 1, "nmax": [128], "shape": [small], "grid_pct": [100]},                       # shape too small
        {"nclass": 1, "nmax": [128], "shape": [init["shape"][-1]], "grid_pct": [0]},            # grid
        {"nclass": 1, "nmax": [128], "shape": [len(shapes)], "grid_pct": [100]},                # no such shape
        {"nclass": 7, "nmax": [128] * 7, "shape": [0] * 7, "grid_pct": [100] * 7},              # too many classes
    ]
    for b in bad:
        with pytest.raises(lupp.LuppError) as e:
            h.set_batched_schedule("f64", b)
        assert e.value.rc == -3, b
    assert h.batched_schedule("f64") == init
    h.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_autotune_choice_valid_and_bit_identical(dtype):
    dt = "f64" if dtype == np.float64 else "f32"
    announce("batched autotune %s" % dt)
    h = lupp.Handle(tuned=False)
    data = _batch(2000, 20210702, dtype, nmin=8)
    ref = _solve(h, *data)
    from paper_2104_05782_amd.autotune import sweep
    r = sweep(h, dt, 64)
    s = r["schedule"]
    assert h.batched_schedule(dt) == s
    shapes = lupp.batched_shapes()
    assert s["nmax"][-1] == 128 and all(a < b for a, b in zip(s["nmax"], s["nmax"][1:]))
    assert all(shapes[v]["nmax"] >= ub for v, ub in zip(s["shape"], s["nmax"]))
    assert 0 < r["tuned_ms"] <= r["default_ms"]
    print("autotune %s: %s" % (dt, r))
    assert _same(ref, _solve(h, *data))
    h.close()
