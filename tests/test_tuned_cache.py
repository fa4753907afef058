"""The committed autotuner cache is well formed: per architecture and
precision, a schedule the library would accept (class bounds increasing and
ending at 128, each class's shape holding its largest order, grids in
1..100), checked against the library's shape table (host-only call)."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_2104_05782_amd", "tuned", "batched.json")


@pytest.mark.skipif(not os.path.exists(CACHE), reason="no cache committed")
def test_cache_schedules_valid():
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2104_05782_amd", "liblupp.so"))
    nshape = lib.lupp_batched_shape_count()
    nmax_of = []
    for v in range(nshape):
        a = [ctypes.c_int32() for _ in range(4)]
        assert lib.lupp_batched_shape(v, *[ctypes.byref(x) for x in a]) == 0
        nmax_of.append(a[3].value)
    cache = json.load(open(CACHE))
    assert cache
    for arch, entry in cache.items():
        assert arch.startswith("gfx")
        for dt in ("f64", "f32"):
            s = entry[dt]["schedule"]
            k = s["nclass"]
            assert 1 <= k <= 6 and len(s["nmax"]) == len(s["shape"]) == len(s["grid_pct"]) == k
            assert s["nmax"][-1] == 128 and all(a < b for a, b in zip(s["nmax"], s["nmax"][1:]))
            assert all(0 <= v < nshape and nmax_of[v] >= ub for v, ub in zip(s["shape"], s["nmax"]))
            assert all(1 <= g <= 100 for g in s["grid_pct"])
            assert entry[dt]["tuned_ms"] <= entry[dt]["default_ms"]
