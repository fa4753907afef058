"""Autotuner of the batched schedules: sweep, choose, keep.

    python -m paper_2104_05782_amd.autotune [--per-bucket N] [--out PATH]

A schedule of the batched calls (include/lupp.h, lupp_batched_schedule) sorts
the systems into up to six size classes, each one persistent launch of a
compiled kernel shape with a grid of some percent of the workgroups of that
shape that fit on the device at once.  The sweep measures the library's own
batched call, captured in a HIP graph as it is meant to be used, on synthetic
systems (entries uniform on [-1, 1)):

1. Eight buckets of orders (16b, 16b + 16] (at least 8), ``per_bucket``
   systems each, each bucket alone under every shape that holds it.
2. Every split of the buckets into at most six contiguous classes, each class
   with the shape of least summed time over its buckets (weighted by how many
   orders of [8, 128] each bucket holds), ranked by that summed time.
3. The six best splits and the best single-class schedule (one launch for the
   whole batch), timed on a mixed batch of 8 * ``per_bucket`` systems with
   orders uniform on [8, 128] against the library's initial schedule.  A
   schedule replaces the best so far only when it is at least 3 % faster (the
   spread between replays is a few percent).
4. Each class's grid at 75 and 50 %, one class at a time, kept when 3 %
   faster.

Every time is the median of seven graph replays after one untimed replay,
inputs restored before each replay outside the timed interval.  The choice is
installed in the handle and can be written to a JSON cache keyed by GPU
architecture (``tuned/batched.json`` in the package by default); every handle
created through the binding installs the cached schedules of its device's
architecture.  Schedules change speed only: every kernel shape computes the
same factors, pivots and solutions bit for bit.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "batched.json")
DTYPES = ("f64", "f32")
BUCKETS = 8
MAX_CLASSES = 6
NMAX = 128


def device_arch(device: int | None = None) -> str:
    """gfx name of a device (e.g. "gfx950"), without feature suffixes."""
    import torch
    d = torch.cuda.current_device() if device is None else device
    return torch.cuda.get_device_properties(d).gcnArchName.split(":")[0]


def load(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply_cached(handle, path: str = CACHE) -> dict:
    """Install the cached schedules for the handle's device; returns what was
    installed, by dtype."""
    cache = load(path)
    entry = cache.get(device_arch(handle.device), {})
    done = {}
    for dt in DTYPES:
        if dt in entry:
            handle.set_batched_schedule(dt, entry[dt]["schedule"])
            done[dt] = entry[dt]["schedule"]
    return done


class _Batch:
    """A packed batch on the device with a pristine copy of its inputs."""

    def __init__(self, sizes: np.ndarray, dtype: str, seed: int):
        import torch
        tdt = torch.float64 if dtype == "f64" else torch.float32
        n64 = sizes.astype(np.int64)
        a_off = np.zeros(len(sizes), np.int64)
        a_off[1:] = np.cumsum(n64 * n64)[:-1]
        p_off = np.zeros(len(sizes), np.int64)
        p_off[1:] = np.cumsum(n64)[:-1]
        g = torch.Generator(device="cuda").manual_seed(seed)
        na, nb = int((n64 * n64).sum()), int(n64.sum())
        self.A0 = torch.rand(na + 1, generator=g, dtype=torch.float64, device="cuda").mul_(2).sub_(1).to(tdt)
        self.B0 = torch.rand(nb + 1, generator=g, dtype=torch.float64, device="cuda").mul_(2).sub_(1).to(tdt)
        self.A, self.B = self.A0.clone(), self.B0.clone()
        self.dn = torch.from_numpy(sizes.astype(np.int32)).cuda()
        self.aoff = torch.from_numpy(a_off).cuda()
        self.poff = torch.from_numpy(p_off).cuda()
        self.ipiv = torch.zeros(nb + 1, dtype=torch.int32, device="cuda")
        self.info = torch.zeros(len(sizes), dtype=torch.int32, device="cuda")

    def call(self, handle):
        from ._binding import lupp_xgesv_batched
        lupp_xgesv_batched(self.dn, self.A, self.aoff, self.ipiv, self.poff, self.B, self.poff, self.info,
                           handle=handle)

    def restore(self):
        self.A.copy_(self.A0)
        self.B.copy_(self.B0)


def graph_time(handle, batch: _Batch, nrep: int = 7) -> float:
    """Median time (ms) of nrep replays of the batched call captured in a
    HIP graph, after one untimed replay; inputs restored before each."""
    import torch
    batch.call(handle)  # class-list workspace sized before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    batch.restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.call(handle)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for r in range(nrep + 1):
        batch.restore()
        torch.cuda.synchronize()
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        if r:
            ts.append(e0.elapsed_time(e1))
    del g
    return float(np.median(ts))


def _splits():
    """Every split of the buckets into at most MAX_CLASSES contiguous classes,
    as lists of (first bucket, last bucket)."""
    for cut in range(1 << (BUCKETS - 1)):
        if bin(cut).count("1") + 1 > MAX_CLASSES:
            continue
        out, b0 = [], 0
        for b in range(BUCKETS):
            if b == BUCKETS - 1 or (cut >> b) & 1:
                out.append((b0, b))
                b0 = b + 1
        yield out


def sweep(handle, dtype: str, per_bucket: int = 2500, seed: int = 20210512) -> dict:
    """Steps 1-4 above on the handle's device; installs and returns the
    choice with every measurement taken."""
    from ._binding import batched_shapes
    shapes = batched_shapes()
    big = max(range(len(shapes)), key=lambda v: (shapes[v]["nmax"], -v))
    rng = np.random.default_rng(seed)
    initial = handle.batched_schedule(dtype)
    handle.set_batched_schedule(dtype, None)
    init = handle.batched_schedule(dtype)
    weight = [9.0] + [16.0] * (BUCKETS - 1)  # orders of [8, 128] per bucket

    # 1. buckets alone
    table = {}
    for b in range(BUCKETS):
        lo, hi = max(8, 16 * b + 1), 16 * b + 16
        batch = _Batch(rng.integers(lo, hi + 1, size=per_bucket), dtype, seed + b)
        for v, sh in enumerate(shapes):
            if sh["nmax"] < hi:
                continue
            if hi == NMAX:
                s = {"nclass": 1, "nmax": [NMAX], "shape": [v], "grid_pct": [100]}
            else:  # the bucket is all in class 0; class 1 gets no system
                s = {"nclass": 2, "nmax": [hi, NMAX], "shape": [v, big], "grid_pct": [100, 100]}
            handle.set_batched_schedule(dtype, s)
            table[(b, v)] = graph_time(handle, batch)
        del batch

    # 2. model ranking of the splits
    def best_shape(b0, b1):
        best = None
        for v, sh in enumerate(shapes):
            if sh["nmax"] < 16 * b1 + 16:
                continue
            cost = sum(weight[q] * table[(q, v)] for q in range(b0, b1 + 1))
            if best is None or cost < best[0]:
                best = (cost, v)
        return best

    ranked = []
    for split in _splits():
        cost, sched = 0.0, {"nclass": len(split), "nmax": [], "shape": [], "grid_pct": []}
        for b0, b1 in split:
            c, v = best_shape(b0, b1)
            cost += c
            sched["nmax"].append(16 * b1 + 16)
            sched["shape"].append(v)
            sched["grid_pct"].append(100)
        ranked.append((cost, sched))
    ranked.sort(key=lambda t: t[0])
    c1, v1 = best_shape(0, BUCKETS - 1)
    trials = [s for _, s in ranked[:6]] + [{"nclass": 1, "nmax": [NMAX], "shape": [v1], "grid_pct": [100]}]

    # 3. the mixed batch decides, against the initial schedule
    mixed = _Batch(rng.integers(8, NMAX + 1, size=BUCKETS * per_bucket), dtype, seed + 100)
    handle.set_batched_schedule(dtype, init)
    init_ms = graph_time(handle, mixed)
    best, best_ms, timed = init, init_ms, [{"schedule": init, "ms": init_ms, "initial": True}]
    for s in trials:
        handle.set_batched_schedule(dtype, s)
        ms = graph_time(handle, mixed)
        timed.append({"schedule": s, "ms": ms})
        if ms < 0.97 * best_ms:
            best, best_ms = s, ms

    # 4. grids, one class at a time
    for c in range(best["nclass"]):
        for pct in (75, 50):
            s = json.loads(json.dumps(best))
            s["grid_pct"][c] = pct
            handle.set_batched_schedule(dtype, s)
            ms = graph_time(handle, mixed)
            timed.append({"schedule": s, "ms": ms})
            if ms < 0.97 * best_ms:
                best, best_ms = s, ms
    handle.set_batched_schedule(dtype, best)
    del mixed
    return {"schedule": best, "tuned_ms": best_ms, "default_ms": init_ms, "systems_per_bucket": per_bucket,
            "previous": initial, "mixed_batch_trials": timed,
            "bucket_ms": {"%d:%d" % k: round(v, 4) for k, v in sorted(table.items())}}


def tune(per_bucket: int = 2500, path: str | None = CACHE) -> dict:
    """Sweep both precisions on the current device; write the cache entry of
    its architecture when path is given."""
    from ._binding import Handle, batched_shapes
    h = Handle(tuned=False)
    result = {dt: sweep(h, dt, per_bucket) for dt in DTYPES}
    shapes = batched_shapes()
    for dt in DTYPES:
        result[dt]["shapes"] = [shapes[v] for v in result[dt]["schedule"]["shape"]]
    h.close()
    if path:
        cache = load(path)
        cache[device_arch()] = result
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
            f.write("\n")
    return result


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--per-bucket", type=int, default=2500)
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    r = tune(a.per_bucket, a.out)
    print(json.dumps({dt: {k: r[dt][k] for k in ("schedule", "tuned_ms", "default_ms")} for dt in DTYPES}))
