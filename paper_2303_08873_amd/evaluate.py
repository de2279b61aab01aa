"""Learned-selector evaluation of the Jacobi region (one GPU).

Training data come from the method itself: a region with the 11 size-sweep
variants runs every training shape once per variant under RoundRobin
exploration (Sec. 2 Apollo paragraph), each run profiled.  The cost model
is trained on those records by the library's GPU kernels.  Held-out shapes
are timed exhaustively (every variant, warmup + repetitions, median) -- the
table that defines the best variant and every regret below.  Compared:
the learned selector, the static default (64x4 = 256-thread direct kernel,
the OpenMP offload default team size, Sec. 4 "GPU threads"), and the
untrained network.  Selection cost: the measured latency of a cold
selector_select against the exhaustive selector's cost sum_v t_v.

Usage: python -m paper_2303_08873_amd.evaluate [--train 2000] [--test 2000]
       [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def _log(msg):
    print(f"[evaluate] {msg}", file=sys.stderr, flush=True)


def _stats(t_sel, t_best):
    r = t_sel / t_best
    return {"geomean_regret_pct": float((np.exp(np.mean(np.log(r))) - 1) * 100),
            "mean_regret_pct": float((np.mean(r) - 1) * 100),
            "p95_regret_pct": float((np.percentile(r, 95) - 1) * 100),
            "hit_rate": float(np.mean(r <= 1.0 + 1e-12)),
            "aggregate_regret_pct": float((t_sel.sum() / t_best.sum() - 1) * 100)}


class ShapeBuffers:
    """One input/output pair per residency, sized for the largest shape of
    the workload; every shape uses a prefix (values U[0,1) from seed 4242)."""

    def __init__(self, max_dim, dev):
        import torch

        import synth
        nmax = max_dim ** 3
        self.u0_d = synth.u01_torch(4242, nmax, dev)
        self.out_d = torch.empty_like(self.u0_d)
        self.u0_h = torch.empty(nmax, dtype=torch.float64).pin_memory()
        self.u0_h.copy_(self.u0_d)
        self.out_h = torch.empty(nmax, dtype=torch.float64).pin_memory()
        torch.cuda.synchronize()

    def args(self, dims, sweeps, resident):
        from . import _lib as ao
        nx, ny, nz = (int(v) for v in dims)
        if resident:
            return ao.jacobi_args(self.u0_d, self.out_d, nx, ny, nz, int(sweeps), 1)
        return ao.jacobi_args(self.u0_h, self.out_h, nx, ny, nz, int(sweeps), 0)


def shape_features(dims, sweeps, resident):
    """The six cost-model features of a Jacobi shape (Sec. 3.1 features
    clause): log2 of each extent, sweeps, log2 of 16 N S bytes, residency."""
    n = int(np.prod(dims))
    return [math.log2(int(dims[0])), math.log2(int(dims[1])), math.log2(int(dims[2])),
            float(sweeps), math.log2(16.0 * n * int(sweeps)), float(resident)]


def collect_training(region, bufs, n_train, seed, max_dim, stream, V):
    """The method's own training data: every training shape runs V times
    under RoundRobin exploration, each run profiled and recorded.  Returns
    the seconds it took."""
    import torch

    import synth

    from . import _lib as ao
    dims, sw, res = synth.selector_shapes(n_train, seed, hi=max_dim)
    t0 = time.perf_counter()
    for q in range(n_train):
        a = bufs.args(dims[q], sw[q], res[q])
        for _ in range(V):
            ao.region_run(region, a, stream=stream)
        if (q + 1) % 500 == 0:
            torch.cuda.synchronize()
            _log(f"training runs: {(q + 1) * V} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def held_out_table(region, bufs, n_test, seed, max_dim, warmup, reps, stream, V):
    """Exhaustive table of the held-out shapes (every variant, `warmup`
    runs then the median of `reps`; not recorded) and their features."""
    import synth

    from . import _lib as ao
    tdims, tsw, tres = synth.selector_shapes(n_test, seed, hi=max_dim)
    table = np.zeros((n_test, V))
    feats = []
    t0 = time.perf_counter()
    for q in range(n_test):
        a = bufs.args(tdims[q], tsw[q], tres[q])
        table[q] = ao.region_profile(region, a, warmup=warmup, reps=reps, stream=stream,
                                     num_variants=V)
        feats.append(shape_features(tdims[q], tsw[q], tres[q]))
        if (q + 1) % 200 == 0:
            _log(f"exhaustive table: {q + 1} shapes ({time.perf_counter() - t0:.0f} s)")
    return table, feats, time.perf_counter() - t0


def judge(region, table, feats, epochs=200, untrained=True):
    """Train the region's cost model on its records and judge it on the
    held-out table: regret statistics of the learned selector, of the
    static default and of the untrained network, and the selection cost
    (cold selector_select latency against the exhaustive cost sum_v t_v)."""
    from . import _lib as ao
    from .variants import STATIC_DEFAULT
    n_test = table.shape[0]
    idx = np.arange(n_test)
    best = table.argmin(axis=1)
    t_best = table[idx, best]
    out = {"best_variant_histogram": np.bincount(best, minlength=table.shape[1]).tolist()}
    if untrained:
        # untrained network (initial weights, normalisation from the data)
        ao.selector_train(region, epochs=0)
        _, ids_u = ao.selector_select(region, feats)
        out["untrained_net"] = _stats(table[idx, np.array(ids_u)], t_best)
    t0 = time.perf_counter()
    loss = ao.selector_train(region, epochs=epochs)
    train_wall = time.perf_counter() - t0
    _, ids = ao.selector_select(region, feats)
    ids = np.array(ids)
    # cold single-vector selection latency (selector_select keeps no memo)
    lat = []
    for f in feats[:min(n_test, 500)]:
        t1 = time.perf_counter()
        ao.selector_select(region, [f])
        lat.append(time.perf_counter() - t1)
    lat = np.array(lat)
    exh_cost = table.sum(axis=1)[:lat.size]
    out.update({
        "train_final_loss": loss, "train_seconds": train_wall,
        "train_kernel_seconds": ao.region_stats(region).last_train_seconds,
        "learned": _stats(table[idx, ids], t_best),
        "static_default": _stats(table[:, STATIC_DEFAULT], t_best),
        "selection_latency_us_median": float(np.median(lat) * 1e6),
        "exhaustive_cost_us_median": float(np.median(exh_cost) * 1e6),
        "selection_cost_ratio_median": float(np.median(exh_cost / lat)),
        "learned_hist": np.bincount(ids, minlength=table.shape[1]).tolist(),
    })
    return out


def run(n_train=2000, n_test=2000, train_seed=4, test_seed=40, max_dim=512, warmup=1, reps=5,
        epochs=200, out=None):
    import torch

    from . import _lib as ao
    from .variants import jacobi_variants_sweep

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    V = len(jacobi_variants_sweep())
    bufs = ShapeBuffers(max_dim, dev)
    region = ao.region_declare_variants(f"eval_{train_seed}_{n_train}", ao.AO_JACOBI7_F64,
                                        jacobi_variants_sweep(), min_train_data=10 ** 9,
                                        model_type="mlp")
    collect_s = collect_training(region, bufs, n_train, train_seed, max_dim, st, V)
    stats0 = ao.region_stats(region)
    table, feats, table_s = held_out_table(region, bufs, n_test, test_seed, max_dim, warmup, reps,
                                           st, V)
    result = {"train_shapes": n_train, "test_shapes": n_test, "variants": V,
              "train_records": int(stats0.records), "train_unique": int(stats0.unique),
              "collect_seconds": collect_s, "table_seconds": table_s,
              "table_protocol": f"warmup {warmup}, median of {reps}"}
    result.update(judge(region, table, feats, epochs=epochs))
    result["selection_cost_ratio_with_protocol_median"] = \
        result["selection_cost_ratio_median"] * (warmup + reps)
    n_test = table.shape[0]
    t_best = table.min(axis=1)

    # the paper's model: depth-2 decision tree on the same records
    import os
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "records.bin")
        ao.region_save(region, path)
        dt = ao.region_declare_variants(f"eval_dt_{train_seed}_{n_train}", ao.AO_JACOBI7_F64,
                                        jacobi_variants_sweep(), min_train_data=10 ** 9,
                                        model_type="dtree")
        ao.region_load(dt, path)
    t0 = time.perf_counter()
    dt_err = ao.selector_train(dt)
    dt_train_s = time.perf_counter() - t0
    _, ids_dt = ao.selector_select(dt, feats)
    ids_dt = np.array(ids_dt)
    lat_dt = []
    for f in feats[:min(n_test, 500)]:
        t1 = time.perf_counter()
        ao.selector_select(dt, [f])
        lat_dt.append(time.perf_counter() - t1)
    ao.region_destroy(dt)
    result.update({
        "dtree_depth2": _stats(table[np.arange(n_test), ids_dt], t_best),
        "dtree_train_error": dt_err, "dtree_train_seconds": dt_train_s,
        "dtree_selection_latency_us_median": float(np.median(lat_dt) * 1e6),
    })
    _log(json.dumps(result))
    if out:
        with open(out, "w") as fh:
            json.dump(result, fh, indent=1)
    ao.region_destroy(region)
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--max-dim", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    r = run(a.train, a.test, max_dim=a.max_dim, reps=a.reps, epochs=a.epochs, out=a.out)
    print(json.dumps(r))


if __name__ == "__main__":
    main()
