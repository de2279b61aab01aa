"""The paper's evaluation protocol on the Jacobi region (Sec. 4, the
"GPU threads" and "CPU-GPU execution" methodology), on one GPU.

Comparators, all measured against one exhaustive table (every variant of
every input timed: warmup 1, median of 5):

* Static default -- the 256-thread direct GPU kernel (the offload default
  team size, Sec. 4 "GPU threads"); Static best -- the one variant with the
  least total time over all inputs.
* Adaptive-100 -- a model trained on the profiles of all inputs and all
  variants, evaluated on the same inputs (Sec. 4 "CPU-GPU execution").
* Adaptive-25 / 50 / 75 -- K-fold-style subsets: the inputs are split into
  K = 4 equal groups, a fraction f of the groups trains a model and the
  others test it; the groups rotate so every input is trained on and
  tested at least once, and the split is redrawn 10 times from a shuffled
  order.
* Online -- one run of an iterative application: the region starts
  untrained, explores every variant once (RoundRobin), trains when it has
  as many unique samples as variants, and uses the model for the remaining
  iterations (Sec. 4 "GPU threads", Online).  This one runs the library's
  own region_run loop on the inputs and sums the recorded times; it is run
  over all variants and over the GPU variants alone (the paper's
  GPU-threads setting, where exploring costs little).

Models: the library's MLP cost model (GPU-trained) and the paper's depth-2
decision tree, each trained through the C ABI from region_record records.

Usage: python -m paper_2303_08873_amd.protocol [--inputs 1000] [--online 100]
       [--iters 100] [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

K = 4
RESHUFFLES = 10
FRACTIONS = (1, 2, 3)  # groups of K used for training: Adaptive-25 / 50 / 75


def _log(msg):
    print(f"[protocol] {msg}", file=sys.stderr, flush=True)


def kfold_groups(count: int, k: int, seed: int, reshuffle: int) -> list:
    """Reshuffle `reshuffle` of `count` inputs into k groups of equal size
    (up to one): the order sorts SplitMix64 keys of substream(seed, 40 +
    reshuffle) (stable), group g takes positions [g*count//k, (g+1)*count//k)."""
    import synth
    keys = synth.splitmix64(synth.substream(seed, 40 + reshuffle), count)
    order = np.argsort(keys, kind="stable")
    return [order[g * count // k:(g + 1) * count // k] for g in range(k)]


def rotations(k: int, m: int) -> list:
    """Training group sets for m of k groups: groups t .. t+m-1 (mod k) for
    t = 0..k-1, so every group is in some training set and (m < k) in some
    test set."""
    return [sorted((t + d) % k for d in range(m)) for t in range(k)]


def _metrics(t_sel, t_best, t_static):
    r = t_sel / t_best
    return {"mean_speedup_vs_static": float(np.mean(t_static / t_sel)),
            "geomean_regret_pct": float((np.exp(np.mean(np.log(r))) - 1) * 100),
            "hit_rate": float(np.mean(r <= 1.0 + 1e-12)),
            "aggregate_speedup_vs_static": float(t_static.sum() / t_sel.sum())}


def _train_and_select(ao, variants, model_type, feats, table, train_idx, test_idx, tag, epochs):
    """A fresh region of `model_type`, fed the exhaustive records of the
    training inputs, trained, asked for the test inputs' variants."""
    V = table.shape[1]
    h = ao.region_declare_variants(f"protocol_{tag}", ao.AO_JACOBI7_F64, variants,
                                   min_train_data=10 ** 9, model_type=model_type)
    try:
        for q in train_idx:
            for v in range(V):
                ao.region_record(h, feats[q], v, float(table[q, v]))
        if model_type == "mlp":
            ao.selector_train(h, epochs=epochs)
        else:
            ao.selector_train(h)
        _, ids = ao.selector_select(h, [feats[q] for q in test_idx])
    finally:
        ao.region_destroy(h)
    return np.array(ids)


def run(n_inputs=1000, n_online=100, iters=100, seed=40, max_dim=512, epochs=200, out=None):
    import torch

    import synth

    from . import _lib as ao
    from .variants import STATIC_DEFAULT, jacobi_variants_sweep

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    variants = jacobi_variants_sweep()
    V = len(variants)
    nmax = max_dim ** 3
    u0_d = synth.u01_torch(4242, nmax, dev)
    out_d = torch.empty_like(u0_d)
    u0_h = torch.empty(nmax, dtype=torch.float64).pin_memory()
    u0_h.copy_(u0_d)
    out_h = torch.empty(nmax, dtype=torch.float64).pin_memory()
    torch.cuda.synchronize()

    dims, sw, res = synth.selector_shapes(n_inputs, seed, hi=max_dim)

    def args_for(q):
        nx, ny, nz = (int(v) for v in dims[q])
        if res[q]:
            return ao.jacobi_args(u0_d, out_d, nx, ny, nz, int(sw[q]), 1)
        return ao.jacobi_args(u0_h, out_h, nx, ny, nz, int(sw[q]), 0)

    # the exhaustive table (the yardstick of every comparator)
    exh = ao.region_declare_variants(f"protocol_table_{seed}", ao.AO_JACOBI7_F64, variants,
                                       min_train_data=10 ** 9, model_type="exhaustive")
    table = np.zeros((n_inputs, V))
    feats = []
    t0 = time.perf_counter()
    for q in range(n_inputs):
        a = args_for(q)
        table[q] = ao.region_profile(exh, a, warmup=1, reps=5, stream=st, num_variants=V)
        feats.append(list(ao.region_features(exh, a)))
        if (q + 1) % 200 == 0:
            _log(f"exhaustive table: {q + 1} inputs ({time.perf_counter() - t0:.0f} s)")
    ao.region_destroy(exh)
    t_best = table.min(axis=1)
    t_static = table[:, STATIC_DEFAULT]
    every = np.arange(n_inputs)
    result = {"inputs": n_inputs, "variants": V, "table_protocol": "warmup 1, median of 5",
              "table_seconds": time.perf_counter() - t0}
    static_best = int(np.argmin(table.sum(axis=0)))
    result["static_default"] = _metrics(t_static, t_best, t_static)
    result["static_best"] = dict(_metrics(table[:, static_best], t_best, t_static),
                                 variant=static_best)

    for model in ("mlp", "dtree"):
        t0 = time.perf_counter()
        ids = _train_and_select(ao, variants, model, feats, table, every, every,
                                f"{model}_a100_{seed}", epochs)
        result[f"adaptive_100_{model}"] = _metrics(table[every, ids], t_best, t_static)
        _log(f"Adaptive-100 {model}: {result[f'adaptive_100_{model}']} "
             f"({time.perf_counter() - t0:.1f} s)")
        for m in FRACTIONS:
            per_model = []
            pooled_sel, pooled_idx = [], []
            for r in range(RESHUFFLES):
                groups = kfold_groups(n_inputs, K, seed, r)
                for t, train_groups in enumerate(rotations(K, m)):
                    train_idx = np.concatenate([groups[g] for g in train_groups])
                    test_idx = np.concatenate([groups[g] for g in range(K) if g not in train_groups])
                    ids = _train_and_select(ao, variants, model, feats, table, train_idx, test_idx,
                                            f"{model}_f{m}_{r}_{t}_{seed}", epochs)
                    sel = table[test_idx, ids]
                    per_model.append(_metrics(sel, t_best[test_idx], t_static[test_idx]))
                    pooled_sel.append(sel)
                    pooled_idx.append(test_idx)
            sel = np.concatenate(pooled_sel)
            idx = np.concatenate(pooled_idx)
            sp = np.array([pm["mean_speedup_vs_static"] for pm in per_model])
            result[f"adaptive_{25 * m}_{model}"] = dict(
                _metrics(sel, t_best[idx], t_static[idx]), models=len(per_model),
                model_speedup_min=float(sp.min()), model_speedup_max=float(sp.max()))
            _log(f"Adaptive-{25 * m} {model}: {result[f'adaptive_{25 * m}_{model}']}")

    # Online: the library's own explore -> train -> exploit loop per input,
    # over all variants (exploration includes the host variants) and over
    # the GPU variants alone (the paper's GPU-threads setting)
    online = {}
    gpu_ids = [v for v in range(V) if variants[v].target == ao.AO_TARGET_GPU]
    for vset_name, vids in (("all_variants", list(range(V))), ("gpu_variants", gpu_ids)):
        for model in ("mlp", "dtree"):
            tot, tot_static, tot_best, per = 0.0, 0.0, 0.0, []
            picks_best = 0
            nq = min(n_online, n_inputs)
            t0 = time.perf_counter()
            for q in range(nq):
                h = ao.region_declare_variants(f"protocol_online_{vset_name}_{model}_{seed}_{q}",
                                               ao.AO_JACOBI7_F64, [variants[v] for v in vids],
                                               model_type=model)  # min_train_data = variants
                a = args_for(q)
                for _ in range(iters):
                    ao.region_run(h, a, stream=st)
                torch.cuda.synchronize()
                _, chosen, seconds = ao.region_records(h)
                run_t = float(np.sum(seconds))
                explored = np.array(seconds[:len(vids)])
                picks_best += int(chosen[-1] == int(np.argmin(explored)))
                ao.region_destroy(h)
                best_q = float(table[q, vids].min())
                per.append(iters * t_static[q] / run_t)
                tot += run_t
                tot_static += iters * t_static[q]
                tot_best += iters * best_q
            online[f"{vset_name}_{model}"] = {
                "inputs": nq, "iterations": iters, "variants": len(vids),
                "mean_speedup_vs_static": float(np.mean(per)),
                "aggregate_speedup_vs_static": float(tot_static / tot),
                "aggregate_regret_vs_best_pct": float((tot / tot_best - 1) * 100),
                "final_choice_is_fastest_explored": picks_best / max(1, nq),
                "seconds": time.perf_counter() - t0}
            _log(f"Online {vset_name} {model}: {online[f'{vset_name}_{model}']}")
    result["online"] = online
    _log(json.dumps(result))
    if out:
        with open(out, "w") as fh:
            json.dump(result, fh, indent=1)
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--inputs", type=int, default=1000)
    ap.add_argument("--online", type=int, default=100)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    r = run(a.inputs, a.online, a.iters, epochs=a.epochs, out=a.out)
    print(json.dumps(r))


if __name__ == "__main__":
    main()
