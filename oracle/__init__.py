"""CPU oracle of the adaptive-region hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct implementations of what the method computes,
written from the paper.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
and its Python binding never do, and the two share no code.

Contents (paper section cited on each function):
  * region arithmetic (serial C, ``oracle.c``): 7-point Jacobi, CSR SpMV in
    plain and in canonical pairwise order, weighted Jacobi relaxation on the
    canonical SpMV;
  * region features (Sec. 3.1 ``features`` clause);
  * numeric variant ranges (Sec. 3.1 ``variants`` clause);
  * RoundRobin exploration and the train trigger (Sec. 2, Apollo paragraph;
    Sec. 3.3 end of region);
  * the exhaustive selector that labels the fastest policy per feature tuple
    (Sec. 2, Apollo paragraph);
  * the MLP cost model, FP64, forward / backward / Adam (the learned
    selector that replaces the paper's depth-2 decision tree of Sec. 3.1
    ``model_type`` and Sec. 4; every detail of it is a reading, see
    ``mlp_*``);
  * the paper's own model, a CART decision-tree classifier on
    fastest-variant labels (``dtree_*``);
  * the K-fold subset construction of the evaluation protocol (Sec. 4,
    Adaptive-25/50/75) and the Online comparator's explore-then-exploit
    choice (Sec. 4, GPU threads).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from collections import OrderedDict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with contraction off (no fused multiply-add)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", os.path.join(_HERE, "oracle.c"), "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_jacobi7.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_spmv_plain.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.orc_spmv_canonical.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.orc_relax.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_double, ctypes.c_int, P]
        for f in (lib.orc_jacobi7, lib.orc_spmv_plain, lib.orc_spmv_canonical, lib.orc_relax):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# Region arithmetic
# --------------------------------------------------------------------------

def jacobi7(u0: np.ndarray, nx: int, ny: int, nz: int, sweeps: int) -> np.ndarray:
    """S sweeps of the 7-point FP64 Jacobi region (Heat-style stencil, Table 3):
    v = (((((xm+xp)+ym)+yp)+zm)+zp) * fl(1/6), ghost zeros outside the grid."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
    assert u0.size == nx * ny * nz
    out = np.empty_like(u0)
    rc = _load().orc_jacobi7(_ptr(u0), _ptr(out), nx, ny, nz, sweeps)
    if rc != 0:
        raise RuntimeError(f"orc_jacobi7 failed ({rc})")
    return out


def _csr_args(row_ptr, col, val, x):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return row_ptr, col, val, x


def spmv_plain(row_ptr, col, val, x) -> np.ndarray:
    """y = A x for CSR A (AMGMk-style sparse region, Table 3): left-to-right
    sum from +0.0 of separately rounded products."""
    row_ptr, col, val, x = _csr_args(row_ptr, col, val, x)
    n = row_ptr.size - 1
    y = np.empty(n, dtype=np.float64)
    rc = _load().orc_spmv_plain(n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    if rc != 0:
        raise RuntimeError(f"orc_spmv_plain failed ({rc})")
    return y


def spmv_canonical(row_ptr, col, val, x) -> np.ndarray:
    """y = A x with each row summed by the aligned pairwise tree over the
    row-local index (padding -0.0 to a power of two; empty row +0.0)."""
    row_ptr, col, val, x = _csr_args(row_ptr, col, val, x)
    n = row_ptr.size - 1
    y = np.empty(n, dtype=np.float64)
    rc = _load().orc_spmv_canonical(n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    if rc != 0:
        raise RuntimeError(f"orc_spmv_canonical failed ({rc})")
    return y


def relax(row_ptr, col, val, x, b, d, omega: float, sweeps: int) -> np.ndarray:
    """Weighted Jacobi relaxation x <- x + (omega * (b - A x)) / d, `sweeps`
    times (the AMGMk relax kernel, Table 3); A x in the canonical order, the
    update rounded step by step (subtract, multiply, divide, add)."""
    row_ptr, col, val, x = _csr_args(row_ptr, col, val, x)
    b = np.ascontiguousarray(b, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = row_ptr.size - 1
    y = np.empty(n, dtype=np.float64)
    rc = _load().orc_relax(n, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(b), _ptr(d),
                           float(omega), int(sweeps), _ptr(y))
    if rc != 0:
        raise RuntimeError(f"orc_relax failed ({rc})")
    return y


def relax_bytes(n: int, nnz: int) -> int:
    """Algorithmic bytes of one relaxation sweep: the SpMV's (matrix once,
    x once, the new x once) plus b and d once."""
    return spmv_bytes(n, nnz) + 16 * n


def jacobi_bytes(nx: int, ny: int, nz: int, sweeps: int) -> int:
    """Algorithmic bytes of a Jacobi region: each sweep reads and writes every
    FP64 point once (16 B per point per sweep)."""
    return 16 * nx * ny * nz * sweeps


def spmv_bytes(n: int, nnz: int) -> int:
    """Algorithmic bytes of one CSR SpMV: col+val per nonzero, row_ptr, x and y once."""
    return 12 * nnz + 4 * (n + 1) + 8 * n + 8 * n


# --------------------------------------------------------------------------
# Features (Sec. 3.1, ``features`` clause: program values fed to the model)
# --------------------------------------------------------------------------

def stencil_features(nx: int, ny: int, nz: int, sweeps: int, resident: int) -> np.ndarray:
    """[log2 nx, log2 ny, log2 nz, S, log2(bytes), device flag], FP32 as the
    Apollo feature values are floats (Table 1).  bytes = 16*N*S.  Reading
    for empty regions (the paper's feature values are never zero): an
    extent of 0 and a byte count of 0 enter as 0, the value of an extent of
    one."""
    b = jacobi_bytes(nx, ny, nz, sweeps)

    def lg(v):
        return math.log2(v) if v > 0 else 0.0

    f = [lg(nx), lg(ny), lg(nz), float(sweeps), lg(b), float(resident)]
    return np.asarray(f, dtype=np.float64).astype(np.float32)


def csr_features(row_ptr) -> np.ndarray:
    """[log2 n, log2 nnz, mean row length, log2(1 + variance), log2 max] of a
    CSR structure (population variance), FP32."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    lengths = np.diff(rp).astype(np.float64)
    nnz = float(rp[-1] - rp[0])
    mean = nnz / n if n > 0 else 0.0
    var = float(np.mean((lengths - mean) ** 2)) if n > 0 else 0.0
    mx = float(lengths.max()) if n > 0 else 0.0
    f = [math.log2(n) if n > 0 else 0.0, math.log2(nnz) if nnz > 0 else 0.0, mean,
         math.log2(1.0 + var), math.log2(mx) if mx > 0 else 0.0]
    return np.asarray(f, dtype=np.float64).astype(np.float32)


# --------------------------------------------------------------------------
# Variants (Sec. 3.1, ``variants`` clause range [BEGIN:END:STEP] and
# ``model_output``)
# --------------------------------------------------------------------------

def expand_range(begin: float, end: float, step: float) -> list:
    """Values begin, begin+step, ... up to end inclusive.  The count is
    floor((end-begin)/step + 0.5) + 1 and value i is begin + i*step
    (computed from i, never accumulated)."""
    if step == 0 or (end - begin) / step < 0:
        raise ValueError("empty or non-terminating range")
    count = int(math.floor((end - begin) / step + 0.5)) + 1
    return [begin + i * step for i in range(count)]


# --------------------------------------------------------------------------
# Exploration and train trigger (Sec. 2 Apollo: RoundRobin cycling of
# policies, training once enough unique samples exist; Sec. 3.1 default
# min_train_data = number of variants; Sec. 3.3 training is triggered at the
# end of a region execution)
# --------------------------------------------------------------------------

class RoundRobinExplorer:
    """Before training, the k-th execution runs policy k mod V.  A sample is
    unique on its (features, variant) pair.  Training fires at the end of the
    execution that brings the unique count to min_train (<= 0 means V)."""

    def __init__(self, num_variants: int, min_train: int = 0):
        self.V = num_variants
        self.min_train = min_train if min_train > 0 else num_variants
        self.k = 0
        self.unique = set()
        self.trained = False

    def step(self, features) -> tuple:
        """One region execution; returns (variant run, whether training fired)."""
        assert not self.trained
        v = self.k % self.V
        self.k += 1
        self.unique.add((tuple(np.asarray(features, dtype=np.float32).tolist()), v))
        fire = len(self.unique) >= self.min_train
        if fire:
            self.trained = True
        return v, fire


# --------------------------------------------------------------------------
# Exhaustive selector (Sec. 2 Apollo: the fastest policy per feature tuple
# is the label)
# --------------------------------------------------------------------------

def exhaustive_select(times) -> tuple:
    """times[V][R] seconds of R timed runs per variant (NaN = variant
    unavailable).  Returns (best variant, medians): best = argmin of the
    median, ties to the lowest id."""
    medians = []
    for row in times:
        row = [t for t in row if not math.isnan(t)]
        medians.append(float(np.median(row)) if row else math.inf)
    best = 0
    for v in range(1, len(medians)):
        if medians[v] < medians[best]:
            best = v
    return best, medians


def regret(t_selected: float, t_best: float) -> float:
    """Relative regret t_sel / t_best - 1, both from the same timing table."""
    return t_selected / t_best - 1.0


# --------------------------------------------------------------------------
# MLP cost model, FP64.  The paper trains a classifier on fastest-policy
# labels (Sec. 2, Sec. 3.1 model_type); here a regressor predicts ln(time)
# of every variant and its argmin is the label.  Readings: z-scored inputs,
# 2 hidden ReLU layers of 64, 12 outputs, masked MSE on the measured
# variant, Adam, He-uniform init.
# --------------------------------------------------------------------------

N_IN, N_H, N_OUT = 6, 64, 12
SHAPES = OrderedDict([("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
                      ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))])
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES.values())  # 5388


def mlp_unflatten(theta) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for k, s in SHAPES.items():
        n = int(np.prod(s))
        out[k] = theta[o:o + n].reshape(s)
        o += n
    return out


def mlp_flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1) for k in SHAPES])


def mlp_init(seed: int) -> np.ndarray:
    """He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)), zero biases.
    Uniforms: SplitMix64 stream ``seed`` drawn in flat parameter order
    (W1, W2, W3 rows, x fastest), u in [0,1) mapped to 2u-1."""
    import synth
    p = {}
    draws = synth.u01(seed, N_H * N_IN + N_H * N_H + N_OUT * N_H)
    o = 0
    for k, s in SHAPES.items():
        if k.startswith("W"):
            n = int(np.prod(s))
            bound = math.sqrt(6.0 / s[1])
            p[k] = ((2.0 * draws[o:o + n] - 1.0) * bound).reshape(s)
            o += n
        else:
            p[k] = np.zeros(s)
    return mlp_flatten(p)


def mlp_forward(theta, X) -> tuple:
    """X [B, 6] already normalised.  Returns (outputs [B, 12], cache)."""
    p = mlp_unflatten(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (X, z1, h1, z2, h2)


def mlp_loss(theta, X, y, mask) -> float:
    """Masked MSE: 0.5 / B * sum_b sum_v mask[b,v] (o[b,v] - y[b])^2."""
    o, _ = mlp_forward(theta, X)
    B = o.shape[0]
    d = (o - np.asarray(y, dtype=np.float64)[:, None]) * mask
    return 0.5 * float(np.sum(d * d)) / B


def mlp_grad(theta, X, y, mask) -> tuple:
    """Analytic gradient of mlp_loss (ReLU derivative taken as [z > 0])."""
    p = mlp_unflatten(theta)
    o, (X, z1, h1, z2, h2) = mlp_forward(theta, X)
    B = o.shape[0]
    mask = np.asarray(mask, dtype=np.float64)
    dO = (o - np.asarray(y, dtype=np.float64)[:, None]) * mask / B
    g = {}
    g["W3"] = dO.T @ h2
    g["b3"] = dO.sum(axis=0)
    dh2 = dO @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    loss = 0.5 * float(np.sum(((o - np.asarray(y)[:, None]) * mask) ** 2)) / B
    return mlp_flatten(g), loss


def adam_step(theta, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> tuple:
    """One Adam update (Kingma and Ba 2015), step count t >= 1, bias-corrected."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def build_dataset(records, num_variants: int) -> dict:
    """Training set from profiling records (features, variant, seconds).
    Duplicate (features, variant) pairs are merged by their median time, in
    order of first appearance.  Inputs are z-scored (population std floored
    at 1e-6, features beyond the region's count stay 0); the target is
    ln(seconds) minus its mean; the mask is one-hot on the measured variant."""
    groups = OrderedDict()
    for feats, var, sec in records:
        key = (tuple(np.asarray(feats, dtype=np.float32).tolist()), int(var))
        groups.setdefault(key, []).append(float(sec))
    keys = list(groups.keys())
    F = np.zeros((len(keys), N_IN))
    for i, (f, _) in enumerate(keys):
        F[i, :len(f)] = f
    var = np.array([k[1] for k in keys], dtype=np.int64)
    t = np.array([float(np.median(groups[k])) for k in keys])
    mu = F.mean(axis=0)
    sd = np.maximum(F.std(axis=0), 1e-6)
    X = (F - mu) / sd
    lt = np.log(t)
    y_mean = float(lt.mean())
    mask = np.zeros((len(keys), N_OUT))
    mask[np.arange(len(keys)), var] = 1.0
    return {"X": X, "y": lt - y_mean, "mask": mask, "mu": mu, "sd": sd, "y_mean": y_mean,
            "variant": var, "features": F, "seconds": t, "V": num_variants}


def epoch_permutation(count: int, seed: int, epoch: int) -> np.ndarray:
    """Shuffle of epoch e: indices ordered by SplitMix64 keys of sub-stream
    e of ``seed`` (stable on equal keys)."""
    import synth
    keys = synth.splitmix64(synth.substream(seed, epoch & 0xFF) ^ (epoch >> 8), count)
    return np.argsort(keys, kind="stable")


def mlp_train(ds: dict, seed: int = 7, epochs: int = 200, batch: int = 256, lr: float = 1e-3) -> tuple:
    """Mini-batch Adam over ds; the last batch of an epoch may be short.
    Returns (theta, final epoch mean loss)."""
    theta = mlp_init(seed)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    n = ds["X"].shape[0]
    last = math.nan
    for e in range(epochs):
        perm = epoch_permutation(n, seed, e)
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            g, loss = mlp_grad(theta, ds["X"][idx], ds["y"][idx], ds["mask"][idx])
            t += 1
            theta, m, v = adam_step(theta, g, m, v, t, lr=lr)
            tot += loss * idx.size
        last = tot / n
    return theta, last


def mlp_select(theta, ds_or_norm: dict, features, num_variants: int) -> int:
    """argmin over v < V of the predicted ln-time, ties to the lowest id."""
    f = np.zeros(N_IN)
    feats = np.asarray(features, dtype=np.float64)
    f[:feats.size] = feats
    x = (f - ds_or_norm["mu"]) / ds_or_norm["sd"]
    o, _ = mlp_forward(theta, x[None, :])
    o = o[0, :num_variants]
    best = 0
    for k in range(1, num_variants):
        if o[k] < o[best]:
            best = k
    return best


# --------------------------------------------------------------------------
# Decision-tree classifier (Sec. 3.1 model_type dtree; depth 2 in Sec. 4),
# the paper's own model: CART grown by minimising the weighted Gini impurity
# sum_child (n_child / n) * (1 - sum_k p_k^2), evaluated exactly with
# rationals; candidate thresholds halfway between consecutive distinct
# values (computed in double from the float32 features); ties to the lower
# feature index, then the lower threshold; growth stops at the depth limit
# or on a pure node.  Labels: fastest variant per feature tuple (Sec. 2).
# --------------------------------------------------------------------------

def label_records(records, num_variants: int):
    """(features, variant, seconds) records -> (feature tuples, labels): per
    distinct float32 feature tuple, in order of first appearance, the
    variant with the lowest median time (ties to the lowest id)."""
    groups = OrderedDict()
    for feats, var, sec in records:
        key = tuple(float(v) for v in np.asarray(feats, dtype=np.float32).tolist())
        groups.setdefault(key, [[] for _ in range(num_variants)])[int(var)].append(float(sec))
    X, y = [], []
    for key, per in groups.items():
        med = [float(np.median(t)) if t else math.inf for t in per]
        best = 0
        for v in range(1, num_variants):
            if med[v] < med[best]:
                best = v
        X.append(list(key))
        y.append(best)
    return X, y


def _gini_weighted(groups, num_classes):
    from fractions import Fraction
    n = sum(len(g) for g in groups)
    total = Fraction(0)
    for g in groups:
        if not g:
            continue
        imp = Fraction(1) - sum(Fraction(sum(1 for c in g if c == k), len(g)) ** 2
                                for k in range(num_classes))
        total += Fraction(len(g), n) * imp
    return total


def dtree_fit(X, y, depth: int, num_classes: int) -> dict:
    """Grow the tree; nodes are dicts {feature (-1 = leaf), threshold, left,
    right, counts}."""
    X = [[float(np.float32(v)) for v in row] + [0.0] * (N_IN - len(row)) for row in X]

    def build(idx, d):
        counts = [sum(1 for i in idx if y[i] == k) for k in range(num_classes)]
        node = {"feature": -1, "threshold": 0.0, "left": None, "right": None, "counts": counts}
        if d >= depth or sum(1 for c in counts if c > 0) <= 1 or len(idx) < 2:
            return node
        best = None
        for f in range(N_IN):
            vals = sorted(set(X[i][f] for i in idx))
            for a, b in zip(vals, vals[1:]):
                thr = 0.5 * (a + b)
                left = [y[i] for i in idx if X[i][f] <= thr]
                right = [y[i] for i in idx if X[i][f] > thr]
                g = _gini_weighted([left, right], num_classes)
                if best is None or g < best[0]:
                    best = (g, f, thr)
        if best is None:
            return node
        _, f, thr = best
        node["feature"], node["threshold"] = f, thr
        node["left"] = build([i for i in idx if X[i][f] <= thr], d + 1)
        node["right"] = build([i for i in idx if X[i][f] > thr], d + 1)
        return node

    return build(list(range(len(X))), 0)


def dtree_predict(tree: dict, features, allowed=None) -> int:
    """Leaf majority among allowed classes (ties to the lowest id)."""
    f = [float(np.float32(v)) for v in features] + [0.0] * (N_IN - len(features))
    node = tree
    while node["feature"] >= 0:
        node = node["left"] if f[node["feature"]] <= node["threshold"] else node["right"]
    best = -1
    for k, c in enumerate(node["counts"]):
        if (allowed is None or k in allowed) and c > 0 and (best < 0 or c > node["counts"][best]):
            best = k
    return best


# --------------------------------------------------------------------------
# Evaluation protocol (Sec. 4, CPU-GPU execution): inputs are split into K
# equal groups, a fraction of the groups trains and the rest tests, each
# input trained on and tested at least once, the split redrawn from a
# shuffled order.  Reading: reshuffle r orders the inputs by SplitMix64
# keys of substream(seed, 40 + r) (ties by index), group g takes the order's
# positions [g*Q//K, (g+1)*Q//K), and m training groups rotate as groups
# t, t+1, ..., t+m-1 (mod K) for t = 0..K-1.
# --------------------------------------------------------------------------

def kfold_groups(count: int, k: int, seed: int, reshuffle: int) -> list:
    import synth
    keys = [int(v) for v in synth.splitmix64(synth.substream(seed, 40 + reshuffle), count)]
    order = [i for _, i in sorted((keys[i], i) for i in range(count))]
    groups = []
    for g in range(k):
        lo, hi = g * count // k, (g + 1) * count // k
        groups.append(order[lo:hi])
    return groups


def rotations(k: int, m: int) -> list:
    out = []
    for t in range(k):
        out.append(sorted((t + d) % k for d in range(m)))
    return out


def online_choice(explored_seconds) -> int:
    """Online comparator (Sec. 4, GPU threads): after one exploration run of
    every variant on a single input, a model trained on those samples picks
    the fastest measured variant (ties to the lowest id)."""
    best = 0
    for v in range(1, len(explored_seconds)):
        if explored_seconds[v] < explored_seconds[best]:
            best = v
    return best
