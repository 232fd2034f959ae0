"""Seeded synthetic inputs for HAP (Gaussian point blobs, small integer matrices, initial
perceptron parameters and minibatch orders for the warm start).

This module only draws random numbers; it holds none of the method's arithmetic
(no similarity, no preference, no message update).  The oracle side and the HIP
side both take their inputs from here and from nowhere else.

The paper clusters image pixels and a 788-point 2-D shape set (Section 4); none
of those datasets is used here.  Gaussian blobs of the sizes below stand in for
them.  All draws use numpy ``Generator(PCG64(seed))`` in float64; the point
matrix is then cast to the run dtype and that cast matrix is the canonical
input for every party.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Blobs:
    X: np.ndarray            # (n, d) points in the run dtype
    truth: np.ndarray        # (n,) generating blob id of every point (int32)
    seed: int
    meta: dict = field(default_factory=dict)


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_blobs(seed, n: int, d: int, k: int, *, centre: str, centre_scale: float,
                   sigma_lo: float, sigma_hi: float, sizes: str, dtype=np.float32,
                   shuffle: bool = True) -> Blobs:
    """Draw n points in d dimensions from k isotropic Gaussian blobs.

    centre='uniform': centres ~ U[-centre_scale, centre_scale]^d.
    centre='normal':  centres ~ N(0, centre_scale^2 I).
    sigma per blob ~ U[sigma_lo, sigma_hi] (equal bounds give a fixed sigma).
    sizes='equal': n/k points each (n must divide); 'multinomial': Multinomial(n, 1/k).
    Draw order is fixed: centres, sigmas, sizes, unit normals, shuffle.
    """
    rng = _rng(seed)
    if centre == "uniform":
        C = rng.uniform(-centre_scale, centre_scale, size=(k, d))
    elif centre == "normal":
        C = rng.standard_normal(size=(k, d)) * centre_scale
    else:
        raise ValueError(centre)
    sig = rng.uniform(sigma_lo, sigma_hi, size=k) if sigma_hi > sigma_lo else np.full(k, float(sigma_lo))
    if sizes == "equal":
        if n % k:
            raise ValueError("equal sizes need k | n")
        cnt = np.full(k, n // k, dtype=np.int64)
    elif sizes == "multinomial":
        cnt = rng.multinomial(n, np.full(k, 1.0 / k))
    else:
        raise ValueError(sizes)
    truth = np.repeat(np.arange(k, dtype=np.int32), cnt)
    Z = rng.standard_normal(size=(n, d))
    X = C[truth] + Z * sig[truth][:, None]
    if shuffle:
        perm = rng.permutation(n)
        X, truth = X[perm], truth[perm]
    return Blobs(X=np.ascontiguousarray(X.astype(dtype)), truth=truth, seed=int(seed) if not isinstance(seed, np.random.SeedSequence) else -1,
                 meta=dict(n=n, d=d, k=k, centre=centre, centre_scale=centre_scale,
                           sigma=(sigma_lo, sigma_hi), sizes=sizes, dtype=np.dtype(dtype).name))


# ---------------------------------------------------------------------------
# Workload registry.  Each entry fixes the seed and every generator argument.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class RunParams:
    levels: int
    damping: float
    max_iters: int
    stable_iters: int        # 0 = run exactly max_iters
    dtype: str               # "f64" or "f32"
    noise_rel: float         # relative tie-break noise on off-diagonal S (0 = off)
    noise_seed: int


def workload_small_f64(seed: int = 1001) -> tuple[Blobs, RunParams]:
    """300 points in 2-D, 3 blobs of 100, centres U[-10,10]^2, sigma 1; FP64 with 1e-12 noise."""
    b = gaussian_blobs(seed, 300, 2, 3, centre="uniform", centre_scale=10.0, sigma_lo=1.0,
                       sigma_hi=1.0, sizes="equal", dtype=np.float64)
    return b, RunParams(levels=3, damping=0.5, max_iters=200, stable_iters=0, dtype="f64",
                        noise_rel=1e-12, noise_seed=seed)


def workload_plain_f32(seed: int = 1002, n: int = 8192) -> tuple[Blobs, RunParams]:
    """8192 points in 2-D, 64 blobs, centres U[-100,100]^2, sigma U[0.5,2], multinomial sizes; FP32."""
    b = gaussian_blobs(seed, n, 2, 64, centre="uniform", centre_scale=100.0, sigma_lo=0.5,
                       sigma_hi=2.0, sizes="multinomial", dtype=np.float32)
    return b, RunParams(levels=3, damping=0.9, max_iters=500, stable_iters=50, dtype="f32",
                        noise_rel=0.0, noise_seed=seed)


def workload_precision(seed: int = 1003, n: int = 32768) -> tuple[Blobs, RunParams]:
    """32768 points in 64-D, 256 blobs, centres N(0,4I), points centre+N(0,I); FP32 inputs."""
    b = gaussian_blobs(seed, n, 64, 256, centre="normal", centre_scale=2.0, sigma_lo=1.0,
                       sigma_hi=1.0, sizes="multinomial", dtype=np.float32)
    return b, RunParams(levels=4, damping=0.9, max_iters=300, stable_iters=0, dtype="f32",
                        noise_rel=0.0, noise_seed=seed)


def workload_batched(seed: int = 1004, count: int = 512, n_lo: int = 64, n_hi: int = 2048):
    """`count` independent instances: N ~ U{n_lo..n_hi}, d=16, k ~ U{4..32}, centres U[-10,10]^16, sigma 1."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for ss in children:
        r = _rng(ss)
        n = int(r.integers(n_lo, n_hi + 1))
        k = int(r.integers(4, 33))
        sub = r.integers(0, 2**63 - 1)
        out.append(gaussian_blobs(int(sub), n, 16, k, centre="uniform", centre_scale=10.0,
                                  sigma_lo=1.0, sigma_hi=1.0, sizes="multinomial", dtype=np.float32))
    return out, RunParams(levels=3, damping=0.8, max_iters=200, stable_iters=0, dtype="f32",
                          noise_rel=0.0, noise_seed=seed)


def workload_warm_eval(seed: int = 1005, n: int = 65536) -> tuple[Blobs, RunParams]:
    """65536 points in 32-D, 1024 blobs, centres N(0,4I), points centre+N(0,I); FP32."""
    b = gaussian_blobs(seed, n, 32, 1024, centre="normal", centre_scale=2.0, sigma_lo=1.0,
                       sigma_hi=1.0, sizes="multinomial", dtype=np.float32)
    return b, RunParams(levels=3, damping=0.9, max_iters=500, stable_iters=50, dtype="f32",
                        noise_rel=0.0, noise_seed=seed)


def workload_warm_train(k: int, rep: int, n: int = 8192) -> Blobs:
    """Training instances for the warm start: 2-D blobs, centres U[-10,10]^2, sigma 1."""
    seed = 2001 + 100 * rep + k
    return gaussian_blobs(seed, n, 2, k, centre="uniform", centre_scale=10.0, sigma_lo=1.0,
                          sigma_hi=1.0, sizes="multinomial", dtype=np.float32)


def rgb_pixels(seed: int, n: int, k: int = 16, sigma_lo: float = 4.0, sigma_hi: float = 20.0) -> Blobs:
    """n RGB pixels from k colour blobs: centres U[0,255]^3, sigma U[sigma_lo, sigma_hi] per
    blob, multinomial sizes, rounded to integer intensities and clipped to [0,255]; FP32."""
    b = gaussian_blobs(seed, n, 3, k, centre="uniform", centre_scale=127.5, sigma_lo=sigma_lo,
                       sigma_hi=sigma_hi, sizes="multinomial", dtype=np.float64)
    X = np.clip(np.rint(b.X + 127.5), 0.0, 255.0).astype(np.float32)
    return Blobs(X=np.ascontiguousarray(X), truth=b.truth, seed=seed, meta=dict(b.meta, kind="rgb"))


def random_preferences(seed: int, n: int, lo: float = -1e6, hi: float = 0.0) -> np.ndarray:
    """Per-point preferences U[lo, hi] (FP64)."""
    return _rng(seed).uniform(lo, hi, size=n)


def workload_image(which: str = "mandrill"):
    """Image-style workload: RGB pixels of the sizes of the paper's two images (103 x 103 and
    120 x 100) from 16 colour blobs, preferences U[-1e6, 0] per point, L = 3, damping 0.5,
    30 iterations (Section 4).  Returns (Blobs, preferences, RunParams)."""
    n, seed = {"mandrill": (103 * 103, 1006), "buttons": (120 * 100, 1007)}[which]
    b = rgb_pixels(seed, n)
    return b, random_preferences(seed + 50, n), RunParams(levels=3, damping=0.5, max_iters=30, stable_iters=0,
                                                          dtype="f32", noise_rel=0.0, noise_seed=seed)


def small_blobs(seed: int, n: int, d: int = 2, k: int = 4, dtype=np.float64, scale: float = 10.0) -> Blobs:
    """Generic small test input: k blobs, centres U[-scale,scale]^d, sigma 1, multinomial sizes."""
    return gaussian_blobs(seed, n, d, k, centre="uniform", centre_scale=scale, sigma_lo=1.0,
                          sigma_hi=1.0, sizes="multinomial", dtype=dtype)


def separated_blobs(seed: int, k: int = 3, m: int = 4, d: int = 2, sep: float = 100.0) -> Blobs:
    """k blobs of m points, sigma 1, centres on a line `sep` apart (well separated)."""
    rng = _rng(seed)
    C = np.zeros((k, d))
    C[:, 0] = sep * np.arange(k)
    truth = np.repeat(np.arange(k, dtype=np.int32), m)
    X = C[truth] + rng.standard_normal(size=(k * m, d))
    perm = rng.permutation(k * m)
    return Blobs(X=X[perm].copy(), truth=truth[perm].copy(), seed=seed, meta=dict(k=k, m=m, sep=sep))


def integer_matrix(seed: int, n: int, lo: int = -20, hi: int = -1) -> np.ndarray:
    """n x n matrix of integers drawn uniformly from [lo, hi] (float64 storage)."""
    rng = _rng(seed)
    return rng.integers(lo, hi + 1, size=(n, n)).astype(np.float64)


def integer_vector(seed: int, n: int, lo: int = -20, hi: int = -1) -> np.ndarray:
    rng = _rng(seed + 7919)
    return rng.integers(lo, hi + 1, size=n).astype(np.float64)


def mlp_init(seed: int, n_in: int, hidden: int, n_out: int) -> np.ndarray:
    """Initial perceptron parameters as one flat FP32 vector (W1, b1, W2, b2, W3, b3; weights
    row-major): weights N(0, 2/fan_in), biases 0."""
    rng = _rng(seed)
    parts = []
    for fan_in, fan_out in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        parts.append(rng.standard_normal(fan_in * fan_out) * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def minibatch_order(seed: int, rows: int, batch: int, steps: int) -> np.ndarray:
    """Row indices for `steps` minibatches of `batch` rows (int32): concatenated random
    permutations of range(rows), one per pass over the data."""
    rng = _rng(seed)
    need = batch * steps
    out = []
    while sum(len(o) for o in out) < need:
        out.append(rng.permutation(rows))
    return np.concatenate(out)[:need].astype(np.int32)
