"""GPU tests of the Gram-matrix (MFMA) similarity builds against the FP64 oracle.

Error bounds are derived from each build's arithmetic (u = 2^-24, FP32 unit roundoff):
  GEMM FP32   S = -((n_i + n_j) - 2 g): FP32 rounding of the norms, of the d-term dot product
              and of the combination: |dS| <= (d + 4) u (n_i + n_j).
  BF16        coordinates rounded to BF16 (8 significant bits: relative error <= 2^-8), norms
              of the rounded points: S is the FP32 distance of the rounded points, so
              |dS| <= 2 |x_i - x_j| |d_i - d_j| + |d_i - d_j|^2 + (d + 4) u (n_i + n_j),
              with |d_i| <= 2^-8 |x_i|.
  BF16x3      x = hi + lo + r, |x - hi| <= 2^-8 |x|, |r| <= 2^-8 |x - hi| <= 2^-16 |x|.  With the
              norms n^_i = sum(hi^2 + 2 hi lo) the build gives exactly
              -|x^_i - x^_j|^2 + |lo_i - lo_j|^2 (x^ = hi + lo) before FP32 rounding, so
              |dS| <= 2 dist 2^-16 (|x_i| + |x_j|) + 2^-16 (|x_i| + |x_j|)^2 (1 + 2^-15)
                      + (3d + 4) u (n_i + n_j).
  GEMM FP64   (d + 4) 2^-53 (n_i + n_j).
"""
import numpy as np
import pytest
import torch

from oracle import similarity as sim
from paper_1403_7394_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24


def _build(hap, X, mode, dtype=torch.float32):
    n = X.shape[0]
    S = torch.full((n, n + 4), 5.0, dtype=dtype, device=DEV)
    hap.build_similarity(X, S[:, :n], mode=mode)
    out = S.cpu().numpy()
    assert np.all(out[:, n:] == 5.0)   # columns past n untouched
    return out[:, :n]


@pytest.mark.parametrize("n,d,seed", [(1000, 64, 1), (257, 33, 2), (130, 5, 3), (64, 2, 4)])
def test_gram_builds_within_derived_bounds(hap_gpu, n, d, seed):
    b = synth.gaussian_blobs(seed, n, d, 7, centre="normal", centre_scale=2.0, sigma_lo=1.0, sigma_hi=1.0,
                             sizes="multinomial", dtype=np.float32)
    X64 = b.X.astype(np.float64)
    ref = sim.similarity(X64)
    nrm = np.sum(X64 * X64, axis=1)
    norm_sum = nrm[:, None] + nrm[None, :]
    xn = np.sqrt(nrm)
    X = torch.from_numpy(b.X).to(DEV)
    dist = np.sqrt(-ref)

    got = _build(hap_gpu, X, hap_gpu.BUILD_GEMM)
    assert np.all(np.abs(got - ref) <= (d + 4) * U32 * norm_sum + 1e-30)

    got = _build(hap_gpu, X, hap_gpu.BUILD_BF16)
    dlt = 2.0 ** -8 * (xn[:, None] + xn[None, :])
    assert np.all(np.abs(got - ref) <= 2 * dist * dlt + dlt ** 2 + (d + 4) * U32 * norm_sum)

    got3 = _build(hap_gpu, X, hap_gpu.BUILD_BF16X3)
    xs = xn[:, None] + xn[None, :]
    bound3 = 2 * dist * 2.0 ** -16 * xs + 2.0 ** -16 * xs ** 2 * (1 + 2.0 ** -15) + (3 * d + 4) * U32 * norm_sum
    assert np.all(np.abs(got3 - ref) <= bound3)
    # the split-precision build is much closer than a single BF16 pass
    assert np.max(np.abs(got3 - ref)) < np.max(np.abs(got - ref)) / 16

    X64t = torch.from_numpy(X64).to(DEV)
    got64 = _build(hap_gpu, X64t, hap_gpu.BUILD_GEMM, torch.float64)
    assert np.all(np.abs(got64 - ref) <= (d + 4) * 2.0 ** -53 * norm_sum)

    for g in (got, got3, got64):
        assert np.all(np.diag(g) == 0) and np.all(g <= 0)


def test_gemm_build_f64_with_noise_within_bound(hap_gpu):
    """The FP64 GEMM build adds the counter-based tie-break noise: within the FP64 GEMM bound
    (plus the noise of that rounding difference) of the oracle's noised similarity."""
    b = synth.small_blobs(9, 200, k=3)
    X64 = b.X.astype(np.float64)
    X = torch.from_numpy(X64).to(DEV)
    S1 = torch.empty((200, 200), dtype=torch.float64, device=DEV)
    hap_gpu.build_similarity(X, S1, mode=hap_gpu.BUILD_GEMM, noise_rel=1e-6, seed=5)
    ref = sim.add_noise(sim.similarity(X64), 1e-6, 5)
    nrm = np.sum(X64 * X64, axis=1)
    bound = (2 + 4) * 2.0 ** -53 * (nrm[:, None] + nrm[None, :]) * (1 + 2e-6)
    assert np.all(np.abs(S1.cpu().numpy() - ref) <= bound)
    # and the noise is there: the noise-free build differs by about 1e-6 relative
    S0 = torch.empty_like(S1)
    hap_gpu.build_similarity(X, S0, mode=hap_gpu.BUILD_GEMM)
    rel = np.abs(S1.cpu().numpy() - S0.cpu().numpy()) / np.maximum(np.abs(ref), 1e-300)
    off = ~np.eye(200, dtype=bool)
    assert 0.3e-6 < np.median(rel[off]) < 0.7e-6


def test_full_size_builds_on_sampled_rows(hap_gpu):
    """The precision workload at its full size (32768 points, d = 64): every build mode, on
    sampled rows against the FP64 oracle's rows, within the bounds above; the whole matrix
    has a zero diagonal and no positive entry."""
    b, _ = synth.workload_precision()
    n, d = b.X.shape
    X64 = b.X.astype(np.float64)
    X = torch.from_numpy(b.X).to(DEV)
    rows = np.array([0, 1, 127, 128, 4095, 16384, 32766, 32767])
    ref = sim.similarity_rows(X64, rows)
    nrm = np.sum(X64 * X64, axis=1)
    norm_sum = nrm[rows][:, None] + nrm[None, :]
    xn = np.sqrt(nrm)
    xs = xn[rows][:, None] + xn[None, :]
    dist = np.sqrt(-ref)
    S = torch.empty((n, n), dtype=torch.float32, device=DEV)
    ridx = torch.from_numpy(rows).to(DEV)
    for mode, bound in (
            (hap_gpu.BUILD_DIRECT, None),
            (hap_gpu.BUILD_GEMM, (d + 4) * U32 * norm_sum),
            (hap_gpu.BUILD_BF16, 2 * dist * 2.0 ** -8 * xs + (2.0 ** -8 * xs) ** 2 + (d + 4) * U32 * norm_sum),
            (hap_gpu.BUILD_BF16X3, 2 * dist * 2.0 ** -16 * xs + 2.0 ** -16 * xs ** 2 * (1 + 2.0 ** -15)
             + (3 * d + 4) * U32 * norm_sum)):
        S.fill_(1.0)
        hap_gpu.build_similarity(X, S, mode=mode)
        got = S[ridx].cpu().numpy().astype(np.float64)
        if bound is None:
            assert np.array_equal(got, ref.astype(np.float32).astype(np.float64)), mode
        else:
            assert np.all(np.abs(got - ref) <= bound), mode
        assert float(S.max()) <= 0.0 and bool(torch.all(torch.diagonal(S) == 0)), mode
    del S
    torch.cuda.empty_cache()
